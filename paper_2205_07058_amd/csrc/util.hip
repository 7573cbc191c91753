// Elementwise training utilities: Adam (the optimiser SVLF trains with,
// section 4.5), FP32 -> bfloat16 copies of parameters, fills, and the
// deterministic reduction of per-block MLP-gradient partial sums.
#include <hip/hip_runtime.h>

#include "svlf_internal.hpp"

namespace svlf {
namespace {

constexpr int kThreads = 256;

// Round-to-nearest-even FP32 -> bfloat16 bits (NaN kept quiet).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 65536) b = 65536;
  return static_cast<int>(b < 1 ? 1 : b);
}

__global__ __launch_bounds__(kThreads) void k_adam(float* __restrict__ p, float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2,
                                                   uint16_t* __restrict__ bf, int zero) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (bf) bf[i] = bf16_bits(pi);
    if (zero) g[i] = 0.0f;
  }
}

__global__ __launch_bounds__(kThreads) void k_to_bf16(const float* __restrict__ s,
                                                      uint16_t* __restrict__ d, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride)
    d[i] = bf16_bits(s[i]);
}

__global__ __launch_bounds__(kThreads) void k_fill(float* __restrict__ d, float v, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride)
    d[i] = v;
}

// out[j] += sum over rows r (in order) of partials[r][j]; loss_out = sum of
// loss partials.  Fixed order: deterministic.
__global__ __launch_bounds__(kThreads) void k_reduce(const float* __restrict__ part, int rows,
                                                     int64_t n, float* __restrict__ out,
                                                     const float* __restrict__ lp,
                                                     float* __restrict__ loss_out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; j < n; j += stride) {
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += part[static_cast<int64_t>(r) * n + j];
    out[j] += s;
  }
  if (loss_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += lp[r];
    *loss_out = s;
  }
}

}  // namespace

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2, uint16_t* bf16, int zero,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(kThreads), 0, s, p, g, m, v, n, lr, b1, b2,
                     eps, bc1, bc2, bf16, zero);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(kThreads), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill(float* dst, float v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, dst, v, n);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* partials, int rows, int64_t n, float* out,
                                  const float* loss_partials, float* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(grid_for(n)), dim3(kThreads), 0, s, partials, rows, n, out,
                     loss_partials, loss_out);
  return hipGetLastError();
}

}  // namespace svlf
