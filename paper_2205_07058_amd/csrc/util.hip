// Elementwise training utilities: Adam (the optimiser SVLF trains with,
// section 4.5), FP32 -> bfloat16 copies of parameters, fills, and the
// deterministic reduction of per-block MLP-gradient partial sums.
#include <hip/hip_runtime.h>

#include <mutex>

#include "svlf_internal.hpp"

// The workspace of svlf_train_step_noalloc: a file-scope device array, one
// copy per device the library runs on, held until the process ends.  Host
// code never uses this name as an address (on the host it is a stand-in
// symbol); it takes the device address from hipGetSymbolAddress, once per
// device, in noalloc_scratch below.
static __device__ __align__(256) char scratch[SVLF_NOALLOC_SCRATCH_BYTES];

namespace svlf {
namespace {

constexpr int kThreads = 256;

// Round-to-nearest-even FP32 -> bfloat16 bits with gfx950's conversion
// instruction, the same one the shading kernels use for their operands (a
// NaN gives a quiet NaN).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
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
#pragma clang fp contract(off)   // the same rounding in every path (no fused multiply-adds)
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

// The same update, four consecutive parameters per thread (16-byte loads
// and stores; identical arithmetic per element).
__global__ __launch_bounds__(kThreads) void k_adam4(float4* __restrict__ p, float4* __restrict__ g,
                                                    float4* __restrict__ m, float4* __restrict__ v,
                                                    int64_t n4, float lr, float b1, float b2,
                                                    float eps, float bc1, float bc2,
                                                    uint2* __restrict__ bf, int zero) {
#pragma clang fp contract(off)   // the same rounding in every path (no fused multiply-adds)
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n4; i += stride) {
    const float4 gi = g[i];
    float4 mi = m[i], vi = v[i], pi = p[i];
    float* mf = &mi.x;
    float* vf = &vi.x;
    float* pf = &pi.x;
    const float* gf = &gi.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      mf[c] = b1 * mf[c] + (1.0f - b1) * gf[c];
      vf[c] = b2 * vf[c] + (1.0f - b2) * gf[c] * gf[c];
      pf[c] = pf[c] - lr * (mf[c] / bc1) / (sqrtf(vf[c] / bc2) + eps);
    }
    m[i] = mi;
    v[i] = vi;
    p[i] = pi;
    if (bf) {
      uint2 b;
      b.x = static_cast<uint32_t>(bf16_bits(pi.x)) | (static_cast<uint32_t>(bf16_bits(pi.y)) << 16);
      b.y = static_cast<uint32_t>(bf16_bits(pi.z)) | (static_cast<uint32_t>(bf16_bits(pi.w)) << 16);
      bf[i] = b;
    }
    if (zero) g[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

// Lazy (row-sparse) Adam: rows of `L4` float4 groups (row length 4*L4
// floats); a row is updated, and its gradient cleared, only if some entry of
// its gradient is nonzero; other rows (their moments included) are left
// untouched.  Bias corrections use the global step.  Each row is handled by
// L4 consecutive lanes of one wave, 64/L4 rows per wave per iteration.
__global__ __launch_bounds__(kThreads) void k_lazy_adam(float4* __restrict__ p,
                                                        float4* __restrict__ g,
                                                        float4* __restrict__ m,
                                                        float4* __restrict__ v, int64_t n_rows,
                                                        int L4, float lr, float b1, float b2,
                                                        float eps, float bc1, float bc2,
                                                        uint2* __restrict__ bf, int zero) {
#pragma clang fp contract(off)   // the same rounding in every path (no fused multiply-adds)
  const int lane = threadIdx.x & 63;
  const int rpw = 64 / L4;
  const int grp = lane / L4;
  const int sub = lane - grp * L4;
  const unsigned long long gmask =
      (L4 == 64 ? ~0ull : ((1ull << L4) - 1ull)) << (grp < rpw ? grp * L4 : 0);
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x) >> 6;
  const int64_t n_waves = (static_cast<int64_t>(gridDim.x) * kThreads) >> 6;
  for (int64_t r0 = wave * rpw; r0 < n_rows; r0 += n_waves * rpw) {
    const int64_t r = r0 + grp;
    const bool ok = grp < rpw && r < n_rows;
    const int64_t i = r * L4 + sub;
    float4 gi = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ok) gi = g[i];
    const bool nz = ok && (gi.x != 0.0f || gi.y != 0.0f || gi.z != 0.0f || gi.w != 0.0f);
    const unsigned long long any = __ballot(nz);
    if (!ok || (any & gmask) == 0ull) continue;
    float4 mi = m[i], vi = v[i], pi = p[i];
    float* mf = &mi.x;
    float* vf = &vi.x;
    float* pf = &pi.x;
    const float* gf = &gi.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      mf[c] = b1 * mf[c] + (1.0f - b1) * gf[c];
      vf[c] = b2 * vf[c] + (1.0f - b2) * gf[c] * gf[c];
      pf[c] = pf[c] - lr * (mf[c] / bc1) / (sqrtf(vf[c] / bc2) + eps);
    }
    m[i] = mi;
    v[i] = vi;
    p[i] = pi;
    if (bf) {
      uint2 b;
      b.x = static_cast<uint32_t>(bf16_bits(pi.x)) | (static_cast<uint32_t>(bf16_bits(pi.y)) << 16);
      b.y = static_cast<uint32_t>(bf16_bits(pi.z)) | (static_cast<uint32_t>(bf16_bits(pi.w)) << 16);
      bf[i] = b;
    }
    if (zero) g[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
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
// Sum of `rows` per-block partial vectors (row-major [rows][n]) into out.
// A block owns 64 columns; thread (column, quarter) sums its quarter of the
// rows in order, the four quarter sums are then added in order: a fixed
// summation order for any launch.  Block 0 also sums the loss partials.
constexpr int kRedCols = 64;
__global__ __launch_bounds__(kThreads) void k_reduce(const float* __restrict__ part, int rows,
                                                     int64_t n, float* __restrict__ out,
                                                     const float* __restrict__ lp,
                                                     float* __restrict__ loss_out) {
  __shared__ float q[kThreads];
  const int t = threadIdx.x, col = t % kRedCols, qt = t / kRedCols;
  constexpr int NQ = kThreads / kRedCols;
  const int r0 = static_cast<int>(static_cast<int64_t>(rows) * qt / NQ);
  const int r1 = static_cast<int>(static_cast<int64_t>(rows) * (qt + 1) / NQ);
  for (int64_t c0 = static_cast<int64_t>(blockIdx.x) * kRedCols; c0 < n;
       c0 += static_cast<int64_t>(gridDim.x) * kRedCols) {
    const int64_t j = c0 + col;
    float s = 0.0f;
    if (j < n) {
#pragma unroll 8
      for (int r = r0; r < r1; ++r) s += part[static_cast<int64_t>(r) * n + j];
    }
    q[t] = s;
    __syncthreads();
    if (qt == 0 && j < n) {
      float tot = q[col];
#pragma unroll
      for (int k = 1; k < NQ; ++k) tot += q[k * kRedCols + col];
      out[j] += tot;
    }
    __syncthreads();
  }
  if (loss_out != nullptr && blockIdx.x == 0) {
    float s = 0.0f;
    for (int r = t; r < rows; r += kThreads) s += lp[r];
    q[t] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (t < w) q[t] += q[t + w];
      __syncthreads();
    }
    if (t == 0) *loss_out = q[0];
  }
}

}  // namespace

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2, uint16_t* bf16, int zero,
                       hipStream_t s) {
  const auto a16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
  const bool vec = n % 4 == 0 && a16(p) && a16(g) && a16(m) && a16(v) &&
                   (bf16 == nullptr || (reinterpret_cast<uintptr_t>(bf16) & 7u) == 0);
  if (vec) {
    hipLaunchKernelGGL(k_adam4, dim3(grid_for(n / 4)), dim3(kThreads), 0, s,
                       reinterpret_cast<float4*>(p), reinterpret_cast<float4*>(g),
                       reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n / 4, lr, b1,
                       b2, eps, bc1, bc2, reinterpret_cast<uint2*>(bf16), zero);
  } else {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(kThreads), 0, s, p, g, m, v, n, lr, b1, b2,
                       eps, bc1, bc2, bf16, zero);
  }
  return hipGetLastError();
}

hipError_t launch_lazy_adam(float* p, float* g, float* m, float* v, int64_t n_rows, int row_len,
                            float lr, float b1, float b2, float eps, float bc1, float bc2,
                            uint16_t* bf16, int zero, hipStream_t s) {
  const int L4 = row_len / 4;
  const int64_t rows_per_block = (kThreads / 64) * (64 / L4);
  int64_t blocks = (n_rows + rows_per_block - 1) / rows_per_block;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_lazy_adam, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s,
                     reinterpret_cast<float4*>(p), reinterpret_cast<float4*>(g),
                     reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n_rows, L4, lr,
                     b1, b2, eps, bc1, bc2, reinterpret_cast<uint2*>(bf16), zero);
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
  int64_t blocks = (n + kRedCols - 1) / kRedCols;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_reduce, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s, partials,
                     rows, n, out, loss_partials, loss_out);
  return hipGetLastError();
}

// Device address of this device's scratch array, looked up on the first
// call with that device current and kept per device.
hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* dev_ptr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (dev_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    dev_ptr[dev] = p;
  }
  *ptr = dev_ptr[dev];
  return hipSuccess;
}

}  // namespace svlf
