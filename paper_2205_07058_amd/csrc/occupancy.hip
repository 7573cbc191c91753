// Occupied leaves from depth maps (SVLF section 4.1: the octree keeps the
// voxels that contain a surface, found from the dataset's depth).
//
// For every ray with a finite target depth t > 0 the surface point
// p = o + t d is computed in binary32 (a rounded product, then a rounded
// sum, no fused multiply-add) and its cell is floor(RN(p + 1) 2^(L-1)) per
// axis; points outside the grid are dropped.  Cells are marked in a bitmap
// indexed by Morton code (so the compacted list comes out in leaf-id
// order), then compacted: per-block bit counts, one exclusive scan over the
// blocks, and an emit pass that writes each set bit's cell coordinates.
#include <hip/hip_runtime.h>

#include "svlf_internal.hpp"

namespace svlf {
namespace {

constexpr int kThreads = 256;
constexpr int kBitsPerBlock = kThreads * 32;

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  // bit b of v -> bit 3b (v < 2^10)
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x3FFu;
  return v;
}

__global__ __launch_bounds__(kThreads) void k_mark(const float* __restrict__ o,
                                                  const float* __restrict__ d,
                                                  const float* __restrict__ t, int64_t n, int level,
                                                  uint32_t* __restrict__ bitmap) {
#pragma clang fp contract(off)
  // (the surface point must round the product and the sum separately)
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (r >= n) return;
  const float tr = t[r];
  if (!(tr > 0.0f) || !isfinite(tr)) return;
  const float scale = __int_as_float((126 + level) << 23);    // 2^(level-1)
  const float side = static_cast<float>(1 << level);
  uint32_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float p = o[3 * r + a] + tr * d[3 * r + a];
    const float q = (p + 1.0f) * scale;
    if (!(q >= 0.0f && q < side)) return;                     // also drops NaN
    c[a] = static_cast<uint32_t>(q);                          // floor of q >= 0
  }
  const uint32_t m = spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
  atomicOr(bitmap + (m >> 5), 1u << (m & 31));
}

__device__ __forceinline__ int block_excl(int v, int* scr, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const int y = __shfl_up(x, k, 64);
    if (lane >= k) x += y;
  }
  if (lane == 63) scr[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) {
    pre += i < w ? scr[i] : 0;
    tot += scr[i];
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

__global__ __launch_bounds__(kThreads) void k_count(const uint32_t* __restrict__ bitmap,
                                                   int* __restrict__ counts) {
  __shared__ int scr[kThreads / 64];
  const int c = __popc(bitmap[static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x]);
  int total;
  block_excl(c, scr, total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// One block: exclusive scan of the block counts in place; n_out = total.
__global__ __launch_bounds__(kThreads) void k_scan(int* __restrict__ counts, int nb,
                                                  int64_t* __restrict__ n_out) {
  __shared__ int scr[kThreads / 64];
  int carry = 0;
  for (int base = 0; base < nb; base += kThreads) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? counts[i] : 0;
    int total;
    const int ex = block_excl(v, scr, total);
    if (i < nb) counts[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *n_out = carry;
}

__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t* __restrict__ bitmap,
                                                  const int* __restrict__ offsets, int64_t cap,
                                                  int32_t* __restrict__ leaf_ijk) {
  __shared__ int scr[kThreads / 64];
  const int64_t word = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  uint32_t bits = bitmap[word];
  int total;
  int64_t pos = offsets[blockIdx.x] + block_excl(__popc(bits), scr, total);
  while (bits) {
    const int b = __builtin_ctz(bits);
    bits &= bits - 1;
    const uint32_t m = static_cast<uint32_t>(word * 32 + b);
    if (pos < cap) {
      leaf_ijk[3 * pos] = static_cast<int32_t>(compact3(m));
      leaf_ijk[3 * pos + 1] = static_cast<int32_t>(compact3(m >> 1));
      leaf_ijk[3 * pos + 2] = static_cast<int32_t>(compact3(m >> 2));
    }
    ++pos;
  }
}

}  // namespace

size_t occupancy_bitmap_words(int level) {
  const uint64_t bits = uint64_t(1) << (3 * level);
  return static_cast<size_t>((bits + kBitsPerBlock - 1) / kBitsPerBlock) * kThreads;
}

hipError_t launch_occupancy(const float* o, const float* d, const float* t, int64_t n, int level,
                            uint32_t* bitmap, int* counts, int32_t* leaf_ijk, int64_t cap,
                            int64_t* n_out, hipStream_t s) {
  const size_t words = occupancy_bitmap_words(level);
  const int nb = static_cast<int>(words / kThreads);
  hipError_t e = launch_fill(reinterpret_cast<float*>(bitmap), 0.0f, static_cast<int64_t>(words), s);
  if (e != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_mark, dim3(static_cast<unsigned>((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, o, d, t, n, level, bitmap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_count, dim3(nb), dim3(kThreads), 0, s, bitmap, counts);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kThreads), 0, s, counts, nb, n_out);
  hipLaunchKernelGGL(k_emit, dim3(nb), dim3(kThreads), 0, s, bitmap, counts, cap, leaf_ijk);
  return hipGetLastError();
}

}  // namespace svlf
