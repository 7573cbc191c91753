// Deterministic reduction of the feature gradient (the alternative to FP32
// atomics in the backward): the backward leaves, per hit slot, the hit's
// cell coordinates u and dL/dx; here the slots are bucketed by leaf
// (counting sort: counts, exclusive scan, placement), each bucket is put in
// ascending slot order, and every vertex sums w_j(u) dL/dx over the hits of
// its (up to 8) adjacent leaves, leaves in a fixed order and hits in slot
// order, then adds the sum to its gradient row.  The result does not depend
// on the order in which threads run.
#include <hip/hip_runtime.h>

#include "svlf_internal.hpp"

namespace svlf {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;                        // scan items per thread
constexpr int kScanBlock = kThreads * kItems;

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct DetLayout {
  size_t lcount, cursor, loff, bsum, bucket, vleaves, total;
};

DetLayout det_layout(int64_t n_rays, int K, int64_t n_leaves, int64_t n_vertices) {
  DetLayout w;
  const size_t nb = static_cast<size_t>((n_leaves + kScanBlock - 1) / kScanBlock) + 1;
  size_t off = 0;
  w.lcount = off;
  off = a256(off + static_cast<size_t>(n_leaves) * 4);
  w.cursor = off;
  off = a256(off + static_cast<size_t>(n_leaves) * 4);
  w.loff = off;
  off = a256(off + static_cast<size_t>(n_leaves + 1) * 4);
  w.bsum = off;
  off = a256(off + nb * 4);
  w.bucket = off;
  off = a256(off + static_cast<size_t>(n_rays) * K * 8);
  w.vleaves = off;
  off = a256(off + static_cast<size_t>(n_vertices) * 8 * 4);
  w.total = off;
  return w;
}

__global__ void k_fill_i32(int* __restrict__ p, int v, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = v;
}

// vleaves[v][7 - j] = the leaf whose corner j is v (each entry has one writer)
__global__ void k_vleaves(const int32_t* __restrict__ leaf_corners, int64_t n_leaves,
                          int* __restrict__ vleaves) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n_leaves * 8) return;
  const int64_t l = e >> 3;
  const int j = static_cast<int>(e & 7);
  vleaves[static_cast<int64_t>(leaf_corners[e]) * 8 + (7 - j)] = static_cast<int>(l);
}

__global__ void k_count(const HitRec* __restrict__ hits, const int32_t* __restrict__ cnt,
                        int64_t n_rays, int K, int* __restrict__ lcount) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  for (int k = 0; k < cnt[r]; ++k) atomicAdd(&lcount[hits[r * K + k].leaf], 1);
}

__device__ __forceinline__ int block_scan_excl(int v, int* scr, int& total) {
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

__global__ __launch_bounds__(kThreads) void k_scan_sums(const int* __restrict__ a, int64_t n,
                                                       int* __restrict__ bsum) {
  __shared__ int scr[kThreads / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * kItems;
  int s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) s += base + i < n ? a[base + i] : 0;
  int total;
  block_scan_excl(s, scr, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(int* __restrict__ bsum, int nb) {
  __shared__ int scr[kThreads / 64];
  int carry = 0;
  for (int base = 0; base < nb; base += kThreads) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int total;
    const int ex = block_scan_excl(v, scr, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kThreads) void k_scan_out(const int* __restrict__ a, int64_t n,
                                                      const int* __restrict__ bsum,
                                                      int* __restrict__ out) {
  __shared__ int scr[kThreads / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * kItems;
  int v[kItems];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = base + i < n ? a[base + i] : 0;
    s += v[i];
  }
  int total;
  int run = bsum[blockIdx.x] + block_scan_excl(s, scr, total);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (base <= n - 1 && n - 1 < base + kItems) out[n] = run;      // the total
}

__global__ void k_place(const HitRec* __restrict__ hits, const int32_t* __restrict__ cnt,
                        int64_t n_rays, int K, const int* __restrict__ loff,
                        int* __restrict__ cursor, int64_t* __restrict__ bucket) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  for (int k = 0; k < cnt[r]; ++k) {
    const int leaf = hits[r * K + k].leaf;
    bucket[loff[leaf] + atomicAdd(&cursor[leaf], 1)] = r * K + k;
  }
}

// insertion sort of each (small) bucket by slot
__global__ void k_sort_buckets(const int* __restrict__ loff, int64_t n_leaves,
                               int64_t* __restrict__ bucket) {
  const int64_t l = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (l >= n_leaves) return;
  const int b = loff[l], e = loff[l + 1];
  for (int i = b + 1; i < e; ++i) {
    const int64_t x = bucket[i];
    int j = i - 1;
    while (j >= b && bucket[j] > x) {
      bucket[j + 1] = bucket[j];
      --j;
    }
    bucket[j + 1] = x;
  }
}

// One vertex per C lanes (lane = channel).
template <int C>
__global__ __launch_bounds__(kThreads) void k_vgrad(const int* __restrict__ vleaves,
                                                   const int* __restrict__ loff,
                                                   const int64_t* __restrict__ bucket,
                                                   const float* __restrict__ gxu,
                                                   int64_t n_vertices, float* __restrict__ grad) {
  constexpr int VPB = kThreads / C;
  const int c = threadIdx.x % C;
  const int64_t v = static_cast<int64_t>(blockIdx.x) * VPB + threadIdx.x / C;
  if (v >= n_vertices) return;
  float acc = 0.0f;
  for (int p = 0; p < 8; ++p) {
    const int l = vleaves[v * 8 + p];
    if (l < 0) continue;
    const int j = 7 - p;                       // v is corner j of leaf l
    const int b = loff[l], e = loff[l + 1];
    for (int i = b; i < e; ++i) {
      const float* rec = gxu + bucket[i] * (C + 4);
      const float ux = rec[0], uy = rec[1], uz = rec[2];
      const float w = ((j & 1) ? ux : 1.0f - ux) * (((j >> 1) & 1) ? uy : 1.0f - uy) *
                      ((j >> 2) ? uz : 1.0f - uz);
      acc += w * rec[4 + c];
    }
  }
  grad[v * C + c] += acc;
}

int grid_of(int64_t n, int per = kThreads) {
  int64_t b = (n + per - 1) / per;
  return static_cast<int>(b < 1 ? 1 : b);
}

}  // namespace

size_t detgrad_bytes(int64_t n_rays, int K, int C, int64_t n_leaves, int64_t n_vertices) {
  (void)C;
  return det_layout(n_rays, K, n_leaves, n_vertices).total;
}

hipError_t launch_detgrad(const DevScene& sc, const HitRec* hits, const int32_t* cnt,
                          int64_t n_rays, int K, int C, const float* gxu, void* scratch,
                          int64_t n_leaves, int64_t n_vertices, hipStream_t s) {
  if (n_leaves == 0 || n_rays == 0) return hipSuccess;
  const DetLayout w = det_layout(n_rays, K, n_leaves, n_vertices);
  char* base = static_cast<char*>(scratch);
  int* lcount = reinterpret_cast<int*>(base + w.lcount);
  int* cursor = reinterpret_cast<int*>(base + w.cursor);
  int* loff = reinterpret_cast<int*>(base + w.loff);
  int* bsum = reinterpret_cast<int*>(base + w.bsum);
  int64_t* bucket = reinterpret_cast<int64_t*>(base + w.bucket);
  int* vleaves = reinterpret_cast<int*>(base + w.vleaves);
  const int nb = static_cast<int>((n_leaves + kScanBlock - 1) / kScanBlock);
  const int fill_grid = 1024;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid), dim3(kThreads), 0, s, lcount, 0, n_leaves);
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid), dim3(kThreads), 0, s, cursor, 0, n_leaves);
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid), dim3(kThreads), 0, s, vleaves, -1, n_vertices * 8);
  hipLaunchKernelGGL(k_vleaves, dim3(grid_of(n_leaves * 8)), dim3(kThreads), 0, s,
                     sc.leaf_corners, n_leaves, vleaves);
  hipLaunchKernelGGL(k_count, dim3(grid_of(n_rays)), dim3(kThreads), 0, s, hits, cnt, n_rays, K,
                     lcount);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(kThreads), 0, s, lcount, n_leaves, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_out, dim3(nb), dim3(kThreads), 0, s, lcount, n_leaves, bsum, loff);
  hipLaunchKernelGGL(k_place, dim3(grid_of(n_rays)), dim3(kThreads), 0, s, hits, cnt, n_rays, K,
                     loff, cursor, bucket);
  hipLaunchKernelGGL(k_sort_buckets, dim3(grid_of(n_leaves)), dim3(kThreads), 0, s, loff,
                     n_leaves, bucket);
  switch (C) {
    case 8:
      hipLaunchKernelGGL(k_vgrad<8>, dim3(grid_of(n_vertices, kThreads / 8)), dim3(kThreads), 0, s,
                         vleaves, loff, bucket, gxu, n_vertices, sc.grad);
      break;
    case 16:
      hipLaunchKernelGGL(k_vgrad<16>, dim3(grid_of(n_vertices, kThreads / 16)), dim3(kThreads), 0, s,
                         vleaves, loff, bucket, gxu, n_vertices, sc.grad);
      break;
    case 32:
      hipLaunchKernelGGL(k_vgrad<32>, dim3(grid_of(n_vertices, kThreads / 32)), dim3(kThreads), 0, s,
                         vleaves, loff, bucket, gxu, n_vertices, sc.grad);
      break;
    default:
      return hipErrorNotSupported;
  }
  return hipGetLastError();
}

}  // namespace svlf
