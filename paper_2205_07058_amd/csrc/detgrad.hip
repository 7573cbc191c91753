// Deterministic reduction of the feature gradient (the alternative to FP32
// atomics in the backward): the backward leaves, per hit slot, the hit's
// cell coordinates u and dL/dx; here the hits are compacted in slot order
// (exclusive scan of the per-ray counts) and put in leaf order by a stable
// LSD radix sort (8-bit digits: per-tile digit counts, a digit-major
// exclusive scan, and a scatter whose ranks within a tile come from wave
// ballots and per-wave counts, never from atomics), so each leaf's bucket
// lists its hits in ascending slot order at a cost linear in the hits,
// whatever their distribution over leaves; the hits' records are then
// copied into that order.  Every vertex sums w_j(u) dL/dx over the hits of
// its (up to 8) adjacent leaves, leaves in a fixed order and hits in slot
// order, and adds the sum to its gradient row.
// The result does not depend on the order in which threads run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "svlf_internal.hpp"

namespace svlf {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 16;                        // scan items per thread
constexpr int kScanBlock = kThreads * kItems;
constexpr int kBins = 256;                        // radix digit: 8 bits
constexpr int kTileChunks = 8;                    // sort tile: chunks of kThreads items
constexpr int kTile = kThreads * kTileChunks;
static_assert(kBins == kThreads, "one digit per thread in the sort kernels");

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

int64_t tiles_of(int64_t n_items) { return (n_items + kTile - 1) / kTile; }

struct DetLayout {
  size_t lrun, hoff, bsum, dcount, doff, keys0, vals0, keys1, vals1, vleaves, recs, total;
};

DetLayout det_layout(int64_t n_rays, int K, int C, int64_t n_leaves, int64_t n_vertices) {
  DetLayout w;
  const int64_t slots = n_rays * K;
  const int64_t ndig = kBins * (tiles_of(slots) > 0 ? tiles_of(slots) : 1);
  const int64_t scan_max = ndig > n_rays ? ndig : n_rays;
  const size_t nb = static_cast<size_t>((scan_max + kScanBlock - 1) / kScanBlock) + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = a256(off + bytes);
    return at;
  };
  w.lrun = take(static_cast<size_t>(n_leaves) * 8);
  w.hoff = take(static_cast<size_t>(n_rays + 1) * 4);
  w.bsum = take(nb * 4);
  w.dcount = take(static_cast<size_t>(ndig) * 4);
  w.doff = take(static_cast<size_t>(ndig + 1) * 4);
  w.keys0 = take(static_cast<size_t>(slots) * 4);
  w.vals0 = take(static_cast<size_t>(slots) * 4);
  w.keys1 = take(static_cast<size_t>(slots) * 4);
  w.vals1 = take(static_cast<size_t>(slots) * 4);
  w.vleaves = take(static_cast<size_t>(n_vertices) * 8 * 4);
  w.recs = take(static_cast<size_t>(slots) * (C + 4) * 4);
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
  for (int i = 0; i < kWaves; ++i) {
    pre += i < w ? scr[i] : 0;
    tot += scr[i];
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_sums(const int* __restrict__ a, int64_t n,
                                                       int* __restrict__ bsum) {
  __shared__ int scr[kWaves];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * kItems;
  int s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) s += base + i < n ? a[base + i] : 0;
  int total;
  block_scan_excl(s, scr, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(int* __restrict__ bsum, int nb) {
  __shared__ int scr[kWaves];
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

// out[0..n) = exclusive prefix sums of a, out[n] = the total
__global__ __launch_bounds__(kThreads) void k_scan_out(const int* __restrict__ a, int64_t n,
                                                      const int* __restrict__ bsum,
                                                      int* __restrict__ out) {
  __shared__ int scr[kWaves];
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

// The hits in slot order: keys = leaf, vals = slot (r K + k).
__global__ void k_emit(const HitRec* __restrict__ hits, const int32_t* __restrict__ cnt,
                       const int* __restrict__ hoff, int64_t n_rays, int K,
                       int* __restrict__ keys, int* __restrict__ vals) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  const int o = hoff[r], c = cnt[r];
  for (int k = 0; k < c; ++k) {
    keys[o + k] = hits[r * K + k].leaf;
    vals[o + k] = static_cast<int>(r * K + k);
  }
}

// Radix pass, step 1: digit counts of each kTile-item tile, digit-major
// (dcount[d * n_tiles + tile]); tiles past the item count write zeros.
__global__ __launch_bounds__(kThreads) void k_digit_count(const int* __restrict__ keys,
                                                         const int* __restrict__ n_items_p,
                                                         int shift, int n_tiles,
                                                         int* __restrict__ dcount) {
  __shared__ int h[kBins];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t n = *n_items_p;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
#pragma unroll
  for (int c = 0; c < kTileChunks; ++c) {
    const int64_t i = base + c * kThreads + tid;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kBins - 1)], 1);
  }
  __syncthreads();
  dcount[static_cast<int64_t>(tid) * n_tiles + blockIdx.x] = h[tid];
}

// Radix pass, step 2 (after the exclusive scan of dcount into doff): each
// tile places its items in item order.  An item's rank among the tile's
// items with its digit = the tile's base for the digit + those in earlier
// chunks + those of lower waves in its chunk + those of lower lanes in its
// wave (lanes with equal digits found by one ballot per digit bit).
__global__ __launch_bounds__(kThreads) void k_digit_scatter(const int* __restrict__ kin,
                                                           const int* __restrict__ vin,
                                                           const int* __restrict__ n_items_p,
                                                           int shift, int n_tiles,
                                                           const int* __restrict__ doff,
                                                           int* __restrict__ kout,
                                                           int* __restrict__ vout) {
  __shared__ int run[kBins];
  __shared__ int wc[kWaves][kBins];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t n = *n_items_p;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
  if (base >= n) return;                          // the whole block: no item
  run[tid] = doff[static_cast<int64_t>(tid) * n_tiles + blockIdx.x];
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int c = 0; c < kTileChunks; ++c) {
#pragma unroll
    for (int q = 0; q < kWaves; ++q) wc[q][tid] = 0;
    __syncthreads();
    const int64_t i = base + c * kThreads + tid;
    const bool valid = i < n;
    int key = 0, val = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
    }
    const int d = (key >> shift) & (kBins - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int wrank = __popcll(peers & below);
    if (valid && wrank == 0) wc[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[d] + wrank;
      for (int q = 0; q < w; ++q) pos += wc[q][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) add += wc[q][tid];
    run[tid] += add;
  }
}

// Each leaf's run [begin, end) in the sorted hit list (leaves without hits
// keep the (0, 0) they were filled with).
__global__ __launch_bounds__(kThreads) void k_runs(const int* __restrict__ keys,
                                                  const int* __restrict__ n_items_p,
                                                  int2* __restrict__ lrun) {
  const int n = *n_items_p;
  const int stride = gridDim.x * kThreads;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    const int k = keys[i];
    if (i == 0 || keys[i - 1] != k) lrun[k].x = i;
    if (i == n - 1 || keys[i + 1] != k) lrun[k].y = i + 1;
  }
}

// The hits' records (u, pad, dL/dx: C + 4 floats, Q = (C + 4) / 4 16-byte
// chunks) in sorted order, so that each leaf's records are contiguous and
// leaves near in Morton order (the leaves around the vertices a block
// handles, as vertices are Morton-ranked too) are near in memory.
template <int C>
__global__ __launch_bounds__(kThreads) void k_order_recs(const int* __restrict__ bucket,
                                                        const int* __restrict__ n_items_p,
                                                        const float4* __restrict__ gxu,
                                                        float4* __restrict__ recs) {
  constexpr int Q = (C + 4) / 4;
  const int n = *n_items_p;
  for (int r0 = blockIdx.x * kThreads; r0 < n; r0 += gridDim.x * kThreads) {
    for (int q = threadIdx.x; q < kThreads * Q; q += kThreads) {
      const int i = r0 + q / Q, part = q % Q;
      if (i < n) recs[static_cast<int64_t>(i) * Q + part] = gxu[static_cast<int64_t>(bucket[i]) * Q + part];
    }
  }
}

// One vertex per thread: its adjacent leaves, their runs, then every record
// of each run, leaves in a fixed order and each run in slot order (a run
// usually holds at most one hit), accumulated per channel in registers; the
// sum is added to the vertex's gradient row (with 16-byte accesses when the
// row pointer allows).  Vertices with no hit leave their row untouched.
template <int C, bool ALIGNED>
__global__ __launch_bounds__(kThreads) void k_vgrad(const int* __restrict__ vleaves,
                                                   const int2* __restrict__ lrun,
                                                   const float4* __restrict__ recs,
                                                   int64_t n_vertices, float* __restrict__ grad) {
  constexpr int Q = (C + 4) / 4;                  // record: u (3), pad, dL/dx (C)
  const int64_t v = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (v >= n_vertices) return;
  const int4 la = *reinterpret_cast<const int4*>(vleaves + v * 8);
  const int4 lb = *reinterpret_cast<const int4*>(vleaves + v * 8 + 4);
  const int lv[8] = {la.x, la.y, la.z, la.w, lb.x, lb.y, lb.z, lb.w};
  int2 run[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) run[p] = lv[p] >= 0 ? lrun[lv[p]] : make_int2(0, 0);
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0f;
  bool any = false;
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int j = 7 - p;                          // v is corner j of leaf lv[p]
    for (int i = run[p].x; i < run[p].y; ++i) {
      any = true;
      const float4* rec = recs + static_cast<int64_t>(i) * Q;
      const float4 u = rec[0];
      const float w = ((j & 1) ? u.x : 1.0f - u.x) * (((j >> 1) & 1) ? u.y : 1.0f - u.y) *
                      ((j >> 2) ? u.z : 1.0f - u.z);
#pragma unroll
      for (int q = 0; q < C / 4; ++q) {
        const float4 g = rec[1 + q];
        acc[4 * q] += w * g.x;
        acc[4 * q + 1] += w * g.y;
        acc[4 * q + 2] += w * g.z;
        acc[4 * q + 3] += w * g.w;
      }
    }
  }
  if (!any) return;
  float* row = grad + v * C;
  if constexpr (ALIGNED) {
    float4* r4 = reinterpret_cast<float4*>(row);
#pragma unroll
    for (int q = 0; q < C / 4; ++q) {
      float4 x = r4[q];
      x.x += acc[4 * q];
      x.y += acc[4 * q + 1];
      x.z += acc[4 * q + 2];
      x.w += acc[4 * q + 3];
      r4[q] = x;
    }
  } else {
#pragma unroll
    for (int c = 0; c < C; ++c) row[c] += acc[c];
  }
}

template <int C>
void launch_vgrad(const int* vleaves, const int2* lrun, const float4* recs, int64_t n_vertices,
                  float* grad, int grid, hipStream_t s) {
  if (reinterpret_cast<uintptr_t>(grad) % 16 == 0)
    hipLaunchKernelGGL((k_vgrad<C, true>), dim3(grid), dim3(kThreads), 0, s, vleaves, lrun, recs,
                       n_vertices, grad);
  else
    hipLaunchKernelGGL((k_vgrad<C, false>), dim3(grid), dim3(kThreads), 0, s, vleaves, lrun, recs,
                       n_vertices, grad);
}

int grid_of(int64_t n, int per = kThreads) {
  int64_t b = (n + per - 1) / per;
  return static_cast<int>(b < 1 ? 1 : b);
}

}  // namespace

size_t detgrad_bytes(int64_t n_rays, int K, int C, int64_t n_leaves, int64_t n_vertices) {
  return det_layout(n_rays, K, C, n_leaves, n_vertices).total;
}

// Exclusive scan of a[0..n) into out[0..n], out[n] = the total.
void scan_excl(const int* a, int64_t n, int* bsum, int* out, hipStream_t s) {
  const int nb = static_cast<int>((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(kThreads), 0, s, a, n, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_out, dim3(nb), dim3(kThreads), 0, s, a, n, bsum, out);
}

namespace {

struct DetPtrs {
  int2* lrun;
  int *hoff, *bsum, *dcount, *doff, *keys[2], *vals[2], *vleaves;
  float4* recs;
  int passes;
};

DetPtrs det_ptrs(void* scratch, int64_t n_rays, int K, int C, int64_t n_leaves,
                 int64_t n_vertices) {
  const DetLayout w = det_layout(n_rays, K, C, n_leaves, n_vertices);
  char* base = static_cast<char*>(scratch);
  auto at = [&](size_t off) { return reinterpret_cast<int*>(base + off); };
  DetPtrs p;
  p.lrun = reinterpret_cast<int2*>(base + w.lrun);
  p.hoff = at(w.hoff);
  p.bsum = at(w.bsum);
  p.dcount = at(w.dcount);
  p.doff = at(w.doff);
  p.keys[0] = at(w.keys0);
  p.keys[1] = at(w.keys1);
  p.vals[0] = at(w.vals0);
  p.vals[1] = at(w.vals1);
  p.vleaves = at(w.vleaves);
  p.recs = reinterpret_cast<float4*>(base + w.recs);
  int bits = 1;
  while ((int64_t(1) << bits) < n_leaves) ++bits;
  p.passes = (bits + 7) / 8;
  return p;
}

constexpr int kFillGrid = 1024, kItemGrid = 1024;

}  // namespace

hipError_t launch_detgrad_order(const DevScene& sc, const HitRec* hits, const int32_t* cnt,
                                int64_t n_rays, int K, int C, void* scratch, int64_t n_leaves,
                                int64_t n_vertices, hipStream_t s) {
  if (n_leaves == 0 || n_rays == 0) return hipSuccess;
  if (C != 8 && C != 16 && C != 32) return hipErrorNotSupported;
  const DetPtrs p = det_ptrs(scratch, n_rays, K, C, n_leaves, n_vertices);
  hipLaunchKernelGGL(k_fill_i32, dim3(kFillGrid), dim3(kThreads), 0, s,
                     reinterpret_cast<int*>(p.lrun), 0, 2 * n_leaves);
  hipLaunchKernelGGL(k_fill_i32, dim3(kFillGrid), dim3(kThreads), 0, s, p.vleaves, -1,
                     n_vertices * 8);
  hipLaunchKernelGGL(k_vleaves, dim3(grid_of(n_leaves * 8)), dim3(kThreads), 0, s,
                     sc.leaf_corners, n_leaves, p.vleaves);
  // the hits in slot order (hoff[n_rays] = their number), then sorted by leaf
  scan_excl(cnt, n_rays, p.bsum, p.hoff, s);
  hipLaunchKernelGGL(k_emit, dim3(grid_of(n_rays)), dim3(kThreads), 0, s, hits, cnt, p.hoff,
                     n_rays, K, p.keys[0], p.vals[0]);
  const int* n_items = p.hoff + n_rays;
  const int64_t n_tiles = tiles_of(n_rays * K);
  for (int pass = 0; pass < p.passes; ++pass) {
    const int src = pass & 1, shift = 8 * pass;
    hipLaunchKernelGGL(k_digit_count, dim3(static_cast<unsigned>(n_tiles)), dim3(kThreads), 0, s,
                       p.keys[src], n_items, shift, static_cast<int>(n_tiles), p.dcount);
    scan_excl(p.dcount, kBins * n_tiles, p.bsum, p.doff, s);
    hipLaunchKernelGGL(k_digit_scatter, dim3(static_cast<unsigned>(n_tiles)), dim3(kThreads), 0, s,
                       p.keys[src], p.vals[src], n_items, shift, static_cast<int>(n_tiles), p.doff,
                       p.keys[src ^ 1], p.vals[src ^ 1]);
  }
  hipLaunchKernelGGL(k_runs, dim3(kItemGrid), dim3(kThreads), 0, s, p.keys[p.passes & 1], n_items,
                     p.lrun);
  return hipGetLastError();
}

hipError_t launch_detgrad_sum(const DevScene& sc, int64_t n_rays, int K, int C, const float* gxu,
                              void* scratch, int64_t n_leaves, int64_t n_vertices, hipStream_t s) {
  if (n_leaves == 0 || n_rays == 0) return hipSuccess;
  if (C != 8 && C != 16 && C != 32) return hipErrorNotSupported;
  const DetPtrs p = det_ptrs(scratch, n_rays, K, C, n_leaves, n_vertices);
  const int* n_items = p.hoff + n_rays;
  const int* bucket = p.vals[p.passes & 1];
  const float4* g4 = reinterpret_cast<const float4*>(gxu);
  const int vgrid = grid_of(n_vertices);
  switch (C) {
    case 8:
      hipLaunchKernelGGL(k_order_recs<8>, dim3(kItemGrid), dim3(kThreads), 0, s, bucket, n_items, g4, p.recs);
      launch_vgrad<8>(p.vleaves, p.lrun, p.recs, n_vertices, sc.grad, vgrid, s);
      break;
    case 16:
      hipLaunchKernelGGL(k_order_recs<16>, dim3(kItemGrid), dim3(kThreads), 0, s, bucket, n_items, g4, p.recs);
      launch_vgrad<16>(p.vleaves, p.lrun, p.recs, n_vertices, sc.grad, vgrid, s);
      break;
    default:
      hipLaunchKernelGGL(k_order_recs<32>, dim3(kItemGrid), dim3(kThreads), 0, s, bucket, n_items, g4, p.recs);
      launch_vgrad<32>(p.vleaves, p.lrun, p.recs, n_vertices, sc.grad, vgrid, s);
      break;
  }
  return hipGetLastError();
}

}  // namespace svlf
