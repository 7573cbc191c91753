// Hit-list kernels: the first K occupied leaves along each ray (SVLF
// sections 4.2-4.3), one ray per lane at a time.
#include <hip/hip_runtime.h>

#include "svlf_internal.hpp"
#include "traverse.hpp"

namespace svlf {
namespace {

constexpr int kTraceThreads = 256;

__device__ __forceinline__ Ray load_ray(const float* __restrict__ o, const float* __restrict__ d,
                                        int64_t r) {
  return make_ray(o[3 * r], o[3 * r + 1], o[3 * r + 2], d[3 * r], d[3 * r + 1], d[3 * r + 2]);
}

// One ray per lane (public layout: separate leaf / t_in / t_out arrays [n][K],
// padded with -1 / 0).
__global__ __launch_bounds__(kTraceThreads) void k_trace_public(
    const svlf_node* __restrict__ nodes, int depth, const float* __restrict__ o,
    const float* __restrict__ d, int64_t n, int K, int32_t* __restrict__ leaf_out,
    float* __restrict__ tin_out, float* __restrict__ tout_out, int32_t* __restrict__ cnt_out) {
  extern __shared__ uint2 stk[];
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kTraceThreads + threadIdx.x;
  if (r >= n) return;
  const int64_t base = r * K;
  auto emit = [&](int slot, int32_t leaf, float t0, float t1, uint32_t) {
    leaf_out[base + slot] = leaf;
    tin_out[base + slot] = t0;
    tout_out[base + slot] = t1;
  };
  Walker wk;
  if (wk.start(load_ray(o, d, r), nodes, depth)) {
    while (!wk.step(K, stk + threadIdx.x, kTraceThreads, emit)) {
    }
  }
  for (int s = wk.count; s < K; ++s) {
    leaf_out[base + s] = -1;
    tin_out[base + s] = 0.0f;
    tout_out[base + s] = 0.0f;
  }
  cnt_out[r] = wk.count;
}

// Persistent traversal with per-lane ray refill (internal hit-slot layout):
// each lane walks one ray; when it finishes it takes the next unprocessed
// ray (one atomic per wave for all lanes that need one), so a wave is not
// held back by its deepest ray while lanes whose rays missed sit idle.
// `next` must be 0 at launch.  Rays are grouped by scene (ray ranges of the
// scene table).
__global__ __launch_bounds__(kTraceThreads) void k_trace_internal(
    SceneTable tab, int64_t n_rays, const float* __restrict__ o, const float* __restrict__ d,
    int K, unsigned long long* __restrict__ next, HitRec* __restrict__ hits,
    int32_t* __restrict__ cnt_out) {
  extern __shared__ uint2 stk[];
  const int lane = threadIdx.x & 63;
  uint2* my_stk = stk + threadIdx.x;
  Walker wk;
  int64_t r = -1;
  bool active = false, exhausted = false;
  auto emit = [&](int slot, int32_t leaf, float t0, float t1, uint32_t ijk) {
    HitRec h;
    h.leaf = leaf;
    h.tin = t0;
    h.tout = t1;
    h.ijk = ijk;
    hits[r * K + slot] = h;
  };
  while (true) {
    // refill the lanes that need a ray
    const bool need = !active && !exhausted;
    const unsigned long long mask = __ballot(need);
    if (mask != 0ull) {
      const int leader = __builtin_ctzll(mask);
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(next, static_cast<unsigned long long>(__popcll(mask)));
      base = __shfl(base, leader, 64);
      if (need) {
        const unsigned long long below = mask & ((1ull << lane) - 1ull);
        const unsigned long long idx = base + static_cast<unsigned long long>(__popcll(below));
        if (idx >= static_cast<unsigned long long>(n_rays)) {
          exhausted = true;
        } else {
          r = static_cast<int64_t>(idx);
          int s = 0;
          while (s + 1 < tab.n && r >= tab.s[s + 1].ray_begin) ++s;
          active = wk.start(load_ray(o, d, r), tab.s[s].nodes, tab.s[s].depth);
          if (!active) cnt_out[r] = 0;
        }
      }
    }
    if (__ballot(active) == 0ull) {
      if (__ballot(!exhausted) == 0ull) break;
      continue;
    }
    if (active && wk.step(K, my_stk, kTraceThreads, emit)) {
      cnt_out[r] = wk.count;
      active = false;
    }
  }
}

__global__ void k_zero_counter(unsigned long long* c) { *c = 0ull; }

size_t stack_bytes(int depth) {
  const int levels = depth > 1 ? depth - 1 : 1;
  return static_cast<size_t>(levels) * kTraceThreads * sizeof(uint2);
}

int trace_grid(int64_t n_rays, int max_depth) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  int per_cu = static_cast<int>((160 * 1024) / stack_bytes(max_depth));
  if (per_cu > 8) per_cu = 8;
  if (per_cu < 1) per_cu = 1;
  int64_t grid = static_cast<int64_t>(cus) * per_cu;
  const int64_t need = (n_rays + kTraceThreads - 1) / kTraceThreads;
  if (grid > need) grid = need;
  return static_cast<int>(grid < 1 ? 1 : grid);
}

}  // namespace

hipError_t launch_trace_public(const svlf_octree& oct, const float* o, const float* d, int64_t n,
                               int K, int32_t* leaf, float* tin, float* tout, int32_t* cnt,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + kTraceThreads - 1) / kTraceThreads;
  hipLaunchKernelGGL(k_trace_public, dim3(static_cast<unsigned>(blocks)), dim3(kTraceThreads),
                     stack_bytes(oct.depth), s, oct.n_leaves > 0 ? oct.nodes : nullptr, oct.depth,
                     o, d, n, K, leaf, tin, tout, cnt);
  return hipGetLastError();
}

hipError_t launch_trace_internal(const SceneTable& tab, const float* o, const float* d, int K,
                                 HitRec* hits, int32_t* cnt, unsigned long long* counter,
                                 hipStream_t s) {
  const int64_t n = tab.s[tab.n - 1].ray_end;
  if (n == 0) return hipSuccess;
  int max_depth = 1;
  for (int i = 0; i < tab.n; ++i) max_depth = tab.s[i].depth > max_depth ? tab.s[i].depth : max_depth;
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, counter);
  hipLaunchKernelGGL(k_trace_internal, dim3(trace_grid(n, max_depth)), dim3(kTraceThreads),
                     stack_bytes(max_depth), s, tab, n, o, d, K, counter, hits, cnt);
  return hipGetLastError();
}

}  // namespace svlf
