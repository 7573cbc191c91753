// Hit-list kernels: the first K occupied leaves along each ray (SVLF
// sections 4.2-4.3), one ray per lane.
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

// Public layout: separate leaf / t_in / t_out arrays [n][K], padded.
__global__ __launch_bounds__(kTraceThreads) void k_trace_public(
    const svlf_node* __restrict__ nodes, int depth, int64_t n_leaves,
    const float* __restrict__ o, const float* __restrict__ d, int64_t n, int K,
    int32_t* __restrict__ leaf_out, float* __restrict__ tin_out, float* __restrict__ tout_out,
    int32_t* __restrict__ cnt_out) {
  extern __shared__ uint2 stk[];
  __shared__ uint8_t mtab[kMirrorTableBytes];
  fill_mirror_table(mtab, threadIdx.x, kTraceThreads);
  __syncthreads();
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kTraceThreads + threadIdx.x;
  if (r >= n) return;
  int count = 0;
  const int64_t base = r * K;
  if (n_leaves > 0) {
    const Ray ray = load_ray(o, d, r);
    count = traverse(ray, nodes, depth, K, stk + threadIdx.x, kTraceThreads, mtab,
                     [&](int slot, int32_t leaf, float t0, float t1, uint32_t) {
                       leaf_out[base + slot] = leaf;
                       tin_out[base + slot] = t0;
                       tout_out[base + slot] = t1;
                     });
  }
  for (int s = count; s < K; ++s) {
    leaf_out[base + s] = -1;
    tin_out[base + s] = 0.0f;
    tout_out[base + s] = 0.0f;
  }
  cnt_out[r] = count;
}

// Internal layout for the shading kernels: one 16-byte record per hit slot
// (unused slots are left unwritten), rays grouped by scene.
__global__ __launch_bounds__(kTraceThreads) void k_trace_internal(
    SceneTable tab, const float* __restrict__ o, const float* __restrict__ d, int K,
    HitRec* __restrict__ hits, int32_t* __restrict__ cnt_out) {
  extern __shared__ uint2 stk[];
  __shared__ uint8_t mtab[kMirrorTableBytes];
  fill_mirror_table(mtab, threadIdx.x, kTraceThreads);
  __syncthreads();
  const int b = blockIdx.x;
  int s = 0;
  while (s + 1 < tab.n && b >= tab.s[s + 1].block_begin) ++s;
  const DevScene& sc = tab.s[s];
  const int64_t r = sc.ray_begin + static_cast<int64_t>(b - sc.block_begin) * kTraceThreads +
                    threadIdx.x;
  if (r >= sc.ray_end) return;
  int count = 0;
  if (sc.nodes != nullptr) {
    const Ray ray = load_ray(o, d, r);
    HitRec* out = hits + r * K;
    count = traverse(ray, sc.nodes, sc.depth, K, stk + threadIdx.x, kTraceThreads, mtab,
                     [&](int slot, int32_t leaf, float t0, float t1, uint32_t ijk) {
                       HitRec h;
                       h.leaf = leaf;
                       h.tin = t0;
                       h.tout = t1;
                       h.ijk = ijk;
                       out[slot] = h;
                     });
  }
  cnt_out[r] = count;
}

size_t stack_bytes(int depth) {
  const int levels = depth > 1 ? depth - 1 : 1;
  return static_cast<size_t>(levels) * kTraceThreads * sizeof(uint2);
}

}  // namespace

hipError_t launch_trace_public(const svlf_octree& oct, const float* o, const float* d, int64_t n,
                               int K, int32_t* leaf, float* tin, float* tout, int32_t* cnt,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + kTraceThreads - 1) / kTraceThreads;
  hipLaunchKernelGGL(k_trace_public, dim3(static_cast<unsigned>(blocks)), dim3(kTraceThreads),
                     stack_bytes(oct.depth), s, oct.nodes, oct.depth, oct.n_leaves, o, d, n, K,
                     leaf, tin, tout, cnt);
  return hipGetLastError();
}

hipError_t launch_trace_internal(const SceneTable& tab, const float* o, const float* d, int K,
                                 HitRec* hits, int32_t* cnt, hipStream_t s) {
  if (tab.n_blocks == 0) return hipSuccess;
  int max_depth = 1;
  for (int i = 0; i < tab.n; ++i) max_depth = tab.s[i].depth > max_depth ? tab.s[i].depth : max_depth;
  hipLaunchKernelGGL(k_trace_internal, dim3(static_cast<unsigned>(tab.n_blocks)),
                     dim3(kTraceThreads), stack_bytes(max_depth), s, tab, o, d, K, hits, cnt);
  return hipGetLastError();
}

}  // namespace svlf
