// Front-to-back sparse-octree traversal of one ray per lane.
//
// SVLF lists, for every ray, the occupied voxels it crosses in order along the
// ray with their entry/exit distances (section 4.3), using a ray-AABB slab
// test (section 4.2).  The paper runs a level-synchronous traversal with
// device-wide scans between levels; on gfx950 this is a per-lane depth-first
// walk instead: children are visited in the order i ^ oct (oct = sign bits of
// the direction), which is the order of their entry distances, so the walk
// can stop after K leaves and needs no global synchronisation.  The per-level
// stack lives in LDS, laid out [level][lane] so that lanes never conflict.
//
// Every plane distance is RN(RN(b - o) * inv) in binary32 with no
// contraction; as each value depends only on the plane b, a child is hit only
// if its parent is, sibling order equals t_in order, and the produced t_in /
// t_out equal those of testing each leaf directly (the library's documented
// predicate).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "svlf.h"

namespace svlf {

struct Ray {
  float ox, oy, oz;
  float ix, iy, iz;   // RN(1 / d)
  bool fx, fy, fz;    // reciprocal finite
  uint32_t oct;       // bit a set iff d_a < 0
  bool valid;
};

__device__ __forceinline__ bool finite32(float x) { return __builtin_isfinite(x); }

__device__ __forceinline__ Ray make_ray(float ox, float oy, float oz, float dx, float dy,
                                        float dz) {
  Ray r;
  r.ox = ox;
  r.oy = oy;
  r.oz = oz;
  r.valid = finite32(ox) && finite32(oy) && finite32(oz) && finite32(dx) && finite32(dy) &&
            finite32(dz) && (dx != 0.0f || dy != 0.0f || dz != 0.0f);
  // correctly rounded division (the library is built without fast-math)
  r.ix = 1.0f / dx;
  r.iy = 1.0f / dy;
  r.iz = 1.0f / dz;
  r.fx = finite32(r.ix);
  r.fy = finite32(r.iy);
  r.fz = finite32(r.iz);
  r.oct = (dx < 0.0f ? 1u : 0u) | (dy < 0.0f ? 2u : 0u) | (dz < 0.0f ? 4u : 0u);
  return r;
}

// Entry/exit intervals of the low (0) and high (1) half of a cell along one
// axis, from the three planes lo < mid < hi.
struct AxisKids {
  float tn0, tf0, tn1, tf1;
};

__device__ __forceinline__ AxisKids axis_kids(float o, float inv, bool fin, float lo, float mid,
                                              float hi) {
#pragma clang fp contract(off)
  AxisKids a;
  const float inf = __builtin_inff();
  if (fin) {
    const float p0 = (lo - o) * inv;
    const float p1 = (mid - o) * inv;
    const float p2 = (hi - o) * inv;
    if (inv > 0.0f) {
      a.tn0 = p0; a.tf0 = p1; a.tn1 = p1; a.tf1 = p2;
    } else {
      a.tn0 = p1; a.tf0 = p0; a.tn1 = p2; a.tf1 = p1;
    }
  } else {
    const bool in0 = (lo <= o) && (o < mid);
    const bool in1 = (mid <= o) && (o < hi);
    a.tn0 = in0 ? -inf : inf; a.tf0 = in0 ? inf : -inf;
    a.tn1 = in1 ? -inf : inf; a.tf1 = in1 ? inf : -inf;
  }
  return a;
}

struct Kids {
  AxisKids x, y, z;
};

__device__ __forceinline__ void kid_interval(const Kids& k, uint32_t c, float& tin, float& tout) {
  const float tnx = (c & 1) ? k.x.tn1 : k.x.tn0, tfx = (c & 1) ? k.x.tf1 : k.x.tf0;
  const float tny = (c & 2) ? k.y.tn1 : k.y.tn0, tfy = (c & 2) ? k.y.tf1 : k.y.tf0;
  const float tnz = (c & 4) ? k.z.tn1 : k.z.tn0, tfz = (c & 4) ? k.z.tf1 : k.z.tf0;
  const float tn = __builtin_fmaxf(__builtin_fmaxf(tnx, tny), tnz);
  tin = tn > 0.0f ? tn : 0.0f;
  tout = __builtin_fminf(__builtin_fminf(tfx, tfy), tfz);
}

// Cell side at level l: 2^(1-l), exact.
__device__ __forceinline__ float cell_size(int level) {
  return __int_as_float((128 - level) << 23);
}

__device__ __forceinline__ Kids node_kids(const Ray& r, int level, uint32_t ci, uint32_t cj,
                                          uint32_t ck) {
  const float h = cell_size(level);
  const float hh = cell_size(level + 1);
  const float lx = -1.0f + static_cast<float>(ci) * h;
  const float ly = -1.0f + static_cast<float>(cj) * h;
  const float lz = -1.0f + static_cast<float>(ck) * h;
  Kids k;
  k.x = axis_kids(r.ox, r.ix, r.fx, lx, lx + hh, lx + h);
  k.y = axis_kids(r.oy, r.iy, r.fy, ly, ly + hh, ly + h);
  k.z = axis_kids(r.oz, r.iz, r.fz, lz, lz + hh, lz + h);
  return k;
}

// Hit children of a node (mask in child space), restricted to `exists`.
__device__ __forceinline__ uint32_t kid_hits(const Kids& k, uint32_t exists) {
  uint32_t m = 0;
#pragma unroll
  for (uint32_t c = 0; c < 8; ++c) {
    float tin, tout;
    kid_interval(k, c, tin, tout);
    m |= ((tin < tout) ? 1u : 0u) << c;
  }
  return m & exists;
}

// Child-space mask -> visiting-order mask (bit i <-> child i ^ oct).
__device__ __forceinline__ uint32_t to_order(uint32_t m, uint32_t oct) {
  uint32_t r = 0;
#pragma unroll
  for (uint32_t i = 0; i < 8; ++i) r |= ((m >> (i ^ oct)) & 1u) << i;
  return r;
}

// Root cell [-1, 1]^3 test.
__device__ __forceinline__ bool root_hit(const Ray& r) {
  const Kids k = node_kids(r, -1, 0, 0, 0);  // level -1 has side 4: planes -1, 1, 3
  float tin, tout;
  kid_interval(k, 0, tin, tout);             // its low child is the root cell
  return tin < tout;
}

// Walks the octree front to back; calls emit(slot, leaf, t_in, t_out, ijk)
// for the first K hit leaves.  `stk` points at this lane's entry of level 0
// of an LDS array laid out [level][stride].  Returns the number of hits.
template <class Emit>
__device__ __forceinline__ int traverse(const Ray& r, const svlf_node* __restrict__ nodes,
                                        int depth, int K, uint2* stk, int stride, Emit emit) {
  if (!r.valid || !root_hit(r)) return 0;
  int count = 0;
  int level = 0;
  uint32_t ci = 0, cj = 0, ck = 0;
  svlf_node nd = nodes[0];
  uint32_t rem = 0;
  bool expand = true;
  while (true) {
    if (expand) {
      expand = false;
      const Kids kd = node_kids(r, level, ci, cj, ck);
      rem = to_order(kid_hits(kd, nd.mask), r.oct);
      if (level == depth - 1) {
        // children are leaves: emit them in order
        while (rem) {
          const uint32_t i = __builtin_ctz(rem);
          rem &= rem - 1;
          const uint32_t c = i ^ r.oct;
          float tin, tout;
          kid_interval(kd, c, tin, tout);
          const int32_t leaf = nd.child + __builtin_popcount(nd.mask & ((1u << c) - 1u));
          const uint32_t li = 2 * ci + (c & 1), lj = 2 * cj + ((c >> 1) & 1),
                         lk = 2 * ck + (c >> 2);
          emit(count, leaf, tin, tout, li | (lj << 10) | (lk << 20));
          if (++count == K) return count;
        }
      }
    }
    if (rem == 0) {
      if (level == 0) break;
      --level;
      ci >>= 1;
      cj >>= 1;
      ck >>= 1;
      const uint2 e = stk[level * stride];
      nd.child = static_cast<int32_t>(e.x);
      nd.mask = e.y & 0xFFu;
      rem = e.y >> 8;
      continue;
    }
    const uint32_t i = __builtin_ctz(rem);
    rem &= rem - 1;
    const uint32_t c = i ^ r.oct;
    const int32_t idx = nd.child + __builtin_popcount(nd.mask & ((1u << c) - 1u));
    stk[level * stride] = make_uint2(static_cast<uint32_t>(nd.child), nd.mask | (rem << 8));
    ++level;
    ci = 2 * ci + (c & 1);
    cj = 2 * cj + ((c >> 1) & 1);
    ck = 2 * ck + (c >> 2);
    nd = nodes[idx];
    expand = true;
  }
  return count;
}

}  // namespace svlf
