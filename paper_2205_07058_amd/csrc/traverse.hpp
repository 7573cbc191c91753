// Front-to-back sparse-octree traversal of one ray per lane.
//
// SVLF lists, for every ray, the occupied voxels it crosses in order along the
// ray with their entry/exit distances (section 4.3), using a ray-AABB slab
// test (section 4.2).  The paper runs a level-synchronous traversal with
// device-wide scans between levels; on gfx950 this is a per-lane depth-first
// walk instead: children are visited in the order of their entry distances,
// so the walk can stop after K leaves and needs no global synchronisation.
// The per-level stack lives in LDS, laid out [level][lane] so that lanes
// never conflict.
//
// Every plane distance is RN(RN(b - o) * inv) in binary32 with no
// contraction; as each value depends only on the plane b, a child is hit only
// if its parent is, sibling order equals t_in order, and the produced t_in /
// t_out equal those of testing each leaf directly (the library's documented
// predicate).
//
// The walk runs in a frame mirrored on every axis where d < 0 (x -> -x):
// there every finite reciprocal is positive, so the half of a cell that a ray
// enters first is always the low half and the visiting order of the children
// is their index in that frame.  Mirroring changes no distance: the mirrored
// cell planes are the negated true planes (exact, as all planes are dyadic
// with at most 11 significant bits), RN(-a) = -RN(a), and the product of two
// negated factors is the original product; only the sign of an exact zero
// distance can differ, which no comparison sees and the t_in clamp removes.
// The child index in the octree's own frame is (mirrored index) ^ oct.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "svlf.h"

namespace svlf {

struct Ray {
  float ox, oy, oz;   // origin, negated on the axes where d < 0
  float ix, iy, iz;   // RN(1 / d), negated likewise
  uint32_t oct;       // bit a set iff d_a < 0
  uint32_t nonfin;    // bit a set iff RN(1 / d_a) is not finite
  bool valid;
};

__device__ __forceinline__ bool finite32(float x) { return __builtin_isfinite(x); }

__device__ __forceinline__ Ray make_ray(float ox, float oy, float oz, float dx, float dy,
                                        float dz) {
  Ray r;
  r.valid = finite32(ox) && finite32(oy) && finite32(oz) && finite32(dx) && finite32(dy) &&
            finite32(dz) && (dx != 0.0f || dy != 0.0f || dz != 0.0f);
  // correctly rounded division (the library is built without fast-math)
  const float ix = 1.0f / dx, iy = 1.0f / dy, iz = 1.0f / dz;
  r.oct = (dx < 0.0f ? 1u : 0u) | (dy < 0.0f ? 2u : 0u) | (dz < 0.0f ? 4u : 0u);
  r.nonfin = (finite32(ix) ? 0u : 1u) | (finite32(iy) ? 0u : 2u) | (finite32(iz) ? 0u : 4u);
  r.ox = (r.oct & 1u) ? -ox : ox;
  r.oy = (r.oct & 2u) ? -oy : oy;
  r.oz = (r.oct & 4u) ? -oz : oz;
  r.ix = (r.oct & 1u) ? -ix : ix;
  r.iy = (r.oct & 2u) ? -iy : iy;
  r.iz = (r.oct & 4u) ? -iz : iz;
  return r;
}

// Distances to the three planes lo < mid < hi of a cell along one axis (in
// the mirrored frame): the low child spans [p0, p1], the high child [p1, p2].
struct Axis {
  float p0, p1, p2;
};

__device__ __forceinline__ Axis axis_planes(float o, float inv, float lo, float mid, float hi) {
#pragma clang fp contract(off)
  Axis a;
  a.p0 = (lo - o) * inv;
  a.p1 = (mid - o) * inv;
  a.p2 = (hi - o) * inv;
  return a;
}

// A ray parallel to the axis (non-finite reciprocal) constrains a child only
// through whether the origin lies in it; the true-frame half-open interval
// [a, b) becomes (-b, -a] after mirroring.  Encoded so that the low child is
// [p0, p1] and the high child [p1, p2] as above: an interval is (-inf, inf)
// when the origin is inside and empty otherwise.
__device__ __forceinline__ bool inside(float o, float lo, float hi, bool mirrored) {
  return mirrored ? (lo < o && o <= hi) : (lo <= o && o < hi);
}

__device__ __forceinline__ Axis axis_parallel(float o, bool mirrored, float lo, float mid,
                                              float hi) {
  const float inf = __builtin_inff();
  const bool in_lo = inside(o, lo, mid, mirrored);
  const bool in_hi = inside(o, mid, hi, mirrored);
  Axis a;
  a.p0 = in_lo ? -inf : inf;
  a.p1 = in_lo ? inf : (in_hi ? -inf : 0.0f);
  a.p2 = in_hi ? inf : -inf;
  return a;
}

struct Kids {
  Axis x, y, z;
};

// Cell side at level l: 2^(1-l), exact.
__device__ __forceinline__ float cell_size(int level) {
  return __int_as_float((128 - level) << 23);
}

// Plane distances of the node at `level` with mirrored cell coordinates
// (ci, cj, ck).  PAR: the ray has an axis with a non-finite reciprocal.
template <bool PAR>
__device__ __forceinline__ Kids node_kids(const Ray& r, int level, uint32_t ci, uint32_t cj,
                                          uint32_t ck) {
  const float h = cell_size(level);
  const float hh = cell_size(level + 1);
  const float lx = -1.0f + static_cast<float>(ci) * h;
  const float ly = -1.0f + static_cast<float>(cj) * h;
  const float lz = -1.0f + static_cast<float>(ck) * h;
  Kids k;
  k.x = axis_planes(r.ox, r.ix, lx, lx + hh, lx + h);
  k.y = axis_planes(r.oy, r.iy, ly, ly + hh, ly + h);
  k.z = axis_planes(r.oz, r.iz, lz, lz + hh, lz + h);
  if (PAR) {
    if (r.nonfin & 1u) k.x = axis_parallel(r.ox, r.oct & 1u, lx, lx + hh, lx + h);
    if (r.nonfin & 2u) k.y = axis_parallel(r.oy, r.oct & 2u, ly, ly + hh, ly + h);
    if (r.nonfin & 4u) k.z = axis_parallel(r.oz, r.oct & 4u, lz, lz + hh, lz + h);
  }
  return k;
}

// Interval of the child with mirrored index i (bit a = high half on axis a).
__device__ __forceinline__ void kid_interval(const Kids& k, uint32_t i, float& tin, float& tout) {
  const float tnx = (i & 1) ? k.x.p1 : k.x.p0, tfx = (i & 1) ? k.x.p2 : k.x.p1;
  const float tny = (i & 2) ? k.y.p1 : k.y.p0, tfy = (i & 2) ? k.y.p2 : k.y.p1;
  const float tnz = (i & 4) ? k.z.p1 : k.z.p0, tfz = (i & 4) ? k.z.p2 : k.z.p1;
  const float tn = __builtin_fmaxf(__builtin_fmaxf(tnx, tny), tnz);
  tin = tn > 0.0f ? tn : 0.0f;
  tout = __builtin_fminf(__builtin_fminf(tfx, tfy), tfz);
}

// Hit children, bit i = mirrored child i (i.e. in visiting order).
__device__ __forceinline__ uint32_t kid_hits(const Kids& k) {
  // max(t_n, 0) < t_out with the clamp folded into the z entries
  const float z0 = __builtin_fmaxf(k.z.p0, 0.0f), z1 = __builtin_fmaxf(k.z.p1, 0.0f);
  uint32_t m = 0;
#pragma unroll
  for (uint32_t i = 0; i < 8; ++i) {
    const float xn = (i & 1) ? k.x.p1 : k.x.p0, xf = (i & 1) ? k.x.p2 : k.x.p1;
    const float yn = (i & 2) ? k.y.p1 : k.y.p0, yf = (i & 2) ? k.y.p2 : k.y.p1;
    const float zn = (i & 4) ? z1 : z0, zf = (i & 4) ? k.z.p2 : k.z.p1;
    // Children of odd index pair x with z first, the others x with y: no
    // two children then share an inner max / min, so each folds into one
    // three-operand max / min (the values are NaN-free, order is immaterial).
    const bool odd = (__builtin_popcount(i) & 1) != 0;
    const float tn = odd ? __builtin_fmaxf(__builtin_fmaxf(xn, zn), yn)
                         : __builtin_fmaxf(__builtin_fmaxf(xn, yn), zn);
    const float tf = odd ? __builtin_fminf(__builtin_fminf(xf, zf), yf)
                         : __builtin_fminf(__builtin_fminf(xf, yf), zf);
    m |= (tn < tf ? 1u : 0u) << i;
  }
  return m;
}

// Child-frame occupancy mask -> mirrored frame: bit i <- bit (i ^ oct).
__device__ __forceinline__ uint32_t mirror_mask(uint32_t m, uint32_t oct) {
  if (oct & 1u) m = ((m & 0x55u) << 1) | ((m >> 1) & 0x55u);
  if (oct & 2u) m = ((m & 0x33u) << 2) | ((m >> 2) & 0x33u);
  if (oct & 4u) m = ((m & 0x0Fu) << 4) | ((m >> 4) & 0x0Fu);
  return m;
}

// mirror_mask for every (oct, m) as a byte table, entry (oct << 8) | m:
// the kernels keep it in LDS, where one lookup replaces the three
// conditional bit swaps in the walk's loop.
constexpr int kMirrorTableBytes = 8 * 256;

__device__ __forceinline__ void fill_mirror_table(uint8_t* t, int tid, int nthreads) {
  for (int e = tid; e < kMirrorTableBytes; e += nthreads)
    t[e] = static_cast<uint8_t>(mirror_mask(static_cast<uint32_t>(e) & 0xFFu, static_cast<uint32_t>(e) >> 8));
}

// Root cell [-1, 1]^3 test (the cell is its own mirror image).
__device__ __forceinline__ bool root_hit(const Ray& r) {
#pragma clang fp contract(off)
  const float inf = __builtin_inff();
  float n[3], f[3];
  const float o[3] = {r.ox, r.oy, r.oz};
  const float v[3] = {r.ix, r.iy, r.iz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (r.nonfin & (1u << a)) {
      const bool in = inside(o[a], -1.0f, 1.0f, r.oct & (1u << a));
      n[a] = in ? -inf : inf;
      f[a] = in ? inf : -inf;
    } else {
      n[a] = (-1.0f - o[a]) * v[a];
      f[a] = (1.0f - o[a]) * v[a];
    }
  }
  const float tn = __builtin_fmaxf(__builtin_fmaxf(n[0], n[1]), n[2]);
  const float tin = tn > 0.0f ? tn : 0.0f;
  const float tout = __builtin_fminf(__builtin_fminf(f[0], f[1]), f[2]);
  return tin < tout;
}

// One node as a single 64-bit buffer load.  A plain load lets the compiler
// merge it with the stack pop into one flat load through a selected pointer
// (LDS or global) behind a full wait at the loop head.
__device__ __forceinline__ svlf_node load_node(__amdgpu_buffer_rsrc_t rs, int32_t idx) {
  typedef unsigned int v2u_t __attribute__((ext_vector_type(2)));
  const v2u_t v = __builtin_bit_cast(
      v2u_t, __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<uint32_t>(idx) * 8u, 0, 0));
  svlf_node n;
  n.child = static_cast<int32_t>(v.x);
  n.mask = v.y;
  return n;
}

template <bool PAR, class Emit>
__device__ __forceinline__ int walk(const Ray& r, const svlf_node* __restrict__ nodes, int depth,
                                    int K, uint2* stk, int stride, const uint8_t* mtab, Emit emit) {
  // node indices are < 2^28, so byte offsets fit the 32-bit buffer range
  const __amdgpu_buffer_rsrc_t nrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<svlf_node*>(nodes), 0, 0x7FFFFFFF, 0x00020000);
  // leaf-level coordinate flips back to the octree's frame
  const uint32_t full = (1u << depth) - 1u;
  const uint32_t fx = (r.oct & 1u) ? full : 0u, fy = (r.oct & 2u) ? full : 0u,
                 fz = (r.oct & 4u) ? full : 0u;
  int count = 0;
  int level = 0;
  uint32_t ci = 0, cj = 0, ck = 0;   // mirrored cell coordinates
  svlf_node nd = load_node(nrs, 0);
  uint32_t rem = 0;
  while (true) {
    {
      const Kids kd = node_kids<PAR>(r, level, ci, cj, ck);
      rem = kid_hits(kd) & mtab[(r.oct << 8) | (nd.mask & 0xFFu)];
      if (level == depth - 1) {
        // children are leaves: emit them in order
        while (rem) {
          const uint32_t i = __builtin_ctz(rem);
          rem &= rem - 1;
          const uint32_t c = i ^ r.oct;
          float tin, tout;
          kid_interval(kd, i, tin, tout);
          const int32_t leaf = nd.child + __builtin_popcount(nd.mask & ((1u << c) - 1u));
          const uint32_t li = (2 * ci + (i & 1)) ^ fx, lj = (2 * cj + ((i >> 1) & 1)) ^ fy,
                         lk = (2 * ck + (i >> 2)) ^ fz;
          emit(count, leaf, tin, tout, li | (lj << 10) | (lk << 20));
          if (++count == K) return count;
        }
      }
    }
    // back up to the nearest level with a sibling left, then descend into it
    // in the same iteration
    while (rem == 0 && level > 0) {
      --level;
      ci >>= 1;
      cj >>= 1;
      ck >>= 1;
      const uint2 e = stk[level * stride];
      nd.child = static_cast<int32_t>(e.x);
      nd.mask = e.y & 0xFFu;
      rem = e.y >> 8;
    }
    if (rem == 0) break;
    const uint32_t i = __builtin_ctz(rem);
    rem &= rem - 1;
    const uint32_t c = i ^ r.oct;
    const int32_t idx = nd.child + __builtin_popcount(nd.mask & ((1u << c) - 1u));
    stk[level * stride] = make_uint2(static_cast<uint32_t>(nd.child), nd.mask | (rem << 8));
    ++level;
    ci = 2 * ci + (i & 1);
    cj = 2 * cj + ((i >> 1) & 1);
    ck = 2 * ck + (i >> 2);
    nd = load_node(nrs, idx);
  }
  return count;
}

// Walks the octree front to back; calls emit(slot, leaf, t_in, t_out, ijk)
// for the first K hit leaves (ijk = i | j << 10 | k << 20 in the octree's own
// frame).  `stk` points at this lane's entry of level 0 of an LDS array laid
// out [level][stride].  Returns the number of hits.  Rays parallel to an
// axis take a separate instance of the walk, so that the common one carries
// no code for them.
template <class Emit>
__device__ __forceinline__ int traverse(const Ray& r, const svlf_node* __restrict__ nodes,
                                        int depth, int K, uint2* stk, int stride,
                                        const uint8_t* mtab, Emit emit) {
  if (!r.valid || !root_hit(r)) return 0;
  if (r.nonfin) return walk<true>(r, nodes, depth, K, stk, stride, mtab, emit);
  return walk<false>(r, nodes, depth, K, stk, stride, mtab, emit);
}

}  // namespace svlf
