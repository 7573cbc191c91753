// Building blocks shared by the shading kernels: gfx950 MFMA wrappers and
// their operand layouts, bfloat16 rounding, block-wide scan and sum.
//
// MFMA layouts (32x32 result tiles, 64 lanes, lane group g = lane / 32):
//  * v_mfma_f32_32x32x16_bf16: A lane l holds row l % 32, K = 8 g + j
//    (j = 0..7); B lane l holds column l % 32, the same K; result register i
//    of lane l is row drow(i, g), column l % 32;
//  * v_mfma_f32_32x32x2f32: A / B lane l holds row / column l % 32, K = g;
//    the result layout is the same.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace svlf {
namespace detail {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// FP32 -> bfloat16 bits, round to nearest even: gfx950 converts in hardware
// (v_cvt_pk_bf16_f32, two values per instruction); on every non-NaN input it
// gives the bits of the integer rounding u + 0x7FFF + ((u >> 16) & 1) >> 16.
typedef __bf16 bf16x8_vt __attribute__((ext_vector_type(8)));
typedef float f32x8_vt __attribute__((ext_vector_type(8)));
__device__ __forceinline__ short bf16_rne(float x) {
  return __builtin_bit_cast(short, static_cast<__bf16>(x));
}
// Eight consecutive values of a tile, packed as one MFMA operand.
__device__ __forceinline__ s16x8 bf16_rne8(float a0, float a1, float a2, float a3, float a4,
                                           float a5, float a6, float a7) {
  const f32x8_vt v = {a0, a1, a2, a3, a4, a5, a6, a7};
  return __builtin_bit_cast(s16x8, __builtin_convertvector(v, bf16x8_vt));
}
__device__ __forceinline__ float bf16_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// The segment midpoint t = (t0 + t1) / 2 as an unevaluated sum hi + lo
// (TwoSum, exact), and the cell coordinate (o + t d - lo_plane) / h of the
// point there, evaluated with error-free transformations (TwoSum, FMA
// residual of the product): its error stays a few ulps of the result even
// when the origin lies far from the cell, where plain binary32 evaluation
// loses about |o| 2^-24 absolutely and 1/h (up to 2^9) scales that up.
__device__ __forceinline__ void midpoint2(float t0, float t1, float& hi, float& lo) {
#pragma clang fp contract(off)
  const float s = t0 + t1;
  const float v = s - t0;
  const float e = (t0 - (s - v)) + (t1 - v);
  hi = 0.5f * s;
  lo = 0.5f * e;
}
__device__ __forceinline__ float cell_coord(float o, float d, float thi, float tlo, float plane,
                                            float inv_h) {
#pragma clang fp contract(off)
  const float a = o - plane;
  const float av = a - o;
  const float ea = (o - (a - av)) + (-plane - av);
  const float b = thi * d;
  const float eb = __builtin_fmaf(thi, d, -b);
  const float s = a + b;
  const float sv = s - a;
  const float es = (a - (s - sv)) + (b - sv);
  return (s + (((ea + eb) + es) + tlo * d)) * inv_h;
}

__device__ __forceinline__ f32x16 mma(s16x8 a, s16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mma(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.0f;
  return z;
}

// Row (output feature within a 32-tile) of register i of a 32x32 MFMA result
// held by a lane of group g = lane / 32.
__device__ __forceinline__ constexpr int drow(int i, int g) { return 8 * (i >> 2) + 4 * g + (i & 3); }

// K index of step s, lane group g, element j for an operand that comes from
// a 32x32 result tile (D layout, see drow).
template <bool BF>
__device__ __forceinline__ int kmap_d(int s, int g, int j) {
  if (BF) return 32 * (s >> 1) + 8 * (2 * (s & 1) + (j >> 2)) + 4 * g + (j & 3);
  return 32 * (s >> 4) + 8 * ((s & 15) >> 2) + 4 * g + (s & 3);
}
// K index of an operand read row-wise from an LDS tile [hit][k].
template <bool BF>
__device__ __forceinline__ int kmap_x(int s, int g, int j) {
  if (BF) return 16 * s + 8 * g + j;
  return 4 * (2 * (s >> 2) + g) + (s & 3);
}

constexpr int align16(int x) { return (x + 15) & ~15; }
constexpr int align8(int x) { return (x + 7) & ~7; }
constexpr int align32(int x) { return (x + 31) & ~31; }

__device__ __forceinline__ void relu16(f32x16& t) {
#pragma unroll
  for (int i = 0; i < 16; ++i) t[i] = t[i] > 0.0f ? t[i] : 0.0f;
}

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// Exclusive prefix sum of v over the block's NW waves (scr: NW ints of LDS).
// `before_sync(prefix)` runs in every thread before the closing barrier, so
// that LDS it writes is visible to the block when the scan returns.
template <int NW, class F>
__device__ __forceinline__ int block_excl_scan(int v, int* scr, int& total, F&& before_sync) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) scr[w] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int t = scr[i];
    pre += (i < w) ? t : 0;
    tot += t;
  }
  before_sync(pre + x - v);
  __syncthreads();
  total = tot;
  return pre + x - v;
}
template <int NW>
__device__ __forceinline__ int block_excl_scan(int v, int* scr, int& total) {
  return block_excl_scan<NW>(v, scr, total, [](int) {});
}

// Transposes the first ROWS columns of an LDS tile X [WIN][XS] (one row per
// hit; columns >= REAL read as zero) into AT [ROWS][TS] (one row per column,
// AT[c * TS + hit]).  Each thread moves a block of 2 hits x 8 columns
// (BF16) or 1 hit x 4 columns (FP32): 16-byte reads of X rows, and for BF16
// 32-bit writes that pack the two hits' values, so that consecutive lanes
// touch consecutive LDS words (a one-element-per-lane transpose reads X at
// the row stride, a 4-way bank conflict for these strides).
template <bool BF, int WIN, int XS, int TS, int REAL, int ROWS, int NT, class El>
__device__ __forceinline__ void transpose_tile(const El* X, El* AT, int tid) {
  if constexpr (BF) {
    static_assert(XS % 8 == 0 && TS % 2 == 0 && WIN % 2 == 0 && ROWS % 8 == 0, "BF16 transpose blocks");
    constexpr int HP = WIN / 2, UNITS = HP * (ROWS / 8);
    for (int u = tid; u < UNITS; u += NT) {
      const int hp = u % HP, ch = u / HP, c0 = 8 * ch;
      uint4 r0 = make_uint4(0u, 0u, 0u, 0u), r1 = r0;
      if (c0 < REAL) {
        r0 = *reinterpret_cast<const uint4*>(X + (2 * hp) * XS + c0);
        r1 = *reinterpret_cast<const uint4*>(X + (2 * hp + 1) * XS + c0);
      }
      const uint32_t a[4] = {r0.x, r0.y, r0.z, r0.w}, b[4] = {r1.x, r1.y, r1.z, r1.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        uint32_t* lo = reinterpret_cast<uint32_t*>(AT + (c0 + 2 * k) * TS + 2 * hp);
        uint32_t* hi = reinterpret_cast<uint32_t*>(AT + (c0 + 2 * k + 1) * TS + 2 * hp);
        *lo = (a[k] & 0xFFFFu) | (b[k] << 16);
        *hi = (a[k] >> 16) | (b[k] & 0xFFFF0000u);
      }
    }
  } else {
    static_assert(XS % 4 == 0 && ROWS % 4 == 0, "FP32 transpose blocks");
    constexpr int UNITS = WIN * (ROWS / 4);
    for (int u = tid; u < UNITS; u += NT) {
      const int hh = u % WIN, c0 = 4 * (u / WIN);
      f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
      if (c0 < REAL) v = *reinterpret_cast<const f32x4*>(X + hh * XS + c0);
#pragma unroll
      for (int k = 0; k < 4; ++k) AT[(c0 + k) * TS + hh] = v[k];
    }
  }
}

template <int NW>
__device__ __forceinline__ float block_sum(float v, float* scr) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) scr[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.0f;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += scr[i];
  __syncthreads();
  return t;
}

}  // namespace detail
}  // namespace svlf
