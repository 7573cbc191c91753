// Shading kernels of the paper's voxel light-field function (SVLF sections
// 4.1-4.3): per crossed voxel, a density decoder F_T reads the features
// interpolated at the entry and exit points x1, x2 together with the ray
// parameterisation r (the two points where the ray meets the voxel's
// bounding sphere, as unit vectors from its centre) and outputs the optical
// thickness tau and the mixing factor eta; a colour decoder F_C reads the
// features interpolated at the surface point x_s = eta x1 + (1 - eta) x2 with
// r (and the view direction on request) and outputs the colour; Eq. 3
// composites front to back.
//
// Each scene's feature table holds the two embedding collections as two
// blocks, Z_T [n_vertices][64] followed by Z_C [n_vertices][32] (so that one
// of them can be trained or frozen as one contiguous array).  Decoder
// inputs are ordered [features | r | (d)].
//
// Three kernels, all persistent over 256-ray items with ray-aligned hit
// windows (as the single-decoder kernels):
//  * k_density: records, gather of the 8 corner rows of Z_T (one gather
//    serves x1 and x2: both lie on the same voxel), r, F_T on MFMA, and per
//    hit tau, eta and the surface point (written to the workspace); in
//    backward mode it recomputes F_T, back-propagates dL/d(o_T0, o_T1) left
//    by the colour kernel, accumulates F_T's weight gradients and scatters
//    dL/dZ_T;
//  * k_color: gather of Z_C at the surface point, F_C on MFMA (hidden
//    activations kept transposed in LDS in backward mode), Eq. 3, and in
//    backward / train mode the compositing backward, F_C's backward, the
//    scatter of dL/dZ_C, and dL/deta through the interpolation at x_s;
//  * k_lf_pack: MFMA operand packs of both decoders (forward and transposed)
//    from the FP32 masters, read by the kernels from global memory (L2).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mfma_common.hpp"
#include "svlf_internal.hpp"

namespace svlf {
namespace {

using namespace detail;

constexpr int kThreads = 256;
static_assert(kThreads == kRaysPerBlock, "one ray per thread in a work item");
constexpr int kWaves = 4;

// ------------------------------------------------------------ decoder geometry

// A ReLU MLP IN0 -> H (NH hidden layers) -> OUT (<= 32); BM0 = number of
// leading inputs whose gradient is needed (the features).
template <bool BF, int IN0_, int H_, int NH_, int OUT_, int BM0_>
struct Mlp {
  static constexpr int IN0 = IN0_, H = H_, NH = NH_, OUT = OUT_, BM0 = BM0_;
  static constexpr int KS = BF ? 16 : 2;
  static constexpr int NL = NH + 1;
  static constexpr int IN0P = BF ? align16(IN0) : align8(IN0);
  static constexpr int MTH = H / 32;
  static constexpr int in_r(int l) { return l == 0 ? IN0 : H; }
  static constexpr int in_p(int l) { return l == 0 ? IN0P : H; }
  static constexpr int out_r(int l) { return l == NH ? OUT : H; }
  static constexpr int out_p(int l) { return l == NH ? 32 : H; }
  static constexpr int bm(int l) { return l == 0 ? BM0 : H; }
  static constexpr int fwd_off(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += out_p(i) * in_p(i);
    return o;
  }
  static constexpr int bwd_off(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += bm(i) * out_p(i);
    return o;
  }
  static constexpr int bias_off(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += out_p(i);
    return o;
  }
  static constexpr int par_w(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += out_r(i) * in_r(i) + out_r(i);
    return o;
  }
  static constexpr int par_b(int l) { return par_w(l) + out_r(l) * in_r(l); }
  static constexpr int dw_mt(int l) { return out_p(l) / 32; }
  static constexpr int dw_nt(int l) { return align32(in_r(l)) / 32; }
  static constexpr int dw_off(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += dw_mt(i) * dw_nt(i);
    return o;
  }
  static constexpr int NPARAMS = par_w(NL);
  static constexpr int FWD = fwd_off(NL);
  static constexpr int BWD = bwd_off(NL);
  static constexpr int BIAS = bias_off(NL);
  static constexpr int NDW = dw_off(NL);
  static constexpr int NBIAS = NH * H + OUT;
  // pack layout (elements of the operand type, then FP32 biases)
  static constexpr size_t pack_bytes(int eb) {
    return ((static_cast<size_t>(FWD + BWD) * eb + 15) / 16) * 16 + BIAS * 4;
  }
  static_assert(OUT <= 32 && H % 32 == 0 && BM0 % 32 == 0 && BM0 <= IN0, "geometry");
};

template <bool BF, int VD>
struct Dec {
  using T = Mlp<BF, 2 * kLfCT + 6, kLfH, kLfNHT, 2, 2 * kLfCT>;
  using C = Mlp<BF, kLfCC + 6 + 3 * VD, kLfH, kLfNHC, 3, kLfCC>;
};

template <bool BF>
struct Types {
  using Elem = typename std::conditional<BF, uint16_t, float>::type;
  using El = Elem;
  using Op = typename std::conditional<BF, s16x8, float>::type;
  static constexpr int EB = BF ? 2 : 4;
};

template <bool BF>
__device__ __forceinline__ typename Types<BF>::Elem to_el(float v) {
  if constexpr (BF) return static_cast<uint16_t>(bf16_rne(v));
  else return v;
}

// operand (mt, s) of a packed matrix in global memory
template <bool BF>
__device__ __forceinline__ typename Types<BF>::Op gop(const typename Types<BF>::Elem* __restrict__ p,
                                                      int mt, int s, int steps, int lane) {
  if constexpr (BF)
    return *reinterpret_cast<const s16x8*>(p + (static_cast<size_t>(mt * steps + s) * 64 + lane) * 8);
  else
    return p[(mt * steps + s) * 64 + lane];
}

// Weight operands are read with buffer loads: the per-(tile, step) offset is
// a scalar (SGPR) and only the lane offset lives in a VGPR, so a fully
// unrolled layer needs no per-load address registers; loads past the end of
// the pack return 0.
typedef int v4i_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pack_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}
template <bool BF>
__device__ __forceinline__ typename Types<BF>::Op gopb(__amdgpu_buffer_rsrc_t rs, int byte_base,
                                                       int mt, int s, int steps, int lane) {
  if constexpr (BF) {
    const v4i_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, lane * 16, byte_base + (mt * steps + s) * 1024, 0);
    return __builtin_bit_cast(s16x8, v);
  } else {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4, byte_base + (mt * steps + s) * 256, 0));
  }
}

// B operand of step s from D-layout tiles
template <bool BF>
__device__ __forceinline__ typename Types<BF>::Op dop(const f32x16* t, int s) {
  if constexpr (BF) {
    s16x8 b;
    const f32x16& tt = t[s >> 1];
    {
      const int o = 8 * (s & 1);
      b = bf16_rne8(tt[o], tt[o + 1], tt[o + 2], tt[o + 3], tt[o + 4], tt[o + 5], tt[o + 6], tt[o + 7]);
    }
    return b;
  } else {
    return t[s >> 4][s & 15];
  }
}

__device__ __forceinline__ f32x16 gbias(const float* __restrict__ b, int mt, int g) {
  f32x16 t;
  const float* p = b + 32 * mt + 4 * g;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = *reinterpret_cast<const float4*>(p + 8 * q);
    t[4 * q + 0] = v.x;
    t[4 * q + 1] = v.y;
    t[4 * q + 2] = v.z;
    t[4 * q + 3] = v.w;
  }
  return t;
}

template <bool BF>
struct ActT;
template <>
struct ActT<true> {
  s16x8 lo, hi;
  __device__ __forceinline__ void set(const f32x16& t) {
    lo = bf16_rne8(t[0], t[1], t[2], t[3], t[4], t[5], t[6], t[7]);
    hi = bf16_rne8(t[8], t[9], t[10], t[11], t[12], t[13], t[14], t[15]);
  }
  __device__ __forceinline__ bool positive(int i) const { return (i < 8 ? lo[i] : hi[i - 8]) > 0; }
  __device__ __forceinline__ uint16_t elem(int i) const {
    return static_cast<uint16_t>(i < 8 ? lo[i] : hi[i - 8]);
  }
};
template <>
struct ActT<false> {
  f32x16 v;
  __device__ __forceinline__ void set(const f32x16& t) { v = t; }
  __device__ __forceinline__ bool positive(int i) const { return v[i] > 0.0f; }
  __device__ __forceinline__ float elem(int i) const { return v[i]; }
};

// Keeps the compiler from hoisting the weight loads of a whole layer ahead
// of its MFMAs (they come from global memory; hoisting them all would need a
// register per operand): no instruction moves across the fence, which is
// placed every CH K-steps of a fully unrolled loop.
template <int CH>
__device__ __forceinline__ void chunk_fence(int s) {
  if ((s + 1) % CH == 0) __builtin_amdgcn_sched_barrier(0);
}
template <bool BF>
constexpr int kChunk = BF ? 4 : 16;

// ------------------------------------------------------------ packing

// Packs one decoder from its FP32 layers (params) into [fwd][bwd] operand
// arrays (elements) followed by the padded biases (FP32).
template <bool BF, class M>
__device__ void pack_decoder(const float* __restrict__ params, char* __restrict__ out) {
  using El = typename Types<BF>::Elem;
  constexpr int E = BF ? 8 : 1;
  El* fp = reinterpret_cast<El*>(out);
  El* bp = fp + M::FWD;
  float* bias = reinterpret_cast<float*>(out + M::pack_bytes(Types<BF>::EB) - M::BIAS * 4);
  const int stride = gridDim.x * blockDim.x;
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
  static_for<M::NL>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    constexpr int IW = M::in_p(l), OW = M::out_p(l), IR = M::in_r(l), OR = M::out_r(l);
    constexpr int STEPS = IW / M::KS;
    const float* W = params + M::par_w(l);
    const float* b = params + M::par_b(l);
    El* f = fp + M::fwd_off(l);
    for (int e = t0; e < OW * IW; e += stride) {
      const int j = e % E, lane = (e / E) % 64, s = (e / (E * 64)) % STEPS, mt = e / (E * 64 * STEPS);
      const int m = 32 * mt + (lane & 31), g = lane >> 5;
      const int k = (l == 0) ? kmap_x<BF>(s, g, j) : kmap_d<BF>(s, g, j);
      f[e] = to_el<BF>((m < OR && k < IR) ? W[m * IR + k] : 0.0f);
    }
    // transposed: M = layer input (the first bm(l) only), K = layer output
    constexpr int BM = M::bm(l), BSTEPS = OW / M::KS;
    El* bb = bp + M::bwd_off(l);
    for (int e = t0; e < BM * OW; e += stride) {
      const int j = e % E, lane = (e / E) % 64, s = (e / (E * 64)) % BSTEPS, mt = e / (E * 64 * BSTEPS);
      const int m = 32 * mt + (lane & 31), g = lane >> 5;
      const int k = kmap_d<BF>(s, g, j);
      bb[e] = to_el<BF>((m < IR && k < OR) ? W[k * IR + m] : 0.0f);
    }
    for (int r = t0; r < OW; r += stride) bias[M::bias_off(l) + r] = r < OR ? b[r] : 0.0f;
  });
}

template <bool BF, int VD>
__global__ __launch_bounds__(kThreads) void k_lf_pack(const float* __restrict__ params,
                                                      char* __restrict__ packs) {
  using D = Dec<BF, VD>;
  pack_decoder<BF, typename D::T>(params, packs);
  pack_decoder<BF, typename D::C>(params + D::T::NPARAMS,
                                  packs + D::T::pack_bytes(Types<BF>::EB));
}

// ------------------------------------------------------------ shared LDS

extern __shared__ __attribute__((aligned(16))) char g_lds[];

// Hit window: the rays of the item whose hits all fit in [s0, s0 + WIN);
// returns s1 (end of the window) and publishes hit -> (ray lane | slot << 16).
// Work items of a persistent light-field kernel: dealt round-robin over the
// grid (the logical block index groups the blocks of one XCD), except the
// last two rounds, which `counter` hands out in order to whichever block
// asks first.  Uniform over the block; scr[10] carries the counter's value.
struct ItemDeal {
  int G, lb, nb, n_static;
  int32_t* counter;
  __device__ int first(int* scr) { return lb < n_static ? lb : tail(scr); }
  __device__ int next(int item, int* scr) { return item + G < n_static ? item + G : tail(scr); }
  __device__ int tail(int* scr) {
    if (n_static == nb) return nb;
    if (threadIdx.x == 0) scr[10] = n_static + atomicAdd(counter, 1);
    __syncthreads();
    const int it = scr[10];
    __syncthreads();
    return it;
  }
};
__device__ __forceinline__ ItemDeal item_deal(const LfArgs& a, int which) {
  ItemDeal d;
  d.G = gridDim.x;
  const int b = blockIdx.x;
  d.lb = (d.G % 8 == 0) ? (b % 8) * (d.G / 8) + b / 8 : b;
  d.nb = a.tab.n_blocks;
  d.counter = a.item_counters != nullptr ? a.item_counters + which : nullptr;
  const int n_tail = d.counter != nullptr ? (d.nb < 2 * d.G ? d.nb : 2 * d.G) : 0;
  d.n_static = d.nb - n_tail;
  return d;
}

template <int WIN>
__device__ __forceinline__ int open_window(int s0, int total, int off, int count, int* scr,
                                           int* hmap, bool& in_win) {
  const int tid = threadIdx.x;
  if (tid == 0) scr[8] = total;
  __syncthreads();
  const bool started = count > 0 && off >= s0;
  in_win = started && off + count <= s0 + WIN;
  if (started && !in_win) atomicMin(&scr[8], off);
  __syncthreads();
  const int s1 = scr[8];
  if (in_win)
    for (int q = 0; q < count; ++q) hmap[off - s0 + q] = tid | (q << 16);
  __syncthreads();
  return s1;
}

// The same window from a map of all of the item's hits (hit -> lane |
// slot << 16, written once per item): the window ends at the start of the
// ray that holds hit s0 + WIN (no ray is longer than a window).  No barrier.
template <int WIN>
__device__ __forceinline__ int open_window_imap(int s0, int total, int off, int count,
                                                const int* imap, bool& in_win) {
  const int p = s0 + WIN;
  const int s1 = p < total ? p - (imap[p] >> 16) : total;
  in_win = count > 0 && off >= s0 && off + count <= s1;
  return s1;
}

__device__ __forceinline__ int scene_of(const SceneTable& tab, int item) {
  int si = 0;
  while (si + 1 < tab.n && item >= tab.s[si + 1].block_begin) ++si;
  return si;
}

__device__ __forceinline__ void trilinear(float ux, float uy, float uz, float (&w)[8]) {
  const float wx[2] = {1.0f - ux, ux}, wy[2] = {1.0f - uy, uy}, wz[2] = {1.0f - uz, uz};
#pragma unroll
  for (int j = 0; j < 8; ++j) w[j] = wx[j & 1] * wy[(j >> 1) & 1] * wz[j >> 2];
}

__device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// Bounding-sphere parameterisation relative to the voxel centre, from the
// entry point's offset y1 = x1 - c (small: on the voxel boundary) and the
// direction d: the sphere |y1 + s d|^2 = R^2 with R^2 = 3 h^2 / 4.
__device__ __forceinline__ void sphere_r(float y0, float y1, float y2, float dx, float dy, float dz,
                                         float h, float (&r)[6]) {
  const float a = dx * dx + dy * dy + dz * dz;
  const float b = dx * y0 + dy * y1 + dz * y2;
  const float cx = dy * y2 - dz * y1, cy = dz * y0 - dx * y2, cz = dx * y1 - dy * y0;
  const float disc = a * (0.75f * h * h) - (cx * cx + cy * cy + cz * cz);
  const float sq = sqrtf(fmaxf(disc, 0.0f));
  const float sa = (-b - sq) / a, sb = (-b + sq) / a;
  const float p[2][3] = {{y0 + sa * dx, y1 + sa * dy, y2 + sa * dz},
                         {y0 + sb * dx, y1 + sb * dy, y2 + sb * dz}};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float inv = 1.0f / sqrtf(p[k][0] * p[k][0] + p[k][1] * p[k][1] + p[k][2] * p[k][2]);
    r[3 * k + 0] = p[k][0] * inv;
    r[3 * k + 1] = p[k][1] * inv;
    r[3 * k + 2] = p[k][2] * inv;
  }
}

// dW tiles of layer l for one window (K = the window's hits, read
// transposed from LDS: GZ rows = layer outputs, AT rows = layer inputs),
// added into this block's partial sums (FP32, parameter layout).  A tile is
// owned by one wave, so the additions never collide; they are
// workgroup-scope atomics only so that the wave does not wait for a load
// of the old values (the block's partials are private to the block and are
// read by the reduction kernel after this kernel ends).  Only one tile is
// live in registers at a time.
template <bool BF, class M, int l, int WIN, int TS>
__device__ __forceinline__ void dw_window(const typename Types<BF>::El* GZ,
                                          const typename Types<BF>::El* AT, float* __restrict__ part,
                                          int wave, int lane) {
  using El = typename Types<BF>::El;
  constexpr int MT = M::dw_mt(l), NT = M::dw_nt(l), T0 = M::dw_off(l);
  constexpr int KSTEPS = WIN / M::KS;
  constexpr int IR = M::in_r(l), OR = M::out_r(l);
  const int g = lane >> 5;
#pragma unroll 1
  for (int t = 0; t < MT * NT; ++t) {
    if ((T0 + t) % kWaves != wave) continue;
    const int mt = t / NT, nt = t % NT;
    const El* ga_ = GZ + (32 * mt + (lane & 31)) * TS;
    const El* gb_ = AT + (32 * nt + (lane & 31)) * TS;
    f32x16 acc = zero16();
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
      if constexpr (BF) {
        const s16x8 av = *reinterpret_cast<const s16x8*>(ga_ + 16 * s + 8 * g);
        const s16x8 bv = *reinterpret_cast<const s16x8*>(gb_ + 16 * s + 8 * g);
        acc = mma(av, bv, acc);
      } else {
        acc = mma(ga_[2 * s + g], gb_[2 * s + g], acc);
      }
      chunk_fence<BF ? 2 : 8>(s);
    }
    const int col = 32 * nt + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int rowo = 32 * mt + drow(i, g);
      if (rowo < OR && col < IR)
        __hip_atomic_fetch_add(part + M::par_w(l) + rowo * IR + col, acc[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// ------------------------------------------------------------ density kernel

template <int P, int MODE>
struct DCfg {
  static constexpr bool BF = P == 1;
  static constexpr bool BWD = MODE != kForward;
  using M = typename Dec<BF, 0>::T;
  using El = typename Types<BF>::Elem;
  static constexpr int EB = Types<BF>::EB;
  static constexpr int WIN = BF ? 128 : 64;
  static constexpr int NTILE = WIN / 32;
  static constexpr int XS = M::IN0P + (BF ? 8 : 4);
  static constexpr int TS = WIN + (BF ? 8 : 1);
  static constexpr int XT_ROWS = align32(M::IN0);        // rows of X^T read by the dW tiles
  // LDS: records (64 B / hit), X, then (backward) GZ [128][TS] and AT [XT_ROWS][TS]
  static constexpr int L_REC = 0;
  static constexpr int L_X = L_REC + WIN * 64;
  static constexpr int L_GZ = align16(L_X + WIN * XS * EB);
  static constexpr int L_AT = align16(L_GZ + (BWD ? kLfH * TS * EB : 0));
  static constexpr int L_MAP = align16(L_AT + (BWD ? XT_ROWS * TS * EB : 0));
  // hit map: all of a work item's hits (IMAP: backward, where it fits) or the window's
  static constexpr bool IMAP = BWD && align16(L_MAP + kThreads * SVLF_MAX_K * 4) + 64 <= 160 * 1024;
  static constexpr int L_SCR = align16(L_MAP + (IMAP ? kThreads * SVLF_MAX_K : WIN) * 4);
  static constexpr int LDS = L_SCR + 64;
  static_assert(LDS <= 160 * 1024, "LDS");
  static_assert(!BWD || WIN * 2 * kLfCT * 4 <= L_MAP - L_GZ, "dL/dz staging fits in GZ + AT");
  static_assert(M::NBIAS <= kThreads, "one thread per bias entry writes its combined gradient");
};

// Bias gradients of layer l (ROWS real rows of width RW in GZ, one column
// per hit of the window): thread (row = tid % RW, part = tid / RW) adds its
// slice of the window's hits to its own register; the parts are combined
// once per block by bias_combine.
template <bool BF, int RW, int ROWS, int WIN, int TS, class El>
__device__ __forceinline__ void bias_part(const El* GZ, int tid, float& acc) {
  constexpr int HP = WIN / (kThreads / RW);
  static_assert(kThreads % RW == 0 && (!BF || HP % 8 == 0), "bias-gradient parts");
  const int row = tid % RW, pt = tid / RW;
  if (row >= ROWS) return;
  const El* gr = GZ + row * TS + pt * HP;
  float sum = 0.0f;
  if constexpr (BF) {
#pragma unroll
    for (int hh = 0; hh < HP; hh += 8) {
      const s16x8 v = *reinterpret_cast<const s16x8*>(gr + hh);
#pragma unroll
      for (int j = 0; j < 8; ++j) sum += bf16_f32(static_cast<uint16_t>(v[j]));
    }
  } else {
#pragma unroll
    for (int hh = 0; hh < HP; ++hh) sum += gr[hh];
  }
  acc += sum;
}

// Sums every layer's parts (through `lds`, NL * kThreads floats) into the
// block's partial gradient.  Called by all threads.
template <class M>
__device__ __forceinline__ void bias_combine(const float (&acc)[M::NL], float* lds, float* part,
                                             int tid) {
  __syncthreads();
#pragma unroll
  for (int l = 0; l < M::NL; ++l) lds[l * kThreads + tid] = acc[l];
  __syncthreads();
  static_for<M::NL>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    constexpr int RW = M::out_p(l);
    if (tid < M::out_r(l)) {
      float sum = 0.0f;
#pragma unroll
      for (int pt = 0; pt < kThreads / RW; ++pt) sum += lds[l * kThreads + pt * RW + tid];
      part[M::par_b(l) + tid] = sum;
    }
  });
}

// Density record (64 B): unclamped cell coordinates of x1 and x2, t_in,
// t_out and the 8 corner ids.
struct DRec {
  float u1[3];
  float u2[3];
  float tin, tout;
  int4 v0, v1;
};

template <class CF>
__device__ __forceinline__ typename CF::El* dX() { return reinterpret_cast<typename CF::El*>(g_lds + CF::L_X); }

template <int P, int MODE>
__global__ __launch_bounds__(kThreads, 1) void k_density(LfArgs a) {
  using CF = DCfg<P, MODE>;
  using M = typename CF::M;
  using El = typename CF::El;
  constexpr bool BF = CF::BF;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;
  DRec* rec = reinterpret_cast<DRec*>(g_lds + CF::L_REC);
  int* hmap = reinterpret_cast<int*>(g_lds + CF::L_MAP);
  int* scr = reinterpret_cast<int*>(g_lds + CF::L_SCR);
  const auto rs = pack_rsrc(a.packs, static_cast<int>(M::pack_bytes(CF::EB)));
  constexpr int BWD_BASE = M::FWD * CF::EB;
  const float* bias = reinterpret_cast<const float*>(static_cast<const char*>(a.packs) +
                                                     M::pack_bytes(CF::EB) - M::BIAS * 4);

  float* part = a.partT + static_cast<int64_t>(blockIdx.x) * M::NPARAMS;
  if constexpr (CF::BWD) {
    for (int i = tid; i < M::NPARAMS; i += kThreads) part[i] = 0.0f;
    __syncthreads();
  }
  float dbp[M::NL];
#pragma unroll
  for (int l = 0; l < M::NL; ++l) dbp[l] = 0.0f;

  ItemDeal deal = item_deal(a, CF::BWD ? 2 : 0);
  for (int item = deal.first(scr); item < deal.nb; item = deal.next(item, scr)) {
    const DevScene& sc = a.tab.s[scene_of(a.tab, item)];
    const ItemRays ir = item_rays(sc, item);
    const int64_t r = ir.ray(tid);
    const int count = r < sc.ray_end ? a.cnt[r] : 0;
    const float h = __int_as_float((128 - sc.depth) << 23);
    const float inv_h = __int_as_float((126 + sc.depth) << 23);
    int total;
    const int off = block_excl_scan<kWaves>(count, scr, total, [&](int o) {
      if constexpr (CF::IMAP)
        for (int q = 0; q < count; ++q) hmap[o + q] = tid | (q << 16);
    });
    for (int s0 = 0; s0 < total;) {
      bool in_win;
      const int s1 = CF::IMAP ? open_window_imap<CF::WIN>(s0, total, off, count, hmap, in_win)
                              : open_window<CF::WIN>(s0, total, off, count, scr, hmap, in_win);
      const int* wmap = CF::IMAP ? hmap + s0 : hmap;    // the window's map entries
      const int tw = s1 - s0;
      (void)in_win;
      if (BF && CF::BWD && a.xsave != nullptr) {
        // the forward pass saved this window's decoder inputs: one thread per
        // hit rebuilds its record, the rows stream back 16 B per thread
        for (int hh = tid; hh < CF::WIN; hh += kThreads) {
          if (hh < tw) {
            const int mp = wmap[hh];
            const int64_t ray = ir.ray(mp & 0xFFFF);
            const HitRec hr = a.hits[ray * a.K + (mp >> 16)];
            const float ox = a.o[3 * ray], oy = a.o[3 * ray + 1], oz = a.o[3 * ray + 2];
            const float dx = a.d[3 * ray], dy = a.d[3 * ray + 1], dz = a.d[3 * ray + 2];
            const int4* lc = reinterpret_cast<const int4*>(sc.leaf_corners + 8 * static_cast<int64_t>(hr.leaf));
            const float lx = -1.0f + static_cast<float>(hr.ijk & 1023u) * h;
            const float ly = -1.0f + static_cast<float>((hr.ijk >> 10) & 1023u) * h;
            const float lz = -1.0f + static_cast<float>(hr.ijk >> 20) * h;
            DRec rc;
            rc.u1[0] = cell_coord(ox, dx, hr.tin, 0.0f, lx, inv_h);
            rc.u1[1] = cell_coord(oy, dy, hr.tin, 0.0f, ly, inv_h);
            rc.u1[2] = cell_coord(oz, dz, hr.tin, 0.0f, lz, inv_h);
            rc.u2[0] = cell_coord(ox, dx, hr.tout, 0.0f, lx, inv_h);
            rc.u2[1] = cell_coord(oy, dy, hr.tout, 0.0f, ly, inv_h);
            rc.u2[2] = cell_coord(oz, dz, hr.tout, 0.0f, lz, inv_h);
            rc.tin = hr.tin;
            rc.tout = hr.tout;
            rc.v0 = lc[0];
            rc.v1 = lc[1];
            rec[hh] = rc;
          }
        }
        constexpr int CPR = M::IN0P * 2 / 16;   // 16-byte chunks per row
        for (int e = tid; e < CF::WIN * CPR; e += kThreads) {
          const int hh = e / CPR, c = e % CPR;
          uint4 v = make_uint4(0u, 0u, 0u, 0u);
          if (hh < tw) {
            const int mp = wmap[hh];
            const int64_t slot = ir.ray(mp & 0xFFFF) * a.K + (mp >> 16);
            v = *reinterpret_cast<const uint4*>(a.xsave + slot * M::IN0P + 8 * c);
          }
          *reinterpret_cast<uint4*>(dX<CF>() + hh * CF::XS + 8 * c) = v;
        }
      } else {
      // gather: thread q of a hit owns VPT channels of psi(x1) and psi(x2)
      {
        constexpr int TPH = kLfCT * CF::EB / 16;
        constexpr int VPT = 16 / CF::EB;
        constexpr int HPP = kThreads / TPH;
        const int q = tid % TPH;
#pragma unroll 1
        for (int hh = tid / TPH; hh < CF::WIN; hh += HPP) {
          float v1[VPT], v2[VPT];
#pragma unroll
          for (int i = 0; i < VPT; ++i) v1[i] = v2[i] = 0.0f;
          float rr[6] = {0, 0, 0, 0, 0, 0};
          if (hh < tw) {
            const int mp = wmap[hh];
            const int64_t ray = ir.ray(mp & 0xFFFF);
            const HitRec hr = a.hits[ray * a.K + (mp >> 16)];
            const float ox = a.o[3 * ray], oy = a.o[3 * ray + 1], oz = a.o[3 * ray + 2];
            const float dx = a.d[3 * ray], dy = a.d[3 * ray + 1], dz = a.d[3 * ray + 2];
            const int4* lc = reinterpret_cast<const int4*>(sc.leaf_corners + 8 * static_cast<int64_t>(hr.leaf));
            const int4 c0 = lc[0], c1 = lc[1];
            const float lx = -1.0f + static_cast<float>(hr.ijk & 1023u) * h;
            const float ly = -1.0f + static_cast<float>((hr.ijk >> 10) & 1023u) * h;
            const float lz = -1.0f + static_cast<float>(hr.ijk >> 20) * h;
            const float u1[3] = {cell_coord(ox, dx, hr.tin, 0.0f, lx, inv_h),
                                 cell_coord(oy, dy, hr.tin, 0.0f, ly, inv_h),
                                 cell_coord(oz, dz, hr.tin, 0.0f, lz, inv_h)};
            const float u2[3] = {cell_coord(ox, dx, hr.tout, 0.0f, lx, inv_h),
                                 cell_coord(oy, dy, hr.tout, 0.0f, ly, inv_h),
                                 cell_coord(oz, dz, hr.tout, 0.0f, lz, inv_h)};
            if (q == 0) {
              DRec rc;
              rc.u1[0] = u1[0]; rc.u1[1] = u1[1]; rc.u1[2] = u1[2];
              rc.u2[0] = u2[0]; rc.u2[1] = u2[1]; rc.u2[2] = u2[2];
              rc.tin = hr.tin;
              rc.tout = hr.tout;
              rc.v0 = c0;
              rc.v1 = c1;
              rec[hh] = rc;
              const float hc = 0.5f * h;
              sphere_r(cell_coord(ox, dx, hr.tin, 0.0f, lx + hc, 1.0f),
                       cell_coord(oy, dy, hr.tin, 0.0f, ly + hc, 1.0f),
                       cell_coord(oz, dz, hr.tin, 0.0f, lz + hc, 1.0f), dx, dy, dz, h, rr);
            }
            float w1[8], w2[8];
            trilinear(clamp01(u1[0]), clamp01(u1[1]), clamp01(u1[2]), w1);
            trilinear(clamp01(u2[0]), clamp01(u2[1]), clamp01(u2[2]), w2);
            const int vid[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              if constexpr (BF) {
                const uint4 raw = *reinterpret_cast<const uint4*>(sc.feat16 + static_cast<int64_t>(vid[j]) * kLfCT + 8 * q);
                const uint32_t w4[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const float f0 = bf16_f32(static_cast<uint16_t>(w4[i] & 0xFFFFu));
                  const float f1 = bf16_f32(static_cast<uint16_t>(w4[i] >> 16));
                  v1[2 * i] += w1[j] * f0;
                  v1[2 * i + 1] += w1[j] * f1;
                  v2[2 * i] += w2[j] * f0;
                  v2[2 * i + 1] += w2[j] * f1;
                }
              } else {
                const float4 f = *reinterpret_cast<const float4*>(sc.feat32 + static_cast<int64_t>(vid[j]) * kLfCT + 4 * q);
                v1[0] += w1[j] * f.x; v1[1] += w1[j] * f.y; v1[2] += w1[j] * f.z; v1[3] += w1[j] * f.w;
                v2[0] += w2[j] * f.x; v2[1] += w2[j] * f.y; v2[2] += w2[j] * f.z; v2[3] += w2[j] * f.w;
              }
            }
          }
          El* xr = dX<CF>() + hh * CF::XS;
#pragma unroll
          for (int i = 0; i < VPT; ++i) {
            xr[VPT * q + i] = to_el<BF>(v1[i]);
            xr[kLfCT + VPT * q + i] = to_el<BF>(v2[i]);
          }
          if (q == 0) {
#pragma unroll
            for (int i = 2 * kLfCT; i < M::IN0P; ++i) xr[i] = to_el<BF>(i < 2 * kLfCT + 6 ? rr[i - 2 * kLfCT] : 0.0f);
          }
        }
      }
      }
      __syncthreads();
      if (BF && !CF::BWD && a.xsave != nullptr) {
        // save the window's decoder inputs for the backward pass
        constexpr int CPR = M::IN0P * 2 / 16;
        for (int e = tid; e < tw * CPR; e += kThreads) {
          const int hh = e / CPR, c = e % CPR;
          const int mp = wmap[hh];
          const int64_t slot = ir.ray(mp & 0xFFFF) * a.K + (mp >> 16);
          *reinterpret_cast<uint4*>(a.xsave + slot * M::IN0P + 8 * c) =
              *reinterpret_cast<const uint4*>(dX<CF>() + hh * CF::XS + 8 * c);
        }
      }

      const int n0 = 32 * wave;
      const bool has_tile = wave < CF::NTILE && n0 < tw;
      ActT<BF> act[M::MTH];
      f32x16 o;
      if (has_tile) {
        const int row = n0 + (lane & 31);
        f32x16 hdn[M::MTH];
        constexpr int S0 = M::IN0P / M::KS;
#pragma unroll
        for (int mt = 0; mt < M::MTH; ++mt) hdn[mt] = gbias(bias, mt, g);
#pragma unroll
        for (int s = 0; s < S0; ++s) {
          typename Types<BF>::Op b;
          if constexpr (BF) b = *reinterpret_cast<const s16x8*>(dX<CF>() + row * CF::XS + 16 * s + 8 * g);
          else b = dX<CF>()[row * CF::XS + 4 * (2 * (s >> 2) + g) + (s & 3)];
#pragma unroll
          for (int mt = 0; mt < M::MTH; ++mt) hdn[mt] = mma(gopb<BF>(rs, 0, mt, s, S0, lane), b, hdn[mt]);
          chunk_fence<kChunk<BF>>(s);
        }
#pragma unroll
        for (int mt = 0; mt < M::MTH; ++mt) {
          relu16(hdn[mt]);
          act[mt].set(hdn[mt]);
        }
        constexpr int S1 = kLfH / M::KS;
        o = gbias(bias + M::bias_off(1), 0, g);
#pragma unroll
        for (int s = 0; s < S1; ++s) {
          o = mma(gopb<BF>(rs, M::fwd_off(1) * CF::EB, 0, s, S1, lane), dop<BF>(hdn, s), o);
          chunk_fence<kChunk<BF>>(s);
        }
      }

      if constexpr (!CF::BWD) {
        // per hit: tau, eta, the surface point (section 4.2) -> workspace
        if (has_tile && g == 0 && n0 + lane < tw) {
          const int hh = n0 + lane;
          const DRec rc = rec[hh];
          const int mp = wmap[hh];
          const int64_t slot = ir.ray(mp & 0xFFFF) * a.K + (mp >> 16);
          const float dt = rc.tout - rc.tin;
          const float ft = a.tau_mode == SVLF_TAU_VOXEL ? dt * inv_h
                           : a.tau_mode == SVLF_TAU_WORLD ? dt : 1.0f;
          const float tau = fmaxf(o[0], 0.0f) * ft;
          const float eta = sigmoidf_(o[1]);
          LfHit st;
          st.us[0] = eta * rc.u1[0] + (1.0f - eta) * rc.u2[0];
          st.us[1] = eta * rc.u1[1] + (1.0f - eta) * rc.u2[1];
          st.us[2] = eta * rc.u1[2] + (1.0f - eta) * rc.u2[2];
          st.ts = eta * rc.tin + (1.0f - eta) * rc.tout;
          st.alpha = -expm1f(-tau);
          st.e = expf(-tau);
          st.dtau = o[0] > 0.0f ? ft : 0.0f;
          st.eta = eta;
          a.st[slot] = st;
        }
      } else {
        // backward of F_T from dL/d(o_0, o_1) left by the colour kernel
        El* GZ = reinterpret_cast<El*>(g_lds + CF::L_GZ);
        El* AT = reinterpret_cast<El*>(g_lds + CF::L_AT);
        f32x16 gz[M::MTH];
#pragma unroll
        for (int mt = 0; mt < M::MTH; ++mt) gz[mt] = zero16();
        if (has_tile && g == 0 && n0 + lane < tw) {
          const int mp = wmap[n0 + lane];
          const int64_t slot = ir.ray(mp & 0xFFFF) * a.K + (mp >> 16);
          const float2 gv = *reinterpret_cast<const float2*>(a.gT + 2 * slot);
          gz[0][0] = gv.x;
          gz[0][1] = gv.y;
        }
        f32x16 gx[2 * kLfCT / 32];
        static_for<M::NL>([&](auto lc) {
          constexpr int l = M::NH - decltype(lc)::value;
          constexpr int OT = M::out_p(l) / 32;
          const int col = n0 + (lane & 31);
          if (wave < CF::NTILE) {
            if (has_tile) {
#pragma unroll
              for (int mt = 0; mt < OT; ++mt)
#pragma unroll
                for (int i = 0; i < 16; ++i) GZ[(32 * mt + drow(i, g)) * CF::TS + col] = to_el<BF>(gz[mt][i]);
              if constexpr (l > 0) {
#pragma unroll
                for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
                  for (int i = 0; i < 16; ++i) AT[(32 * mt + drow(i, g)) * CF::TS + col] = act[mt].elem(i);
              }
            } else {
              for (int rr = g; rr < 32 * OT; rr += 2) GZ[rr * CF::TS + col] = to_el<BF>(0.0f);
              if constexpr (l > 0)
                for (int rr = g; rr < kLfH; rr += 2) AT[rr * CF::TS + col] = to_el<BF>(0.0f);
            }
          }
          if constexpr (l == 0)
            transpose_tile<BF, CF::WIN, CF::XS, CF::TS, M::IN0P, CF::XT_ROWS, kThreads>(dX<CF>(), AT, tid);
          __syncthreads();
          dw_window<BF, M, l, CF::WIN, CF::TS>(GZ, AT, part, wave, lane);
          bias_part<BF, M::out_p(l), M::out_r(l), CF::WIN, CF::TS>(GZ, tid, dbp[l]);
          if (has_tile) {
            constexpr int BMT = M::bm(l) / 32;
            constexpr int S = M::out_p(l) / M::KS;
            constexpr int BB = BWD_BASE + M::bwd_off(l) * CF::EB;
            f32x16 rr_[BMT];
#pragma unroll
            for (int mt = 0; mt < BMT; ++mt) rr_[mt] = zero16();
#pragma unroll
            for (int s = 0; s < S; ++s) {
              const typename Types<BF>::Op bo = dop<BF>(gz, s);
#pragma unroll
              for (int mt = 0; mt < BMT; ++mt) rr_[mt] = mma(gopb<BF>(rs, BB, mt, s, S, lane), bo, rr_[mt]);
              chunk_fence<kChunk<BF>>(s);
            }
            if constexpr (l > 0) {
#pragma unroll
              for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
                for (int i = 0; i < 16; ++i) gz[mt][i] = act[mt].positive(i) ? rr_[mt][i] : 0.0f;
            } else {
#pragma unroll
              for (int mt = 0; mt < BMT; ++mt) gx[mt] = rr_[mt];
            }
          }
          __syncthreads();
        });
        // scatter dL/dZ_T: dL/dpsi(x1) and dL/dpsi(x2) share the voxel's corners
        float* gxs = reinterpret_cast<float*>(g_lds + CF::L_GZ);      // [WIN][128]
        if (has_tile) {
          const int row = n0 + (lane & 31);
#pragma unroll
          for (int mt = 0; mt < 2 * kLfCT / 32; ++mt)
#pragma unroll
            for (int i = 0; i < 16; ++i) gxs[row * 2 * kLfCT + 32 * mt + drow(i, g)] = gx[mt][i];
        }
        __syncthreads();
        if (has_tile) {
          for (int k = 0; k < 32; ++k) {
            const int hh = n0 + k;
            if (hh >= tw) break;
            const DRec rc = rec[hh];
            float w1[8], w2[8];
            trilinear(clamp01(rc.u1[0]), clamp01(rc.u1[1]), clamp01(rc.u1[2]), w1);
            trilinear(clamp01(rc.u2[0]), clamp01(rc.u2[1]), clamp01(rc.u2[2]), w2);
            const int vid[8] = {rc.v0.x, rc.v0.y, rc.v0.z, rc.v0.w, rc.v1.x, rc.v1.y, rc.v1.z, rc.v1.w};
            const float g1 = gxs[hh * 2 * kLfCT + lane];
            const float g2 = gxs[hh * 2 * kLfCT + kLfCT + lane];
#pragma unroll
            for (int j = 0; j < 8; ++j)
              unsafeAtomicAdd(sc.grad + static_cast<int64_t>(vid[j]) * kLfCT + lane, w1[j] * g1 + w2[j] * g2);
          }
        }
      }
      __syncthreads();
      s0 = s1;
    }
  }

  if constexpr (CF::BWD) {
    static_assert(M::NL * kThreads * 4 <= kLfH * CF::TS * CF::EB, "bias parts fit in GZ");
    bias_combine<M>(dbp, reinterpret_cast<float*>(g_lds + CF::L_GZ), part, tid);
  }
}

// ------------------------------------------------------------ colour kernel

template <int P, int MODE, int VD>
struct CCfg {
  static constexpr bool BF = P == 1;
  static constexpr bool BWD = MODE != kForward;
  using M = typename Dec<BF, VD>::C;
  using El = typename Types<BF>::Elem;
  static constexpr int EB = Types<BF>::EB;
  // BF16 backward keeps the activations of hidden layers 1 and 2 in
  // registers (packed) and those of layer 0 transposed in LDS, staging one
  // register layer at a time for the weight gradients; this allows 128-hit
  // windows (all four waves own a tile).  FP32 keeps all three layers
  // transposed in LDS at 32-hit windows.
  static constexpr bool ACT_REG = BF;
  static constexpr int L0_ROW = ACT_REG ? kLfH : 0;     // LDS row of layer 0's activations
  static constexpr int WIN = BWD ? (BF ? 128 : 32) : (BF ? 128 : 64);
  static constexpr int NTILE = WIN / 32;
  static constexpr int XS = M::IN0P + (BF ? 8 : 4);
  static constexpr int TS = WIN + (BF ? 8 : 1);
  static constexpr int XT_ROWS = align32(M::IN0);
  // LDS: records, X, per-hit out (8 floats), then (backward) the hidden
  // activations [NH][H][TS] (or, with ACT_REG, one staged layer [H][TS] that
  // also takes X^T), X^T [XT_ROWS][TS] and GZ [H][TS]
  static constexpr int ACT_ROWS = ACT_REG ? 2 * kLfH : kLfNHC * kLfH;
  static constexpr int L_REC = 0;
  static constexpr int L_X = L_REC + WIN * 64;
  static constexpr int L_OUT = align16(L_X + WIN * XS * EB);
  static constexpr int L_ACT = align16(L_OUT + WIN * 32);
  static constexpr int L_XT = align16(L_ACT + (BWD ? ACT_ROWS * TS * EB : 0));
  static constexpr int L_GZ = align16(L_XT + ((BWD && !ACT_REG) ? XT_ROWS * TS * EB : 0));
  static constexpr int L_MAP = align16(L_GZ + (BWD ? kLfH * TS * EB : 0));
  // hit map: all of a work item's hits (IMAP: backward, where it fits) or the window's
  static constexpr bool IMAP = BWD && align16(L_MAP + kThreads * SVLF_MAX_K * 4) + 64 <= 160 * 1024;
  static constexpr int L_SCR = align16(L_MAP + (IMAP ? kThreads * SVLF_MAX_K : WIN) * 4);
  static constexpr int LDS = L_SCR + 64;
  static_assert(LDS <= 160 * 1024, "LDS");
  static_assert(!BWD || WIN * kLfCC * 4 <= kLfH * TS * EB, "dL/dz_C staging fits in GZ");
  static_assert(XT_ROWS <= kLfH, "X^T fits in the staged-activation area");
};

// Colour record (64 B): unclamped surface point in cell units, t_in, t_out,
// eta, the slot's ray index within the item, and the 8 corner ids.
struct CRec {
  float us[3];
  float tin, tout, eta;
  int ray_lane;
  int pad;
  int4 v0, v1;
};

template <class CF>
__device__ __forceinline__ typename CF::El* cX() { return reinterpret_cast<typename CF::El*>(g_lds + CF::L_X); }
template <class CF>
__device__ __forceinline__ typename CF::El* cACT() { return reinterpret_cast<typename CF::El*>(g_lds + CF::L_ACT); }

template <int P, int MODE, int VD>
__global__ __launch_bounds__(kThreads, 1) void k_color(LfArgs a) {
  using CF = CCfg<P, MODE, VD>;
  using M = typename CF::M;
  using El = typename CF::El;
  constexpr bool BF = CF::BF;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;
  CRec* rec = reinterpret_cast<CRec*>(g_lds + CF::L_REC);
  float* out = reinterpret_cast<float*>(g_lds + CF::L_OUT);
  int* hmap = reinterpret_cast<int*>(g_lds + CF::L_MAP);
  int* scr = reinterpret_cast<int*>(g_lds + CF::L_SCR);
  using MT_ = typename Dec<BF, VD>::T;
  const char* cpack = static_cast<const char*>(a.packs) + MT_::pack_bytes(CF::EB);
  const auto rs = pack_rsrc(cpack, static_cast<int>(M::pack_bytes(CF::EB)));
  constexpr int BWD_BASE = M::FWD * CF::EB;
  const float* bias = reinterpret_cast<const float*>(cpack + M::pack_bytes(CF::EB) - M::BIAS * 4);

  float* part = a.partC + static_cast<int64_t>(blockIdx.x) * M::NPARAMS;
  if constexpr (CF::BWD) {
    for (int i = tid; i < M::NPARAMS; i += kThreads) part[i] = 0.0f;
    __syncthreads();
  }
  float dbp[M::NL];
#pragma unroll
  for (int l = 0; l < M::NL; ++l) dbp[l] = 0.0f;
  float loss_acc = 0.0f;

  ItemDeal deal = item_deal(a, 1);
  for (int item = deal.first(scr); item < deal.nb; item = deal.next(item, scr)) {
    const DevScene& sc = a.tab.s[scene_of(a.tab, item)];
    const int64_t zc = sc.n_vertices * kLfCT;       // Z_C follows Z_T
    const float* featC32 = sc.feat32 + zc;
    const uint16_t* featC16 = sc.feat16 != nullptr ? sc.feat16 + zc : nullptr;
    float* gradC = sc.grad != nullptr ? sc.grad + zc : nullptr;
    const ItemRays ir = item_rays(sc, item);
    const int64_t r = ir.ray(tid);
    const bool live = r < sc.ray_end;
    const int count = live ? a.cnt[r] : 0;
    const float h = __int_as_float((128 - sc.depth) << 23);
    const float inv_h = __int_as_float((126 + sc.depth) << 23);
    int total;
    const int off = block_excl_scan<kWaves>(count, scr, total, [&](int o) {
      if constexpr (CF::IMAP)
        for (int q = 0; q < count; ++q) hmap[o + q] = tid | (q << 16);
    });
    float cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, acc = 0.0f;
    for (int s0 = 0; s0 < total;) {
      bool in_win;
      const int s1 = CF::IMAP ? open_window_imap<CF::WIN>(s0, total, off, count, hmap, in_win)
                              : open_window<CF::WIN>(s0, total, off, count, scr, hmap, in_win);
      const int* wmap = CF::IMAP ? hmap + s0 : hmap;    // the window's map entries
      const int tw = s1 - s0;
      {
        constexpr int TPH = kLfCC * CF::EB / 16;
        constexpr int VPT = 16 / CF::EB;
        constexpr int HPP = kThreads / TPH;
        const int q = tid % TPH;
#pragma unroll 1
        for (int hh = tid / TPH; hh < CF::WIN; hh += HPP) {
          float v[VPT];
#pragma unroll
          for (int i = 0; i < VPT; ++i) v[i] = 0.0f;
          float rr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
          if (hh < tw) {
            const int mp = wmap[hh];
            const int64_t ray = ir.ray(mp & 0xFFFF);
            const int64_t slot = ray * a.K + (mp >> 16);
            const HitRec hr = a.hits[slot];
            const LfHit st = a.st[slot];
            const int4* lc = reinterpret_cast<const int4*>(sc.leaf_corners + 8 * static_cast<int64_t>(hr.leaf));
            const int4 c0 = lc[0], c1 = lc[1];
            if (q == 0) {
              CRec rc;
              rc.us[0] = st.us[0];
              rc.us[1] = st.us[1];
              rc.us[2] = st.us[2];
              rc.tin = hr.tin;
              rc.tout = hr.tout;
              rc.eta = st.eta;
              rc.ray_lane = mp & 0xFFFF;
              rc.pad = 0;
              rc.v0 = c0;
              rc.v1 = c1;
              rec[hh] = rc;
              // per-hit compositing inputs: {e^-tau, dtau/do_0, t_s, alpha}
              *reinterpret_cast<f32x4*>(out + 8 * hh + 4) = f32x4{st.e, st.dtau, st.ts, st.alpha};
              const float ox = a.o[3 * ray], oy = a.o[3 * ray + 1], oz = a.o[3 * ray + 2];
              const float dx = a.d[3 * ray], dy = a.d[3 * ray + 1], dz = a.d[3 * ray + 2];
              const float lx = -1.0f + static_cast<float>(hr.ijk & 1023u) * h;
              const float ly = -1.0f + static_cast<float>((hr.ijk >> 10) & 1023u) * h;
              const float lz = -1.0f + static_cast<float>(hr.ijk >> 20) * h;
              const float hc = 0.5f * h;
              float r6[6];
              sphere_r(cell_coord(ox, dx, hr.tin, 0.0f, lx + hc, 1.0f),
                       cell_coord(oy, dy, hr.tin, 0.0f, ly + hc, 1.0f),
                       cell_coord(oz, dz, hr.tin, 0.0f, lz + hc, 1.0f), dx, dy, dz, h, r6);
#pragma unroll
              for (int i = 0; i < 6; ++i) rr[i] = r6[i];
              rr[6] = dx;
              rr[7] = dy;
              rr[8] = dz;
            }
            float w[8];
            trilinear(clamp01(st.us[0]), clamp01(st.us[1]), clamp01(st.us[2]), w);
            const int vid[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              if constexpr (BF) {
                const uint4 raw = *reinterpret_cast<const uint4*>(featC16 + static_cast<int64_t>(vid[j]) * kLfCC + 8 * q);
                const uint32_t w4[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  v[2 * i] += w[j] * bf16_f32(static_cast<uint16_t>(w4[i] & 0xFFFFu));
                  v[2 * i + 1] += w[j] * bf16_f32(static_cast<uint16_t>(w4[i] >> 16));
                }
              } else {
                const float4 f = *reinterpret_cast<const float4*>(featC32 + static_cast<int64_t>(vid[j]) * kLfCC + 4 * q);
                v[0] += w[j] * f.x; v[1] += w[j] * f.y; v[2] += w[j] * f.z; v[3] += w[j] * f.w;
              }
            }
          }
          El* xr = cX<CF>() + hh * CF::XS;
#pragma unroll
          for (int i = 0; i < VPT; ++i) xr[VPT * q + i] = to_el<BF>(v[i]);
          if (q == 0) {
#pragma unroll
            for (int i = kLfCC; i < M::IN0P; ++i)
              xr[i] = to_el<BF>(i < kLfCC + 6 + 3 * VD ? rr[i - kLfCC] : 0.0f);
          }
        }
      }
      __syncthreads();

      // colour decoder: one 32-hit tile per wave
      const int n0 = 32 * wave;
      const bool has_tile = wave < CF::NTILE && n0 < tw;
      const int col = n0 + (lane & 31);
      ActT<BF> act[CF::ACT_REG && CF::BWD ? M::NH - 1 : 1][M::MTH];   // layers 1 .. NH-1
      if (has_tile) {
        const int row = col;
        f32x16 cur[M::MTH];
        {
          constexpr int S0 = M::IN0P / M::KS;
#pragma unroll
          for (int mt = 0; mt < M::MTH; ++mt) cur[mt] = gbias(bias, mt, g);
#pragma unroll
          for (int s = 0; s < S0; ++s) {
            typename Types<BF>::Op b;
            if constexpr (BF) b = *reinterpret_cast<const s16x8*>(cX<CF>() + row * CF::XS + 16 * s + 8 * g);
            else b = cX<CF>()[row * CF::XS + 4 * (2 * (s >> 2) + g) + (s & 3)];
#pragma unroll
            for (int mt = 0; mt < M::MTH; ++mt) cur[mt] = mma(gopb<BF>(rs, 0, mt, s, S0, lane), b, cur[mt]);
            chunk_fence<kChunk<BF>>(s);
          }
#pragma unroll
          for (int mt = 0; mt < M::MTH; ++mt) relu16(cur[mt]);
          if constexpr (CF::BWD) {
#pragma unroll
            for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
              for (int i = 0; i < 16; ++i)
                cACT<CF>()[(CF::L0_ROW + 32 * mt + drow(i, g)) * CF::TS + col] = to_el<BF>(cur[mt][i]);
          }
        }
        static_for<M::NH - 1>([&](auto lc) {
          constexpr int l = decltype(lc)::value + 1;
          constexpr int S = kLfH / M::KS;
          f32x16 nxt[M::MTH];
#pragma unroll
          for (int mt = 0; mt < M::MTH; ++mt) nxt[mt] = gbias(bias + M::bias_off(l), mt, g);
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const typename Types<BF>::Op b = dop<BF>(cur, s);
#pragma unroll
            for (int mt = 0; mt < M::MTH; ++mt) nxt[mt] = mma(gopb<BF>(rs, M::fwd_off(l) * CF::EB, mt, s, S, lane), b, nxt[mt]);
            chunk_fence<kChunk<BF>>(s);
          }
#pragma unroll
          for (int mt = 0; mt < M::MTH; ++mt) {
            relu16(nxt[mt]);
            cur[mt] = nxt[mt];
          }
          if constexpr (CF::BWD && CF::ACT_REG) {
#pragma unroll
            for (int mt = 0; mt < M::MTH; ++mt) act[l - 1][mt].set(cur[mt]);
          } else if constexpr (CF::BWD) {
#pragma unroll
            for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
              for (int i = 0; i < 16; ++i)
                cACT<CF>()[(l * kLfH + 32 * mt + drow(i, g)) * CF::TS + col] = to_el<BF>(cur[mt][i]);
          }
        });
        constexpr int S = kLfH / M::KS;
        f32x16 o = gbias(bias + M::bias_off(M::NH), 0, g);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          o = mma(gopb<BF>(rs, M::fwd_off(M::NH) * CF::EB, 0, s, S, lane), dop<BF>(cur, s), o);
          chunk_fence<kChunk<BF>>(s);
        }
        if (g == 0 && col < tw)
          *reinterpret_cast<f32x4*>(out + 8 * col) = f32x4{sigmoidf_(o[0]), sigmoidf_(o[1]), sigmoidf_(o[2]), 0.0f};
      } else if (CF::BWD && wave < CF::NTILE) {
        // no hits for this tile: its activation columns must not hold stale data
        constexpr int R0 = CF::ACT_REG ? CF::L0_ROW : 0;
        constexpr int R1 = CF::ACT_REG ? CF::L0_ROW + kLfH : kLfNHC * kLfH;
        for (int rr = R0 + g; rr < R1; rr += 2) cACT<CF>()[rr * CF::TS + col] = to_el<BF>(0.0f);
      }
      __syncthreads();

      // Eq. 3 front to back by the owning lanes, and its backward
      if (in_win) {
        const int p0 = off - s0;
        float T = 1.0f;
        for (int k = 0; k < count; ++k) {
          float* hp = out + 8 * (p0 + k);
          const f32x4 va = *reinterpret_cast<const f32x4*>(hp);
          const f32x4 vb = *reinterpret_cast<const f32x4*>(hp + 4);
          const float w = T * vb[3];
          cr += w * va[0];
          cg += w * va[1];
          cb += w * va[2];
          dep += w * vb[2];
          acc += w;
          if constexpr (CF::BWD) hp[3] = T;
          T *= vb[0];
        }
        if constexpr (CF::BWD) {
          float gr, gg, gb, gd, ga;
          // the hit holding the target surface point (staged losses)
          int surf = -1;
          float tgt_r = 0.0f, tgt_g = 0.0f, tgt_b = 0.0f;
          if (MODE == kTrain) {
            tgt_r = a.t_rgb[3 * r];
            tgt_g = a.t_rgb[3 * r + 1];
            tgt_b = a.t_rgb[3 * r + 2];
          }
          if (MODE == kTrain && a.loss_kind != kLfLossDefault) {
            const float ts_ = a.t_depth[r];
            for (int k = 0; k < count; ++k) {
              const CRec& rc = rec[p0 + k];
              if (rc.tin <= ts_ && ts_ < rc.tout) surf = k;
            }
          }
          if (MODE == kTrain && a.loss_kind == kLfLossSurface) {
            gr = gg = gb = gd = ga = 0.0f;
          } else if (MODE == kTrain && a.loss_kind == kLfLossVolume) {
            const float k2 = 2.0f * a.loss_scale;
            gr = k2 * (cr - tgt_r);
            gg = k2 * (cg - tgt_g);
            gb = k2 * (cb - tgt_b);
            gd = 0.0f;
            ga = 0.0f;
          } else if (MODE == kTrain) {
            const float er = cr - tgt_r, eg = cg - tgt_g, eb = cb - tgt_b, ed = dep - a.t_depth[r];
            const float k2 = a.loss_scale * (2.0f / 3.0f);
            gr = k2 * er;
            gg = k2 * eg;
            gb = k2 * eb;
            gd = a.loss_scale * a.lambda_depth * (ed > 0.0f ? 1.0f : (ed < 0.0f ? -1.0f : 0.0f));
            ga = 0.0f;
          } else {
            gr = a.g_rgb[3 * r];
            gg = a.g_rgb[3 * r + 1];
            gb = a.g_rgb[3 * r + 2];
            gd = a.g_depth[r];
            ga = a.g_acc ? a.g_acc[r] : 0.0f;
          }
          float Sr = 0.0f, Sg = 0.0f, Sb = 0.0f, St = 0.0f, Sa = 0.0f;
          float surf_loss = 0.0f;
          for (int k = count - 1; k >= 0; --k) {
            float* hp = out + 8 * (p0 + k);
            const f32x4 va = *reinterpret_cast<const f32x4*>(hp);
            const f32x4 vb = *reinterpret_cast<const f32x4*>(hp + 4);
            const float Tq = va[3];
            const float w = Tq * vb[3];
            const float Tn = Tq * vb[0];
            const float c0 = va[0], c1 = va[1], c2 = va[2], ts = vb[2];
            const float gtau = gr * (Tn * c0 - Sr) + gg * (Tn * c1 - Sg) + gb * (Tn * c2 - Sb) +
                               gd * (Tn * ts - St) + ga * (Tn - Sa);
            Sr += w * c0;
            Sg += w * c1;
            Sb += w * c2;
            St += w * ts;
            Sa += w;
            // direct terms of the staged losses on the surface hit: colour
            // (surface stage), eta against the target's within-voxel depth,
            // and the opacity term lambda_tau e^{-2 tau}
            float gc0 = gr * w, gc1 = gg * w, gc2 = gb * w, gt = gtau, geta = 0.0f;
            if (k == surf) {
              const CRec& rc = rec[p0 + k];
              const float ls2 = 2.0f * a.loss_scale;
              const float eta_gt = (rc.tout - a.t_depth[r]) / (rc.tout - rc.tin);
              const float e2 = vb[0] * vb[0];
              if (a.loss_kind == kLfLossSurface) {
                gc0 = ls2 * (c0 - tgt_r);
                gc1 = ls2 * (c1 - tgt_g);
                gc2 = ls2 * (c2 - tgt_b);
                surf_loss += (c0 - tgt_r) * (c0 - tgt_r) + (c1 - tgt_g) * (c1 - tgt_g) +
                             (c2 - tgt_b) * (c2 - tgt_b);
              }
              geta = ls2 * a.lambda_eta * (rc.eta - eta_gt);
              gt -= ls2 * a.lambda_tau * e2;
              surf_loss += a.lambda_eta * (rc.eta - eta_gt) * (rc.eta - eta_gt) + a.lambda_tau * e2;
            }
            *reinterpret_cast<f32x4*>(hp) =
                f32x4{gc0 * c0 * (1.0f - c0), gc1 * c1 * (1.0f - c1), gc2 * c2 * (1.0f - c2),
                      gt * vb[1]};
            hp[4] = w * gd;                     // dL/dt_s
            hp[5] = geta;                       // direct dL/deta
          }
          // surface-voxel terms of the staged losses (the photometric term
          // of the volume kind is added for every ray below, hits or not)
          if (MODE == kTrain && a.loss_kind != kLfLossDefault) loss_acc += a.loss_scale * surf_loss;
        }
      }

      if constexpr (CF::BWD) {
        __syncthreads();
        El* GZ = reinterpret_cast<El*>(g_lds + CF::L_GZ);
        El* XT = reinterpret_cast<El*>(g_lds + CF::L_XT);
        f32x16 gz[M::MTH];
#pragma unroll
        for (int mt = 0; mt < M::MTH; ++mt) gz[mt] = zero16();
        if (has_tile && g == 0 && col < tw) {
          const f32x4 go = *reinterpret_cast<const f32x4*>(out + 8 * col);
          gz[0][0] = go[0];
          gz[0][1] = go[1];
          gz[0][2] = go[2];
        }
        f32x16 gx[1];
        static_for<M::NL>([&](auto lc) {
          constexpr int l = M::NH - decltype(lc)::value;
          constexpr int OT = M::out_p(l) / 32;
          if (wave < CF::NTILE) {
            if (has_tile) {
#pragma unroll
              for (int mt = 0; mt < OT; ++mt)
#pragma unroll
                for (int i = 0; i < 16; ++i) GZ[(32 * mt + drow(i, g)) * CF::TS + col] = to_el<BF>(gz[mt][i]);
              if constexpr (CF::ACT_REG && l > 1) {
#pragma unroll
                for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
                  for (int i = 0; i < 16; ++i) cACT<CF>()[(32 * mt + drow(i, g)) * CF::TS + col] = act[l - 2][mt].elem(i);
              }
            } else {
              for (int rr = g; rr < 32 * OT; rr += 2) GZ[rr * CF::TS + col] = to_el<BF>(0.0f);
              if constexpr (CF::ACT_REG && l > 1)
                for (int rr = g; rr < kLfH; rr += 2) cACT<CF>()[rr * CF::TS + col] = to_el<BF>(0.0f);
            }
          }
          El* XTs = CF::ACT_REG ? cACT<CF>() : XT;      // X^T (layer 0)
          if constexpr (l == 0)
            transpose_tile<BF, CF::WIN, CF::XS, CF::TS, M::IN0P, CF::XT_ROWS, kThreads>(cX<CF>(), XTs, tid);
          __syncthreads();
          // layer l's input: X^T (l = 0), layer 0 from LDS, or the staged register layer
          const El* AT = (l == 0) ? XTs
                         : CF::ACT_REG ? cACT<CF>() + (l == 1 ? CF::L0_ROW * CF::TS : 0)
                                       : cACT<CF>() + (l - 1) * kLfH * CF::TS;
          if (!a.freeze_color) dw_window<BF, M, l, CF::WIN, CF::TS>(GZ, AT, part, wave, lane);
          if (!a.freeze_color)
            bias_part<BF, M::out_p(l), M::out_r(l), CF::WIN, CF::TS>(GZ, tid, dbp[l]);
          if (has_tile) {
            constexpr int BMT = M::bm(l) / 32;
            constexpr int S = M::out_p(l) / M::KS;
            constexpr int BB = BWD_BASE + M::bwd_off(l) * CF::EB;
            f32x16 rr_[BMT];
#pragma unroll
            for (int mt = 0; mt < BMT; ++mt) rr_[mt] = zero16();
#pragma unroll
            for (int s = 0; s < S; ++s) {
              const typename Types<BF>::Op bo = dop<BF>(gz, s);
#pragma unroll
              for (int mt = 0; mt < BMT; ++mt) rr_[mt] = mma(gopb<BF>(rs, BB, mt, s, S, lane), bo, rr_[mt]);
              chunk_fence<kChunk<BF>>(s);
            }
            if constexpr (l > 1 && CF::ACT_REG) {
#pragma unroll
              for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
                for (int i = 0; i < 16; ++i) gz[mt][i] = act[l - 2][mt].positive(i) ? rr_[mt][i] : 0.0f;
            } else if constexpr (l > 0) {
              const El* actl = cACT<CF>() + (CF::ACT_REG ? CF::L0_ROW : (l - 1) * kLfH) * CF::TS;
#pragma unroll
              for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                  const El av = actl[(32 * mt + drow(i, g)) * CF::TS + col];
                  bool pos;
                  if constexpr (BF) pos = static_cast<short>(av) > 0;
                  else pos = av > 0.0f;
                  gz[mt][i] = pos ? rr_[mt][i] : 0.0f;
                }
            } else {
              gx[0] = rr_[0];
            }
          }
          __syncthreads();
        });
        // scatter dL/dZ_C and carry dL/deta through the interpolation at x_s
        float* gxs = reinterpret_cast<float*>(g_lds + CF::L_GZ);       // [WIN][C_C]
        if (has_tile) {
#pragma unroll
          for (int i = 0; i < 16; ++i) gxs[col * kLfCC + drow(i, g)] = gx[0][i];
        }
        __syncthreads();
        if (has_tile) {
          const int c = lane & 31, hs = lane >> 5;
#pragma unroll 4
          for (int k = 0; k < 32; k += 2) {
            const int hh = n0 + k + hs;
            const bool ok = hh < tw;
            float proj[8];
            CRec rc;
            float wv[8];
            if (ok) {
              rc = rec[hh];
              trilinear(clamp01(rc.us[0]), clamp01(rc.us[1]), clamp01(rc.us[2]), wv);
              const int vid[8] = {rc.v0.x, rc.v0.y, rc.v0.z, rc.v0.w, rc.v1.x, rc.v1.y, rc.v1.z, rc.v1.w};
              const float gv = gxs[hh * kLfCC + c];
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                const int64_t idx = static_cast<int64_t>(vid[j]) * kLfCC + c;
                float fv;
                if constexpr (BF) fv = bf16_f32(featC16[idx]);
                else fv = featC32[idx];
                proj[j] = fv * gv;
                if (!a.freeze_color) unsafeAtomicAdd(gradC + idx, wv[j] * gv);
              }
            } else {
#pragma unroll
              for (int j = 0; j < 8; ++j) proj[j] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
#pragma unroll
              for (int m = 16; m > 0; m >>= 1) proj[j] += __shfl_xor(proj[j], m, 64);
            }
            if (ok && c == 0) {
              // dL/du_s from the trilinear weights' derivatives
              const float u[3] = {clamp01(rc.us[0]), clamp01(rc.us[1]), clamp01(rc.us[2])};
              float gu[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
              for (int j = 0; j < 8; ++j) {
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                  float dwv = ((j >> ax) & 1) ? 1.0f : -1.0f;
#pragma unroll
                  for (int bx = 0; bx < 3; ++bx)
                    if (bx != ax) dwv *= ((j >> bx) & 1) ? u[bx] : 1.0f - u[bx];
                  gu[ax] += dwv * proj[j];
                }
              }
              const int64_t ray = ir.ray(rc.ray_lane);
              const float dir[3] = {a.d[3 * ray], a.d[3 * ray + 1], a.d[3 * ray + 2]};
              float gx_d = 0.0f;
#pragma unroll
              for (int ax = 0; ax < 3; ++ax) {
                const bool inside = rc.us[ax] >= 0.0f && rc.us[ax] <= 1.0f;
                gx_d += inside ? gu[ax] * dir[ax] : 0.0f;
              }
              const float* hp = out + 8 * hh;
              const float g_eta = (rc.tin - rc.tout) * (hp[4] + gx_d * inv_h) + hp[5];
              const int mp = wmap[hh];
              const int64_t slot = ray * a.K + (mp >> 16);
              *reinterpret_cast<float2*>(a.gT + 2 * slot) =
                  make_float2(hp[3], g_eta * rc.eta * (1.0f - rc.eta));
            }
          }
        }
      }
      __syncthreads();
      s0 = s1;
    }

    if (live) {
      if (MODE != kBackward) {
        if (a.rgb) {
          a.rgb[3 * r] = cr;
          a.rgb[3 * r + 1] = cg;
          a.rgb[3 * r + 2] = cb;
        }
        if (a.depth) a.depth[r] = dep;
        if (a.acc) a.acc[r] = acc;
      }
      if (MODE == kTrain && a.loss_kind == kLfLossDefault) {
        const float er = cr - a.t_rgb[3 * r], eg = cg - a.t_rgb[3 * r + 1],
                    eb = cb - a.t_rgb[3 * r + 2], ed = dep - a.t_depth[r];
        loss_acc += a.loss_scale * ((er * er + eg * eg + eb * eb) * (1.0f / 3.0f) +
                                    a.lambda_depth * fabsf(ed));
      } else if (MODE == kTrain && a.loss_kind == kLfLossVolume) {
        const float er = cr - a.t_rgb[3 * r], eg = cg - a.t_rgb[3 * r + 1],
                    eb = cb - a.t_rgb[3 * r + 2];
        loss_acc += a.loss_scale * (er * er + eg * eg + eb * eb);
      }
    }
  }

  if constexpr (CF::BWD) {
    static_assert(M::NL * kThreads * 4 <= kLfH * CF::TS * CF::EB, "bias parts fit in GZ");
    bias_combine<M>(dbp, reinterpret_cast<float*>(g_lds + CF::L_GZ), part, tid);
    if (MODE == kTrain) {
      const float tot = block_sum<kWaves>(loss_acc, reinterpret_cast<float*>(scr));
      if (tid == 0) a.ws_loss[blockIdx.x] = tot;
    } else if (tid == 0) {
      a.ws_loss[blockIdx.x] = 0.0f;
    }
  }
}

// ------------------------------------------------------------ dispatch

int lf_num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, v = 0;
    n = (hipGetDevice(&dev) == hipSuccess &&
         hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            ? v
            : 256;
  }
  return n;
}

// Persistent launch: as many blocks as fit on the device at once (registers
// and LDS), at most `cap` (the backward kernels' partial sums are sized for
// lf_grid_limit() blocks).
template <class K>
hipError_t launch_persistent(K kern, int lds, const LfArgs& a, hipStream_t s, int* grid_out,
                             int cap) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  int per_cu = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                   kThreads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int grid = lf_num_cus() * per_cu;
  if (grid > cap) grid = cap;
  if (grid > a.tab.n_blocks) grid = a.tab.n_blocks;
  if (grid < 1) grid = 1;
  *grid_out = grid;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <int P, int VD>
hipError_t run_lf(const LfArgs& a, int mode, hipStream_t s) {
  constexpr bool BF = P == 1;
  using D = Dec<BF, VD>;
  hipLaunchKernelGGL((k_lf_pack<BF, VD>), dim3(64), dim3(kThreads), 0, s, a.params,
                     static_cast<char*>(a.packs));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && a.item_counters != nullptr)
    e = launch_fill(reinterpret_cast<float*>(a.item_counters), 0.0f, 3, s);   // 0.0f has zero bits
  if (e != hipSuccess) return e;
  int g1 = 0, g2 = 0, g3 = 0;
  const int fwd_cap = 4096, bwd_cap = lf_grid_limit();
  e = launch_persistent(k_density<P, kForward>, DCfg<P, kForward>::LDS, a, s, &g1, fwd_cap);
  if (e != hipSuccess) return e;
  if (mode == kForward)
    return launch_persistent(k_color<P, kForward, VD>, CCfg<P, kForward, VD>::LDS, a, s, &g2,
                             fwd_cap);
  if (mode == kTrain)
    e = launch_persistent(k_color<P, kTrain, VD>, CCfg<P, kTrain, VD>::LDS, a, s, &g2, bwd_cap);
  else
    e = launch_persistent(k_color<P, kBackward, VD>, CCfg<P, kBackward, VD>::LDS, a, s, &g2,
                          bwd_cap);
  if (e != hipSuccess) return e;
  e = launch_persistent(k_density<P, kBackward>, DCfg<P, kBackward>::LDS, a, s, &g3, bwd_cap);
  if (e != hipSuccess) return e;
  e = launch_reduce_partials(a.partT, g3, D::T::NPARAMS, a.grad_params, nullptr, nullptr, s);
  if (e != hipSuccess) return e;
  return launch_reduce_partials(a.partC, g2, D::C::NPARAMS, a.grad_params + D::T::NPARAMS,
                                a.ws_loss, mode == kTrain ? a.loss_out : nullptr, s);
}

}  // namespace

int lf_grid_limit() { return 256; }
int lf_x_row() { return Dec<true, 0>::T::IN0P; }
int64_t lf_params_density() { return Dec<true, 0>::T::NPARAMS; }
int64_t lf_params_color(int viewdir) {
  return viewdir ? Dec<true, 1>::C::NPARAMS : Dec<true, 0>::C::NPARAMS;
}
size_t lf_pack_bytes(int precision, int viewdir) {
  const bool bf = precision == SVLF_BF16;
  if (bf) {
    return viewdir ? Dec<true, 1>::T::pack_bytes(2) + Dec<true, 1>::C::pack_bytes(2)
                   : Dec<true, 0>::T::pack_bytes(2) + Dec<true, 0>::C::pack_bytes(2);
  }
  return viewdir ? Dec<false, 1>::T::pack_bytes(4) + Dec<false, 1>::C::pack_bytes(4)
                 : Dec<false, 0>::T::pack_bytes(4) + Dec<false, 0>::C::pack_bytes(4);
}

hipError_t launch_lf(const LfArgs& a, int mode, hipStream_t s) {
  const int P = a.precision == SVLF_BF16 ? 1 : 0;
  if (P) return a.viewdir ? run_lf<1, 1>(a, mode, s) : run_lf<1, 0>(a, mode, s);
  return a.viewdir ? run_lf<0, 1>(a, mode, s) : run_lf<0, 0>(a, mode, s);
}

}  // namespace svlf
