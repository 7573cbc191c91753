// Shading kernels of the SVLF per-ray path (gfx950).
//
// For every hit (leaf, t_in, t_out) found by the traversal: trilinear
// interpolation of the leaf's corner features at the segment midpoint
// (section 4.1), one ReLU decoder C -> H ... -> 4 (section 4.5), optical
// thickness from sigma (section 4 footnote) and front-to-back alpha
// compositing (Eq. 3); the backward variant recomputes all of it and
// propagates dL/d(rgb, depth, acc) to the features (FP32 atomics) and the
// decoder parameters (per-block partial sums, reduced deterministically).
//
// Organisation (one block = 4 waves = 256 rays per work item, persistent):
//  * the rays' hits are consumed in windows of up to WIN hits that never
//    split a ray, so compositing and its backward are window-local;
//  * the window's hit records and the interpolated MLP inputs live in LDS;
//    each wave runs the decoder on a 32-hit tile with MFMA (32x32x16 BF16 or
//    32x32x2 FP32), hits on the N dimension: a layer's result (D layout:
//    lane = hit, registers = output features) is fed to the next layer's B
//    operand directly, the K order of every weight matrix being permuted at
//    pack time to match the D layout (no shuffles between layers);
//  * backward: dL/dz of each layer and the layer's input are written to LDS
//    transposed ([feature][hit]) and every wave accumulates the dW tiles it
//    owns over all windows in registers (K = hits); the data gradient uses a
//    second, transposed weight pack;
//  * backward: a window's feature-gradient atomics are issued after the next
//    window's gather, and the next window's hit records and corner ids are
//    loaded while the current window computes (the window loop);
//  * the rays of groups of consecutive full work items are interleaved
//    (item_rays), which shortened both the train and the forward pass.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "mfma_common.hpp"
#include "svlf_internal.hpp"

namespace svlf {
namespace {

using namespace detail;

constexpr int kThreads = 256;
static_assert(kThreads == kRaysPerBlock, "one ray per thread in a work item");
static_assert(kThreads <= 256 && SVLF_MAX_K <= 256, "hit map entries: 8-bit lane, 8-bit slot");
constexpr int kWaves = 4;

// ------------------------------------------------------------ geometry

constexpr int in_w(int l, int CI, int H) { return l == 0 ? CI : H; }
constexpr int out_w(int l, int H, int NH) { return l == NH ? 32 : H; }
constexpr int in_real(int l, int C, int H) { return l == 0 ? C : H; }
constexpr int out_real(int l, int H, int NH) { return l == NH ? 4 : H; }
constexpr int bwd_m(int l, int H) { return l == 0 ? 32 : H; }

constexpr int fwd_off(int l, int CI, int H, int NH) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += out_w(i, H, NH) * in_w(i, CI, H);
  return o;
}
constexpr int bwd_off(int l, int H, int NH) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += bwd_m(i, H) * out_w(i, H, NH);
  return o;
}
constexpr int bias_off(int l, int H, int NH) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += out_w(i, H, NH);
  return o;
}
constexpr int par_w(int l, int C, int H, int NH) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += out_real(i, H, NH) * in_real(i, C, H) + out_real(i, H, NH);
  return o;
}
constexpr int par_b(int l, int C, int H, int NH) {
  return par_w(l, C, H, NH) + out_real(l, H, NH) * in_real(l, C, H);
}
// dW tiles per layer: (out tiles) x (in tiles)
constexpr int dw_mt(int l, int H, int NH) { return out_w(l, H, NH) / 32; }
constexpr int dw_nt(int l, int H, int CIN) { return l == 0 ? (CIN + 31) / 32 : H / 32; }
constexpr int dw_tile_off(int l, int H, int NH, int CIN) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += dw_mt(i, H, NH) * dw_nt(i, H, CIN);
  return o;
}

// VD = 1: the decoder input is [psi (C) | ray direction (3)].
template <int P, int C_, int H_, int NH_, int MODE_, int VD_ = 0>
struct Cfg {
  static constexpr bool BF = P == 1;
  static constexpr int C = C_, H = H_, NH = NH_, MODE = MODE_, VD = VD_;
  static constexpr bool BWD = MODE != kForward;
  static constexpr int KS = BF ? 16 : 2;            // K per MFMA
  static constexpr int CIN = C + 3 * VD;            // decoder input width
  static constexpr int CI = BF ? align16(CIN) : align8(CIN);  // padded to the K steps
  static constexpr int NL = NH + 1;
  static constexpr int MTH = H / 32;
  static constexpr int WIN = (BWD && !BF) ? 64 : 128;
  static constexpr int NTILE = WIN / 32;
  static constexpr int EB = BF ? 2 : 4;
  using Op = typename std::conditional<BF, s16x8, float>::type;
  using Elem = typename std::conditional<BF, uint16_t, float>::type;
  static constexpr int FWD_ELEMS = fwd_off(NL, CI, H, NH);
  static constexpr int BWD_ELEMS = BWD ? bwd_off(NL, H, NH) : 0;
  static constexpr int BIAS_ELEMS = bias_off(NL, H, NH);
  static constexpr int NPARAMS = par_w(NL, CIN, H, NH);
  static constexpr int NDW = dw_tile_off(NL, H, NH, CIN);     // dW tiles
  static constexpr int DW_SLOTS = (NDW + kWaves - 1) / kWaves;
  static constexpr int NBIAS = NH * H + 4;
  static constexpr int XS = CI + (BF ? 8 : 4);                  // X row stride
  static constexpr int TS = WIN + (BF ? 8 : 1);                 // transposed row stride
  static constexpr int TROWS = H > 32 ? H : 32;
  // LDS byte layout
  static constexpr int L_FP = 0;
  static constexpr int L_BP = align16(L_FP + FWD_ELEMS * EB);
  static constexpr int L_BI = align16(L_BP + BWD_ELEMS * EB);
  static constexpr int L_REC = align16(L_BI + BIAS_ELEMS * 4);
  static constexpr int L_X = align16(L_REC + WIN * 64);
  static constexpr int L_OUT = align16(L_X + WIN * XS * EB);
  static constexpr int L_GZ = align16(L_OUT + WIN * 32);
  static constexpr int L_AT = align16(L_GZ + (BWD ? TROWS * TS * EB : 0));
  // hit map: all of a work item's hits, 16 bits per hit (IMAP: backward
  // kernels where it fits), else the window's hits, 32 bits per hit
  // (backward: two windows, the current one and the next)
  static constexpr int L_MAP = align16(L_AT + (BWD ? TROWS * TS * EB : 0));
  static constexpr int map_end(int entries) {
    return align16(align16(L_MAP + entries * 2) + (BWD ? WIN * 64 : 0)) + 64;
  }
  static constexpr bool IMAP = BWD && map_end(kThreads * SVLF_MAX_K) <= 160 * 1024;
  using MapT = typename std::conditional<IMAP, uint16_t, int32_t>::type;
  static constexpr int MAP_ENTRIES = IMAP ? kThreads * SVLF_MAX_K : (BWD ? 2 : 1) * WIN;
  // backward: records of the window awaiting its scatter
  static constexpr int L_REC2 = align16(L_MAP + MAP_ENTRIES * static_cast<int>(sizeof(MapT)));
  static constexpr int L_SCR = align16(L_REC2 + (BWD ? WIN * 64 : 0));
  static constexpr int LDS_BYTES = L_SCR + 64;
  static_assert(NBIAS <= kThreads, "one thread per bias entry writes its combined gradient");
  static_assert(C <= 32 && CI <= TROWS, "feature gradients come from one 32-row tile");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS budget");
  static_assert(!BWD || WIN * C * 4 <= 2 * TROWS * TS * EB, "dL/dx staging fits in GZ + AT");
};

// Hit record in LDS (64 bytes): the leaf's corner vertex ids are fetched
// once by the ray's lane, so the gather and the gradient scatter start with
// independent feature-row accesses.
struct RecL {
  int32_t leaf;
  float ux, uy, uz;
  float tmid;
  float dt;
  float T;
  float pad;
  int4 v0, v1;
};

// Dynamic LDS of the shading kernels.  Every LDS address is derived from
// this array directly, so the compiler keeps LDS accesses as ds_* operations
// (an LDS pointer stored in an object would be accessed as a generic address,
// and each generic access waits for all outstanding global memory traffic).
extern __shared__ __attribute__((aligned(16))) char g_smem[];

template <class CF>
struct Smem {
  __device__ __forceinline__ typename CF::Elem* fpack() const { return reinterpret_cast<typename CF::Elem*>(g_smem + CF::L_FP); }
  __device__ __forceinline__ typename CF::Elem* bpack() const { return reinterpret_cast<typename CF::Elem*>(g_smem + CF::L_BP); }
  __device__ __forceinline__ float* bias() const { return reinterpret_cast<float*>(g_smem + CF::L_BI); }
  __device__ __forceinline__ RecL* rec(int b) const {
    return reinterpret_cast<RecL*>(g_smem + (b ? CF::L_REC2 : CF::L_REC));
  }
  __device__ __forceinline__ typename CF::Elem* X() const { return reinterpret_cast<typename CF::Elem*>(g_smem + CF::L_X); }
  __device__ __forceinline__ float* out() const { return reinterpret_cast<float*>(g_smem + CF::L_OUT); }
  __device__ __forceinline__ typename CF::Elem* GZ() const { return reinterpret_cast<typename CF::Elem*>(g_smem + CF::L_GZ); }
  __device__ __forceinline__ typename CF::Elem* AT() const { return reinterpret_cast<typename CF::Elem*>(g_smem + CF::L_AT); }
  __device__ __forceinline__ int* scr() const { return reinterpret_cast<int*>(g_smem + CF::L_SCR); }
  // entry = the hit's ray lane | (its slot in the ray's hit list << 8)
  __device__ __forceinline__ typename CF::MapT* hmap() const {
    return reinterpret_cast<typename CF::MapT*>(g_smem + CF::L_MAP);
  }
};

template <class CF>
__device__ __forceinline__ typename CF::Elem to_elem(float v) {
  if constexpr (CF::BF) return static_cast<uint16_t>(bf16_rne(v));
  else return v;
}

// ------------------------------------------------------------ weight packs

template <class CF>
__device__ __forceinline__ void build_packs(const Smem<CF>& sm, const float* __restrict__ params) {
  constexpr int E = CF::BF ? 8 : 1;
  static_for<CF::NL>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    constexpr int IW = in_w(l, CF::CI, CF::H), OW = out_w(l, CF::H, CF::NH);
    constexpr int IR = in_real(l, CF::CIN, CF::H), OR = out_real(l, CF::H, CF::NH);
    constexpr int STEPS = IW / CF::KS;
    const float* W = params + par_w(l, CF::CIN, CF::H, CF::NH);
    const float* b = params + par_b(l, CF::CIN, CF::H, CF::NH);
    typename CF::Elem* fp = sm.fpack() + fwd_off(l, CF::CI, CF::H, CF::NH);
    for (int e = threadIdx.x; e < OW * IW; e += kThreads) {
      const int j = e % E, lane = (e / E) % 64, s = (e / (E * 64)) % STEPS, mt = e / (E * 64 * STEPS);
      const int m = 32 * mt + (lane & 31), g = lane >> 5;
      const int k = (l == 0) ? kmap_x<CF::BF>(s, g, j) : kmap_d<CF::BF>(s, g, j);
      fp[e] = to_elem<CF>((m < OR && k < IR) ? W[m * IR + k] : 0.0f);
    }
    for (int r = threadIdx.x; r < OW; r += kThreads)
      sm.bias()[bias_off(l, CF::H, CF::NH) + r] = r < OR ? b[r] : 0.0f;
    if constexpr (CF::BWD) {
      // transposed pack: M = layer input (padded), K = layer output (D layout)
      constexpr int BM = bwd_m(l, CF::H), BSTEPS = OW / CF::KS;
      typename CF::Elem* bp = sm.bpack() + bwd_off(l, CF::H, CF::NH);
      for (int e = threadIdx.x; e < BM * OW; e += kThreads) {
        const int j = e % E, lane = (e / E) % 64, s = (e / (E * 64)) % BSTEPS, mt = e / (E * 64 * BSTEPS);
        const int m = 32 * mt + (lane & 31), g = lane >> 5;
        const int k = kmap_d<CF::BF>(s, g, j);
        bp[e] = to_elem<CF>((m < IR && k < OR) ? W[k * IR + m] : 0.0f);
      }
    }
  });
}

template <class CF>
__device__ __forceinline__ typename CF::Op pack_operand(const typename CF::Elem* pack, int mt, int s,
                                                        int steps, int lane) {
  if constexpr (CF::BF)
    return *reinterpret_cast<const s16x8*>(pack + ((mt * steps + s) * 64 + lane) * 8);
  else
    return pack[(mt * steps + s) * 64 + lane];
}

template <class CF>
__device__ __forceinline__ typename CF::Op d_operand(const f32x16* t, int s) {
  if constexpr (CF::BF) {
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

template <class CF>
__device__ __forceinline__ typename CF::Op x_operand(const Smem<CF>& sm, int row, int s, int g) {
  if constexpr (CF::BF) {
    return *reinterpret_cast<const s16x8*>(sm.X() + row * CF::XS + 16 * s + 8 * g);
  } else {
    return sm.X()[row * CF::XS + 4 * (2 * (s >> 2) + g) + (s & 3)];
  }
}

template <class CF>
__device__ __forceinline__ f32x16 bias_tile(const Smem<CF>& sm, int l_off, int mt, int g) {
  f32x16 t;
  const float* b = sm.bias() + l_off + 32 * mt + 4 * g;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(b + 8 * q);
    t[4 * q + 0] = v[0];
    t[4 * q + 1] = v[1];
    t[4 * q + 2] = v[2];
    t[4 * q + 3] = v[3];
  }
  return t;
}

// Kept hidden activations of a 32x32 tile (backward only): FP32 values, or
// on the BF16 path the bfloat16 values the MFMA operands were made of.
template <bool BF>
struct ActTile;
template <>
struct ActTile<true> {
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
struct ActTile<false> {
  f32x16 v;
  __device__ __forceinline__ void set(const f32x16& t) { v = t; }
  __device__ __forceinline__ bool positive(int i) const { return v[i] > 0.0f; }
  __device__ __forceinline__ float elem(int i) const { return v[i]; }
};

// Decoder forward on the 32 hits [n0, n0+32) of the window.  Returns the
// output tile (rows 0..3 = raw o_0..o_3 in registers 0..3 of lanes 0..31);
// with SAVE, the post-ReLU activations of every hidden layer are kept.
template <class CF, bool SAVE>
__device__ __forceinline__ f32x16 mlp_tile(const Smem<CF>& sm, int n0, int lane,
                                           ActTile<CF::BF> (&act)[CF::NH][CF::MTH]) {
  const int g = lane >> 5, row = n0 + (lane & 31);
  f32x16 cur[CF::MTH];
  {
    constexpr int S0 = CF::CI / CF::KS;
    const typename CF::Elem* A = sm.fpack();
#pragma unroll
    for (int mt = 0; mt < CF::MTH; ++mt) cur[mt] = bias_tile(sm, 0, mt, g);
#pragma unroll
    for (int s = 0; s < S0; ++s) {
      const typename CF::Op b = x_operand(sm, row, s, g);
#pragma unroll
      for (int mt = 0; mt < CF::MTH; ++mt) cur[mt] = mma(pack_operand<CF>(A, mt, s, S0, lane), b, cur[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < CF::MTH; ++mt) relu16(cur[mt]);
    if constexpr (SAVE) {
#pragma unroll
      for (int mt = 0; mt < CF::MTH; ++mt) act[0][mt].set(cur[mt]);
    }
  }
  static_for<CF::NH - 1>([&](auto lc) {
    constexpr int l = decltype(lc)::value + 1;
    constexpr int S = CF::H / CF::KS;
    const typename CF::Elem* A = sm.fpack() + fwd_off(l, CF::CI, CF::H, CF::NH);
    f32x16 nxt[CF::MTH];
#pragma unroll
    for (int mt = 0; mt < CF::MTH; ++mt) nxt[mt] = bias_tile(sm, bias_off(l, CF::H, CF::NH), mt, g);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const typename CF::Op b = d_operand<CF>(cur, s);
#pragma unroll
      for (int mt = 0; mt < CF::MTH; ++mt) nxt[mt] = mma(pack_operand<CF>(A, mt, s, S, lane), b, nxt[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < CF::MTH; ++mt) {
      relu16(nxt[mt]);
      cur[mt] = nxt[mt];
      if constexpr (SAVE) act[l][mt].set(nxt[mt]);
    }
  });
  constexpr int S = CF::H / CF::KS;
  const typename CF::Elem* A = sm.fpack() + fwd_off(CF::NH, CF::CI, CF::H, CF::NH);
  f32x16 o = bias_tile(sm, bias_off(CF::NH, CF::H, CF::NH), 0, g);
#pragma unroll
  for (int s = 0; s < S; ++s) o = mma(pack_operand<CF>(A, 0, s, S, lane), d_operand<CF>(cur, s), o);
  return o;
}

// Data gradient through layer l: r = W_l^T gt (gt in D layout over the
// layer's outputs, r in D layout over its inputs).
template <class CF, int l>
__device__ __forceinline__ void bwd_data(const Smem<CF>& sm, const f32x16* gt, f32x16* r, int lane) {
  constexpr int MT = bwd_m(l, CF::H) / 32;
  constexpr int S = out_w(l, CF::H, CF::NH) / CF::KS;
  const typename CF::Elem* B = sm.bpack() + bwd_off(l, CF::H, CF::NH);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) r[mt] = zero16();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const typename CF::Op b = d_operand<CF>(gt, s);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) r[mt] = mma(pack_operand<CF>(B, mt, s, S, lane), b, r[mt]);
  }
}

// Writes kept activation tiles of the hits [n0, n0+32) transposed into T.
template <class CF, int NT>
__device__ __forceinline__ void store_act_T(typename CF::Elem* T, const ActTile<CF::BF>* t, int n0,
                                            int lane) {
  const int g = lane >> 5, col = n0 + (lane & 31);
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
#pragma unroll
    for (int i = 0; i < 16; ++i) T[(32 * mt + drow(i, g)) * CF::TS + col] = t[mt].elem(i);
  }
}

// Writes `nt` D-layout tiles of the hits [n0, n0+32) transposed into T
// ([feature][hit], row stride TS).
template <class CF, int NT>
__device__ __forceinline__ void store_T(typename CF::Elem* T, const f32x16* t, int n0, int lane) {
  const int g = lane >> 5, col = n0 + (lane & 31);
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
#pragma unroll
    for (int i = 0; i < 16; ++i) T[(32 * mt + drow(i, g)) * CF::TS + col] = to_elem<CF>(t[mt][i]);
  }
}

// ------------------------------------------------------------ the kernel

template <class CF>
__global__ __launch_bounds__(kThreads, CF::BWD ? 1 : 3) void k_shade(ShadeArgs a) {
  const Smem<CF> sm{};
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;

  build_packs<CF>(sm, a.params);

  // dW tiles owned by this wave (accumulated over everything this block does)
  f32x16 dw[CF::DW_SLOTS > 0 ? CF::DW_SLOTS : 1];
#pragma unroll
  for (int i = 0; i < CF::DW_SLOTS; ++i) dw[i] = zero16();
  // bias gradients: for layer l, thread (row = tid % out_w, part = tid /
  // out_w) sums its share of every window's hits; the parts are combined
  // once at the end
  float dbp[CF::NL];
#pragma unroll
  for (int l = 0; l < CF::NL; ++l) dbp[l] = 0.0f;
  float loss_acc = 0.0f;

  // Items (256-ray blocks) are dealt round-robin over the persistent grid
  // for balance; the logical block index groups the blocks of one XCD
  // (hardware places block b on XCD b % 8) so that each XCD works on
  // neighbouring rays in every round and shares their features in its L2.
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int NB = a.tab.n_blocks;
  // The last two rounds of items are handed out in order by a counter to
  // whichever block is free, so that blocks whose items held fewer hits
  // take more of them and the launch does not wait on the slowest block.
  const int n_tail = a.item_counter != nullptr ? (NB < 2 * G ? NB : 2 * G) : 0;
  const int n_static = NB - n_tail;
  auto tail_item = [&]() -> int {
    if (n_tail == 0) return NB;                 // no counter: every item is dealt statically
    if (tid == 0) sm.scr()[9] = n_static + atomicAdd(a.item_counter, 1);
    __syncthreads();
    const int it = sm.scr()[9];
    __syncthreads();
    return it;
  };

  // Backward: a window's feature-gradient atomics are issued after the next
  // window's gather, so that the gather's loads do not queue behind them
  // (the vector-memory counter a wave waits on counts both); the window's
  // records stay in the other record buffer, its dL/dx in the GZ region
  // (untouched until the next window's backward).
  int rb = 0;                    // record buffer of the current window
  int pend_tw = 0;               // hits of the window awaiting its scatter
  float* pend_grad = nullptr;
  auto scatter = [&](int ptw, float* pgrad, const RecL* prec) {
    const int n0p = 32 * wave;
    if (wave < CF::NTILE && n0p < ptw) {
      constexpr int HPI = 64 / CF::C;            // hits per instruction
      const int c = lane % CF::C, hs = lane / CF::C;
      const float* gxs = reinterpret_cast<const float*>(sm.GZ());
      for (int k = 0; k < 32; k += HPI) {
        const int hh = n0p + k + hs;
        if (hh < ptw) {
          const RecL rc = prec[hh];
          const int vid[8] = {rc.v0.x, rc.v0.y, rc.v0.z, rc.v0.w, rc.v1.x, rc.v1.y, rc.v1.z, rc.v1.w};
          const float wx[2] = {1.0f - rc.ux, rc.ux}, wy[2] = {1.0f - rc.uy, rc.uy},
                      wz[2] = {1.0f - rc.uz, rc.uz};
          const float gv = gxs[hh * CF::C + c];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float wj = wx[j & 1] * wy[(j >> 1) & 1] * wz[j >> 2];
            unsafeAtomicAdd(pgrad + static_cast<int64_t>(vid[j]) * CF::C + c, wj * gv);
          }
        }
      }
    }
  };

  __syncthreads();

  for (int item = lb < n_static ? lb : tail_item(); item < NB;
       item = item + G < n_static ? item + G : tail_item()) {
    int si = 0;
    while (si + 1 < a.tab.n && item >= a.tab.s[si + 1].block_begin) ++si;
    const DevScene& sc = a.tab.s[si];
    const ItemRays ir = item_rays(sc, item);
    const int64_t r = ir.ray(tid);
    const bool live = r < sc.ray_end;
    const int count = live ? a.cnt[r] : 0;
    // the ray's target (train) or upstream gradient (backward), read before
    // any window so that no load waits behind pending atomics
    float tg0 = 0.0f, tg1 = 0.0f, tg2 = 0.0f, tg3 = 0.0f, tg4 = 0.0f;
    if (CF::MODE == kTrain && live) {
      tg0 = a.t_rgb[3 * r]; tg1 = a.t_rgb[3 * r + 1]; tg2 = a.t_rgb[3 * r + 2]; tg3 = a.t_depth[r];
    } else if (CF::MODE == kBackward && live) {
      tg0 = a.g_rgb[3 * r]; tg1 = a.g_rgb[3 * r + 1]; tg2 = a.g_rgb[3 * r + 2]; tg3 = a.g_depth[r];
      tg4 = a.g_acc ? a.g_acc[r] : 0.0f;
    }
    const float h = __int_as_float((128 - sc.depth) << 23);       // 2^(1-depth)
    const float inv_h = __int_as_float((126 + sc.depth) << 23);   // 2^(depth-1)
    int total;
    // with IMAP all of the item's hits are mapped (hit -> ray lane, slot)
    // once, as part of the scan
    const int off = block_excl_scan<kWaves>(count, sm.scr(), total, [&](int o) {
      if constexpr (CF::IMAP)
        for (int q = 0; q < count; ++q) sm.hmap()[o + q] = static_cast<typename CF::MapT>(tid | (q << 8));
    });
    float cr = 0.0f, cg = 0.0f, cb = 0.0f, dep = 0.0f, acc = 0.0f;

    // Window: the rays whose hits all fit in [w0, w0 + WIN).  Returns the
    // window's end; `inw` = this ray is in it.  With the item's map the end
    // is the start of the ray that holds hit w0 + WIN (no ray is longer than
    // a window), read without a barrier; otherwise the ray's lane alone
    // publishes its map entries into window map `hb`.
    auto open_win = [&](int w0, int hb, bool& inw) -> int {
      if constexpr (CF::IMAP) {
        const int p = w0 + CF::WIN;
        const int w1 = p < total ? p - (sm.hmap()[p] >> 8) : total;
        inw = count > 0 && off >= w0 && off + count <= w1;
        return w1;
      } else {
        if (tid == 0) sm.scr()[8] = total;
        __syncthreads();
        const bool started = count > 0 && off >= w0;
        inw = started && off + count <= w0 + CF::WIN;
        if (started && !inw) atomicMin(&sm.scr()[8], off);
        __syncthreads();
        const int w1 = sm.scr()[8];
        if (inw) {
          for (int q = 0; q < count; ++q)
            sm.hmap()[hb * CF::WIN + off - w0 + q] = static_cast<typename CF::MapT>(tid | (q << 8));
        }
        __syncthreads();
        return w1;
      }
    };
    // map entry of hit hh of the window starting at w0 (map `hb`)
    auto map_at = [&](int w0, int hb, int hh) -> int {
      return sm.hmap()[CF::IMAP ? w0 + hh : hb * CF::WIN + hh];
    };
    // Gather in three dependent stages: (A) hit records and rays, (B) the
    // leaves' corner ids, (C) the 8 corner rows (issued into registers, then
    // consumed with the trilinear weights into X).  A thread serves GRP hits
    // (in the backward kernels one group covers the window).  There (PIPE)
    // windows are opened one ahead: the next window's stage A is issued
    // before this window's rows are consumed, its stage B after the forward
    // decoder and its stage C loads after the compositing, so that they are
    // in flight while this window's backward runs; only an item's first
    // window waits on all three.
    constexpr int ROWB = CF::C * CF::EB;
    constexpr int TPH = ROWB / 16;
    constexpr int VPT = 16 / CF::EB;             // values per thread
    constexpr int HPP = kThreads / TPH;
    constexpr int NPASS = (CF::WIN + HPP - 1) / HPP;
    constexpr int GRP = (CF::BWD && NPASS >= 2) ? 2 : 1;
    constexpr bool PIPE = CF::BWD;   // forward kernels: slower so (at their register cap)
    static_assert(!PIPE || NPASS == GRP, "one gather group per window");
    const int q = tid % TPH;
    // raw feature rows of a hit's 8 corners: 16 bytes per corner and thread
    using Raw = typename std::conditional<CF::BF, uint4, float4>::type;
    struct Stage {
      int hh[GRP];
      bool val[GRP];
      HitRec hr[GRP];
      float ro[GRP][3], rd[GRP][3];
      int4 c0[GRP], c1[GRP];
    };
    // one window's raw rows: filled for the next window after this one's
    // compositing, consumed when the next window starts
    Raw raw[GRP][8];
    auto stage_a = [&](Stage& st, int pb, int w0, int hb, int twin) {
#pragma unroll
      for (int k = 0; k < GRP; ++k) {
        st.hh[k] = (pb + k) * HPP + tid / TPH;
        st.val[k] = st.hh[k] < twin;
        if (st.val[k]) {
          const int mp = map_at(w0, hb, st.hh[k]);
          const int64_t rr = ir.ray(mp & 0xFF);
          st.hr[k] = a.hits[rr * a.K + (mp >> 8)];
          st.ro[k][0] = a.o[3 * rr]; st.ro[k][1] = a.o[3 * rr + 1]; st.ro[k][2] = a.o[3 * rr + 2];
          st.rd[k][0] = a.d[3 * rr]; st.rd[k][1] = a.d[3 * rr + 1]; st.rd[k][2] = a.d[3 * rr + 2];
        }
      }
    };
    auto stage_b = [&](Stage& st) {
#pragma unroll
      for (int k = 0; k < GRP; ++k) {
        if (st.val[k]) {
          const int4* lc = reinterpret_cast<const int4*>(sc.leaf_corners + 8 * static_cast<int64_t>(st.hr[k].leaf));
          st.c0[k] = lc[0];
          st.c1[k] = lc[1];
        }
      }
    };
    // (C, issue) the 8 corner rows of each hit into registers
    auto stage_c_issue = [&](const Stage& st) {
#pragma unroll
      for (int k = 0; k < GRP; ++k) {
        if (!st.val[k]) continue;
        const int vid[8] = {st.c0[k].x, st.c0[k].y, st.c0[k].z, st.c0[k].w,
                            st.c1[k].x, st.c1[k].y, st.c1[k].z, st.c1[k].w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if constexpr (CF::BF)
            raw[k][j] = *reinterpret_cast<const uint4*>(sc.feat16 + static_cast<int64_t>(vid[j]) * CF::C + 8 * q);
          else
            raw[k][j] = *reinterpret_cast<const float4*>(sc.feat32 + static_cast<int64_t>(vid[j]) * CF::C + 4 * q);
        }
      }
    };
    // (C, consume) trilinear weights, the hit's LDS record and its row of X
    auto stage_c_consume = [&](Stage& st) {
      float v[GRP][VPT];
#pragma unroll
      for (int k = 0; k < GRP; ++k) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) v[k][i] = 0.0f;
        if (!st.val[k]) continue;
        float tm, tml;
        midpoint2(st.hr[k].tin, st.hr[k].tout, tm, tml);
        const float lx = -1.0f + static_cast<float>(st.hr[k].ijk & 1023u) * h;
        const float ly = -1.0f + static_cast<float>((st.hr[k].ijk >> 10) & 1023u) * h;
        const float lz = -1.0f + static_cast<float>(st.hr[k].ijk >> 20) * h;
        const float ux = fminf(fmaxf(cell_coord(st.ro[k][0], st.rd[k][0], tm, tml, lx, inv_h), 0.0f), 1.0f);
        const float uy = fminf(fmaxf(cell_coord(st.ro[k][1], st.rd[k][1], tm, tml, ly, inv_h), 0.0f), 1.0f);
        const float uz = fminf(fmaxf(cell_coord(st.ro[k][2], st.rd[k][2], tm, tml, lz, inv_h), 0.0f), 1.0f);
        if (q == 0) {
          RecL rc;
          rc.leaf = st.hr[k].leaf;
          rc.ux = ux;
          rc.uy = uy;
          rc.uz = uz;
          rc.tmid = tm;
          rc.dt = st.hr[k].tout - st.hr[k].tin;
          rc.T = 0.0f;
          rc.pad = 0.0f;
          rc.v0 = st.c0[k];
          rc.v1 = st.c1[k];
          sm.rec(rb)[st.hh[k]] = rc;
        }
        const float wx[2] = {1.0f - ux, ux}, wy[2] = {1.0f - uy, uy}, wz[2] = {1.0f - uz, uz};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float wj = wx[j & 1] * wy[(j >> 1) & 1] * wz[j >> 2];
          if constexpr (CF::BF) {
            const uint32_t w4[4] = {raw[k][j].x, raw[k][j].y, raw[k][j].z, raw[k][j].w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              v[k][2 * i] += wj * bf16_f32(static_cast<uint16_t>(w4[i] & 0xFFFFu));
              v[k][2 * i + 1] += wj * bf16_f32(static_cast<uint16_t>(w4[i] >> 16));
            }
          } else {
            const float4 f = raw[k][j];
            v[k][0] += wj * f.x;
            v[k][1] += wj * f.y;
            v[k][2] += wj * f.z;
            v[k][3] += wj * f.w;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < GRP; ++k) {
        if (st.hh[k] >= CF::WIN) continue;
        typename CF::Elem* xr = sm.X() + st.hh[k] * CF::XS + VPT * q;
#pragma unroll
        for (int i = 0; i < VPT; ++i) xr[i] = to_elem<CF>(v[k][i]);
        if (CF::CI > CF::C && q == 0) {
          // view direction (VD) and zero padding up to the K steps
#pragma unroll
          for (int i = CF::C; i < CF::CI; ++i) {
            float xv = 0.0f;
            if (CF::VD && i < CF::C + 3 && st.val[k]) xv = st.rd[k][i - CF::C];
            sm.X()[st.hh[k] * CF::XS + i] = to_elem<CF>(xv);
          }
        }
      }
    };
    auto stage_c = [&](Stage& st) {
      stage_c_issue(st);
      stage_c_consume(st);
    };

    Stage cur, nxt;
    int hb = 0;                    // window map of the current window (without IMAP)
    bool have_next = false;        // nxt holds stages A and B of the next window
    bool in_win_n = false;
    int s1n = 0;
    int s0 = 0;
    while (s0 < total) {
      bool in_win;
      int s1;
      if (have_next) {
        cur = nxt;
        in_win = in_win_n;
        s1 = s1n;
      } else {
        s1 = open_win(s0, hb, in_win);
      }
      const int tw = s1 - s0;
      const bool pre = PIPE && s1 < total;
      if (pre) s1n = open_win(s1, hb ^ 1, in_win_n);
      if (PIPE) {
        if (!have_next) {
          stage_a(cur, 0, s0, hb, tw);
          stage_b(cur);
          stage_c_issue(cur);
        }
        if (pre) stage_a(nxt, 0, s1, hb ^ 1, s1n - s1);
        stage_c_consume(cur);
      } else {
#pragma unroll 1
        for (int pb = 0; pb < NPASS; pb += GRP) {
          stage_a(cur, pb, s0, hb, tw);
          stage_b(cur);
          stage_c(cur);
        }
      }
      __syncthreads();

      if constexpr (CF::BWD) {
        if (pend_tw > 0) scatter(pend_tw, pend_grad, sm.rec(rb ^ 1));
        pend_tw = 0;
      }

      // decoder on the window: one 32-hit tile per wave
      ActTile<CF::BF> act[CF::NH][CF::MTH];
      const int n0 = 32 * wave;
      const bool has_tile = wave < CF::NTILE && n0 < tw;
      if (has_tile) {
        const f32x16 o = mlp_tile<CF, CF::BWD>(sm, n0, lane, act);
        // per-hit epilogue, one hit per lane: colour, opacity and
        // transmittance factor of the segment (section 4 footnote, Eq. 3)
        if (g == 0 && n0 + lane < tw) {
          const RecL& rc = sm.rec(rb)[n0 + lane];
          const float ft = a.tau_mode == SVLF_TAU_VOXEL ? rc.dt * inv_h
                           : a.tau_mode == SVLF_TAU_WORLD ? rc.dt : 1.0f;
          const float tau = fmaxf(o[3], 0.0f) * ft;
          const f32x4 va = {sigmoidf_(o[0]), sigmoidf_(o[1]), sigmoidf_(o[2]), -expm1f(-tau)};
          const f32x4 vb = {expf(-tau), o[3] > 0.0f ? ft : 0.0f, rc.tmid, 0.0f};
          *reinterpret_cast<f32x4*>(sm.out() + 8 * (n0 + lane)) = va;
          *reinterpret_cast<f32x4*>(sm.out() + 8 * (n0 + lane) + 4) = vb;
        }
      }
      if (pre) stage_b(nxt);
      __syncthreads();

      // Eq. 3 front to back (owner lanes), and its backward
      // Eq. 3 front to back (owner lanes), and its backward
      if (in_win) {
        const int p0 = off - s0;
        float T = 1.0f;
        for (int q = 0; q < count; ++q) {
          float* hp = sm.out() + 8 * (p0 + q);
          const f32x4 va = *reinterpret_cast<const f32x4*>(hp);
          const f32x4 vb = *reinterpret_cast<const f32x4*>(hp + 4);
          const float w = T * va[3];
          cr += w * va[0];
          cg += w * va[1];
          cb += w * va[2];
          dep += w * vb[2];
          acc += w;
          if constexpr (CF::BWD) hp[7] = T;
          T *= vb[0];
        }
        if constexpr (CF::BWD) {
          float gr, gg, gb, gd, ga;
          if (CF::MODE == kTrain) {
            const float er = cr - tg0, eg = cg - tg1, eb = cb - tg2, ed = dep - tg3;
            const float k2 = a.loss_scale * (2.0f / 3.0f);
            gr = k2 * er;
            gg = k2 * eg;
            gb = k2 * eb;
            gd = a.loss_scale * a.lambda_depth * (ed > 0.0f ? 1.0f : (ed < 0.0f ? -1.0f : 0.0f));
            ga = 0.0f;
          } else {
            gr = tg0;
            gg = tg1;
            gb = tg2;
            gd = tg3;
            ga = tg4;
          }
          float Sr = 0.0f, Sg = 0.0f, Sb = 0.0f, St = 0.0f, Sa = 0.0f;
          for (int q = count - 1; q >= 0; --q) {
            float* hp = sm.out() + 8 * (p0 + q);
            const f32x4 va = *reinterpret_cast<const f32x4*>(hp);
            const f32x4 vb = *reinterpret_cast<const f32x4*>(hp + 4);
            const float Tq = vb[3];
            const float w = Tq * va[3];
            const float Tn = Tq * vb[0];
            const float c0 = va[0], c1 = va[1], c2 = va[2], tm = vb[2];
            const float gtau = gr * (Tn * c0 - Sr) + gg * (Tn * c1 - Sg) + gb * (Tn * c2 - Sb) +
                               gd * (Tn * tm - St) + ga * (Tn - Sa);
            Sr += w * c0;
            Sg += w * c1;
            Sb += w * c2;
            St += w * tm;
            Sa += w;
            f32x4 go;
            go[0] = gr * w * c0 * (1.0f - c0);
            go[1] = gg * w * c1 * (1.0f - c1);
            go[2] = gb * w * c2 * (1.0f - c2);
            go[3] = gtau * vb[1];
            *reinterpret_cast<f32x4*>(hp) = go;
          }
        }
      }

      if constexpr (CF::BWD) {
        // the next window's corner rows: loaded while this window's
        // backward runs from LDS and registers
        if (pre) stage_c_issue(nxt);
        __syncthreads();
        // output-layer gradient tile (rows 0..3 = dL/do, zero elsewhere)
        f32x16 gz[CF::MTH];
#pragma unroll
        for (int mt = 0; mt < CF::MTH; ++mt) gz[mt] = zero16();
        if (has_tile && g == 0 && n0 + lane < tw) {
          const f32x4 go = *reinterpret_cast<const f32x4*>(sm.out() + 8 * (n0 + lane));
          gz[0][0] = go[0];
          gz[0][1] = go[1];
          gz[0][2] = go[2];
          gz[0][3] = go[3];
        }
        f32x16 gx[1];
        static_for<CF::NL>([&](auto lc) {
          constexpr int l = CF::NH - decltype(lc)::value;
          constexpr int OT = out_w(l, CF::H, CF::NH) / 32;
          // stage dL/dz_l and the layer input, transposed, for the dW tiles
          if (wave < CF::NTILE) {
            if (has_tile) {
              store_T<CF, OT>(sm.GZ(), gz, n0, lane);
              if constexpr (l > 0) store_act_T<CF, CF::MTH>(sm.AT(), act[l - 1], n0, lane);
            } else {
              // empty tile: zero its columns
              const int col = n0 + (lane & 31);
              for (int rr = g; rr < 32 * OT; rr += 2) sm.GZ()[rr * CF::TS + col] = to_elem<CF>(0.0f);
              if constexpr (l > 0)
                for (int rr = g; rr < CF::H; rr += 2) sm.AT()[rr * CF::TS + col] = to_elem<CF>(0.0f);
            }
          }
          if constexpr (l == 0)
            transpose_tile<CF::BF, CF::WIN, CF::XS, CF::TS, CF::CI, CF::CI, kThreads>(sm.X(), sm.AT(), tid);
          __syncthreads();
          // owned dW tiles of layer l: K = the window's hits
          {
            constexpr int MT = dw_mt(l, CF::H, CF::NH), NT = dw_nt(l, CF::H, CF::CIN);
            constexpr int T0 = dw_tile_off(l, CF::H, CF::NH, CF::CIN);
            constexpr int KSTEPS = CF::WIN / CF::KS;
            static_for<MT * NT>([&](auto tc) {
              constexpr int t = decltype(tc)::value;
              constexpr int tau_i = T0 + t, mt = t / NT, nt = t % NT, slot = tau_i / kWaves;
              if (tau_i % kWaves == wave) {
                const typename CF::Elem* ga_ = sm.GZ() + (32 * mt + (lane & 31)) * CF::TS;
                const typename CF::Elem* gb_ = sm.AT() + (32 * nt + (lane & 31)) * CF::TS;
#pragma unroll
                for (int s = 0; s < KSTEPS; ++s) {
                  if constexpr (CF::BF) {
                    const s16x8 av = *reinterpret_cast<const s16x8*>(ga_ + 16 * s + 8 * g);
                    const s16x8 bv = *reinterpret_cast<const s16x8*>(gb_ + 16 * s + 8 * g);
                    dw[slot] = mma(av, bv, dw[slot]);
                  } else {
                    dw[slot] = mma(ga_[2 * s + g], gb_[2 * s + g], dw[slot]);
                  }
                }
              }
            });
          }
          {
            constexpr int RW = out_w(l, CF::H, CF::NH);
            constexpr int HP = CF::WIN / (kThreads / RW);     // hits per part
            static_assert(kThreads % RW == 0 && (!CF::BF || HP % 8 == 0), "bias-gradient parts");
            const int row = tid % RW, pt = tid / RW;
            if (row < out_real(l, CF::H, CF::NH)) {
              const typename CF::Elem* gr_ = sm.GZ() + row * CF::TS + pt * HP;
              float sacc = 0.0f;
              if constexpr (CF::BF) {
#pragma unroll
                for (int hh = 0; hh < HP; hh += 8) {
                  const s16x8 v = *reinterpret_cast<const s16x8*>(gr_ + hh);
#pragma unroll
                  for (int j = 0; j < 8; ++j) sacc += bf16_f32(static_cast<uint16_t>(v[j]));
                }
              } else {
#pragma unroll
                for (int hh = 0; hh < HP; ++hh) sacc += gr_[hh];
              }
              dbp[l] += sacc;
            }
          }
          // data gradient to the layer input
          if (has_tile) {
            if constexpr (l > 0) {
              f32x16 ga[CF::MTH];
              bwd_data<CF, l>(sm, gz, ga, lane);
#pragma unroll
              for (int mt = 0; mt < CF::MTH; ++mt) {
#pragma unroll
                for (int i = 0; i < 16; ++i) gz[mt][i] = act[l - 1][mt].positive(i) ? ga[mt][i] : 0.0f;
              }
            } else {
              bwd_data<CF, 0>(sm, gz, gx, lane);
            }
          }
          __syncthreads();
        });
        // scatter dL/dx to the 8 corner features of each hit.  dL/dx is
        // staged through LDS so that the lanes of one atomic instruction
        // cover whole contiguous feature rows (lane = channel): the memory
        // system then merges them per cache line instead of issuing one
        // transaction per lane.
        float* gxs = reinterpret_cast<float*>(sm.GZ());      // [WIN][C] FP32
        if (has_tile) {
          const int row = n0 + (lane & 31);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (8 * q + 4 * g < CF::C) {
#pragma unroll
              for (int p = 0; p < 4; ++p) gxs[row * CF::C + 8 * q + 4 * g + p] = gx[0][4 * q + p];
            }
          }
        }
        __syncthreads();
        if (a.gxu != nullptr) {
          // deterministic mode: keep (u, dL/dx) per hit slot; the feature
          // gradient is reduced afterwards in a fixed order
          if (has_tile) {
            constexpr int HPI = 64 / CF::C;
            const int c = lane % CF::C, hs = lane / CF::C;
            for (int k = 0; k < 32; k += HPI) {
              const int hh = n0 + k + hs;
              if (hh < tw) {
                const RecL rc = sm.rec(rb)[hh];
                const int mp = map_at(s0, hb, hh);
                const int64_t slot = ir.ray(mp & 0xFF) * a.K + (mp >> 8);
                float* rec_out = a.gxu + slot * (CF::C + 4);
                rec_out[4 + c] = gxs[hh * CF::C + c];
                if (c < 3) rec_out[c] = c == 0 ? rc.ux : (c == 1 ? rc.uy : rc.uz);
              }
            }
          }
        } else {
          pend_tw = tw;
          pend_grad = sc.grad;
          rb ^= 1;
        }
      }
      __syncthreads();
      s0 = s1;
      have_next = pre;
      if (pre) hb ^= 1;
    }

    if (live) {
      if (CF::MODE != kBackward) {
        if (a.rgb) {
          a.rgb[3 * r] = cr;
          a.rgb[3 * r + 1] = cg;
          a.rgb[3 * r + 2] = cb;
        }
        if (a.depth) a.depth[r] = dep;
        if (a.acc) a.acc[r] = acc;
      }
      if (CF::MODE == kTrain) {
        const float er = cr - tg0, eg = cg - tg1, eb = cb - tg2, ed = dep - tg3;
        loss_acc += a.loss_scale * ((er * er + eg * eg + eb * eb) * (1.0f / 3.0f) +
                                    a.lambda_depth * fabsf(ed));
      }
    }
  }

  if constexpr (CF::BWD) {
    if (pend_tw > 0) scatter(pend_tw, pend_grad, sm.rec(rb ^ 1));
    // this block's partial sums of dL/dparams (every entry written once)
    float* part = a.ws_partials + static_cast<int64_t>(blockIdx.x) * CF::NPARAMS;
    static_for<CF::NL>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      constexpr int MT = dw_mt(l, CF::H, CF::NH), NT = dw_nt(l, CF::H, CF::CIN);
      constexpr int T0 = dw_tile_off(l, CF::H, CF::NH, CF::CIN);
      constexpr int IR = in_real(l, CF::CIN, CF::H), OR = out_real(l, CF::H, CF::NH);
      static_for<MT * NT>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        constexpr int tau_i = T0 + t, mt = t / NT, nt = t % NT, slot = tau_i / kWaves;
        if (tau_i % kWaves == wave) {
          const int col = 32 * nt + (lane & 31);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int rowo = 32 * mt + drow(i, g);
            if (rowo < OR && col < IR) part[par_w(l, CF::CIN, CF::H, CF::NH) + rowo * IR + col] = dw[slot][i];
          }
        }
      });
    });
    // bias gradients: combine the parts through LDS ([layer][part][row])
    static_assert(CF::NL * kThreads * 4 <= CF::TROWS * CF::TS * CF::EB, "bias parts fit in GZ");
    float* bsc = reinterpret_cast<float*>(sm.GZ());
    __syncthreads();
#pragma unroll
    for (int l = 0; l < CF::NL; ++l) bsc[l * kThreads + tid] = dbp[l];
    __syncthreads();
    if (tid < CF::NBIAS) {
      const int bl = tid / CF::H < CF::NH ? tid / CF::H : CF::NH;
      const int br = tid - bl * CF::H;
      static_for<CF::NL>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        constexpr int RW = out_w(l, CF::H, CF::NH);
        if (l == bl) {
          float sum = 0.0f;
#pragma unroll
          for (int pt = 0; pt < kThreads / RW; ++pt) sum += bsc[l * kThreads + pt * RW + br];
          part[par_b(l, CF::CIN, CF::H, CF::NH) + br] = sum;
        }
      });
    }
    if (CF::MODE == kTrain) {
      const float tot = block_sum<kWaves>(loss_acc, reinterpret_cast<float*>(sm.scr()));
      if (tid == 0) a.ws_loss[blockIdx.x] = tot;
    } else if (tid == 0) {
      a.ws_loss[blockIdx.x] = 0.0f;
    }
  }
}

// Decoder alone on rows of X (diagnostics / tests): 128 rows per block pass.
template <class CF>
__global__ __launch_bounds__(kThreads) void k_mlp_rows(const float* __restrict__ params,
                                                       const float* __restrict__ X, int64_t n,
                                                       float* __restrict__ out) {
  const Smem<CF> sm{};
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5;
  build_packs<CF>(sm, params);
  __syncthreads();
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * CF::WIN; base < n;
       base += static_cast<int64_t>(gridDim.x) * CF::WIN) {
    for (int e = tid; e < CF::WIN * CF::CI; e += kThreads) {
      const int hh = e / CF::CI, c = e % CF::CI;
      const int64_t row = base + hh;
      sm.X()[hh * CF::XS + c] = to_elem<CF>((row < n && c < CF::CIN) ? X[row * CF::CIN + c] : 0.0f);
    }
    __syncthreads();
    ActTile<CF::BF> act[CF::NH][CF::MTH];
    if (wave < CF::NTILE) {
      const int n0 = 32 * wave;
      const f32x16 o = mlp_tile<CF, false>(sm, n0, lane, act);
      const int64_t row = base + n0 + (lane & 31);
      if (g == 0 && row < n) {
        out[4 * row] = o[0];
        out[4 * row + 1] = o[1];
        out[4 * row + 2] = o[2];
        out[4 * row + 3] = o[3];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ dispatch

int g_num_cus = 0;

int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      g_num_cus = n;
    else
      g_num_cus = 256;
  }
  return g_num_cus;
}

template <class CF>
hipError_t run(const ShadeArgs& a, hipStream_t s, int* grid_used) {
  const auto kern = k_shade<CF>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, CF::LDS_BYTES);
  if (e != hipSuccess) return e;
  // resident blocks per CU: LDS and registers (the persistent grid must fit
  // in one round, or the blocks of a second round would run after the rest)
  int per_cu = (160 * 1024) / CF::LDS_BYTES;
  static int occ = -1;                         // per kernel instance, queried once
  if (occ < 0 && hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     &occ, reinterpret_cast<const void*>(kern), kThreads, CF::LDS_BYTES) != hipSuccess)
    occ = 0;
  if (occ > 0 && occ < per_cu) per_cu = occ;
  int grid = num_cus() * (per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu));
  if (grid > shade_grid_limit()) grid = shade_grid_limit();
  if (grid > a.tab.n_blocks) grid = a.tab.n_blocks;
  if (grid < 1) grid = 1;
  *grid_used = grid;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), CF::LDS_BYTES, s, a);
  return hipGetLastError();
}

template <int P, int C, int H, int NH, int VD>
hipError_t run_mode(const ShadeArgs& a, int mode, hipStream_t s, int* grid) {
  if (mode == kForward) return run<Cfg<P, C, H, NH, kForward, VD>>(a, s, grid);
  if (mode == kBackward) return run<Cfg<P, C, H, NH, kBackward, VD>>(a, s, grid);
  return run<Cfg<P, C, H, NH, kTrain, VD>>(a, s, grid);
}

template <int P, int C, int H, int NH, int VD>
hipError_t run_mlp(const float* params, const float* X, int64_t n, float* out, hipStream_t s) {
  using CF = Cfg<P, C, H, NH, kForward, VD>;
  const auto kern = k_mlp_rows<CF>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, CF::LDS_BYTES);
  if (e != hipSuccess) return e;
  int64_t blocks = (n + CF::WIN - 1) / CF::WIN;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), CF::LDS_BYTES, s,
                     params, X, n, out);
  return hipGetLastError();
}

// Supported decoder shapes (C, H, hidden layers, view-direction input).
#define SVLF_SHAPES(X) \
  X(8, 32, 2, 0) X(16, 64, 3, 0) X(32, 64, 3, 0) X(8, 32, 2, 1) X(32, 64, 3, 1)

}  // namespace

int shade_grid_limit() { return 1024; }

hipError_t launch_shade(const ShadeArgs& a, int mode, hipStream_t s, int* grid_used) {
  *grid_used = 0;
  const int P = a.precision == SVLF_BF16 ? 1 : 0;
  const int vd = a.viewdir ? 1 : 0;
#define SVLF_CASE(C_, H_, NH_, VD_)                                                    \
  if (a.C == C_ && a.H == H_ && a.n_hidden == NH_ && vd == VD_)                        \
    return P ? run_mode<1, C_, H_, NH_, VD_>(a, mode, s, grid_used)                    \
             : run_mode<0, C_, H_, NH_, VD_>(a, mode, s, grid_used);
  SVLF_SHAPES(SVLF_CASE)
#undef SVLF_CASE
  return hipErrorNotSupported;
}

hipError_t launch_mlp_forward(const float* params, int C, int H, int n_hidden, int viewdir,
                              int precision, const float* X, int64_t n, float* out,
                              hipStream_t s) {
  const int P = precision == SVLF_BF16 ? 1 : 0;
  const int vd = viewdir ? 1 : 0;
#define SVLF_CASE(C_, H_, NH_, VD_)                                                    \
  if (C == C_ && H == H_ && n_hidden == NH_ && vd == VD_)                              \
    return P ? run_mlp<1, C_, H_, NH_, VD_>(params, X, n, out, s)                      \
             : run_mlp<0, C_, H_, NH_, VD_>(params, X, n, out, s);
  SVLF_SHAPES(SVLF_CASE)
#undef SVLF_CASE
  return hipErrorNotSupported;
}

}  // namespace svlf
