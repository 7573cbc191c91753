// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "svlf.h"

namespace svlf {

// Per-thread error string behind svlf_last_error().
void set_error(const std::string& msg);
void clear_error();
const char* error_cstr();

// One scene as the kernels see it (passed by value in kernel arguments).
struct DevScene {
  const svlf_node* nodes;
  const int32_t* leaf_corners;
  const float* feat32;
  const uint16_t* feat16;
  float* grad;            // backward only
  int64_t n_vertices;
  int64_t ray_begin;      // first ray of this scene
  int64_t ray_end;
  int32_t depth;
  int32_t block_begin;    // first 256-ray block of this scene in the grid
};

struct SceneTable {
  DevScene s[SVLF_MAX_SCENES];
  int32_t n;
  int32_t n_blocks;       // total 256-ray blocks over all scenes
};

// Internal hit record, one per (ray, slot): leaf id, t_in, t_out and the
// leaf's cell coordinates packed as i | j << 10 | k << 20.
struct HitRec {
  int32_t leaf;
  float tin;
  float tout;
  uint32_t ijk;
};

constexpr int kRaysPerBlock = 256;

// Rays of one work item (kRaysPerBlock rays) of the shading kernels.  The
// rays of kIlvItems consecutive full items of a scene are interleaved: item
// j of such a group takes rays j, j + kIlvItems, j + 2 kIlvItems, ... of
// the group, so that one item's rays lie far apart in the caller's order
// while the group, whose items run at about the same time, covers one
// contiguous range.  Other items take kRaysPerBlock consecutive rays.
// Lane t of the item handles ray base + t * stride (it may be past the
// scene's last ray only in a scene's last, partial item).
constexpr int kIlvItems = 256;

struct ItemRays {
  int64_t base;
  int stride;
  __device__ __forceinline__ int64_t ray(int lane) const {
    return base + static_cast<int64_t>(lane) * stride;
  }
};

__device__ __forceinline__ ItemRays item_rays(const DevScene& sc, int item) {
  const int64_t li = item - sc.block_begin, g0 = li / kIlvItems * kIlvItems;
  if ((g0 + kIlvItems) * kRaysPerBlock <= sc.ray_end - sc.ray_begin)
    return {sc.ray_begin + g0 * kRaysPerBlock + (li - g0), kIlvItems};
  return {sc.ray_begin + li * kRaysPerBlock, 1};
}

// Launchers (defined in the .hip files).
hipError_t launch_trace_public(const svlf_octree& oct, const float* o, const float* d,
                               int64_t n, int K, int32_t* leaf, float* tin, float* tout,
                               int32_t* cnt, hipStream_t s);
hipError_t launch_trace_internal(const SceneTable& tab, const float* o, const float* d,
                                 int K, HitRec* hits, int32_t* cnt, hipStream_t s);

struct ShadeArgs {
  SceneTable tab;
  const float* o;
  const float* d;
  const HitRec* hits;
  const int32_t* cnt;
  int32_t K;
  int32_t tau_mode;
  int32_t precision;
  int32_t C;              // features per vertex
  int32_t H;
  int32_t n_hidden;
  int32_t viewdir;        // decoder input [psi | d] (width C + 3)
  const float* params;
  // forward outputs
  float* rgb;
  float* depth;
  float* acc;
  // backward inputs
  const float* g_rgb;
  const float* g_depth;
  const float* g_acc;
  // train-step inputs
  const float* t_rgb;
  const float* t_depth;
  float lambda_depth;
  float loss_scale;
  float* loss_out;
  // backward outputs
  float* grad_params;
  float* ws_partials;     // [grid][n_params] per-block dW partial sums
  float* ws_loss;         // [grid] per-block loss partial sums
  int64_t n_params;
  float* gxu;             // deterministic mode: [n][K][C + 4] (u, dL/dx) per hit, else null
  int32_t* item_counter;  // zeroed before the launch: hands out the last work items (nullable)
};

// Deterministic feature-gradient reduction (detgrad.hip): the order step
// (needs only the hit lists) sorts the hits by leaf, stably in slot order,
// and builds the vertex-to-leaf table; the sum step (after the backward has
// written the per-hit records gxu) sums per vertex over its (up to 8)
// adjacent leaves in a fixed order.
size_t detgrad_bytes(int64_t n_rays, int K, int C, int64_t n_leaves, int64_t n_vertices);
hipError_t launch_detgrad_order(const DevScene& sc, const HitRec* hits, const int32_t* cnt,
                                int64_t n_rays, int K, int C, void* scratch, int64_t n_leaves,
                                int64_t n_vertices, hipStream_t s);
hipError_t launch_detgrad_sum(const DevScene& sc, int64_t n_rays, int K, int C, const float* gxu,
                              void* scratch, int64_t n_leaves, int64_t n_vertices, hipStream_t s);

enum ShadeMode { kForward = 0, kBackward = 1, kTrain = 2 };

// ---------------------------------------------------------------- light field
// The paper's two-decoder function (svlf_lf_*): per-hit state written by the
// density kernel and read by the colour kernel.
struct LfHit {
  float us[3];            // surface point in cell units (unclamped)
  float ts;               // its ray parameter
  float alpha;            // 1 - e^-tau
  float e;                // e^-tau
  float dtau;             // d tau / d o_T0 (0 where the ReLU is off)
  float eta;
};

// Train-mode losses of the light-field path: the photometric + depth loss of
// the single-decoder train step, or the paper's staged loss (Eq. 4) on the
// voxel holding the target surface point (surface stage) or with the
// composited colour (volumetric stages).
enum LfLossKind { kLfLossDefault = 0, kLfLossSurface = 1, kLfLossVolume = 2 };

// Supported light-field decoders: C_T = 64, C_C = 32, H = 128, one hidden
// layer in the density decoder and three in the colour decoder.
constexpr int kLfCT = 64, kLfCC = 32, kLfH = 128, kLfNHT = 1, kLfNHC = 3;
int lf_grid_limit();      // blocks of each light-field kernel (workspace partials)
int64_t lf_params_density();
int64_t lf_params_color(int viewdir);
size_t lf_pack_bytes(int precision, int viewdir);   // both decoders' MFMA packs
int lf_x_row();           // BF16 elements of one saved density-decoder input row

struct LfArgs {
  SceneTable tab;
  const float* o;
  const float* d;
  const HitRec* hits;
  const int32_t* cnt;
  int32_t K;
  int32_t tau_mode;
  int32_t precision;
  int32_t viewdir;
  const float* params;    // FP32 masters: density layers then colour layers
  LfHit* st;              // [n][K]
  float* gT;              // [n][K][2]: dL/d(o_T0, o_T1)
  uint16_t* xsave;        // [n][K][lf_x_row()] BF16 density-decoder inputs written by
                          // the forward density pass for the backward one (nullable)
  void* packs;            // lf_pack_bytes()
  float* rgb;
  float* depth;
  float* acc;
  const float* g_rgb;
  const float* g_depth;
  const float* g_acc;
  const float* t_rgb;
  const float* t_depth;
  float lambda_depth;
  float loss_scale;
  float* loss_out;
  float* grad_params;
  int32_t loss_kind;      // kLfLoss*: train-mode loss
  float lambda_eta;       // staged losses: weight of (eta - eta_target)^2
  float lambda_tau;       // staged losses: weight of e^{-2 tau}
  int32_t freeze_color;   // nonzero: no gradients for Z_C and the colour decoder
  int32_t* item_counters; // [3] zeroed before the kernels: density forward, colour,
                          // density backward; each hands out its launch's last items
  float* partT;           // [grid][params_density]
  float* partC;           // [grid][params_color]
  float* ws_loss;         // [grid]
};

// Occupied leaves from depth maps (occupancy.hip).
size_t occupancy_bitmap_words(int level);
hipError_t launch_occupancy(const float* o, const float* d, const float* t, int64_t n, int level,
                            uint32_t* bitmap, int* counts, int32_t* leaf_ijk, int64_t cap,
                            int64_t* n_out, hipStream_t s);

// Runs packing, the density kernel, the colour kernel and (backward / train)
// the density backward and the reductions of the decoder gradients.
hipError_t launch_lf(const LfArgs& a, int mode, hipStream_t s);

hipError_t launch_shade(const ShadeArgs& a, int mode, hipStream_t s, int* grid_used);
size_t shade_workspace_bytes(int64_t n_params, int n_rays_hint);
int shade_grid_limit();

hipError_t launch_reduce_partials(const float* partials, int rows, int64_t n, float* out,
                                  const float* loss_partials, float* loss_out, hipStream_t s);

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2, uint16_t* bf16, int zero,
                       hipStream_t s);
hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t n, hipStream_t s);
hipError_t launch_fill(float* dst, float v, int64_t n, hipStream_t s);
hipError_t launch_lazy_adam(float* p, float* g, float* m, float* v, int64_t n_rows, int row_len,
                            float lr, float b1, float b2, float eps, float bc1, float bc2,
                            uint16_t* bf16, int zero, hipStream_t s);
hipError_t launch_mlp_forward(const float* params, int C, int H, int n_hidden, int viewdir,
                              int precision, const float* X, int64_t n, float* out,
                              hipStream_t s);

// This device's copy of the library's scratch array of
// svlf_train_step_noalloc (util.hip; SVLF_NOALLOC_SCRATCH_BYTES).
hipError_t noalloc_scratch(void** ptr);

// Host octree build (octree_build.cpp).
struct HostOctree {
  svlf_octree_sizes sizes;
  std::vector<svlf_node> nodes;
  std::vector<int32_t> leaf_corners;
  std::vector<int32_t> leaf_ijk_sorted;
};
int build_octree_host(const int32_t* ijk, int64_t n, int depth, HostOctree* out,
                      bool want_arrays);

}  // namespace svlf
