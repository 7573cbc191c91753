/*
 * svlf.h -- C-ABI of the SVLF per-ray render library (libsvlf.so, gfx950).
 *
 * SVLF ("Sparse Voxel Light Field", RTMV paper arxiv 2205.07058, section 4)
 * renders a pixel by listing the occupied voxels of a sparse octree that its
 * ray crosses, decoding every crossed voxel once with a small network into an
 * optical thickness and a colour, and alpha compositing the results in order
 * along the ray (section 4.3, Eq. 3).  This library implements that per-ray
 * path with one decoder C -> H ... -> 4 (RGB + sigma) whose input is the
 * feature interpolated at the middle of the ray's segment in the voxel:
 *
 *   svlf_build_octree   sparse octree over occupied leaves (section 4.1)
 *   svlf_occupancy_from_depth  occupied leaves from depth maps (section 4.1)
 *   svlf_trace_hits     first K leaves crossed by each ray (sections 4.2-4.3)
 *   svlf_render         traversal + trilinear features + MLP + Eq. 3
 *   svlf_render_backward  gradients of rgb/depth/acc w.r.t. the features and
 *                       the MLP parameters (re-traces and recomputes)
 *   svlf_train_step     render + MSE/L1 loss + backward in one pass
 *   svlf_adam_step      Adam update of an FP32 parameter vector (section 4.5
 *                       trains with Adam)
 *   svlf_lazy_adam_step Adam restricted to the feature rows a batch touched
 *   svlf_lf_*           the same path with the paper's two-decoder light-field
 *                       function (ray parameterisation, tau and eta from the
 *                       entry / exit features, colour at the surface point)
 *
 * Conventions shared by every call
 * --------------------------------
 * Scene cube [-1,1]^3.  A leaf of an octree of depth L (1 <= L <= 10) is the
 * cell (i,j,k) of the 2^L grid, lo = -1 + (i,j,k) h, hi = lo + h, h = 2/2^L.
 * Leaf ids are ranks in ascending Morton order (bit b of i,j,k at bits 3b,
 * 3b+1, 3b+2).  Vertex ids are ranks of the Morton codes (L+1 bits per axis)
 * of all corners of occupied leaves; each vertex owns one feature row
 * (features are shared by adjacent voxels, section 4.1).  Corner j of a leaf
 * is the vertex (i + (j&1), j + ((j>>1)&1), k + (j>>2)).
 *
 * Hit predicate (the ray-AABB test of section 4.2, fixed here so hit lists
 * are reproducible bit for bit): binary32 round-to-nearest-even arithmetic,
 * no FMA contraction, no flush to zero; inv_a = 1/d_a; finite inv_a:
 * t0 = (lo_a-o_a)*inv_a, t1 = (hi_a-o_a)*inv_a, tn_a = min, tf_a = max;
 * infinite inv_a: the axis is unconstrained if lo_a <= o_a < hi_a (half-open)
 * and excludes the cell otherwise; t_in = max(tn) clamped below at +0,
 * t_out = min(tf); hit iff t_in < t_out.  Rays with a non-finite component
 * or d = 0 hit nothing.  A ray's hit list is its first K hit leaves in
 * ascending t_in (no ties can occur).
 *
 * Per hit: t_mid = (t_in+t_out)/2, p = o + t_mid d, u = clamp((p-lo)/h,0,1),
 * x = sum_j w_j(u) F[corner j] (trilinear, section 4.1).  MLP: hidden layers
 * ReLU; rgb = sigmoid(o_0..2); sigma = ReLU(o_3) (section 4.5).  Optical
 * thickness (section 4 footnote): tau = sigma*(t_out-t_in)/h (VOXEL mode),
 * sigma (DIRECT) or sigma*(t_out-t_in) (WORLD).  Eq. 3 over the first
 * min(N,K) hits: w_i = T_i (1 - e^{-tau_i}), T_i = prod_{j<i} e^{-tau_j};
 * rgb = sum w_i c_i, depth = sum w_i t_mid_i, acc = sum w_i; zero hits give 0.
 *
 * Memory and streams
 * ------------------
 * Every pointer documented "device" is device memory of the current HIP
 * device; "host" pointers are host memory.  All arrays are dense, row-major,
 * little-endian.  The caller owns every buffer and keeps it alive until the
 * work queued on `stream` (a hipStream_t, NULL = default stream) completes.
 * The library keeps no pointer after a call returns and holds no global
 * state besides the per-thread error string; calls are reentrant across
 * streams.  Calls are asynchronous with respect to the host unless stated.
 *
 * Errors
 * ------
 * Every call returns SVLF_OK (0) or a negative svlf_status.  Arguments are
 * validated on the host before anything is queued; a call that fails
 * validation writes nothing.  HIP launch failures return SVLF_E_HIP;
 * faults inside a kernel surface at the caller's next synchronisation.
 * svlf_last_error() returns a message for the last failing call on the
 * calling thread.  No C++ exception crosses this interface.
 */
#ifndef SVLF_H
#define SVLF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SVLF_OK = 0,
  SVLF_E_INVAL = -1,        /* NULL pointer, negative size, malformed input */
  SVLF_E_RANGE = -2,        /* value outside the supported range            */
  SVLF_E_WORKSPACE = -3,    /* workspace missing or too small               */
  SVLF_E_UNSUPPORTED = -4,  /* valid but not implemented (e.g. MLP shape)   */
  SVLF_E_HIP = -5           /* a HIP runtime call failed                    */
} svlf_status;

#define SVLF_MAX_DEPTH 10
#define SVLF_MAX_K 16
#define SVLF_MAX_SCENES 16
#define SVLF_MAX_LAYERS 8

/* One internal octree node (levels 0 .. depth-1), 8 bytes.
 * mask bit c (0..7) is set iff child c = x | y<<1 | z<<2 exists.
 * child: for a node at level < depth-1, the index in the node array of its
 * first existing child (children of a node are consecutive, in increasing
 * child index); for a node at level depth-1, the leaf id of its first leaf.
 * The node array is in level order: level 0 (the root, index 0), then every
 * level in ascending Morton order. */
typedef struct {
  int32_t child;
  uint32_t mask;
} svlf_node;

typedef struct {
  int32_t depth;
  int64_t n_leaves;
  int64_t n_vertices;
  int64_t n_nodes;                              /* internal nodes            */
  int64_t level_offset[SVLF_MAX_DEPTH + 1];     /* first node of level l;
                                                   level_offset[depth] = n_nodes */
} svlf_octree_sizes;

/* A built octree (device arrays owned by the caller). */
typedef struct {
  int32_t depth;
  int64_t n_leaves;
  int64_t n_vertices;
  int64_t n_nodes;
  const svlf_node* nodes;        /* device [n_nodes]                         */
  const int32_t* leaf_corners;   /* device [n_leaves][8] vertex ids          */
} svlf_octree;

/* A scene = octree + per-vertex features (section 4.1: one learnable
 * embedding per octree vertex). */
typedef struct {
  svlf_octree octree;
  const float* features;         /* device [n_vertices][C] FP32 (masters)     */
  const uint16_t* features_bf16; /* device [n_vertices][C] bfloat16 bits, RNE
                                    of `features`; required for BF16 precision,
                                    may be NULL for FP32                     */
} svlf_scene;

/* The decoder.  widths[0] = C, widths[n_layers] = 4, hidden layers ReLU.
 * params: device FP32, per layer W[out][in] row-major then b[out], layers
 * concatenated (n = sum out*in + out).  Supported shapes (C, hidden width,
 * hidden layers): (8, 32, 2), (16, 64, 3), (32, 64, 3); other shapes return
 * SVLF_E_UNSUPPORTED from the render calls. */
typedef struct {
  int32_t n_layers;
  int32_t widths[SVLF_MAX_LAYERS + 1];
  const float* params;
} svlf_mlp;

typedef enum { SVLF_TAU_VOXEL = 0, SVLF_TAU_DIRECT = 1, SVLF_TAU_WORLD = 2 } svlf_tau_mode;
typedef enum { SVLF_FP32 = 0, SVLF_BF16 = 1 } svlf_precision;

typedef struct {
  int32_t K;                     /* hit cap per ray, 1..SVLF_MAX_K           */
  int32_t tau_mode;              /* svlf_tau_mode                            */
  int32_t precision;             /* svlf_precision: MLP operand type; BF16
                                    rounds features, weights, the MLP input
                                    and hidden activations to bfloat16 (RNE)
                                    with FP32 accumulation; traversal, slabs,
                                    interpolation weights, compositing and
                                    gradient accumulation stay FP32          */
  int32_t flags;                 /* 0, or SVLF_FLAG_* bits                   */
} svlf_render_opts;

/* svlf_render_opts.flags.  SVLF_FLAG_TRACE_ONLY runs only the traversal,
 * leaving the hit slots and counts in the workspace; SVLF_FLAG_REUSE_HITS
 * skips the traversal and shades the hits left in the workspace by an
 * earlier call with the same scenes, rays, ray_offsets and K (the caller
 * guarantees this; nothing is checked).  Together they split one call into
 * its two kernels, e.g. to reuse one traversal for several evaluations. */
#define SVLF_FLAG_TRACE_ONLY 1
#define SVLF_FLAG_REUSE_HITS 2
/* SVLF_FLAG_VIEWDIR: the decoder input is the interpolated feature followed
 * by the ray direction d as given (3 values), [psi(p; Z) | d], so that
 * colour and density may depend on the viewing direction: the input the
 * paper proposes for view-dependent appearance (section 6, limitations).
 * mlp->widths[0] is then C + 3 (C = features per vertex); supported
 * decoders 11-32-32-4 and 35-64-64-64-4.  The direction takes no gradient;
 * grad_features keep C columns. */
#define SVLF_FLAG_VIEWDIR 4
/* SVLF_FLAG_DETERMINISTIC (svlf_render_backward, svlf_train_step; one scene):
 * the feature gradient is reduced in a fixed order instead of with FP32
 * atomics, and every work item stays on a fixed block, so repeated calls on
 * the same inputs give bit-identical feature and decoder gradients and
 * loss.  The backward keeps (u, dL/dx) per hit; the hits are sorted by leaf
 * (stable, each leaf's hits in ascending hit-slot order) and every vertex
 * sums over its up to 8 adjacent leaves in a fixed order.  The workspace
 * must then come from svlf_workspace_bytes_scenes.  Without the flag the
 * feature gradient takes FP32 atomics and the last work items go to
 * whichever block is free, so both gradients and the loss may differ in
 * their last bits between calls. */
#define SVLF_FLAG_DETERMINISTIC 8

/* ---------------------------------------------------------------- octree */

/* Sizes of the octree over `n` occupied leaves (host int32 [n][3], any
 * order, unique, 0 <= coord < 2^depth).  Host-only, synchronous.
 * Section 4.1 ("Scene volume"). */
int svlf_build_octree_sizes(const int32_t* leaf_ijk_host, int64_t n, int32_t depth,
                            svlf_octree_sizes* out);

/* Workspace bytes of svlf_occupancy_from_depth at grid level `level`
 * (1..10): a bitmap of 8^level bits and per-block counts (0 if out of
 * range). */
size_t svlf_occupancy_workspace_bytes(int32_t level);

/* Occupied leaves from depth maps (section 4.1: the octree keeps the voxels
 * that contain a surface, found from the depth the dataset provides).  For
 * every ray r with a finite target depth t[r] > 0 the surface point
 * p = o + t d is computed in binary32 (rounded product, then rounded sum,
 * no fused multiply-add) and its leaf at `level` is
 * floor(RN(p + 1) * 2^(level-1)) per axis; points outside the grid are
 * dropped.  ray_o, ray_d: device FP32 [n][3]; target_depth: device FP32 [n].
 * leaf_ijk_out: device int32 [n][3] (capacity n; a ray marks at most one
 * leaf) receives the unique leaves in ascending Morton order (leaf-id
 * order), n_leaves_out (device int64) their number.  Feed the leaves to
 * svlf_build_octree (host copy).  Asynchronous on `stream`. */
int svlf_occupancy_from_depth(const float* ray_o, const float* ray_d, const float* target_depth,
                              int64_t n, int32_t level, int32_t* leaf_ijk_out,
                              int64_t* n_leaves_out, void* workspace, size_t ws_bytes,
                              void* stream);

/* Builds the octree on the host and copies it to the device arrays
 * nodes_dev (n_nodes entries) and leaf_corners_dev (n_leaves*8 entries), sized
 * by svlf_build_octree_sizes.  leaf_ijk_sorted_host (nullable, host int32
 * [n][3]) receives the leaves in leaf-id order.  Synchronous: returns after
 * the copies on `stream` complete.  Section 4.1. */
int svlf_build_octree(const int32_t* leaf_ijk_host, int64_t n, int32_t depth,
                      svlf_node* nodes_dev, int32_t* leaf_corners_dev,
                      int32_t* leaf_ijk_sorted_host, void* stream);

/* Same build, host outputs only: nodes_host (n_nodes entries),
 * leaf_corners_host (n_leaves*8 entries), leaf_ijk_sorted_host (nullable,
 * n_leaves*3 entries).  Host-only, synchronous, no HIP call.  Section 4.1. */
int svlf_build_octree_host(const int32_t* leaf_ijk_host, int64_t n, int32_t depth,
                           svlf_node* nodes_host, int32_t* leaf_corners_host,
                           int32_t* leaf_ijk_sorted_host);

/* ---------------------------------------------------------------- trace */

/* First K hit leaves of each ray (sections 4.2-4.3).  ray_o, ray_d: device
 * FP32 [n_rays][3].  Outputs (device): hit_leaf int32 [n_rays][K] (-1 padded),
 * hit_tin / hit_tout FP32 [n_rays][K] (0 padded), hit_count int32 [n_rays]. */
int svlf_trace_hits(const svlf_octree* oct, const float* ray_o, const float* ray_d,
                    int64_t n_rays, int32_t K, int32_t* hit_leaf, float* hit_tin,
                    float* hit_tout, int32_t* hit_count, void* stream);

/* ---------------------------------------------------------------- render */

/* Workspace bytes needed by svlf_render / svlf_render_backward /
 * svlf_train_step for n_rays rays (all scenes together) with this MLP and
 * these options: per-ray hit slots (16 bytes x K), per-ray hit counts and
 * per-block partial sums of the MLP gradient.  Returns 0 on invalid
 * arguments (see svlf_last_error).  The workspace is device memory owned by
 * the caller, needs no initialisation, and may not be shared by calls that
 * run concurrently. */
size_t svlf_workspace_bytes(const svlf_mlp* mlp, const svlf_render_opts* opts, int64_t n_rays);

/* Forward render of rays grouped by scene (section 4.3, Eq. 3).  Scenes
 * 0..n_scenes-1 (1 <= n_scenes <= SVLF_MAX_SCENES) share the MLP and C; the
 * rays of scene s are rows ray_offsets_host[s] .. ray_offsets_host[s+1]-1 of
 * ray_o / ray_d (device FP32 [n][3], n = ray_offsets_host[n_scenes]).
 * Outputs (device FP32): out_rgb [n][3], out_depth [n], out_acc [n] (nullable).
 * All scenes are rendered by one persistent kernel launch. */
int svlf_render(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                const svlf_mlp* mlp, const svlf_render_opts* opts,
                const float* ray_o, const float* ray_d,
                float* out_rgb, float* out_depth, float* out_acc,
                void* workspace, size_t ws_bytes, void* stream);

/* Backward of svlf_render for upstream gradients grad_rgb [n][3],
 * grad_depth [n] and grad_acc [n] (device FP32; grad_acc nullable = 0).
 * Re-traces every ray and recomputes the forward activations.
 * ACCUMULATES into grad_features[s] (device FP32 [n_vertices_s][C], one per
 * scene, with FP32 atomics: order-dependent rounding) and grad_params
 * (device FP32, layout of svlf_mlp.params, reduced deterministically). */
int svlf_render_backward(const svlf_scene* scenes, int32_t n_scenes,
                         const int64_t* ray_offsets_host, const svlf_mlp* mlp,
                         const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                         const float* grad_rgb, const float* grad_depth, const float* grad_acc,
                         float* const* grad_features, float* grad_params,
                         void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes for calls over these scenes (the scene sizes matter with
 * SVLF_FLAG_DETERMINISTIC; otherwise equal to svlf_workspace_bytes).
 * 0 on invalid arguments. */
size_t svlf_workspace_bytes_scenes(const svlf_mlp* mlp, const svlf_render_opts* opts,
                                   const svlf_scene* scenes, int32_t n_scenes, int64_t n_rays);

/* One fused training pass: render, loss
 *   L = sum over rays of ( |rgb - rgb*|^2 / 3 + lambda_depth |depth - depth*| ) * loss_scale
 * (loss_scale = 1/n gives the mean MSE over channels + lambda times the mean
 * L1 of depth; sign(0) = 0), and its backward, as svlf_render_backward with
 * the loss gradient as upstream gradient.  target_rgb [n][3], target_depth [n]
 * (device FP32).  out_rgb / out_depth (nullable) receive the render.
 * loss_out (device FP32 scalar, nullable) is overwritten with L. */
int svlf_train_step(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                    const svlf_mlp* mlp, const svlf_render_opts* opts,
                    const float* ray_o, const float* ray_d,
                    const float* target_rgb, const float* target_depth,
                    float lambda_depth, float loss_scale,
                    float* out_rgb, float* out_depth, float* loss_out,
                    float* const* grad_features, float* grad_params,
                    void* workspace, size_t ws_bytes, void* stream);

/* Size of the device scratch array that svlf_train_step_noalloc uses in
 * place of a workspace (one array per device, held until the process ends). */
#define SVLF_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* svlf_train_step for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same pass, arguments and results as svlf_train_step without the
 * workspace: the per-ray hit slots and counts and the per-block partial sums
 * live in a library-owned file-scope device array of
 * SVLF_NOALLOC_SCRATCH_BYTES (its address is looked up once per device, on
 * the first call with that device current).  Nothing is allocated or freed.
 * A call whose workspace (svlf_workspace_bytes_scenes for the same arguments)
 * exceeds SVLF_NOALLOC_SCRATCH_BYTES fails with SVLF_E_WORKSPACE before
 * anything is queued (with K = 8 and the 32-64-64-64-4 decoder about 1.7M
 * rays fit).  The array needs no initialisation; every call on a device
 * uses the same array, so calls that overlap on one device (other streams,
 * other host threads) race and must be serialised by the caller. */
int svlf_train_step_noalloc(const svlf_scene* scenes, int32_t n_scenes,
                            const int64_t* ray_offsets_host, const svlf_mlp* mlp,
                            const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                            const float* target_rgb, const float* target_depth,
                            float lambda_depth, float loss_scale, float* out_rgb, float* out_depth,
                            float* loss_out, float* const* grad_features, float* grad_params,
                            void* stream);

/* ---------------------------------------------------------------- light field */

/* The paper's voxel light-field function (section 4.2, Eq. 1-2) in place of
 * the single decoder: for every crossed voxel (entry point x1 = o + t_in d,
 * exit point x2 = o + t_out d),
 *   r      = the two points where the ray meets the voxel's bounding sphere
 *            (centre lo + h/2, radius h sqrt(3)/2), as unit vectors from the
 *            centre, in order along the ray (6 values; section 4.1);
 *   (tau, eta) from the density decoder F_T on [psi(x1; Z_T) | psi(x2; Z_T) | r]
 *            (2 C_T + 6 inputs): tau = ReLU(o_0) (scaled by dt/h or dt in the
 *            VOXEL / WORLD tau modes; DIRECT is the paper's form), eta =
 *            sigmoid(o_1);
 *   x_s    = eta x1 + (1 - eta) x2, t_s = eta t_in + (1 - eta) t_out;
 *   c      = sigmoid of the colour decoder F_C on [psi(x_s; Z_C) | r]
 *            (C_C + 6 inputs, + 3 for the ray direction d with
 *            SVLF_FLAG_VIEWDIR);
 * composited with Eq. 3 (depth = sum w_i t_s,i).  psi is the trilinear
 * interpolation of the voxel's corner embeddings with u clamped to [0,1].
 * Features: one table per scene holding the two collections as blocks, Z_T
 * [n_vertices][C_T] followed by Z_C [n_vertices][C_C] (FP32; features_bf16
 * the same layout in BF16 for the BF16 precision); grad_features likewise.
 * params: FP32, F_T's layers then F_C's, each W[out][in] then b[out]
 * (svlf_lf_param_count()).  Supported: C_T = 64, C_C = 32, hidden width
 * 128, one hidden layer in F_T and three in F_C (the paper's sizes, section
 * 4.5).  Hidden layers ReLU; BF16 rounds features, weights, both decoders'
 * inputs and hidden activations (and each layer's dL/dz in the backward). */
typedef struct {
  int32_t c_density;          /* C_T: 64                                     */
  int32_t c_color;            /* C_C: 32                                     */
  int32_t hidden;             /* 128                                         */
  int32_t n_hidden_density;   /* 1                                           */
  int32_t n_hidden_color;     /* 3                                           */
  const float* params;        /* device FP32 [svlf_lf_param_count()]         */
} svlf_lf_model;

/* Number of parameters of the model (with opts->flags' SVLF_FLAG_VIEWDIR),
 * or 0 with the error set if the model is unsupported. */
int64_t svlf_lf_param_count(const svlf_lf_model* model, const svlf_render_opts* opts);

/* Workspace bytes for n_rays rays, enough for every light-field call (0 on
 * invalid arguments).  With BF16 precision, calls that run a backward pass
 * (svlf_lf_render_backward, svlf_lf_train_step, svlf_lf_train_stage) keep
 * the density decoder's input row of every hit slot in it (n_rays * K * 288
 * bytes) instead of gathering the features a second time. */
size_t svlf_lf_workspace_bytes(const svlf_lf_model* model, const svlf_render_opts* opts,
                               int64_t n_rays);

/* Workspace bytes sufficient for svlf_lf_render alone (forward only); never
 * larger than svlf_lf_workspace_bytes. */
size_t svlf_lf_render_workspace_bytes(const svlf_lf_model* model, const svlf_render_opts* opts,
                                      int64_t n_rays);

/* Forward render with the light-field function; arguments as svlf_render. */
int svlf_lf_render(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                   const svlf_lf_model* model, const svlf_render_opts* opts,
                   const float* ray_o, const float* ray_d,
                   float* out_rgb, float* out_depth, float* out_acc,
                   void* workspace, size_t ws_bytes, void* stream);

/* Backward of svlf_lf_render (re-traces and recomputes); gradients are
 * ADDED to grad_features[s] (the features' layout, FP32 atomics)
 * and grad_params (FP32 [svlf_lf_param_count()]); arguments otherwise as
 * svlf_render_backward.  The gradient reaches eta through t_s and through
 * the interpolation at x_s (the clamp of the cell coordinates passes it
 * where the unclamped coordinate is in [0, 1]). */
int svlf_lf_render_backward(const svlf_scene* scenes, int32_t n_scenes,
                            const int64_t* ray_offsets_host, const svlf_lf_model* model,
                            const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                            const float* grad_rgb, const float* grad_depth, const float* grad_acc,
                            float* const* grad_features, float* grad_params,
                            void* workspace, size_t ws_bytes, void* stream);

/* Render + the loss of svlf_train_step + backward, with the light-field
 * function; arguments as svlf_train_step. */
int svlf_lf_train_step(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                       const svlf_lf_model* model, const svlf_render_opts* opts,
                       const float* ray_o, const float* ray_d,
                       const float* target_rgb, const float* target_depth,
                       float lambda_depth, float loss_scale,
                       float* out_rgb, float* out_depth, float* loss_out,
                       float* const* grad_features, float* grad_params,
                       void* workspace, size_t ws_bytes, void* stream);

/* The paper's staged training loss (section 4.4, Eq. 4) for the light-field
 * function.  Per ray with target colour c* and target depth t* (same units
 * as depth), the surface voxel is the hit whose [t_in, t_out) holds t*
 * (none if no hit does); its within-voxel depth target is
 * eta* = (t_out - t*) / (t_out - t_in), the eta that places x_s on the
 * target surface point.  With e_v = e^{-tau_v} of the surface voxel:
 *   SVLF_LF_LOSS_SURFACE (voxel training):
 *     L = loss_scale * sum over rays with a surface voxel v of
 *         ( |c_v - c*|^2 + lambda_eta (eta_v - eta*)^2 + lambda_tau e_v^2 )
 *   SVLF_LF_LOSS_VOLUME (volumetric training and fine-tuning):
 *     L = loss_scale * sum over rays of ( |c(r) - c*|^2
 *         + [surface voxel v] (lambda_eta (eta_v - eta*)^2 + lambda_tau e_v^2) )
 *     with c(r) the composited colour (Eq. 3); the paper sets lambda_tau = 0.
 * freeze_color != 0 leaves the colour embeddings Z_C and the colour decoder
 * without gradient (the volumetric stage trains the density side only);
 * the gradient still flows through them to eta. */
typedef enum { SVLF_LF_LOSS_SURFACE = 1, SVLF_LF_LOSS_VOLUME = 2 } svlf_lf_loss_kind;
typedef struct {
  int32_t kind;          /* svlf_lf_loss_kind                                */
  float lambda_eta;      /* >= 0                                             */
  float lambda_tau;      /* >= 0                                             */
  float loss_scale;      /* e.g. 1 / n_rays                                   */
  int32_t freeze_color;  /* nonzero: no gradients for Z_C and F_C            */
} svlf_lf_loss;

/* One training pass with a staged loss: render (out_rgb / out_depth
 * nullable), the loss (loss_out nullable, overwritten) and its gradients,
 * ADDED to grad_features and grad_params as in svlf_lf_train_step. */
int svlf_lf_train_stage(const svlf_scene* scenes, int32_t n_scenes,
                        const int64_t* ray_offsets_host, const svlf_lf_model* model,
                        const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                        const float* target_rgb, const float* target_depth,
                        const svlf_lf_loss* loss, float* out_rgb, float* out_depth,
                        float* loss_out, float* const* grad_features, float* grad_params,
                        void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- training utilities */

/* Adam (Kingma & Ba; the optimiser of section 4.5) on n FP32 parameters:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).  All device FP32
 * [n].  If bf16_out (device uint16 [n], nullable) is given, it receives the
 * RNE bfloat16 bits of the updated p.  If zero_grad != 0, grad is set to 0
 * after it is read.  step_t >= 1. */
int svlf_adam_step(float* param, float* grad, float* m, float* v, int64_t n,
                   float lr, float beta1, float beta2, float eps, int64_t step_t,
                   uint16_t* bf16_out, int32_t zero_grad, void* stream);

/* Lazy (row-sparse) Adam over a table of n_rows rows of row_len FP32
 * entries (e.g. the per-vertex feature rows): a row takes the Adam update of
 * svlf_adam_step, with bias corrections from the global step_t, only if its
 * gradient row holds a nonzero entry; the parameters and both moments of any
 * other row are left as they are.  This is the update of rows touched by the
 * batch only (the dense optimiser's cost over an untouched row is what it
 * saves; a row that no ray reached does not decay its moments).  The same
 * bf16_out / zero_grad semantics as svlf_adam_step, applied to updated rows
 * (untouched rows keep an all-zero gradient).  row_len: a multiple of 4 in
 * [4, 256]; all arrays device, 16-byte aligned ([n_rows][row_len], bf16_out
 * 8-byte aligned).  Errors: E_INVAL (NULL, misaligned, n_rows < 0),
 * E_RANGE (hyper-parameters, step_t < 1), E_UNSUPPORTED (row_len). */
int svlf_lazy_adam_step(float* param, float* grad, float* m, float* v, int64_t n_rows,
                        int32_t row_len, float lr, float beta1, float beta2, float eps,
                        int64_t step_t, uint16_t* bf16_out, int32_t zero_grad, void* stream);

/* dst[i] = RNE bfloat16 bits of src[i] (device, n elements). */
int svlf_to_bf16(const float* src, uint16_t* dst, int64_t n, void* stream);

/* dst[i] = value (device FP32, n elements); a kernel, never a memset node. */
int svlf_fill(float* dst, float value, int64_t n, void* stream);

/* ---------------------------------------------------------------- diagnostics */

/* Evaluates the decoder alone on X (device FP32 [n][widths[0]]: C features,
 * plus the 3 direction values with SVLF_FLAG_VIEWDIR) with the precision
 * of opts, writing the 4 raw outputs (before sigmoid/ReLU) to out (device
 * FP32 [n][4]).  Exposes the MLP of the render kernels for testing. */
int svlf_mlp_forward(const svlf_mlp* mlp, const svlf_render_opts* opts, const float* X,
                     int64_t n, float* out, void* stream);

/* Message for the last failing call on this thread ("" if none). */
const char* svlf_last_error(void);

/* Library version string. */
const char* svlf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SVLF_H */
