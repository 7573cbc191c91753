// C-ABI entry points of libsvlf: argument validation, error reporting and
// launch set-up.  All device work is queued on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "svlf_internal.hpp"

namespace svlf {
namespace {
thread_local std::string g_error;
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }
const char* error_cstr() { return g_error.c_str(); }

}  // namespace svlf

using namespace svlf;

namespace {

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(SVLF_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

std::string who_str(const char* who, const char* what) { return std::string(who) + ": " + what; }

int check_octree(const svlf_octree* oct, const char* who) {
  if (oct == nullptr) return fail(SVLF_E_INVAL, who_str(who, "octree is NULL"));
  if (oct->depth < 1 || oct->depth > SVLF_MAX_DEPTH)
    return fail(SVLF_E_RANGE, who_str(who, "octree depth must be in [1, 10]"));
  if (oct->n_leaves < 0 || oct->n_nodes < 0 || oct->n_vertices < 0)
    return fail(SVLF_E_INVAL, who_str(who, "negative octree size"));
  if (oct->n_leaves > 0 &&
      (oct->nodes == nullptr || oct->leaf_corners == nullptr || oct->n_nodes < 1))
    return fail(SVLF_E_INVAL, who_str(who, "octree arrays are NULL"));
  return SVLF_OK;
}

struct MlpShape {
  int C, H, n_hidden;
  int64_t n_params;
};

// The decoder input is the C interpolated features, followed by the ray
// direction (3 values) when `viewdir` is set.
int check_mlp(const svlf_mlp* mlp, bool viewdir, MlpShape* sh, const char* who) {
  if (mlp == nullptr || mlp->params == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "mlp or mlp->params is NULL"));
  const int L = mlp->n_layers;
  if (L < 2 || L > SVLF_MAX_LAYERS)
    return fail(SVLF_E_UNSUPPORTED, who_str(who, "n_layers must be in [2, 5]"));
  int64_t np = 0;
  for (int l = 0; l < L; ++l) {
    if (mlp->widths[l] < 1 || mlp->widths[l + 1] < 1)
      return fail(SVLF_E_INVAL, who_str(who, "non-positive layer width"));
    np += static_cast<int64_t>(mlp->widths[l]) * mlp->widths[l + 1] + mlp->widths[l + 1];
  }
  const int c = mlp->widths[0] - (viewdir ? 3 : 0), h = mlp->widths[1];
  if (mlp->widths[L] != 4)
    return fail(SVLF_E_INVAL, who_str(who, "the last layer must have 4 outputs (RGB, sigma)"));
  if (c != 8 && c != 16 && c != 32)
    return fail(SVLF_E_UNSUPPORTED,
                who_str(who, viewdir ? "widths[0] must be C + 3 with C = 8, 16 or 32"
                                     : "C must be 8, 16 or 32"));
  if (h != 32 && h != 64)
    return fail(SVLF_E_UNSUPPORTED, who_str(who, "hidden width must be 32 or 64"));
  for (int l = 1; l < L; ++l)
    if (mlp->widths[l] != h)
      return fail(SVLF_E_UNSUPPORTED, who_str(who, "hidden layers must have equal widths"));
  if (L - 1 > 4) return fail(SVLF_E_UNSUPPORTED, who_str(who, "at most 4 hidden layers"));
  if (viewdir && !((c == 8 && h == 32 && L == 3) || (c == 32 && h == 64 && L == 4)))
    return fail(SVLF_E_UNSUPPORTED,
                who_str(who, "view-direction input: decoders 11-32-32-4 and 35-64-64-64-4 only"));
  sh->C = c;
  sh->H = h;
  sh->n_hidden = L - 1;
  sh->n_params = np;
  return SVLF_OK;
}

int check_opts(const svlf_render_opts* opts, const char* who) {
  if (opts == nullptr) return fail(SVLF_E_INVAL, who_str(who, "opts is NULL"));
  if (opts->K < 1 || opts->K > SVLF_MAX_K)
    return fail(SVLF_E_RANGE, who_str(who, "K must be in [1, 16]"));
  if (opts->tau_mode < 0 || opts->tau_mode > 2)
    return fail(SVLF_E_RANGE, who_str(who, "unknown tau_mode"));
  if (opts->precision != SVLF_FP32 && opts->precision != SVLF_BF16)
    return fail(SVLF_E_RANGE, who_str(who, "unknown precision"));
  if (opts->flags &
      ~(SVLF_FLAG_TRACE_ONLY | SVLF_FLAG_REUSE_HITS | SVLF_FLAG_VIEWDIR | SVLF_FLAG_DETERMINISTIC))
    return fail(SVLF_E_INVAL, who_str(who, "unknown flags"));
  if ((opts->flags & SVLF_FLAG_TRACE_ONLY) && (opts->flags & SVLF_FLAG_REUSE_HITS))
    return fail(SVLF_E_INVAL, who_str(who, "TRACE_ONLY and REUSE_HITS exclude each other"));
  return SVLF_OK;
}

// Validates the scene list and builds the kernels' scene table.
int make_table(const svlf_scene* scenes, int n_scenes, const int64_t* offs, bool bf16,
               float* const* grads, bool need_grads, SceneTable* tab, const char* who) {
  if (scenes == nullptr) return fail(SVLF_E_INVAL, who_str(who, "scenes is NULL"));
  if (n_scenes < 1 || n_scenes > SVLF_MAX_SCENES)
    return fail(SVLF_E_RANGE, who_str(who, "n_scenes must be in [1, 16]"));
  if (offs == nullptr) return fail(SVLF_E_INVAL, who_str(who, "ray_offsets is NULL"));
  if (offs[0] != 0) return fail(SVLF_E_INVAL, who_str(who, "ray_offsets[0] must be 0"));
  if (need_grads && grads == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "grad_features is NULL"));
  std::memset(tab, 0, sizeof(*tab));
  tab->n = n_scenes;
  int64_t blocks = 0;
  for (int s = 0; s < n_scenes; ++s) {
    const svlf_scene& sc = scenes[s];
    int rc = check_octree(&sc.octree, who);
    if (rc) return rc;
    if (offs[s + 1] < offs[s])
      return fail(SVLF_E_INVAL, who_str(who, "ray_offsets must be non-decreasing"));
    const bool empty = sc.octree.n_leaves == 0;
    if (!empty) {
      if (sc.features == nullptr) return fail(SVLF_E_INVAL, who_str(who, "features is NULL"));
      if (bf16 && sc.features_bf16 == nullptr)
        return fail(SVLF_E_INVAL, who_str(who, "BF16 precision needs features_bf16"));
      if (need_grads && grads[s] == nullptr)
        return fail(SVLF_E_INVAL, who_str(who, "grad_features[s] is NULL"));
    }
    DevScene& d = tab->s[s];
    d.nodes = empty ? nullptr : sc.octree.nodes;
    d.leaf_corners = sc.octree.leaf_corners;
    d.feat32 = sc.features;
    d.feat16 = sc.features_bf16;
    d.grad = need_grads ? grads[s] : nullptr;
    d.n_vertices = sc.octree.n_vertices;
    d.ray_begin = offs[s];
    d.ray_end = offs[s + 1];
    d.depth = sc.octree.depth;
    d.block_begin = static_cast<int32_t>(blocks);
    blocks += (offs[s + 1] - offs[s] + kRaysPerBlock - 1) / kRaysPerBlock;
  }
  if (blocks > (int64_t(1) << 30))
    return fail(SVLF_E_RANGE, who_str(who, "too many rays"));
  tab->n_blocks = static_cast<int32_t>(blocks);
  return SVLF_OK;
}

// A roctx range over one library call, named after its entry point:
// `rocprofv3 --marker-trace` shows it around the call's kernels (without a
// tracer attached the calls do nothing).
struct CallRange {
  explicit CallRange(const char* name) { roctxRangePush(name); }
  ~CallRange() { roctxRangePop(); }
  CallRange(const CallRange&) = delete;
  CallRange& operator=(const CallRange&) = delete;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace: [hit slots n*K][counts n][per-block dW partials][per-block loss]
// [work-item counter]
struct WsLayout {
  size_t hits, cnt, partials, loss, counter, total;
};

WsLayout ws_layout(int64_t n_rays, int K, int64_t n_params) {
  WsLayout w;
  size_t off = 0;
  w.hits = off;
  off = align256(off + static_cast<size_t>(n_rays) * K * sizeof(HitRec));
  w.cnt = off;
  off = align256(off + static_cast<size_t>(n_rays) * sizeof(int32_t));
  w.partials = off;
  off = align256(off + static_cast<size_t>(shade_grid_limit()) * n_params * sizeof(float));
  w.loss = off;
  off = align256(off + static_cast<size_t>(shade_grid_limit()) * sizeof(float));
  w.counter = off;
  off = align256(off + sizeof(int32_t));
  w.total = off;
  return w;
}

// Deterministic mode: [per-hit (u, dL/dx) records][reduction scratch] after
// the standard layout.
struct DetExtra {
  size_t gxu, scratch, total;
};

DetExtra det_extra(size_t base_total, int64_t n, int K, int C, const svlf_scene& sc) {
  DetExtra d;
  d.gxu = align256(base_total);
  d.scratch = align256(d.gxu + static_cast<size_t>(n) * K * (C + 4) * sizeof(float));
  d.total = align256(d.scratch + detgrad_bytes(n, K, C, sc.octree.n_leaves, sc.octree.n_vertices));
  return d;
}

// The library's side stream on the current device (default priority,
// non-blocking) with the two events of a fork / join, created on first use
// and kept until the process ends.  The returned lock serialises the
// fork-join sequences of concurrent calls.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

hipError_t side_stream(SideStream** out, std::unique_lock<std::mutex>* lock) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static SideStream per[kMaxDevices];
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::unique_lock<std::mutex> l(mu);
  SideStream& ss = per[dev];
  if (ss.stream == nullptr) {
    hipStream_t st = nullptr;
    hipEvent_t f = nullptr, j = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    ss.stream = st;
    ss.fork = f;
    ss.join = j;
  }
  *out = &ss;
  *lock = std::move(l);
  return hipSuccess;
}

// Shared body of render / render_backward / train_step.
// noalloc: no workspace argument; the library's per-device scratch array
// (svlf_train_step_noalloc) holds the workspace if it is large enough.
int run_shade(int mode, const svlf_scene* scenes, int32_t n_scenes, const int64_t* offs,
              const svlf_mlp* mlp, const svlf_render_opts* opts, const float* ray_o,
              const float* ray_d, ShadeArgs a, float* const* grad_features, void* ws,
              size_t ws_bytes, void* stream, const char* who, bool noalloc = false) {
  int rc = check_opts(opts, who);
  if (rc) return rc;
  MlpShape sh;
  rc = check_mlp(mlp, (opts->flags & SVLF_FLAG_VIEWDIR) != 0, &sh, who);
  if (rc) return rc;
  const bool need_grads = mode != kForward;
  rc = make_table(scenes, n_scenes, offs, opts->precision == SVLF_BF16, grad_features, need_grads,
                  &a.tab, who);
  if (rc) return rc;
  const int64_t n = offs[n_scenes];
  if (n > 0 && (ray_o == nullptr || ray_d == nullptr))
    return fail(SVLF_E_INVAL, who_str(who, "ray_o / ray_d is NULL"));
  const WsLayout w = ws_layout(n, opts->K, sh.n_params);
  const bool det = (opts->flags & SVLF_FLAG_DETERMINISTIC) != 0 && mode != kForward;
  if (det && n_scenes != 1)
    return fail(SVLF_E_UNSUPPORTED, who_str(who, "SVLF_FLAG_DETERMINISTIC supports one scene"));
  if (det && n * opts->K >= (int64_t(1) << 31))
    return fail(SVLF_E_RANGE, who_str(who, "too many hit slots for SVLF_FLAG_DETERMINISTIC"));
  const DetExtra dx = det ? det_extra(w.total, n, opts->K, sh.C, scenes[0]) : DetExtra{0, 0, w.total};
  if (noalloc) {
    if (dx.total > SVLF_NOALLOC_SCRATCH_BYTES)
      return fail(SVLF_E_WORKSPACE,
                  who_str(who, "the call's workspace (svlf_workspace_bytes_scenes) exceeds "
                               "SVLF_NOALLOC_SCRATCH_BYTES"));
    if (n == 0) return SVLF_OK;
    const hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess) return hip_fail(e, who);
    ws_bytes = SVLF_NOALLOC_SCRATCH_BYTES;
  } else if (ws == nullptr || ws_bytes < dx.total) {
    return fail(SVLF_E_WORKSPACE, who_str(who, det ? "workspace smaller than svlf_workspace_bytes_scenes()"
                                                   : "workspace missing or smaller than svlf_workspace_bytes()"));
  }
  if (n == 0) return SVLF_OK;
  char* base = static_cast<char*>(ws);
  a.gxu = det ? reinterpret_cast<float*>(base + dx.gxu) : nullptr;
  a.o = ray_o;
  a.d = ray_d;
  a.hits = reinterpret_cast<HitRec*>(base + w.hits);
  a.cnt = reinterpret_cast<int32_t*>(base + w.cnt);
  a.ws_partials = reinterpret_cast<float*>(base + w.partials);
  a.ws_loss = reinterpret_cast<float*>(base + w.loss);
  // deterministic mode keeps every item on a fixed block (fixed-order decoder-gradient partials)
  a.item_counter = det ? nullptr : reinterpret_cast<int32_t*>(base + w.counter);
  a.K = opts->K;
  a.tau_mode = opts->tau_mode;
  a.precision = opts->precision;
  a.C = sh.C;
  a.H = sh.H;
  a.n_hidden = sh.n_hidden;
  a.viewdir = (opts->flags & SVLF_FLAG_VIEWDIR) ? 1 : 0;
  a.params = mlp->params;
  a.n_params = sh.n_params;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (!(opts->flags & SVLF_FLAG_REUSE_HITS)) {
    e = launch_trace_internal(a.tab, ray_o, ray_d, opts->K, const_cast<HitRec*>(a.hits),
                              const_cast<int32_t*>(a.cnt), s);
    if (e != hipSuccess) return hip_fail(e, who);
  }
  if (opts->flags & SVLF_FLAG_TRACE_ONLY) return SVLF_OK;
  const int64_t n_leaves = scenes[0].octree.n_leaves, n_vertices = scenes[0].octree.n_vertices;
  void* det_scratch = base + dx.scratch;
  // Deterministic mode: the ordering of the hits needs only the hit lists,
  // so it runs on the library's side stream while the shading kernel runs
  // (fork after the traversal, join before the per-vertex sum); calls
  // without a workspace argument keep everything on the caller's stream.
  std::unique_lock<std::mutex> fork_lock;
  SideStream* side = nullptr;
  if (det && !noalloc) {
    e = side_stream(&side, &fork_lock);
    if (e != hipSuccess) return hip_fail(e, who);
    e = hipEventRecord(side->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side->stream, side->fork, 0);
    if (e == hipSuccess)
      e = launch_detgrad_order(a.tab.s[0], a.hits, a.cnt, n, opts->K, sh.C, det_scratch, n_leaves,
                               n_vertices, side->stream);
    if (e == hipSuccess) e = hipEventRecord(side->join, side->stream);
    if (e != hipSuccess) return hip_fail(e, who);
  }
  int grid = 0;
  if (a.item_counter != nullptr)
    e = launch_fill(reinterpret_cast<float*>(a.item_counter), 0.0f, 1, s);   // 0.0f has zero bits
  if (e == hipSuccess) e = launch_shade(a, mode, s, &grid);
  if (e == hipSuccess && mode != kForward)
    e = launch_reduce_partials(a.ws_partials, grid, sh.n_params, a.grad_params, a.ws_loss,
                               mode == kTrain ? a.loss_out : nullptr, s);
  if (e != hipSuccess) {
    if (side) hipStreamWaitEvent(s, side->join, 0);     // join the fork on every path
    if (e == hipErrorNotSupported)
      return fail(SVLF_E_UNSUPPORTED, who_str(who, "no kernel for this MLP shape / precision"));
    return hip_fail(e, who);
  }
  if (det) {
    if (side) {
      e = hipStreamWaitEvent(s, side->join, 0);
    } else {
      e = launch_detgrad_order(a.tab.s[0], a.hits, a.cnt, n, opts->K, sh.C, det_scratch, n_leaves,
                               n_vertices, s);
    }
    if (e == hipSuccess)
      e = launch_detgrad_sum(a.tab.s[0], n, opts->K, sh.C, a.gxu, det_scratch, n_leaves,
                             n_vertices, s);
    if (e != hipSuccess) return hip_fail(e, who);
  }
  return SVLF_OK;
}

// ---------------------------------------------------------------- light field

int check_lf_shape(const svlf_lf_model* m, const svlf_render_opts* opts, int64_t* np,
                   const char* who) {
  if (m == nullptr) return fail(SVLF_E_INVAL, who_str(who, "model is NULL"));
  if (m->c_density != kLfCT || m->c_color != kLfCC || m->hidden != kLfH ||
      m->n_hidden_density != kLfNHT || m->n_hidden_color != kLfNHC)
    return fail(SVLF_E_UNSUPPORTED,
                who_str(who, "supported light-field model: C_T 64, C_C 32, hidden 128, 1 + 3 hidden layers"));
  *np = lf_params_density() + lf_params_color((opts->flags & SVLF_FLAG_VIEWDIR) ? 1 : 0);
  return SVLF_OK;
}

int check_lf_model(const svlf_lf_model* m, const svlf_render_opts* opts, int64_t* np,
                   const char* who) {
  int rc = check_lf_shape(m, opts, np, who);
  if (rc) return rc;
  if (m->params == nullptr) return fail(SVLF_E_INVAL, who_str(who, "model->params is NULL"));
  return SVLF_OK;
}

// Workspace: [hit slots][counts][per-hit state][dL/d(o_T0, o_T1)][decoder
// packs][per-block partials of F_T][of F_C][per-block loss][BF16 calls with
// a backward pass: the density decoder's input rows per hit slot][work-item
// counters]
struct LfLayout {
  size_t hits, cnt, st, gT, packs, partT, partC, loss, xs, ctr, total;
};

LfLayout lf_layout(int64_t n, int K, int precision, int viewdir, bool backward) {
  LfLayout w;
  const size_t slots = static_cast<size_t>(n) * K;
  const size_t grid = static_cast<size_t>(lf_grid_limit());
  size_t off = 0;
  w.hits = off;
  off = align256(off + slots * sizeof(HitRec));
  w.cnt = off;
  off = align256(off + static_cast<size_t>(n) * sizeof(int32_t));
  w.st = off;
  off = align256(off + slots * sizeof(LfHit));
  w.gT = off;
  off = align256(off + slots * 2 * sizeof(float));
  w.packs = off;
  off = align256(off + lf_pack_bytes(precision, viewdir));
  w.partT = off;
  off = align256(off + grid * lf_params_density() * sizeof(float));
  w.partC = off;
  off = align256(off + grid * lf_params_color(viewdir) * sizeof(float));
  w.loss = off;
  off = align256(off + grid * sizeof(float));
  w.xs = off;
  if (backward && precision == SVLF_BF16)
    off = align256(off + slots * static_cast<size_t>(lf_x_row()) * sizeof(uint16_t));
  w.ctr = off;
  off = align256(off + 3 * sizeof(int32_t));
  w.total = off;
  return w;
}

int run_lf_call(int mode, const svlf_scene* scenes, int32_t n_scenes, const int64_t* offs,
                const svlf_lf_model* model, const svlf_render_opts* opts, const float* ray_o,
                const float* ray_d, LfArgs a, float* const* grad_features, void* ws,
                size_t ws_bytes, void* stream, const char* who) {
  int rc = check_opts(opts, who);
  if (rc) return rc;
  int64_t np = 0;
  rc = check_lf_model(model, opts, &np, who);
  if (rc) return rc;
  const bool need_grads = mode != kForward;
  rc = make_table(scenes, n_scenes, offs, opts->precision == SVLF_BF16, grad_features, need_grads,
                  &a.tab, who);
  if (rc) return rc;
  const int64_t n = offs[n_scenes];
  if (n > 0 && (ray_o == nullptr || ray_d == nullptr))
    return fail(SVLF_E_INVAL, who_str(who, "ray_o / ray_d is NULL"));
  const int vd = (opts->flags & SVLF_FLAG_VIEWDIR) ? 1 : 0;
  const LfLayout w = lf_layout(n, opts->K, opts->precision, vd, need_grads);
  if (ws == nullptr || ws_bytes < w.total)
    return fail(SVLF_E_WORKSPACE,
                who_str(who, need_grads ? "workspace missing or smaller than svlf_lf_workspace_bytes()"
                                        : "workspace missing or smaller than svlf_lf_render_workspace_bytes()"));
  if (n == 0) return SVLF_OK;
  char* base = static_cast<char*>(ws);
  a.o = ray_o;
  a.d = ray_d;
  a.hits = reinterpret_cast<HitRec*>(base + w.hits);
  a.cnt = reinterpret_cast<int32_t*>(base + w.cnt);
  a.st = reinterpret_cast<LfHit*>(base + w.st);
  a.gT = reinterpret_cast<float*>(base + w.gT);
  a.packs = base + w.packs;
  a.partT = reinterpret_cast<float*>(base + w.partT);
  a.partC = reinterpret_cast<float*>(base + w.partC);
  a.ws_loss = reinterpret_cast<float*>(base + w.loss);
  a.item_counters = reinterpret_cast<int32_t*>(base + w.ctr);
  a.xsave = (need_grads && opts->precision == SVLF_BF16) ? reinterpret_cast<uint16_t*>(base + w.xs)
                                                         : nullptr;
  a.K = opts->K;
  a.tau_mode = opts->tau_mode;
  a.precision = opts->precision;
  a.viewdir = vd;
  a.params = model->params;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (!(opts->flags & SVLF_FLAG_REUSE_HITS)) {
    e = launch_trace_internal(a.tab, ray_o, ray_d, opts->K, const_cast<HitRec*>(a.hits),
                              const_cast<int32_t*>(a.cnt), s);
    if (e != hipSuccess) return hip_fail(e, who);
  }
  if (opts->flags & SVLF_FLAG_TRACE_ONLY) return SVLF_OK;
  e = launch_lf(a, mode, s);
  if (e != hipSuccess) return hip_fail(e, who);
  return SVLF_OK;
}

}  // namespace

extern "C" {

int64_t svlf_lf_param_count(const svlf_lf_model* model, const svlf_render_opts* opts) {
  const char* who = "svlf_lf_param_count";
  if (check_opts(opts, who)) return 0;
  int64_t np = 0;
  if (check_lf_shape(model, opts, &np, who)) return 0;
  return np;
}

size_t svlf_lf_workspace_bytes(const svlf_lf_model* model, const svlf_render_opts* opts,
                               int64_t n_rays) {
  const char* who = "svlf_lf_workspace_bytes";
  if (check_opts(opts, who)) return 0;
  if (svlf_lf_param_count(model, opts) == 0) return 0;
  if (n_rays < 0) {
    fail(SVLF_E_INVAL, who_str(who, "n_rays < 0"));
    return 0;
  }
  return lf_layout(n_rays, opts->K, opts->precision, (opts->flags & SVLF_FLAG_VIEWDIR) ? 1 : 0, true)
      .total;
}

size_t svlf_lf_render_workspace_bytes(const svlf_lf_model* model, const svlf_render_opts* opts,
                                      int64_t n_rays) {
  const char* who = "svlf_lf_render_workspace_bytes";
  if (check_opts(opts, who)) return 0;
  if (svlf_lf_param_count(model, opts) == 0) return 0;
  if (n_rays < 0) {
    fail(SVLF_E_INVAL, who_str(who, "n_rays < 0"));
    return 0;
  }
  return lf_layout(n_rays, opts->K, opts->precision, (opts->flags & SVLF_FLAG_VIEWDIR) ? 1 : 0, false)
      .total;
}

int svlf_lf_render(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                   const svlf_lf_model* model, const svlf_render_opts* opts, const float* ray_o,
                   const float* ray_d, float* out_rgb, float* out_depth, float* out_acc,
                   void* workspace, size_t ws_bytes, void* stream) {
  const char* who = "svlf_lf_render";
  const CallRange range(who);
  if (out_rgb == nullptr || out_depth == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "out_rgb / out_depth is NULL"));
  LfArgs a{};
  a.rgb = out_rgb;
  a.depth = out_depth;
  a.acc = out_acc;
  return run_lf_call(kForward, scenes, n_scenes, ray_offsets_host, model, opts, ray_o, ray_d, a,
                     nullptr, workspace, ws_bytes, stream, who);
}

int svlf_lf_render_backward(const svlf_scene* scenes, int32_t n_scenes,
                            const int64_t* ray_offsets_host, const svlf_lf_model* model,
                            const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                            const float* grad_rgb, const float* grad_depth, const float* grad_acc,
                            float* const* grad_features, float* grad_params, void* workspace,
                            size_t ws_bytes, void* stream) {
  const char* who = "svlf_lf_render_backward";
  const CallRange range(who);
  if (grad_rgb == nullptr || grad_depth == nullptr || grad_params == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "grad_rgb / grad_depth / grad_params is NULL"));
  LfArgs a{};
  a.g_rgb = grad_rgb;
  a.g_depth = grad_depth;
  a.g_acc = grad_acc;
  a.grad_params = grad_params;
  return run_lf_call(kBackward, scenes, n_scenes, ray_offsets_host, model, opts, ray_o, ray_d, a,
                     grad_features, workspace, ws_bytes, stream, who);
}

int svlf_lf_train_stage(const svlf_scene* scenes, int32_t n_scenes,
                        const int64_t* ray_offsets_host, const svlf_lf_model* model,
                        const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                        const float* target_rgb, const float* target_depth,
                        const svlf_lf_loss* loss, float* out_rgb, float* out_depth,
                        float* loss_out, float* const* grad_features, float* grad_params,
                        void* workspace, size_t ws_bytes, void* stream) {
  const char* who = "svlf_lf_train_stage";
  const CallRange range(who);
  if (loss == nullptr) return fail(SVLF_E_INVAL, who_str(who, "loss is NULL"));
  if (loss->kind != SVLF_LF_LOSS_SURFACE && loss->kind != SVLF_LF_LOSS_VOLUME)
    return fail(SVLF_E_RANGE, who_str(who, "unknown loss kind"));
  if (!(loss->lambda_eta >= 0.0f) || !(loss->lambda_tau >= 0.0f) ||
      !std::isfinite(loss->lambda_eta) || !std::isfinite(loss->lambda_tau) ||
      !std::isfinite(loss->loss_scale))
    return fail(SVLF_E_RANGE, who_str(who, "loss weights must be finite and >= 0"));
  if (target_rgb == nullptr || target_depth == nullptr || grad_params == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "targets / grad_params is NULL"));
  LfArgs a{};
  a.t_rgb = target_rgb;
  a.t_depth = target_depth;
  a.loss_scale = loss->loss_scale;
  a.loss_kind = loss->kind == SVLF_LF_LOSS_SURFACE ? kLfLossSurface : kLfLossVolume;
  a.lambda_eta = loss->lambda_eta;
  a.lambda_tau = loss->lambda_tau;
  a.freeze_color = loss->freeze_color ? 1 : 0;
  a.rgb = out_rgb;
  a.depth = out_depth;
  a.loss_out = loss_out;
  a.grad_params = grad_params;
  return run_lf_call(kTrain, scenes, n_scenes, ray_offsets_host, model, opts, ray_o, ray_d, a,
                     grad_features, workspace, ws_bytes, stream, who);
}

int svlf_lf_train_step(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                       const svlf_lf_model* model, const svlf_render_opts* opts,
                       const float* ray_o, const float* ray_d, const float* target_rgb,
                       const float* target_depth, float lambda_depth, float loss_scale,
                       float* out_rgb, float* out_depth, float* loss_out,
                       float* const* grad_features, float* grad_params, void* workspace,
                       size_t ws_bytes, void* stream) {
  const char* who = "svlf_lf_train_step";
  const CallRange range(who);
  if (target_rgb == nullptr || target_depth == nullptr || grad_params == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "targets / grad_params is NULL"));
  if (!std::isfinite(lambda_depth) || !std::isfinite(loss_scale))
    return fail(SVLF_E_INVAL, who_str(who, "lambda_depth / loss_scale must be finite"));
  LfArgs a{};
  a.t_rgb = target_rgb;
  a.t_depth = target_depth;
  a.lambda_depth = lambda_depth;
  a.loss_scale = loss_scale;
  a.rgb = out_rgb;
  a.depth = out_depth;
  a.loss_out = loss_out;
  a.grad_params = grad_params;
  return run_lf_call(kTrain, scenes, n_scenes, ray_offsets_host, model, opts, ray_o, ray_d, a,
                     grad_features, workspace, ws_bytes, stream, who);
}


const char* svlf_last_error(void) { return svlf::error_cstr(); }

const char* svlf_version(void) { return "svlf-mi355x 0.1 (gfx950)"; }

int svlf_build_octree_sizes(const int32_t* leaf_ijk_host, int64_t n, int32_t depth,
                            svlf_octree_sizes* out) {
  if (out == nullptr) return fail(SVLF_E_INVAL, "svlf_build_octree_sizes: out is NULL");
  HostOctree h;
  int rc = build_octree_host(leaf_ijk_host, n, depth, &h, false);
  if (rc) return rc;
  *out = h.sizes;
  return SVLF_OK;
}

int svlf_build_octree(const int32_t* leaf_ijk_host, int64_t n, int32_t depth,
                      svlf_node* nodes_dev, int32_t* leaf_corners_dev,
                      int32_t* leaf_ijk_sorted_host, void* stream) {
  const CallRange range("svlf_build_octree");
  HostOctree h;
  int rc = build_octree_host(leaf_ijk_host, n, depth, &h, true);
  if (rc) return rc;
  if (n > 0 && (nodes_dev == nullptr || leaf_corners_dev == nullptr))
    return fail(SVLF_E_INVAL, "svlf_build_octree: device arrays are NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0) {
    hipError_t e = hipMemcpyAsync(nodes_dev, h.nodes.data(), h.nodes.size() * sizeof(svlf_node),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(leaf_corners_dev, h.leaf_corners.data(),
                         h.leaf_corners.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "svlf_build_octree");
  }
  if (leaf_ijk_sorted_host != nullptr && n > 0)
    std::memcpy(leaf_ijk_sorted_host, h.leaf_ijk_sorted.data(), h.leaf_ijk_sorted.size() * 4);
  return SVLF_OK;
}

int svlf_build_octree_host(const int32_t* leaf_ijk_host, int64_t n, int32_t depth,
                           svlf_node* nodes_host, int32_t* leaf_corners_host,
                           int32_t* leaf_ijk_sorted_host) {
  const CallRange range("svlf_build_octree_host");
  HostOctree h;
  int rc = build_octree_host(leaf_ijk_host, n, depth, &h, true);
  if (rc) return rc;
  if (n > 0 && (nodes_host == nullptr || leaf_corners_host == nullptr))
    return fail(SVLF_E_INVAL, "svlf_build_octree_host: output arrays are NULL");
  if (n > 0) {
    std::memcpy(nodes_host, h.nodes.data(), h.nodes.size() * sizeof(svlf_node));
    std::memcpy(leaf_corners_host, h.leaf_corners.data(), h.leaf_corners.size() * sizeof(int32_t));
    if (leaf_ijk_sorted_host != nullptr)
      std::memcpy(leaf_ijk_sorted_host, h.leaf_ijk_sorted.data(), h.leaf_ijk_sorted.size() * 4);
  }
  return SVLF_OK;
}

size_t svlf_occupancy_workspace_bytes(int32_t level) {
  if (level < 1 || level > SVLF_MAX_DEPTH) {
    fail(SVLF_E_RANGE, "svlf_occupancy_workspace_bytes: level must be in [1, 10]");
    return 0;
  }
  const size_t words = occupancy_bitmap_words(level);
  return align256(words * sizeof(uint32_t)) + align256((words / 256) * sizeof(int));
}

int svlf_occupancy_from_depth(const float* ray_o, const float* ray_d, const float* target_depth,
                              int64_t n, int32_t level, int32_t* leaf_ijk_out,
                              int64_t* n_leaves_out, void* workspace, size_t ws_bytes,
                              void* stream) {
  const char* who = "svlf_occupancy_from_depth";
  const CallRange range(who);
  if (level < 1 || level > SVLF_MAX_DEPTH)
    return fail(SVLF_E_RANGE, who_str(who, "level must be in [1, 10]"));
  if (n < 0) return fail(SVLF_E_INVAL, who_str(who, "n < 0"));
  if (n_leaves_out == nullptr) return fail(SVLF_E_INVAL, who_str(who, "n_leaves_out is NULL"));
  if (n > 0 && (ray_o == nullptr || ray_d == nullptr || target_depth == nullptr ||
                leaf_ijk_out == nullptr))
    return fail(SVLF_E_INVAL, who_str(who, "NULL array"));
  const size_t need = svlf_occupancy_workspace_bytes(level);
  if (workspace == nullptr || ws_bytes < need)
    return fail(SVLF_E_WORKSPACE, who_str(who, "workspace missing or smaller than svlf_occupancy_workspace_bytes()"));
  const size_t words = occupancy_bitmap_words(level);
  char* base = static_cast<char*>(workspace);
  hipError_t e = launch_occupancy(ray_o, ray_d, target_depth, n, level,
                                  reinterpret_cast<uint32_t*>(base),
                                  reinterpret_cast<int*>(base + align256(words * sizeof(uint32_t))),
                                  leaf_ijk_out, n, n_leaves_out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, who);
  return SVLF_OK;
}

int svlf_trace_hits(const svlf_octree* oct, const float* ray_o, const float* ray_d,
                    int64_t n_rays, int32_t K, int32_t* hit_leaf, float* hit_tin,
                    float* hit_tout, int32_t* hit_count, void* stream) {
  const char* who = "svlf_trace_hits";
  const CallRange range(who);
  int rc = check_octree(oct, who);
  if (rc) return rc;
  if (n_rays < 0) return fail(SVLF_E_INVAL, who_str(who, "n_rays < 0"));
  if (K < 1 || K > SVLF_MAX_K) return fail(SVLF_E_RANGE, who_str(who, "K must be in [1, 16]"));
  if (n_rays > (int64_t(1) << 34)) return fail(SVLF_E_RANGE, who_str(who, "too many rays"));
  if (n_rays == 0) return SVLF_OK;
  if (ray_o == nullptr || ray_d == nullptr || hit_leaf == nullptr || hit_tin == nullptr ||
      hit_tout == nullptr || hit_count == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "NULL array"));
  hipError_t e = launch_trace_public(*oct, ray_o, ray_d, n_rays, K, hit_leaf, hit_tin, hit_tout,
                                     hit_count, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, who);
  return SVLF_OK;
}

size_t svlf_workspace_bytes(const svlf_mlp* mlp, const svlf_render_opts* opts, int64_t n_rays) {
  const char* who = "svlf_workspace_bytes";
  if (check_opts(opts, who)) return 0;
  MlpShape sh;
  if (check_mlp(mlp, (opts->flags & SVLF_FLAG_VIEWDIR) != 0, &sh, who)) return 0;
  if (n_rays < 0) {
    fail(SVLF_E_INVAL, who_str(who, "n_rays < 0"));
    return 0;
  }
  if (opts->flags & SVLF_FLAG_DETERMINISTIC) {
    fail(SVLF_E_INVAL, who_str(who, "with SVLF_FLAG_DETERMINISTIC use svlf_workspace_bytes_scenes"));
    return 0;
  }
  return ws_layout(n_rays, opts->K, sh.n_params).total;
}

size_t svlf_workspace_bytes_scenes(const svlf_mlp* mlp, const svlf_render_opts* opts,
                                   const svlf_scene* scenes, int32_t n_scenes, int64_t n_rays) {
  const char* who = "svlf_workspace_bytes_scenes";
  if (check_opts(opts, who)) return 0;
  MlpShape sh;
  if (check_mlp(mlp, (opts->flags & SVLF_FLAG_VIEWDIR) != 0, &sh, who)) return 0;
  if (n_rays < 0 || scenes == nullptr || n_scenes < 1 || n_scenes > SVLF_MAX_SCENES) {
    fail(SVLF_E_INVAL, who_str(who, "invalid scenes / n_rays"));
    return 0;
  }
  const size_t base = ws_layout(n_rays, opts->K, sh.n_params).total;
  if (!(opts->flags & SVLF_FLAG_DETERMINISTIC) || n_scenes != 1) return base;
  return det_extra(base, n_rays, opts->K, sh.C, scenes[0]).total;
}

int svlf_render(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                const svlf_mlp* mlp, const svlf_render_opts* opts, const float* ray_o,
                const float* ray_d, float* out_rgb, float* out_depth, float* out_acc,
                void* workspace, size_t ws_bytes, void* stream) {
  const char* who = "svlf_render";
  const CallRange range(who);
  if (out_rgb == nullptr || out_depth == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "out_rgb / out_depth is NULL"));
  ShadeArgs a{};
  a.rgb = out_rgb;
  a.depth = out_depth;
  a.acc = out_acc;
  return run_shade(kForward, scenes, n_scenes, ray_offsets_host, mlp, opts, ray_o, ray_d, a,
                   nullptr, workspace, ws_bytes, stream, who);
}

int svlf_render_backward(const svlf_scene* scenes, int32_t n_scenes,
                         const int64_t* ray_offsets_host, const svlf_mlp* mlp,
                         const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                         const float* grad_rgb, const float* grad_depth, const float* grad_acc,
                         float* const* grad_features, float* grad_params, void* workspace,
                         size_t ws_bytes, void* stream) {
  const char* who = "svlf_render_backward";
  const CallRange range(who);
  if (grad_rgb == nullptr || grad_depth == nullptr || grad_params == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "grad_rgb / grad_depth / grad_params is NULL"));
  ShadeArgs a{};
  a.g_rgb = grad_rgb;
  a.g_depth = grad_depth;
  a.g_acc = grad_acc;
  a.grad_params = grad_params;
  return run_shade(kBackward, scenes, n_scenes, ray_offsets_host, mlp, opts, ray_o, ray_d, a,
                   grad_features, workspace, ws_bytes, stream, who);
}

int svlf_train_step(const svlf_scene* scenes, int32_t n_scenes, const int64_t* ray_offsets_host,
                    const svlf_mlp* mlp, const svlf_render_opts* opts, const float* ray_o,
                    const float* ray_d, const float* target_rgb, const float* target_depth,
                    float lambda_depth, float loss_scale, float* out_rgb, float* out_depth,
                    float* loss_out, float* const* grad_features, float* grad_params,
                    void* workspace, size_t ws_bytes, void* stream) {
  const char* who = "svlf_train_step";
  const CallRange range(who);
  if (target_rgb == nullptr || target_depth == nullptr || grad_params == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "targets / grad_params is NULL"));
  if (!std::isfinite(lambda_depth) || !std::isfinite(loss_scale))
    return fail(SVLF_E_INVAL, who_str(who, "lambda_depth / loss_scale must be finite"));
  ShadeArgs a{};
  a.t_rgb = target_rgb;
  a.t_depth = target_depth;
  a.lambda_depth = lambda_depth;
  a.loss_scale = loss_scale;
  a.rgb = out_rgb;
  a.depth = out_depth;
  a.loss_out = loss_out;
  a.grad_params = grad_params;
  return run_shade(kTrain, scenes, n_scenes, ray_offsets_host, mlp, opts, ray_o, ray_d, a,
                   grad_features, workspace, ws_bytes, stream, who);
}

int svlf_train_step_noalloc(const svlf_scene* scenes, int32_t n_scenes,
                            const int64_t* ray_offsets_host, const svlf_mlp* mlp,
                            const svlf_render_opts* opts, const float* ray_o, const float* ray_d,
                            const float* target_rgb, const float* target_depth,
                            float lambda_depth, float loss_scale, float* out_rgb, float* out_depth,
                            float* loss_out, float* const* grad_features, float* grad_params,
                            void* stream) {
  const char* who = "svlf_train_step_noalloc";
  const CallRange range(who);
  if (target_rgb == nullptr || target_depth == nullptr || grad_params == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "targets / grad_params is NULL"));
  if (!std::isfinite(lambda_depth) || !std::isfinite(loss_scale))
    return fail(SVLF_E_INVAL, who_str(who, "lambda_depth / loss_scale must be finite"));
  ShadeArgs a{};
  a.t_rgb = target_rgb;
  a.t_depth = target_depth;
  a.lambda_depth = lambda_depth;
  a.loss_scale = loss_scale;
  a.rgb = out_rgb;
  a.depth = out_depth;
  a.loss_out = loss_out;
  a.grad_params = grad_params;
  return run_shade(kTrain, scenes, n_scenes, ray_offsets_host, mlp, opts, ray_o, ray_d, a,
                   grad_features, nullptr, 0, stream, who, true);
}

int svlf_adam_step(float* param, float* grad, float* m, float* v, int64_t n, float lr,
                   float beta1, float beta2, float eps, int64_t step_t, uint16_t* bf16_out,
                   int32_t zero_grad, void* stream) {
  const char* who = "svlf_adam_step";
  const CallRange range(who);
  if (n < 0) return fail(SVLF_E_INVAL, who_str(who, "n < 0"));
  if (step_t < 1) return fail(SVLF_E_RANGE, who_str(who, "step_t must be >= 1"));
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
      !std::isfinite(lr))
    return fail(SVLF_E_RANGE, who_str(who, "invalid hyper-parameters"));
  if (n == 0) return SVLF_OK;
  if (param == nullptr || grad == nullptr || m == nullptr || v == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "NULL array"));
  const double bc1 = 1.0 - std::pow(static_cast<double>(beta1), static_cast<double>(step_t));
  const double bc2 = 1.0 - std::pow(static_cast<double>(beta2), static_cast<double>(step_t));
  hipError_t e = launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, static_cast<float>(bc1),
                             static_cast<float>(bc2), bf16_out, zero_grad,
                             static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, who);
  return SVLF_OK;
}

int svlf_lazy_adam_step(float* param, float* grad, float* m, float* v, int64_t n_rows,
                        int32_t row_len, float lr, float beta1, float beta2, float eps,
                        int64_t step_t, uint16_t* bf16_out, int32_t zero_grad, void* stream) {
  const char* who = "svlf_lazy_adam_step";
  const CallRange range(who);
  if (n_rows < 0) return fail(SVLF_E_INVAL, who_str(who, "n_rows < 0"));
  if (row_len < 4 || row_len > 256 || row_len % 4 != 0)
    return fail(SVLF_E_UNSUPPORTED, who_str(who, "row_len must be a multiple of 4 in [4, 256]"));
  if (step_t < 1) return fail(SVLF_E_RANGE, who_str(who, "step_t must be >= 1"));
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
      !std::isfinite(lr))
    return fail(SVLF_E_RANGE, who_str(who, "invalid hyper-parameters"));
  if (n_rows == 0) return SVLF_OK;
  if (param == nullptr || grad == nullptr || m == nullptr || v == nullptr)
    return fail(SVLF_E_INVAL, who_str(who, "NULL array"));
  auto misaligned = [](const void* q, uintptr_t a) {
    return (reinterpret_cast<uintptr_t>(q) & (a - 1)) != 0;
  };
  if (misaligned(param, 16) || misaligned(grad, 16) || misaligned(m, 16) || misaligned(v, 16) ||
      (bf16_out != nullptr && misaligned(bf16_out, 8)))
    return fail(SVLF_E_INVAL, who_str(who, "arrays must be 16-byte aligned (bf16_out 8-byte)"));
  const double bc1 = 1.0 - std::pow(static_cast<double>(beta1), static_cast<double>(step_t));
  const double bc2 = 1.0 - std::pow(static_cast<double>(beta2), static_cast<double>(step_t));
  hipError_t e = launch_lazy_adam(param, grad, m, v, n_rows, row_len, lr, beta1, beta2, eps,
                                  static_cast<float>(bc1), static_cast<float>(bc2), bf16_out,
                                  zero_grad, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, who);
  return SVLF_OK;
}

int svlf_to_bf16(const float* src, uint16_t* dst, int64_t n, void* stream) {
  const CallRange range("svlf_to_bf16");
  if (n < 0) return fail(SVLF_E_INVAL, "svlf_to_bf16: n < 0");
  if (n == 0) return SVLF_OK;
  if (src == nullptr || dst == nullptr) return fail(SVLF_E_INVAL, "svlf_to_bf16: NULL array");
  hipError_t e = launch_to_bf16(src, dst, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "svlf_to_bf16");
  return SVLF_OK;
}

int svlf_fill(float* dst, float value, int64_t n, void* stream) {
  const CallRange range("svlf_fill");
  if (n < 0) return fail(SVLF_E_INVAL, "svlf_fill: n < 0");
  if (n == 0) return SVLF_OK;
  if (dst == nullptr) return fail(SVLF_E_INVAL, "svlf_fill: NULL array");
  hipError_t e = launch_fill(dst, value, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "svlf_fill");
  return SVLF_OK;
}

int svlf_mlp_forward(const svlf_mlp* mlp, const svlf_render_opts* opts, const float* X, int64_t n,
                     float* out, void* stream) {
  const char* who = "svlf_mlp_forward";
  const CallRange range(who);
  int rc = check_opts(opts, who);
  if (rc) return rc;
  MlpShape sh;
  rc = check_mlp(mlp, (opts->flags & SVLF_FLAG_VIEWDIR) != 0, &sh, who);
  if (rc) return rc;
  if (n < 0) return fail(SVLF_E_INVAL, who_str(who, "n < 0"));
  if (n == 0) return SVLF_OK;
  if (X == nullptr || out == nullptr) return fail(SVLF_E_INVAL, who_str(who, "NULL array"));
  hipError_t e = launch_mlp_forward(mlp->params, sh.C, sh.H, sh.n_hidden,
                                    (opts->flags & SVLF_FLAG_VIEWDIR) ? 1 : 0, opts->precision, X,
                                    n, out, static_cast<hipStream_t>(stream));
  if (e == hipErrorNotSupported)
    return fail(SVLF_E_UNSUPPORTED, who_str(who, "no kernel for this MLP shape / precision"));
  if (e != hipSuccess) return hip_fail(e, who);
  return SVLF_OK;
}

}  // extern "C"
