"""ctypes binding of libsvlf (include/svlf.h), argument marshalling only.

Every function keeps the name of the C entry point without the ``svlf_``
prefix, takes torch tensors (device memory and streams come from PyTorch),
checks dtype / device / contiguity / shape, and calls the library on the
current torch stream.  All arithmetic of the render path runs in the HIP
kernels of libsvlf.so; there is no fallback: if the library cannot be
loaded, every call raises.
"""

from __future__ import annotations

import ctypes as ct
import os
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SVLF_LIBRARY names another build of the same library (the host-sanitizer
# build of the ABI tests); by default the in-tree libsvlf.so is loaded.
LIB_PATH = os.environ.get("SVLF_LIBRARY") or os.path.join(HERE, "libsvlf.so")

MAX_DEPTH = 10
MAX_K = 16
MAX_SCENES = 16
MAX_LAYERS = 8
NOALLOC_SCRATCH_BYTES = 256 << 20      # SVLF_NOALLOC_SCRATCH_BYTES

OK, E_INVAL, E_RANGE, E_WORKSPACE, E_UNSUPPORTED, E_HIP = 0, -1, -2, -3, -4, -5
TAU_MODES = {"voxel": 0, "direct": 1, "world": 2}
PRECISIONS = {"fp32": 0, "bf16": 1}
FLAG_TRACE_ONLY = 1
FLAG_REUSE_HITS = 2
FLAG_VIEWDIR = 4
FLAG_DETERMINISTIC = 8


class Node(ct.Structure):
    _fields_ = [("child", ct.c_int32), ("mask", ct.c_uint32)]


class OctreeSizes(ct.Structure):
    _fields_ = [("depth", ct.c_int32), ("n_leaves", ct.c_int64), ("n_vertices", ct.c_int64),
                ("n_nodes", ct.c_int64), ("level_offset", ct.c_int64 * (MAX_DEPTH + 1))]


class Octree(ct.Structure):
    _fields_ = [("depth", ct.c_int32), ("n_leaves", ct.c_int64), ("n_vertices", ct.c_int64),
                ("n_nodes", ct.c_int64), ("nodes", ct.c_void_p), ("leaf_corners", ct.c_void_p)]


class Scene(ct.Structure):
    _fields_ = [("octree", Octree), ("features", ct.c_void_p), ("features_bf16", ct.c_void_p)]


class Mlp(ct.Structure):
    _fields_ = [("n_layers", ct.c_int32), ("widths", ct.c_int32 * (MAX_LAYERS + 1)),
                ("params", ct.c_void_p)]


class RenderOpts(ct.Structure):
    _fields_ = [("K", ct.c_int32), ("tau_mode", ct.c_int32), ("precision", ct.c_int32),
                ("flags", ct.c_int32)]


class LfModel(ct.Structure):
    _fields_ = [("c_density", ct.c_int32), ("c_color", ct.c_int32), ("hidden", ct.c_int32),
                ("n_hidden_density", ct.c_int32), ("n_hidden_color", ct.c_int32),
                ("params", ct.c_void_p)]


class LfLoss(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("lambda_eta", ct.c_float), ("lambda_tau", ct.c_float),
                ("loss_scale", ct.c_float), ("freeze_color", ct.c_int32)]


LF_LOSS_SURFACE = 1
LF_LOSS_VOLUME = 2

# The light-field decoders the library supports (the paper's sizes):
# (C_T, C_C, hidden, hidden layers of F_T, hidden layers of F_C)
LF_DECODERS = (64, 32, 128, 1, 3)

_lib = None

_SIGS = {
    "svlf_last_error": ([], ct.c_char_p),
    "svlf_version": ([], ct.c_char_p),
    "svlf_build_octree_sizes": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.POINTER(OctreeSizes)], ct.c_int),
    "svlf_build_octree": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_void_p,
                           ct.c_void_p, ct.c_void_p], ct.c_int),
    "svlf_build_octree_host": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                ct.c_void_p], ct.c_int),
    "svlf_trace_hits": ([ct.POINTER(Octree), ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32,
                         ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p], ct.c_int),
    "svlf_workspace_bytes": ([ct.POINTER(Mlp), ct.POINTER(RenderOpts), ct.c_int64], ct.c_size_t),
    "svlf_render": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(Mlp),
                     ct.POINTER(RenderOpts), ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                     ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p], ct.c_int),
    "svlf_render_backward": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(Mlp),
                              ct.POINTER(RenderOpts), ct.c_void_p, ct.c_void_p, ct.c_void_p,
                              ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_void_p), ct.c_void_p,
                              ct.c_void_p, ct.c_size_t, ct.c_void_p], ct.c_int),
    "svlf_train_step": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(Mlp),
                         ct.POINTER(RenderOpts), ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                         ct.c_float, ct.c_float, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                         ct.POINTER(ct.c_void_p), ct.c_void_p, ct.c_void_p, ct.c_size_t,
                         ct.c_void_p], ct.c_int),
    "svlf_train_step_noalloc": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(Mlp),
                                 ct.POINTER(RenderOpts), ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                 ct.c_void_p, ct.c_float, ct.c_float, ct.c_void_p, ct.c_void_p,
                                 ct.c_void_p, ct.POINTER(ct.c_void_p), ct.c_void_p, ct.c_void_p],
                                ct.c_int),
    "svlf_adam_step": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_float,
                        ct.c_float, ct.c_float, ct.c_float, ct.c_int64, ct.c_void_p, ct.c_int32,
                        ct.c_void_p], ct.c_int),
    "svlf_lazy_adam_step": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64,
                             ct.c_int32, ct.c_float, ct.c_float, ct.c_float, ct.c_float, ct.c_int64,
                             ct.c_void_p, ct.c_int32, ct.c_void_p], ct.c_int),
    "svlf_lf_param_count": ([ct.POINTER(LfModel), ct.POINTER(RenderOpts)], ct.c_int64),
    "svlf_lf_workspace_bytes": ([ct.POINTER(LfModel), ct.POINTER(RenderOpts), ct.c_int64], ct.c_size_t),
    "svlf_lf_render_workspace_bytes": ([ct.POINTER(LfModel), ct.POINTER(RenderOpts), ct.c_int64],
                                       ct.c_size_t),
    "svlf_lf_render": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(LfModel),
                        ct.POINTER(RenderOpts), ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                        ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p], ct.c_int),
    "svlf_lf_render_backward": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64),
                                 ct.POINTER(LfModel), ct.POINTER(RenderOpts), ct.c_void_p,
                                 ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                 ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p], ct.c_int),
    "svlf_lf_train_step": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64),
                            ct.POINTER(LfModel), ct.POINTER(RenderOpts), ct.c_void_p, ct.c_void_p,
                            ct.c_void_p, ct.c_void_p, ct.c_float, ct.c_float, ct.c_void_p,
                            ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                            ct.c_size_t, ct.c_void_p], ct.c_int),
    "svlf_lf_train_stage": ([ct.POINTER(Scene), ct.c_int32, ct.POINTER(ct.c_int64),
                             ct.POINTER(LfModel), ct.POINTER(RenderOpts), ct.c_void_p, ct.c_void_p,
                             ct.c_void_p, ct.c_void_p, ct.POINTER(LfLoss), ct.c_void_p, ct.c_void_p,
                             ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t,
                             ct.c_void_p], ct.c_int),
    "svlf_occupancy_workspace_bytes": ([ct.c_int32], ct.c_size_t),
    "svlf_occupancy_from_depth": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32,
                                   ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p],
                                  ct.c_int),
    "svlf_workspace_bytes_scenes": ([ct.POINTER(Mlp), ct.POINTER(RenderOpts), ct.POINTER(Scene),
                                     ct.c_int32, ct.c_int64], ct.c_size_t),
    "svlf_to_bf16": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p], ct.c_int),
    "svlf_fill": ([ct.c_void_p, ct.c_float, ct.c_int64, ct.c_void_p], ct.c_int),
    "svlf_mlp_forward": ([ct.POINTER(Mlp), ct.POINTER(RenderOpts), ct.c_void_p, ct.c_int64,
                          ct.c_void_p, ct.c_void_p], ct.c_int),
}

EXPORTED = tuple(_SIGS)


def load(path: str = LIB_PATH):
    """Loads libsvlf.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libsvlf.so not found at {path}; build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ct.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def last_error() -> str:
    return load().svlf_last_error().decode()


def version() -> str:
    return load().svlf_version().decode()


class SvlfError(RuntimeError):
    def __init__(self, name, code, msg):
        super().__init__(f"{name} failed with status {code}: {msg}")
        self.code = code


def _check(name, rc):
    if rc != OK:
        raise SvlfError(name, rc, last_error())


# ------------------------------------------------------------------ helpers

def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, shape=None, name="tensor", allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ct.c_void_p(t.data_ptr()) if t.numel() else ct.c_void_p(0)


def make_mlp(params, widths: Sequence[int]) -> Mlp:
    torch = _torch()
    m = Mlp()
    m.n_layers = len(widths) - 1
    for i, w in enumerate(widths):
        m.widths[i] = int(w)
    m.params = _ptr(params, torch.float32, name="params").value
    return m


def make_opts(K, tau_mode="voxel", precision="fp32", flags=0) -> RenderOpts:
    o = RenderOpts()
    o.K = int(K)
    o.tau_mode = TAU_MODES[tau_mode] if isinstance(tau_mode, str) else int(tau_mode)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.flags = int(flags)
    return o


# ------------------------------------------------------------------ octree

def build_octree_sizes(leaf_ijk: np.ndarray, depth: int) -> OctreeSizes:
    ijk = np.ascontiguousarray(leaf_ijk, dtype=np.int32).reshape(-1, 3)
    out = OctreeSizes()
    _check("svlf_build_octree_sizes",
           load().svlf_build_octree_sizes(ijk.ctypes.data_as(ct.c_void_p), ijk.shape[0], depth,
                                          ct.byref(out)))
    return out


def build_octree_host(leaf_ijk: np.ndarray, depth: int):
    """Host build: returns (sizes, nodes (n_nodes, 2) int32 [child, mask],
    leaf_corners (n_leaves, 8) int32, leaf_ijk_sorted (n_leaves, 3) int32)."""
    ijk = np.ascontiguousarray(leaf_ijk, dtype=np.int32).reshape(-1, 3)
    sz = build_octree_sizes(ijk, depth)
    nodes = np.zeros((max(1, sz.n_nodes), 2), np.int32)
    corners = np.zeros((max(1, sz.n_leaves), 8), np.int32)
    srt = np.zeros((max(1, ijk.shape[0]), 3), np.int32)
    _check("svlf_build_octree_host",
           load().svlf_build_octree_host(ijk.ctypes.data_as(ct.c_void_p), ijk.shape[0], depth,
                                         nodes.ctypes.data_as(ct.c_void_p),
                                         corners.ctypes.data_as(ct.c_void_p),
                                         srt.ctypes.data_as(ct.c_void_p)))
    return sz, nodes[:sz.n_nodes], corners[:sz.n_leaves], srt[:ijk.shape[0]]


class DeviceOctree:
    """Device arrays of an octree built by svlf_build_octree."""

    def __init__(self, leaf_ijk: np.ndarray, depth: int, device="cuda"):
        torch = _torch()
        ijk = np.ascontiguousarray(leaf_ijk, dtype=np.int32).reshape(-1, 3)
        sz = build_octree_sizes(ijk, depth)
        self.sizes = sz
        self.depth = depth
        self.n_leaves = sz.n_leaves
        self.n_vertices = sz.n_vertices
        self.n_nodes = sz.n_nodes
        self.nodes = torch.empty((max(1, sz.n_nodes), 2), dtype=torch.int32, device=device)
        self.leaf_corners = torch.empty((max(1, sz.n_leaves), 8), dtype=torch.int32, device=device)
        self.leaf_ijk_sorted = np.empty((ijk.shape[0], 3), np.int32)
        build_octree(ijk, depth, self.nodes, self.leaf_corners, self.leaf_ijk_sorted)

    def struct(self) -> Octree:
        o = Octree()
        o.depth = self.depth
        o.n_leaves = self.n_leaves
        o.n_vertices = self.n_vertices
        o.n_nodes = self.n_nodes
        o.nodes = self.nodes.data_ptr()
        o.leaf_corners = self.leaf_corners.data_ptr()
        return o


def build_octree(leaf_ijk, depth, nodes, leaf_corners, leaf_ijk_sorted=None):
    torch = _torch()
    ijk = np.ascontiguousarray(leaf_ijk, dtype=np.int32).reshape(-1, 3)
    out_ptr = None
    if leaf_ijk_sorted is not None:
        if leaf_ijk_sorted.dtype != np.int32 or not leaf_ijk_sorted.flags.c_contiguous:
            raise ValueError("leaf_ijk_sorted must be a C-contiguous int32 array")
        out_ptr = leaf_ijk_sorted.ctypes.data_as(ct.c_void_p)
    _check("svlf_build_octree",
           load().svlf_build_octree(ijk.ctypes.data_as(ct.c_void_p), ijk.shape[0], depth,
                                    _ptr(nodes, torch.int32, name="nodes"),
                                    _ptr(leaf_corners, torch.int32, name="leaf_corners"),
                                    out_ptr, _stream()))


# ------------------------------------------------------------------ trace

def trace_hits(octree: DeviceOctree, ray_o, ray_d, K):
    torch = _torch()
    n = ray_o.shape[0]
    dev = ray_o.device
    leaf = torch.empty((n, K), dtype=torch.int32, device=dev)
    tin = torch.empty((n, K), dtype=torch.float32, device=dev)
    tout = torch.empty((n, K), dtype=torch.float32, device=dev)
    cnt = torch.empty((n,), dtype=torch.int32, device=dev)
    st = octree.struct()
    _check("svlf_trace_hits",
           load().svlf_trace_hits(ct.byref(st), _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                  _ptr(ray_d, torch.float32, (n, 3), "ray_d"), n, K,
                                  _ptr(leaf), _ptr(tin), _ptr(tout), _ptr(cnt), _stream()))
    return leaf, tin, tout, cnt


# ------------------------------------------------------------------ scenes

class DeviceScene:
    """Octree + FP32 feature masters (+ BF16 copy) on the device."""

    def __init__(self, octree: DeviceOctree, features, features_bf16=None):
        self.octree = octree
        self.features = features
        self.features_bf16 = features_bf16

    @classmethod
    def from_host(cls, leaf_ijk, depth, features: np.ndarray, bf16=True, device="cuda"):
        torch = _torch()
        oc = DeviceOctree(leaf_ijk, depth, device)
        if features.shape[0] != oc.n_vertices:
            raise ValueError(f"features has {features.shape[0]} rows, octree has {oc.n_vertices} vertices")
        f = torch.from_numpy(np.ascontiguousarray(features, np.float32)).to(device)
        sc = cls(oc, f)
        if bf16:
            sc.refresh_bf16()
        return sc

    @classmethod
    def lf_from_host(cls, leaf_ijk, depth, features: np.ndarray, bf16=True, device="cuda"):
        """Scene for the light-field functions: features given per vertex as
        [n_vertices][C_T + C_C], stored on the device in the library's block
        layout (a flat array: Z_T block, then Z_C block)."""
        torch = _torch()
        oc = DeviceOctree(leaf_ijk, depth, device)
        if features.shape != (oc.n_vertices, LF_DECODERS[0] + LF_DECODERS[1]):
            raise ValueError(f"features must be [{oc.n_vertices}][{LF_DECODERS[0] + LF_DECODERS[1]}]")
        f = torch.from_numpy(lf_feature_blocks(features)).to(device)
        sc = cls(oc, f)
        if bf16:
            sc.refresh_bf16()
        return sc

    def refresh_bf16(self):
        torch = _torch()
        if self.features_bf16 is None:
            self.features_bf16 = torch.empty(self.features.shape, dtype=torch.int16,
                                             device=self.features.device)
        to_bf16(self.features, self.features_bf16)

    def struct(self) -> Scene:
        s = Scene()
        s.octree = self.octree.struct()
        s.features = self.features.data_ptr()
        s.features_bf16 = self.features_bf16.data_ptr() if self.features_bf16 is not None else None
        return s


def _scene_array(scenes, ray_counts):
    arr = (Scene * len(scenes))(*[s.struct() for s in scenes])
    offs = np.zeros(len(scenes) + 1, np.int64)
    offs[1:] = np.cumsum(ray_counts)
    offs_c = (ct.c_int64 * len(offs))(*offs.tolist())
    return arr, offs_c, int(offs[-1])


def workspace_bytes(params, widths, opts: RenderOpts, n_rays, scene_array=None, n_scenes=1) -> int:
    m = make_mlp(params, widths)
    if opts.flags & FLAG_DETERMINISTIC:
        nb = load().svlf_workspace_bytes_scenes(ct.byref(m), ct.byref(opts), scene_array, n_scenes,
                                                int(n_rays))
        name = "svlf_workspace_bytes_scenes"
    else:
        nb = load().svlf_workspace_bytes(ct.byref(m), ct.byref(opts), int(n_rays))
        name = "svlf_workspace_bytes"
    if nb == 0:
        raise SvlfError(name, E_INVAL, last_error())
    return nb


class Workspace:
    """Grows on demand; one per stream."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        return self.buf


_default_ws = Workspace()


def render(scenes, ray_counts, params, widths, opts: RenderOpts, ray_o, ray_d, out_rgb=None,
           out_depth=None, out_acc=None, workspace: Workspace = None):
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    dev = ray_o.device
    out_rgb = torch.empty((n, 3), dtype=torch.float32, device=dev) if out_rgb is None else out_rgb
    out_depth = torch.empty((n,), dtype=torch.float32, device=dev) if out_depth is None else out_depth
    if out_acc is None:
        out_acc = torch.empty((n,), dtype=torch.float32, device=dev)
    m = make_mlp(params, widths)
    nb = workspace_bytes(params, widths, opts, n, arr, len(scenes))
    ws = (workspace or _default_ws).get(nb, dev)
    _check("svlf_render",
           load().svlf_render(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                              _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                              _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                              _ptr(out_rgb, torch.float32, (n, 3), "out_rgb"),
                              _ptr(out_depth, torch.float32, (n,), "out_depth"),
                              _ptr(out_acc, torch.float32, (n,), "out_acc"),
                              _ptr(ws, torch.uint8), nb, _stream()))
    return out_rgb, out_depth, out_acc


def _grad_ptrs(grad_features):
    return (ct.c_void_p * len(grad_features))(*[g.data_ptr() for g in grad_features])


def render_backward(scenes, ray_counts, params, widths, opts: RenderOpts, ray_o, ray_d,
                    grad_rgb, grad_depth, grad_acc, grad_features, grad_params,
                    workspace: Workspace = None):
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    m = make_mlp(params, widths)
    nb = workspace_bytes(params, widths, opts, n, arr, len(scenes))
    ws = (workspace or _default_ws).get(nb, ray_o.device)
    for g, s in zip(grad_features, scenes):
        _ptr(g, torch.float32, tuple(s.features.shape), "grad_features")
    _check("svlf_render_backward",
           load().svlf_render_backward(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                                       _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                       _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                       _ptr(grad_rgb, torch.float32, (n, 3), "grad_rgb"),
                                       _ptr(grad_depth, torch.float32, (n,), "grad_depth"),
                                       _ptr(grad_acc, torch.float32, (n,), "grad_acc", allow_none=True),
                                       _grad_ptrs(grad_features),
                                       _ptr(grad_params, torch.float32, tuple(params.shape), "grad_params"),
                                       _ptr(ws, torch.uint8), nb, _stream()))


def train_step(scenes, ray_counts, params, widths, opts: RenderOpts, ray_o, ray_d, target_rgb,
               target_depth, lambda_depth, loss_scale, grad_features, grad_params,
               out_rgb=None, out_depth=None, loss_out=None, workspace: Workspace = None):
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    m = make_mlp(params, widths)
    nb = workspace_bytes(params, widths, opts, n, arr, len(scenes))
    ws = (workspace or _default_ws).get(nb, ray_o.device)
    for g, s in zip(grad_features, scenes):
        _ptr(g, torch.float32, tuple(s.features.shape), "grad_features")
    _check("svlf_train_step",
           load().svlf_train_step(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                                  _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                  _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                  _ptr(target_rgb, torch.float32, (n, 3), "target_rgb"),
                                  _ptr(target_depth, torch.float32, (n,), "target_depth"),
                                  float(lambda_depth), float(loss_scale),
                                  _ptr(out_rgb, torch.float32, (n, 3), "out_rgb", allow_none=True),
                                  _ptr(out_depth, torch.float32, (n,), "out_depth", allow_none=True),
                                  _ptr(loss_out, torch.float32, (1,), "loss_out", allow_none=True),
                                  _grad_ptrs(grad_features),
                                  _ptr(grad_params, torch.float32, tuple(params.shape), "grad_params"),
                                  _ptr(ws, torch.uint8), nb, _stream()))


def train_step_noalloc(scenes, ray_counts, params, widths, opts: RenderOpts, ray_o, ray_d, target_rgb,
                       target_depth, lambda_depth, loss_scale, grad_features, grad_params,
                       out_rgb=None, out_depth=None, loss_out=None):
    """train_step without a workspace (svlf_train_step_noalloc: the library's
    per-device scratch array; nothing is allocated)."""
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    m = make_mlp(params, widths)
    for g, s in zip(grad_features, scenes):
        _ptr(g, torch.float32, tuple(s.features.shape), "grad_features")
    _check("svlf_train_step_noalloc",
           load().svlf_train_step_noalloc(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                                          _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                          _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                          _ptr(target_rgb, torch.float32, (n, 3), "target_rgb"),
                                          _ptr(target_depth, torch.float32, (n,), "target_depth"),
                                          float(lambda_depth), float(loss_scale),
                                          _ptr(out_rgb, torch.float32, (n, 3), "out_rgb", allow_none=True),
                                          _ptr(out_depth, torch.float32, (n,), "out_depth", allow_none=True),
                                          _ptr(loss_out, torch.float32, (1,), "loss_out", allow_none=True),
                                          _grad_ptrs(grad_features),
                                          _ptr(grad_params, torch.float32, tuple(params.shape), "grad_params"),
                                          _stream()))


# ------------------------------------------------------------------ utilities

def adam_step(param, grad, m, v, lr, beta1, beta2, eps, step_t, bf16_out=None, zero_grad=True):
    torch = _torch()
    n = param.numel()
    for t, nm in ((grad, "grad"), (m, "m"), (v, "v")):
        _ptr(t, torch.float32, tuple(param.shape), nm)
    _check("svlf_adam_step",
           load().svlf_adam_step(_ptr(param, torch.float32, name="param"), _ptr(grad), _ptr(m),
                                 _ptr(v), n, lr, beta1, beta2, eps, int(step_t),
                                 _ptr(bf16_out, torch.int16, tuple(param.shape), "bf16_out",
                                      allow_none=True),
                                 1 if zero_grad else 0, _stream()))


def lazy_adam_step(param, grad, m, v, lr, beta1, beta2, eps, step_t, bf16_out=None,
                   zero_grad=True):
    """Row-sparse Adam over a 2-D table [rows][row_len] (rows whose gradient
    is all zero are left untouched)."""
    torch = _torch()
    if param.dim() != 2:
        raise ValueError("lazy_adam_step: param must be 2-D [rows][row_len]")
    rows, row_len = param.shape
    for t, nm in ((grad, "grad"), (m, "m"), (v, "v")):
        _ptr(t, torch.float32, tuple(param.shape), nm)
    _check("svlf_lazy_adam_step",
           load().svlf_lazy_adam_step(_ptr(param, torch.float32, name="param"), _ptr(grad),
                                      _ptr(m), _ptr(v), rows, row_len, lr, beta1, beta2, eps,
                                      int(step_t),
                                      _ptr(bf16_out, torch.int16, tuple(param.shape), "bf16_out",
                                           allow_none=True),
                                      1 if zero_grad else 0, _stream()))


def to_bf16(src, dst):
    torch = _torch()
    _ptr(dst, torch.int16, tuple(src.shape), "dst")
    _check("svlf_to_bf16", load().svlf_to_bf16(_ptr(src, torch.float32, name="src"), _ptr(dst),
                                              src.numel(), _stream()))


def fill(dst, value):
    torch = _torch()
    _check("svlf_fill", load().svlf_fill(_ptr(dst, torch.float32, name="dst"), float(value),
                                        dst.numel(), _stream()))


def mlp_forward(params, widths, opts: RenderOpts, X):
    torch = _torch()
    n = X.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device=X.device)
    m = make_mlp(params, widths)
    _check("svlf_mlp_forward",
           load().svlf_mlp_forward(ct.byref(m), ct.byref(opts),
                                   _ptr(X, torch.float32, (n, widths[0]), "X"), n, _ptr(out),
                                   _stream()))
    return out


# ------------------------------------------------------------------ light field

def make_lf_model(params=None) -> LfModel:
    m = LfModel()
    m.c_density, m.c_color, m.hidden, m.n_hidden_density, m.n_hidden_color = LF_DECODERS
    m.params = params.data_ptr() if params is not None else None
    return m


def lf_param_count(opts: RenderOpts) -> int:
    m = make_lf_model()
    n = load().svlf_lf_param_count(ct.byref(m), ct.byref(opts))
    if n == 0:
        raise SvlfError("svlf_lf_param_count", E_INVAL, last_error())
    return int(n)


def lf_workspace_bytes(opts: RenderOpts, n_rays) -> int:
    m = make_lf_model()
    nb = load().svlf_lf_workspace_bytes(ct.byref(m), ct.byref(opts), int(n_rays))
    if nb == 0:
        raise SvlfError("svlf_lf_workspace_bytes", E_INVAL, last_error())
    return nb


def lf_render_workspace_bytes(opts: RenderOpts, n_rays) -> int:
    m = make_lf_model()
    nb = load().svlf_lf_render_workspace_bytes(ct.byref(m), ct.byref(opts), int(n_rays))
    if nb == 0:
        raise SvlfError("svlf_lf_render_workspace_bytes", E_INVAL, last_error())
    return nb


def _lf_params(params, opts):
    torch = _torch()
    return _ptr(params, torch.float32, (lf_param_count(opts),), "params").value


def lf_render(scenes, ray_counts, params, opts: RenderOpts, ray_o, ray_d, out_rgb=None,
              out_depth=None, out_acc=None, workspace: Workspace = None):
    """Render with the paper's two-decoder light-field function; features of
    each scene are [n_vertices][C_T + C_C]."""
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    dev = ray_o.device
    out_rgb = torch.empty((n, 3), dtype=torch.float32, device=dev) if out_rgb is None else out_rgb
    out_depth = torch.empty((n,), dtype=torch.float32, device=dev) if out_depth is None else out_depth
    if out_acc is None:
        out_acc = torch.empty((n,), dtype=torch.float32, device=dev)
    m = make_lf_model()
    m.params = _lf_params(params, opts)
    nb = lf_render_workspace_bytes(opts, n)
    ws = (workspace or _default_ws).get(nb, dev)
    _check("svlf_lf_render",
           load().svlf_lf_render(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                                 _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                 _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                 _ptr(out_rgb, torch.float32, (n, 3), "out_rgb"),
                                 _ptr(out_depth, torch.float32, (n,), "out_depth"),
                                 _ptr(out_acc, torch.float32, (n,), "out_acc"),
                                 _ptr(ws, torch.uint8), nb, _stream()))
    return out_rgb, out_depth, out_acc


def lf_render_backward(scenes, ray_counts, params, opts: RenderOpts, ray_o, ray_d, grad_rgb,
                       grad_depth, grad_acc, grad_features, grad_params,
                       workspace: Workspace = None):
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    m = make_lf_model()
    m.params = _lf_params(params, opts)
    nb = lf_workspace_bytes(opts, n)
    ws = (workspace or _default_ws).get(nb, ray_o.device)
    for g, s in zip(grad_features, scenes):
        _ptr(g, torch.float32, tuple(s.features.shape), "grad_features")
    _check("svlf_lf_render_backward",
           load().svlf_lf_render_backward(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                                          _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                          _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                          _ptr(grad_rgb, torch.float32, (n, 3), "grad_rgb"),
                                          _ptr(grad_depth, torch.float32, (n,), "grad_depth"),
                                          _ptr(grad_acc, torch.float32, (n,), "grad_acc", allow_none=True),
                                          _grad_ptrs(grad_features),
                                          _ptr(grad_params, torch.float32, tuple(params.shape), "grad_params"),
                                          _ptr(ws, torch.uint8), nb, _stream()))


def lf_train_step(scenes, ray_counts, params, opts: RenderOpts, ray_o, ray_d, target_rgb,
                  target_depth, lambda_depth, loss_scale, grad_features, grad_params,
                  out_rgb=None, out_depth=None, loss_out=None, workspace: Workspace = None):
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    m = make_lf_model()
    m.params = _lf_params(params, opts)
    nb = lf_workspace_bytes(opts, n)
    ws = (workspace or _default_ws).get(nb, ray_o.device)
    for g, s in zip(grad_features, scenes):
        _ptr(g, torch.float32, tuple(s.features.shape), "grad_features")
    _check("svlf_lf_train_step",
           load().svlf_lf_train_step(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                                     _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                     _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                     _ptr(target_rgb, torch.float32, (n, 3), "target_rgb"),
                                     _ptr(target_depth, torch.float32, (n,), "target_depth"),
                                     float(lambda_depth), float(loss_scale),
                                     _ptr(out_rgb, torch.float32, (n, 3), "out_rgb", allow_none=True),
                                     _ptr(out_depth, torch.float32, (n,), "out_depth", allow_none=True),
                                     _ptr(loss_out, torch.float32, (1,), "loss_out", allow_none=True),
                                     _grad_ptrs(grad_features),
                                     _ptr(grad_params, torch.float32, tuple(params.shape), "grad_params"),
                                     _ptr(ws, torch.uint8), nb, _stream()))


def make_lf_loss(kind, lambda_eta=1.0, lambda_tau=0.0, loss_scale=1.0, freeze_color=False) -> LfLoss:
    k = {"surface": LF_LOSS_SURFACE, "volume": LF_LOSS_VOLUME}.get(kind, kind)
    return LfLoss(int(k), float(lambda_eta), float(lambda_tau), float(loss_scale),
                  1 if freeze_color else 0)


def lf_train_stage(scenes, ray_counts, params, opts: RenderOpts, ray_o, ray_d, target_rgb,
                   target_depth, loss: LfLoss, grad_features, grad_params, out_rgb=None,
                   out_depth=None, loss_out=None, workspace: Workspace = None):
    torch = _torch()
    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    arr, offs, n = _scene_array(scenes, ray_counts)
    m = make_lf_model()
    m.params = _lf_params(params, opts)
    nb = lf_workspace_bytes(opts, n)
    ws = (workspace or _default_ws).get(nb, ray_o.device)
    for g, s in zip(grad_features, scenes):
        _ptr(g, torch.float32, tuple(s.features.shape), "grad_features")
    _check("svlf_lf_train_stage",
           load().svlf_lf_train_stage(arr, len(scenes), offs, ct.byref(m), ct.byref(opts),
                                      _ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                      _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                      _ptr(target_rgb, torch.float32, (n, 3), "target_rgb"),
                                      _ptr(target_depth, torch.float32, (n,), "target_depth"),
                                      ct.byref(loss),
                                      _ptr(out_rgb, torch.float32, (n, 3), "out_rgb", allow_none=True),
                                      _ptr(out_depth, torch.float32, (n,), "out_depth", allow_none=True),
                                      _ptr(loss_out, torch.float32, (1,), "loss_out", allow_none=True),
                                      _grad_ptrs(grad_features),
                                      _ptr(grad_params, torch.float32, tuple(params.shape), "grad_params"),
                                      _ptr(ws, torch.uint8), nb, _stream()))


def lf_feature_blocks(features: np.ndarray) -> np.ndarray:
    """[n_vertices][C_T + C_C] per-vertex rows -> the library's block layout
    (Z_T [n][C_T] then Z_C [n][C_C]) as one flat FP32 array."""
    ct_ = LF_DECODERS[0]
    f = np.asarray(features, np.float32)
    return np.concatenate([np.ascontiguousarray(f[:, :ct_]).ravel(),
                           np.ascontiguousarray(f[:, ct_:]).ravel()])


def lf_feature_rows(blocks, n_vertices) -> np.ndarray:
    """Inverse of lf_feature_blocks."""
    ct_, cc_ = LF_DECODERS[0], LF_DECODERS[1]
    b = np.asarray(blocks, np.float32).ravel()
    return np.concatenate([b[:n_vertices * ct_].reshape(n_vertices, ct_),
                           b[n_vertices * ct_:].reshape(n_vertices, cc_)], axis=1)


def occupancy_from_depth(ray_o, ray_d, target_depth, level):
    """Occupied leaves (device int32 [m][3], Morton order) of the depth maps'
    surface points at grid level `level`."""
    torch = _torch()
    n = ray_o.shape[0]
    nb = load().svlf_occupancy_workspace_bytes(int(level))
    if nb == 0:
        raise SvlfError("svlf_occupancy_workspace_bytes", E_RANGE, last_error())
    ws = torch.empty(nb, dtype=torch.uint8, device=ray_o.device)
    out = torch.empty((max(n, 1), 3), dtype=torch.int32, device=ray_o.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=ray_o.device)
    _check("svlf_occupancy_from_depth",
           load().svlf_occupancy_from_depth(_ptr(ray_o, torch.float32, (n, 3), "ray_o"),
                                            _ptr(ray_d, torch.float32, (n, 3), "ray_d"),
                                            _ptr(target_depth, torch.float32, (n,), "target_depth"),
                                            n, int(level), _ptr(out), _ptr(cnt), _ptr(ws), nb,
                                            _stream()))
    return out[:int(cnt.item())]
