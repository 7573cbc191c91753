"""The synthetic workloads (shapes follow the RTMV/SVLF setup).

=================== ================================================ ==========
name                scene                                            rays
=================== ================================================ ==========
shell_d4            depth 4, shell 0.6 +- 0.05, C=8, MLP 8-32-32-4,  64x64 view
                    K=4
ellipsoids_d7       depth 7, 12 solid rotated ellipsoids (~3%),      800x800
                    C=16, MLP 16-64-64-64-4, K=8                     view
ellipsoids_d7_train the ellipsoids_d7 scene, 50 training + 5         2^18 batch
                    held-out views, analytic Lambertian targets
surfaces_d9         depth 9, 40 rotated ellipsoids + 20 boxes,       1600^2 view,
                    surface cells scaled to ~1%, C=32,               2^20 batch
                    MLP 32-64-64-64-4, K=8
(get_multi)         8 scenes, depths {7,8,8,9,9,10,10,10}, 0.5-3%,   2^16..2^20
                    C=32, MLP 32-64-64-64-4, K=8                     per scene
=================== ================================================ ==========

Features are N(0, 0.1^2) per vertex; MLP weights are Xavier-uniform with zero
biases, laid out per layer as W[out][in] (row-major) followed by b[out], all
layers concatenated into one flat FP32 vector.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import scenes
from .cameras import Camera, sphere_camera
from .targets import render_targets

_STREAMS = ("scene", "features", "mlp", "cameras", "batch")


def streams(seed):
    """Independent PCG64 generators, one per purpose, from one seed."""
    children = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    return {k: np.random.Generator(np.random.PCG64(s)) for k, s in zip(_STREAMS, children)}


def xavier_params(rng, widths):
    chunks = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        chunks.append(rng.uniform(-lim, lim, (fan_out, fan_in)).astype(np.float32).ravel())
        chunks.append(np.zeros(fan_out, np.float32))
    return np.concatenate(chunks)


def param_count(widths):
    return sum(o * i + o for i, o in zip(widths[:-1], widths[1:]))


# The light-field model's sizes (C_T, C_C, hidden, hidden layers of the
# density decoder, of the colour decoder) and its decoders' layer widths.
LF_DECODERS = (64, 32, 128, 1, 3)


def lf_widths(viewdir=False):
    ct, cc, h, nht, nhc = LF_DECODERS
    return ((2 * ct + 6,) + (h,) * nht + (2,),
            (cc + 6 + (3 if viewdir else 0),) + (h,) * nhc + (3,))


def lf_inputs(seed, n_vertices, feat_sd=0.1, tau_bias=0.5, viewdir=False):
    """Seeded inputs of the light-field model for a scene: the per-vertex
    table [Z_T | Z_C] (N(0, feat_sd^2)) and Xavier decoders (density then
    colour), with the optical-thickness output bias set to tau_bias."""
    st = streams(seed + 7919)
    ct, cc = LF_DECODERS[0], LF_DECODERS[1]
    F = st["features"].normal(0.0, feat_sd, (n_vertices, ct + cc)).astype(np.float32)
    wt, wc = lf_widths(viewdir)
    pt = xavier_params(st["mlp"], wt)
    pt[-2] = tau_bias
    return F, np.concatenate([pt, xavier_params(st["mlp"], wc)])


@dataclasses.dataclass
class Scene:
    depth: int
    leaf_ijk: np.ndarray        # int32 (n, 3), Morton-sorted, unique
    n_vertices: int
    objects: list
    albedo: Optional[np.ndarray] = None
    light: Optional[np.ndarray] = None

    @property
    def fraction(self):
        return scenes.occupancy_fraction(self.leaf_ijk, self.depth)


@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    depth: int
    C: int
    widths: tuple
    K: int
    image: int                  # square view size for forward renders
    cam_radius: float
    n_views: int = 1
    n_heldout: int = 0
    batch: int = 0
    description: str = ""

    # lazily generated
    _scene: Optional[Scene] = None
    _features: Optional[np.ndarray] = None
    _params: Optional[np.ndarray] = None
    _cams: Optional[List[Camera]] = None

    # -------------------------------------------------------------- scene
    def scene(self) -> Scene:
        if self._scene is None:
            self._scene = _SCENE_BUILDERS[self.name](self)
        return self._scene

    def features(self) -> np.ndarray:
        if self._features is None:
            sc = self.scene()
            rng = streams(self.seed)["features"]
            self._features = rng.normal(0.0, 0.1, (sc.n_vertices, self.C)).astype(np.float32)
        return self._features

    def params(self) -> np.ndarray:
        if self._params is None:
            self._params = xavier_params(streams(self.seed)["mlp"], self.widths)
        return self._params

    # ------------------------------------------------------------ cameras
    def cameras(self) -> List[Camera]:
        if self._cams is None:
            rng = streams(self.seed)["cameras"]
            n = max(1, self.n_views + self.n_heldout)
            self._cams = [sphere_camera(rng, self.cam_radius, self.image, self.image)
                          for _ in range(n)]
        return self._cams

    def view_rays(self, view=0):
        return self.cameras()[view].rays()

    def heldout_views(self):
        return list(range(self.n_views, self.n_views + self.n_heldout))

    def targets(self, o, d):
        sc = self.scene()
        return render_targets(sc.objects, sc.albedo, sc.light, o, d)

    def train_batch(self, n=None, step=0):
        """n rays sampled uniformly from the training views' pixels, sorted
        by (view, pixel) so that a batch is a set of image-coherent rays;
        returns o, d, rgb*, depth* (FP32)."""
        n = self.batch if n is None else n
        rng = np.random.Generator(np.random.PCG64(
            np.random.SeedSequence([self.seed, 1000003, step])))
        npix = self.image * self.image
        flat = np.sort(rng.integers(0, self.n_views * npix, n, dtype=np.int64))
        view = flat // npix
        pix = flat % npix
        cams = self.cameras()
        o = np.empty((n, 3), np.float32)
        d = np.empty((n, 3), np.float32)
        for v in np.unique(view):
            sel = view == v
            o[sel], d[sel] = cams[v].rays(pix[sel])
        rgb, depth = self.targets(o, d)
        return o, d, rgb, depth


# ------------------------------------------------------------ scene makers


def _scene_shell(w):
    shell = scenes.Shell(0.55, 0.65)
    leaves = scenes.scene_leaves([shell], w.depth, "shell")
    return Scene(w.depth, leaves, scenes.count_vertices(leaves), [shell])


def _lights(rng, n_obj):
    albedo = rng.uniform(0.0, 1.0, (n_obj, 3))
    v = rng.standard_normal(3)
    return albedo, v / np.linalg.norm(v)


def _scene_ellipsoids12(w):
    rng = streams(w.seed)["scene"]
    objs = scenes.random_ellipsoids(rng, 12, 0.05, 0.3)
    leaves = scenes.scene_leaves(objs, w.depth, "solid")
    albedo, light = _lights(rng, len(objs))
    return Scene(w.depth, leaves, scenes.count_vertices(leaves), objs, albedo, light)


def _mixed_objects(seed, n_ell, n_box, scale):
    rng = streams(seed)["scene"]
    objs = scenes.random_ellipsoids(rng, n_ell, 0.05, 0.3, scale=scale)
    objs += scenes.random_boxes(rng, n_box, 0.05, 0.3, scale=scale)
    albedo, light = _lights(rng, len(objs))
    return objs, albedo, light


def calibrated_surface_scene(seed, depth, n_ell, n_box, target, tol=0.2):
    """Surface-rule scene whose object scale s is tuned so the occupied
    fraction lands within +-tol of ``target``.  The fraction of surface cells
    scales ~ s^2 / 2^depth, so s is iterated at depth-1 (target doubled) and
    corrected once more at full depth if needed."""
    s = 1.0
    coarse = max(1, depth - 1)
    ctarget = target * (1 << (depth - coarse))
    for _ in range(4):
        objs, _, _ = _mixed_objects(seed, n_ell, n_box, s)
        f = scenes.occupancy_fraction(scenes.scene_leaves(objs, coarse, "surface"), coarse)
        if abs(f / ctarget - 1.0) < 0.05:
            break
        s *= np.sqrt(ctarget / max(f, 1e-12))
        s = min(s, 3.0)
    for _ in range(3):
        objs, albedo, light = _mixed_objects(seed, n_ell, n_box, s)
        leaves = scenes.scene_leaves(objs, depth, "surface")
        f = scenes.occupancy_fraction(leaves, depth)
        if abs(f / target - 1.0) <= tol:
            break
        s *= np.sqrt(target / max(f, 1e-12))
    return Scene(depth, leaves, scenes.count_vertices(leaves), objs, albedo, light), s


def _scene_paper_scale(w):
    sc, _ = calibrated_surface_scene(w.seed, w.depth, 40, 20, 0.01)
    return sc


_SCENE_BUILDERS = {
    "shell_d4": _scene_shell,
    "ellipsoids_d7": _scene_ellipsoids12,
    "ellipsoids_d7_train": _scene_ellipsoids12,
    "surfaces_d9": _scene_paper_scale,
}


def _make(name, seed=None):
    if name == "shell_d4":
        return Workload("shell_d4", 0 if seed is None else seed, 4, 8, (8, 32, 32, 4), 4, 64, 3.0,
                        description="forward FP32, depth 4 shell, 64x64, K=4")
    if name == "ellipsoids_d7":
        return Workload("ellipsoids_d7", 1 if seed is None else seed, 7, 16, (16, 64, 64, 64, 4), 8, 800,
                        4.0, description="forward FP32, depth 7, 12 ellipsoids, 800x800, K=8")
    if name == "ellipsoids_d7_train":
        # same scene as ellipsoids_d7 (same seed drives the scene stream)
        return Workload("ellipsoids_d7_train", 1 if seed is None else seed, 7, 16, (16, 64, 64, 64, 4), 8,
                        800, 4.0, n_views=50, n_heldout=5, batch=1 << 18,
                        description="train step FP32 on the depth-7 ellipsoid scene, batch 2^18 from 50 views")
    if name == "surfaces_d9":
        return Workload("surfaces_d9", 3 if seed is None else seed, 9, 32, (32, 64, 64, 64, 4), 8, 1600, 4.0,
                        n_views=50, n_heldout=5, batch=1 << 20,
                        description="depth 9, 40 ellipsoids + 20 boxes (~1%), 1600^2, batch 2^20")
    raise KeyError(name)


WORKLOADS = ("shell_d4", "ellipsoids_d7", "ellipsoids_d7_train", "surfaces_d9")

# The multi-scene workload: ragged batch of scenes sharing one decoder (C = 32, MLP
# 32-64-64-64-4, K = 8).  Depths as specified; occupied fractions are fixed
# points of the stated 0.5-3% range (largest at the coarsest depth, so no
# scene exceeds ~6M leaves); ray counts are seeded log-uniform in
# [2^16, 2^20] per scene.
MULTI_DEPTHS = (7, 8, 8, 9, 9, 10, 10, 10)
MULTI_FRACTIONS = (0.03, 0.02, 0.015, 0.01, 0.008, 0.006, 0.005, 0.005)


@dataclasses.dataclass
class MultiScene:
    seed: int
    depths: tuple
    fractions: tuple
    C: int = 32
    widths: tuple = (32, 64, 64, 64, 4)
    K: int = 8
    n_ell: int = 12
    n_box: int = 6
    ray_lo: int = 1 << 16
    ray_hi: int = 1 << 20

    def ray_counts(self):
        rng = streams(self.seed)["batch"]
        lg = rng.uniform(np.log2(self.ray_lo), np.log2(self.ray_hi), len(self.depths))
        return [int(2 ** x) for x in lg]

    def scene(self, i):
        sc, _ = calibrated_surface_scene(self.seed * 100 + i, self.depths[i], self.n_ell,
                                         self.n_box, self.fractions[i])
        return sc

    def params(self):
        return xavier_params(streams(self.seed)["mlp"], self.widths)

    def rays(self, i, n):
        """n rays of scene i from cameras on a sphere of radius 4 (one random
        camera per ray, random pixel of a 1600^2 view)."""
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([self.seed, 77, i])))
        v = rng.standard_normal((n, 3))
        pos = 4.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
        f = -pos / np.linalg.norm(pos, axis=1, keepdims=True)
        up = np.where(np.abs(f[:, 2:3]) > 0.999, [[0.0, 1.0, 0.0]], [[0.0, 0.0, 1.0]])
        r = np.cross(f, up)
        r /= np.linalg.norm(r, axis=1, keepdims=True)
        u = np.cross(r, f)
        t = np.tan(np.deg2rad(25.0))
        px = rng.uniform(-1, 1, (n, 1)) * t
        py = rng.uniform(-1, 1, (n, 1)) * t
        d = f + px * r + py * u
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        return pos.astype(np.float32), d.astype(np.float32)


def get_multi(seed=4, small=False) -> MultiScene:
    if small:
        # the same structure at test scale (depths 3..6, 2^8..2^12 rays)
        return MultiScene(seed, (3, 4, 4, 5, 5, 6, 6, 6), MULTI_FRACTIONS, n_ell=4, n_box=2,
                          ray_lo=1 << 8, ray_hi=1 << 12)
    return MultiScene(seed, MULTI_DEPTHS, MULTI_FRACTIONS)


def get_workload(name, seed=None) -> Workload:
    """One of the named workloads (WORKLOADS)."""
    return _make(name, seed)


def tiny_workload(seed, depth, C, widths, K, image=16, kind="ellipsoids", n_obj=3,
                  rule="solid"):
    """Small scene for oracle self-tests and parity at small sizes."""
    w = Workload(f"tiny{seed}", seed, depth, C, tuple(widths), K, image, 3.0)
    rng = streams(seed)["scene"]
    if kind == "shell":
        objs = [scenes.Shell(0.45, 0.7)]
        rule = "shell"
    else:
        objs = scenes.random_ellipsoids(rng, n_obj, 0.15, 0.6)
    leaves = scenes.scene_leaves(objs, depth, rule)
    albedo, light = _lights(rng, len(objs))
    w._scene = Scene(depth, leaves, scenes.count_vertices(leaves), objs, albedo, light)
    return w


def scene_from_leaves(seed, depth, C, widths, K, leaf_ijk, image=16):
    """Workload over an explicit leaf set (crafted test scenes)."""
    leaf_ijk = np.asarray(leaf_ijk, np.int32).reshape(-1, 3)
    if leaf_ijk.shape[0]:
        key = scenes.morton_key(leaf_ijk)
        _, first = np.unique(key, return_index=True)
        leaf_ijk = leaf_ijk[first]
    w = Workload(f"crafted{seed}", seed, depth, C, tuple(widths), K, image, 3.0)
    w._scene = Scene(depth, leaf_ijk, scenes.count_vertices(leaf_ijk), [])
    return w
