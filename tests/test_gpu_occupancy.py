"""GPU parity of the depth-map occupancy (svlf_occupancy_from_depth): the
leaves holding the surface points of depth maps, bit-exact against the
oracle, and the octree built from them."""

import numpy as np
import pytest

from oracle.octree import occupancy_from_depth
from synth.configs import get_workload, tiny_workload

pytestmark = pytest.mark.gpu


def _gpu(gpu_lib, o, d, t, level):
    import torch
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    out = gpu_lib.occupancy_from_depth(T(o), T(d), T(t), level)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("level", [1, 3, 6, 10])
def test_occupancy_random_points(gpu_lib, level):
    rng = np.random.default_rng(level)
    n = 20000
    o = rng.uniform(-1.3, 1.3, (n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    t = rng.uniform(0, 0.5, n).astype(np.float32)
    t[::13] = 0.0
    t[5::97] = np.nan
    o[:500, 0] = (rng.integers(-8, 8, 500) / 8.0).astype(np.float32)   # points on cell faces
    d[:500, 0] = 0.0
    got = _gpu(gpu_lib, o, d, t, level)
    exp = occupancy_from_depth(o, d, t, level)
    np.testing.assert_array_equal(got, exp)


def test_occupancy_from_rendered_depth_maps(gpu_lib):
    """Analytic depth maps of a synthetic scene: the leaves found from them
    are a subset of the scene's surface occupancy, match the oracle
    bit-exactly, and build an octree whose traversal finds the surface."""
    import torch
    w = tiny_workload(11, 7, 8, (8, 32, 32, 4), 8, n_obj=3, image=96, rule="surface")
    w.n_views, w.n_heldout = 6, 0
    w.cam_radius = 3.0
    os_, ds_, ts_ = [], [], []
    for v in range(w.n_views):
        o, d = w.view_rays(v)
        _, dep = w.targets(o, d)
        os_.append(o), ds_.append(d), ts_.append(dep)
    o, d, t = np.concatenate(os_), np.concatenate(ds_), np.concatenate(ts_)
    got = _gpu(gpu_lib, o, d, t, 7)
    exp = occupancy_from_depth(o, d, t, 7)
    np.testing.assert_array_equal(got, exp)
    assert got.shape[0] > 500
    scene = {tuple(c) for c in w.scene().leaf_ijk.tolist()}
    inside = np.mean([tuple(c) in scene for c in got.tolist()])
    assert inside > 0.99, inside          # FP32 surface points may round into a neighbour
    oc = gpu_lib.DeviceOctree(got.astype(np.int32), 7)
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    leaf, tin, tout, cnt = gpu_lib.trace_hits(oc, T(os_[0]), T(ds_[0]), 4)
    c = cnt.cpu().numpy()
    hit_gt = ts_[0] > 0
    assert np.mean(c[hit_gt] > 0) > 0.99


def test_occupancy_paper_scale_view(gpu_lib):
    """One 1600^2 view of the paper-scale scene at level 9."""
    w = get_workload("surfaces_d9")
    o, d = w.view_rays(0)
    _, t = w.targets(o, d)
    got = _gpu(gpu_lib, o, d, t, 9)
    exp = occupancy_from_depth(o, d, t, 9)
    np.testing.assert_array_equal(got, exp)
    assert got.shape[0] > 10000
