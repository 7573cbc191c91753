"""GPU parity of svlf_build_octree + svlf_trace_hits against the oracle:
hit lists (leaf ids, FP32 t_in / t_out bit patterns, counts) must be
identical (sections 4.2-4.3 with the library's documented predicate)."""

import numpy as np
import pytest

from oracle.octree import Octree
from oracle.trace import trace_hits as oracle_trace
from synth.configs import get_workload, tiny_workload
from tests.helpers import crafted_occupancy, golden_case_arrays, load_golden, random_rays

pytestmark = pytest.mark.gpu


def _gpu_trace(svlf, ijk, depth, o, d, K):
    import torch
    oc = svlf.DeviceOctree(ijk, depth)
    to = torch.from_numpy(np.ascontiguousarray(o, np.float32)).cuda()
    td = torch.from_numpy(np.ascontiguousarray(d, np.float32)).cuda()
    leaf, tin, tout, cnt = svlf.trace_hits(oc, to, td, K)
    torch.cuda.synchronize()
    return leaf.cpu().numpy(), tin.cpu().numpy(), tout.cpu().numpy(), cnt.cpu().numpy()


def _assert_identical(got, exp, ctx=""):
    gl, gi, go, gc = got
    el, ei, eo, ec = exp
    np.testing.assert_array_equal(gc, ec, err_msg=f"counts {ctx}")
    np.testing.assert_array_equal(gl, el, err_msg=f"leaf ids {ctx}")
    np.testing.assert_array_equal(gi.view(np.int32), ei.view(np.int32), err_msg=f"t_in bits {ctx}")
    np.testing.assert_array_equal(go.view(np.int32), eo.view(np.int32), err_msg=f"t_out bits {ctx}")


def test_golden_degenerate_rays(gpu_lib):
    g = load_golden("degenerate_rays.json")
    depth = g["depth"]
    for case in g["cases"]:
        cells = crafted_occupancy(case["occupancy"], depth)
        oc = Octree(cells, depth)
        o, d = golden_case_arrays(case)
        K = case["K"]
        got = _gpu_trace(gpu_lib, cells, depth, o, d, K)
        _assert_identical(got, oracle_trace(oc, o, d, K), case["name"])
        # and the hand-derived values directly
        assert got[3][0] == len(case["hits"]), case["name"]
        for s, (i, j, k, t0, t1) in enumerate(case["hits"]):
            assert oc.leaf_ijk[got[0][0, s]].tolist() == [i, j, k]
            assert got[1][0, s] == np.float32(t0) and got[2][0, s] == np.float32(t1)


@pytest.mark.parametrize("kind,depth", [("full", 3), ("checker", 4), ("random30", 5), ("single", 6),
                                        ("empty", 3)])
@pytest.mark.parametrize("K", [1, 5, 16])
def test_crafted_scenes_random_rays(gpu_lib, kind, depth, K):
    cells = crafted_occupancy(kind, depth, seed=depth) if depth <= 5 else \
        np.array([[13, 40, 27]])
    rng = np.random.default_rng(depth * 7 + K)
    o, d = random_rays(rng, 3001, inside_frac=0.3, axis_frac=0.15)   # ragged tail
    # add degenerate rays: zero, NaN, Inf, subnormal components
    o[:4] = [[0.1, 0.2, 0.3], [-2, 0.1, 0.1], [np.inf, 0, 0], [-2, 0.25, -0.25]]
    d[:4] = [[0, 0, 0], [1, np.nan, 0], [1, 0, 0], [1, 1e-40, -0.0]]
    exp = oracle_trace(Octree(cells, depth), o, d, K)
    _assert_identical(_gpu_trace(gpu_lib, cells, depth, o, d, K), exp, f"{kind} d{depth} K{K}")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_ellipsoid_scenes(gpu_lib, seed):
    w = tiny_workload(seed, 6, 8, (8, 32, 32, 4), 8, n_obj=4)
    sc = w.scene()
    o, d = w.view_rays()
    o2, d2 = random_rays(np.random.default_rng(seed), 2000)
    o = np.concatenate([o, o2]); d = np.concatenate([d, d2])
    exp = oracle_trace(Octree(sc.leaf_ijk, sc.depth), o, d, 8)
    _assert_identical(_gpu_trace(gpu_lib, sc.leaf_ijk, sc.depth, o, d, 8), exp, f"seed {seed}")


def test_workload0_full_view(gpu_lib):
    w = get_workload("shell_d4")
    sc = w.scene()
    o, d = w.view_rays()
    exp = oracle_trace(Octree(sc.leaf_ijk, sc.depth), o, d, w.K)
    _assert_identical(_gpu_trace(gpu_lib, sc.leaf_ijk, sc.depth, o, d, w.K), exp, "shell_d4")


def test_workload1_full_view_sampled(gpu_lib):
    """800x800 view traced on the GPU; a seeded sample of 4096 rays (plus the
    last ray) compared against the oracle."""
    w = get_workload("ellipsoids_d7")
    sc = w.scene()
    o, d = w.view_rays()
    got = _gpu_trace(gpu_lib, sc.leaf_ijk, sc.depth, o, d, w.K)
    rng = np.random.default_rng(123)
    idx = np.concatenate([rng.choice(o.shape[0], 4096, replace=False), [o.shape[0] - 1]])
    exp = oracle_trace(Octree(sc.leaf_ijk, sc.depth), o[idx], d[idx], w.K)
    _assert_identical(tuple(a[idx] for a in got), exp, "ellipsoids_d7 sample")
    # whole-view invariants
    leaf, tin, tout, cnt = got
    assert cnt.max() <= w.K and (cnt > 0).mean() > 0.02
    valid = leaf >= 0
    assert np.array_equal(valid.sum(axis=1), cnt)
    assert np.all(tin[valid] < tout[valid])
