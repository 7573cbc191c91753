"""C-ABI checks that need no GPU: the library loads, exports every function
include/svlf.h declares, rejects invalid arguments before queuing any work,
and builds the octree (host part) exactly as the oracle defines it."""

import ctypes as ct
import os
import re

import numpy as np
import pytest

from oracle.octree import Octree
from paper_2205_07058_amd import svlf
from synth.configs import get_workload, tiny_workload
from tests.helpers import crafted_occupancy

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "svlf.h")


@pytest.fixture(scope="module")
def lib():
    return svlf.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svlf_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(svlf.EXPORTED)


def test_version_and_empty_error(lib):
    assert "gfx950" in svlf.version()


def _mlp(widths=(8, 32, 32, 4), null_params=False):
    m = svlf.Mlp()
    m.n_layers = len(widths) - 1
    for i, w in enumerate(widths):
        m.widths[i] = w
    m.params = None if null_params else 0x1000
    return m


def test_validation_errors_before_any_device_work(lib):
    oc = svlf.Octree()
    oc.depth = 3
    # NULL octree
    rc = lib.svlf_trace_hits(None, None, None, 10, 4, None, None, None, None, None)
    assert rc == svlf.E_INVAL and "octree" in svlf.last_error()
    # K out of range
    rc = lib.svlf_trace_hits(ct.byref(oc), None, None, 10, 0, None, None, None, None, None)
    assert rc == svlf.E_RANGE and "K" in svlf.last_error()
    rc = lib.svlf_trace_hits(ct.byref(oc), None, None, 10, 17, None, None, None, None, None)
    assert rc == svlf.E_RANGE
    # depth out of range
    oc.depth = 11
    rc = lib.svlf_trace_hits(ct.byref(oc), None, None, 10, 4, None, None, None, None, None)
    assert rc == svlf.E_RANGE and "depth" in svlf.last_error()
    oc.depth = 3
    # negative ray count
    rc = lib.svlf_trace_hits(ct.byref(oc), None, None, -1, 4, None, None, None, None, None)
    assert rc == svlf.E_INVAL
    # non-empty octree with NULL arrays
    oc.n_leaves = 5
    rc = lib.svlf_trace_hits(ct.byref(oc), None, None, 10, 4, None, None, None, None, None)
    assert rc == svlf.E_INVAL


def test_render_validation(lib):
    opts = svlf.make_opts(8)
    m = _mlp()
    sc = (svlf.Scene * 1)()
    sc[0].octree.depth = 4
    offs = (ct.c_int64 * 2)(0, 100)
    args = lambda s, n, o, mm, op, ws, wsb: lib.svlf_render(s, n, o, mm, op, ct.c_void_p(0x10),
                                                            ct.c_void_p(0x10), ct.c_void_p(0x10),
                                                            ct.c_void_p(0x10), None, ws, wsb, None)
    assert args(None, 1, offs, ct.byref(m), ct.byref(opts), None, 0) == svlf.E_INVAL
    assert args(sc, 0, offs, ct.byref(m), ct.byref(opts), None, 0) == svlf.E_RANGE
    assert args(sc, 17, offs, ct.byref(m), ct.byref(opts), None, 0) == svlf.E_RANGE
    bad = svlf.make_opts(0)
    assert args(sc, 1, offs, ct.byref(m), ct.byref(bad), None, 0) == svlf.E_RANGE
    bad = svlf.make_opts(4, flags=16)
    assert args(sc, 1, offs, ct.byref(m), ct.byref(bad), None, 0) == svlf.E_INVAL
    bad = svlf.make_opts(4, flags=svlf.FLAG_TRACE_ONLY | svlf.FLAG_REUSE_HITS)
    assert args(sc, 1, offs, ct.byref(m), ct.byref(bad), None, 0) == svlf.E_INVAL
    bad = svlf.make_opts(4, precision=7)
    assert args(sc, 1, offs, ct.byref(m), ct.byref(bad), None, 0) == svlf.E_RANGE
    # unsupported MLP shapes
    for widths, code in (((12, 32, 32, 4), svlf.E_UNSUPPORTED), ((8, 48, 48, 4), svlf.E_UNSUPPORTED),
                         ((8, 32, 64, 4), svlf.E_UNSUPPORTED), ((8, 32, 32, 3), svlf.E_INVAL)):
        mm = _mlp(widths)
        assert args(sc, 1, offs, ct.byref(mm), ct.byref(opts), None, 0) == code, widths
    mm = _mlp(null_params=True)
    assert args(sc, 1, offs, ct.byref(mm), ct.byref(opts), None, 0) == svlf.E_INVAL
    # view-direction input: widths[0] = C + 3 for the two supported decoders
    vopts = svlf.make_opts(8, flags=svlf.FLAG_VIEWDIR)
    for widths in ((8, 32, 32, 4), (19, 64, 64, 64, 4), (11, 64, 64, 64, 4), (35, 32, 32, 4)):
        mm = _mlp(widths)
        assert args(sc, 1, offs, ct.byref(mm), ct.byref(vopts), None, 0) == svlf.E_UNSUPPORTED, widths
    for widths in ((11, 32, 32, 4), (35, 64, 64, 64, 4)):
        mm = _mlp(widths)
        assert lib.svlf_workspace_bytes(ct.byref(mm), ct.byref(vopts), 100) > 0, widths
        # accepted shapes fail later, at the (missing) workspace
        assert args(sc, 1, offs, ct.byref(mm), ct.byref(vopts), None, 0) == svlf.E_WORKSPACE, widths
    # workspace too small (empty scene: only the workspace check can fail)
    ws_need = lib.svlf_workspace_bytes(ct.byref(m), ct.byref(opts), 100)
    assert ws_need > 100 * 8 * 16
    assert args(sc, 1, offs, ct.byref(m), ct.byref(opts), ct.c_void_p(0x100), ws_need - 1) == svlf.E_WORKSPACE
    assert "workspace" in svlf.last_error()
    # BF16 without a BF16 feature copy
    sc[0].octree.n_leaves = 1
    sc[0].octree.n_nodes = 1
    sc[0].octree.nodes = 0x100
    sc[0].octree.leaf_corners = 0x100
    sc[0].features = 0x100
    bopts = svlf.make_opts(4, precision="bf16")
    assert args(sc, 1, offs, ct.byref(m), ct.byref(bopts), ct.c_void_p(0x100), 1 << 40) == svlf.E_INVAL
    assert "features_bf16" in svlf.last_error()
    # decreasing offsets
    offs2 = (ct.c_int64 * 2)(0, -1)
    assert args(sc, 1, offs2, ct.byref(m), ct.byref(opts), ct.c_void_p(0x100), 1 << 40) == svlf.E_INVAL


def test_adam_and_util_validation(lib):
    assert lib.svlf_adam_step(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None, 1, None) == svlf.E_RANGE
    assert lib.svlf_adam_step(None, None, None, None, 10, 1e-3, 1.0, 0.999, 1e-8, 1, None, 1, None) == svlf.E_RANGE
    assert lib.svlf_adam_step(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.E_INVAL
    assert lib.svlf_adam_step(None, None, None, None, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.OK
    la = lib.svlf_lazy_adam_step
    assert la(None, None, None, None, 10, 6, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.E_UNSUPPORTED
    assert la(None, None, None, None, 10, 260, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.E_UNSUPPORTED
    assert la(None, None, None, None, 10, 32, 1e-3, 0.9, 0.999, 1e-8, 0, None, 1, None) == svlf.E_RANGE
    assert la(None, None, None, None, 10, 32, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.E_INVAL
    assert la(None, None, None, None, -1, 32, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.E_INVAL
    assert la(None, None, None, None, 0, 32, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.OK
    # misaligned pointers are rejected on the host (never dereferenced)
    assert la(16, 32, 48, 68, 10, 32, 1e-3, 0.9, 0.999, 1e-8, 1, None, 1, None) == svlf.E_INVAL
    assert la(16, 32, 48, 64, 10, 32, 1e-3, 0.9, 0.999, 1e-8, 1, 4, 1, None) == svlf.E_INVAL
    assert lib.svlf_to_bf16(None, None, 5, None) == svlf.E_INVAL
    assert lib.svlf_fill(None, 0.0, -1, None) == svlf.E_INVAL


def test_build_validation(lib):
    ijk = np.array([[0, 0, 0], [0, 0, 0]], np.int32)
    with pytest.raises(svlf.SvlfError) as e:
        svlf.build_octree_host(ijk, 2)
    assert e.value.code == svlf.E_INVAL and "duplicate" in str(e.value)
    with pytest.raises(svlf.SvlfError) as e:
        svlf.build_octree_host(np.array([[4, 0, 0]], np.int32), 2)
    assert e.value.code == svlf.E_RANGE
    with pytest.raises(svlf.SvlfError) as e:
        svlf.build_octree_host(np.array([[0, 0, 0]], np.int32), 11)
    assert e.value.code == svlf.E_RANGE
    sz, nodes, corners, srt = svlf.build_octree_host(np.zeros((0, 3), np.int32), 3)
    assert sz.n_leaves == 0 and sz.n_nodes == 0 and sz.n_vertices == 0


def _expected_nodes(oc: Octree):
    """Level-order node records derived from the oracle's level codes."""
    L = oc.depth
    offs = np.cumsum([0] + [len(oc.level_codes[l]) for l in range(L)])
    rows = []
    for l in range(L):
        first, _ = oc.children(l, np.arange(len(oc.level_codes[l])))
        child = first + (offs[l + 1] if l + 1 < L else 0)
        rows.append(np.stack([child, oc.masks[l].astype(np.int64)], axis=1))
    return np.concatenate(rows, axis=0), offs


@pytest.mark.parametrize("case", ["shell_d4", "tiny_d3", "checker_d4", "single_d5", "full_d2", "random_d6"])
def test_host_octree_matches_oracle(case):
    if case == "shell_d4":
        sc = get_workload("shell_d4").scene()
        ijk, depth = sc.leaf_ijk, sc.depth
    elif case == "tiny_d3":
        sc = tiny_workload(4, 3, 8, (8, 32, 32, 4), 4).scene()
        ijk, depth = sc.leaf_ijk, sc.depth
    elif case == "checker_d4":
        ijk, depth = crafted_occupancy("checker", 4), 4
    elif case == "single_d5":
        ijk, depth = np.array([[31, 0, 17]]), 5
    elif case == "full_d2":
        ijk, depth = crafted_occupancy("full", 2), 2
    else:
        rng = np.random.default_rng(9)
        ijk, depth = np.unique(rng.integers(0, 64, (3000, 3)), axis=0), 6
    rng = np.random.default_rng(0)
    shuffled = np.asarray(ijk)[rng.permutation(len(ijk))]
    sz, nodes, corners, srt = svlf.build_octree_host(shuffled, depth)
    oc = Octree(ijk, depth)
    exp_nodes, offs = _expected_nodes(oc)
    assert sz.n_leaves == oc.n_leaves and sz.n_vertices == oc.n_vertices
    assert sz.n_nodes == exp_nodes.shape[0]
    assert [sz.level_offset[l] for l in range(depth + 1)] == offs.tolist()
    np.testing.assert_array_equal(nodes.astype(np.int64), exp_nodes)
    np.testing.assert_array_equal(corners, oc.leaf_corners)
    np.testing.assert_array_equal(srt, oc.leaf_ijk)


def test_host_octree_threaded_sort_matches_oracle():
    """200,000 leaves at depth 8: 1.6M corner codes, above the size from
    which the host builder sorts with several threads."""
    rng = np.random.default_rng(21)
    ijk = np.unique(rng.integers(0, 256, (205000, 3)), axis=0)
    assert 8 * ijk.shape[0] >= 1 << 20
    sz, nodes, corners, srt = svlf.build_octree_host(ijk[rng.permutation(len(ijk))], 8)
    oc = Octree(ijk, 8)
    exp_nodes, offs = _expected_nodes(oc)
    assert sz.n_leaves == oc.n_leaves and sz.n_vertices == oc.n_vertices
    np.testing.assert_array_equal(nodes.astype(np.int64), exp_nodes)
    np.testing.assert_array_equal(corners, oc.leaf_corners)
    np.testing.assert_array_equal(srt, oc.leaf_ijk)


def test_lf_validation(lib):
    """Light-field entry points reject unsupported models, NULL parameters and
    short workspaces on the host before any device work."""
    opts = svlf.make_opts(8)
    m = svlf.make_lf_model()
    assert lib.svlf_lf_param_count(ct.byref(m), ct.byref(opts)) > 0
    n_plain = lib.svlf_lf_param_count(ct.byref(m), ct.byref(opts))
    vopts = svlf.make_opts(8, flags=svlf.FLAG_VIEWDIR)
    assert lib.svlf_lf_param_count(ct.byref(m), ct.byref(vopts)) == n_plain + 3 * 128
    from oracle.lightfield import n_params
    assert n_plain == n_params(svlf.LF_DECODERS)
    bad = svlf.make_lf_model()
    bad.hidden = 64
    assert lib.svlf_lf_param_count(ct.byref(bad), ct.byref(opts)) == 0
    assert "light-field" in svlf.last_error()
    sc = (svlf.Scene * 1)()
    sc[0].octree.depth = 4
    offs = (ct.c_int64 * 2)(0, 100)
    call = lambda mm, ws, wsb: lib.svlf_lf_render(sc, 1, offs, ct.byref(mm), ct.byref(opts),
                                                  ct.c_void_p(0x10), ct.c_void_p(0x10),
                                                  ct.c_void_p(0x10), ct.c_void_p(0x10), None,
                                                  ws, wsb, None)
    assert call(bad, None, 0) == svlf.E_UNSUPPORTED
    assert call(m, None, 0) == svlf.E_INVAL                     # params NULL
    m.params = 0x100
    need_r = lib.svlf_lf_render_workspace_bytes(ct.byref(m), ct.byref(opts), 100)
    assert need_r > 100 * 8 * (16 + 32 + 8)
    assert call(m, ct.c_void_p(0x100), need_r - 1) == svlf.E_WORKSPACE
    assert "svlf_lf_render_workspace_bytes" in svlf.last_error()
    # FP32 calls need the same space in both modes; BF16 calls with a backward
    # pass keep the density decoder's inputs per hit slot
    assert need_r == lib.svlf_lf_workspace_bytes(ct.byref(m), ct.byref(opts), 100)
    bopts = svlf.make_opts(8, precision="bf16")
    need_rb = lib.svlf_lf_render_workspace_bytes(ct.byref(m), ct.byref(bopts), 100)
    need = lib.svlf_lf_workspace_bytes(ct.byref(m), ct.byref(bopts), 100)
    assert need >= need_rb + 100 * 8 * 288
    gp = ct.c_void_p(0x100)
    gf = ct.cast((ct.c_void_p * 1)(0x100), ct.c_void_p)
    back = lambda wsb: lib.svlf_lf_render_backward(sc, 1, offs, ct.byref(m), ct.byref(bopts),
                                                   gp, gp, gp, gp, None, gf, gp,
                                                   ct.c_void_p(0x100), wsb, None)
    assert back(need - 1) == svlf.E_WORKSPACE
    assert "svlf_lf_workspace_bytes" in svlf.last_error()


def test_occupancy_validation(lib):
    assert lib.svlf_occupancy_workspace_bytes(0) == 0
    assert lib.svlf_occupancy_workspace_bytes(11) == 0
    assert lib.svlf_occupancy_workspace_bytes(1) > 0
    assert lib.svlf_occupancy_workspace_bytes(10) >= (1 << 30) // 8
    f = lib.svlf_occupancy_from_depth
    cnt = ct.c_void_p(0x100)
    assert f(None, None, None, 10, 0, None, cnt, None, 0, None) == svlf.E_RANGE
    assert f(None, None, None, -1, 5, None, cnt, None, 0, None) == svlf.E_INVAL
    assert f(None, None, None, 10, 5, None, cnt, None, 0, None) == svlf.E_INVAL
    assert f(None, None, None, 10, 5, None, None, None, 0, None) == svlf.E_INVAL
    p = ct.c_void_p(0x100)
    need = lib.svlf_occupancy_workspace_bytes(5)
    assert f(p, p, p, 10, 5, p, cnt, p, need - 1, None) == svlf.E_WORKSPACE


def test_deterministic_workspace_query(lib):
    """With SVLF_FLAG_DETERMINISTIC the scene-less workspace query refuses
    and the scene-aware one adds the reduction's space."""
    m = _mlp()
    opts = svlf.make_opts(8, flags=svlf.FLAG_DETERMINISTIC)
    assert lib.svlf_workspace_bytes(ct.byref(m), ct.byref(opts), 100) == 0
    assert "svlf_workspace_bytes_scenes" in svlf.last_error()
    sc = (svlf.Scene * 1)()
    sc[0].octree.depth = 4
    sc[0].octree.n_leaves = 1000
    sc[0].octree.n_vertices = 3000
    plain = svlf.make_opts(8)
    base = lib.svlf_workspace_bytes_scenes(ct.byref(m), ct.byref(plain), sc, 1, 100)
    assert base == lib.svlf_workspace_bytes(ct.byref(m), ct.byref(plain), 100)
    det = lib.svlf_workspace_bytes_scenes(ct.byref(m), ct.byref(opts), sc, 1, 100)
    assert det >= base + 100 * 8 * (8 + 4) * 4 + 3000 * 32


def test_noalloc_train_step_rejects_oversized_calls_before_device_work(lib):
    """svlf_train_step_noalloc: a call whose workspace exceeds the library's
    scratch array fails with SVLF_E_WORKSPACE during host validation (here on
    a machine without a GPU: nothing reaches the device)."""
    m = _mlp((32, 64, 64, 64, 4))
    opts = svlf.make_opts(8)
    sc = (svlf.Scene * 1)()
    sc[0].octree.depth = 4        # empty scene: only the size check can fail
    n = 4 << 20
    offs = (ct.c_int64 * 2)(0, n)
    need = lib.svlf_workspace_bytes(ct.byref(m), ct.byref(opts), n)
    assert need > svlf.NOALLOC_SCRATCH_BYTES
    grads = (ct.c_void_p * 1)(0x100)
    p = ct.c_void_p(0x100)
    rc = lib.svlf_train_step_noalloc(sc, 1, offs, ct.byref(m), ct.byref(opts), p, p, p, p, 0.1, 1.0,
                                     None, None, None, grads, p, None)
    assert rc == svlf.E_WORKSPACE and "SVLF_NOALLOC_SCRATCH_BYTES" in svlf.last_error()
    # the size limit is the documented one: the largest ray count that fits
    fit = 1
    while lib.svlf_workspace_bytes(ct.byref(m), ct.byref(opts), 2 * fit) <= svlf.NOALLOC_SCRATCH_BYTES:
        fit *= 2
    assert fit >= 1 << 20
    # other validation still comes first
    rc = lib.svlf_train_step_noalloc(sc, 1, offs, ct.byref(m), ct.byref(opts), p, p, None, p, 0.1, 1.0,
                                     None, None, None, grads, p, None)
    assert rc == svlf.E_INVAL
