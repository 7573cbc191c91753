"""svlf_train_step_noalloc (the train step without a workspace, for callers
that cannot allocate device memory) against svlf_train_step: two calls in a
row on the library's scratch array, the second with fewer rays, each
compared with the workspace entry point on the same inputs."""

import numpy as np
import pytest

from synth.configs import tiny_workload
from tests.gpu_cases import Case
from tests.helpers import random_rays

pytestmark = pytest.mark.gpu


def _run(gpu_lib, case, o, d, t_rgb, t_dep, opts, noalloc):
    import torch
    n = o.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    gF = torch.zeros_like(case.scene.features)
    gp = torch.zeros_like(case.params)
    loss = torch.zeros(1, device="cuda")
    rgb = torch.empty((n, 3), device="cuda")
    dep = torch.empty(n, device="cuda")
    step = gpu_lib.train_step_noalloc if noalloc else gpu_lib.train_step
    step([case.scene], [n], case.params, case.widths, opts, T(o), T(d), T(t_rgb), T(t_dep), 0.1,
         1.0 / n, [gF], gp, out_rgb=rgb, out_depth=dep, loss_out=loss)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (rgb, dep, loss, gF, gp)]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_train_step_matches_workspace_entry_point(gpu_lib, precision):
    w = tiny_workload(31, 6, 32, (32, 64, 64, 64, 4), 8, n_obj=4)
    case = Case.from_workload(gpu_lib, w, feat_scale=4.0, sigma_bias=0.5)
    rng = np.random.default_rng(3)
    for n in (70001, 5003):                 # several 65,536-ray groups, then a smaller call
        o, d = random_rays(rng, n, inside_frac=0.1)
        t_rgb = rng.uniform(0, 1, (n, 3)).astype(np.float32)
        t_dep = rng.uniform(0, 5, n).astype(np.float32)
        for flags in (0, gpu_lib.FLAG_DETERMINISTIC):
            opts = gpu_lib.make_opts(case.K, "voxel", precision, flags)
            ref = _run(gpu_lib, case, o, d, t_rgb, t_dep, opts, False)
            got = _run(gpu_lib, case, o, d, t_rgb, t_dep, opts, True)
            assert np.count_nonzero(ref[3]) > 1000
            # per-ray outputs: identical bits
            for k in (0, 1):
                assert np.array_equal(got[k].view(np.int32), ref[k].view(np.int32)), (n, flags, k)
            if flags:
                # fixed-order reductions and a fixed item-to-block assignment:
                # loss, feature and decoder gradients with identical bits
                for k in (2, 3, 4):
                    assert np.array_equal(got[k].view(np.int32), ref[k].view(np.int32)), (n, flags, k)
            else:
                # feature gradients: FP32 atomics in any order; the loss and
                # the decoder gradient: per-block partials of items handed
                # out to whichever block is free
                for k in (2, 3, 4):
                    s = np.abs(ref[k]).max()
                    np.testing.assert_allclose(got[k], ref[k], rtol=1e-5, atol=1e-6 * s)
