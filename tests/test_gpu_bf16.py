"""The FP32 -> bfloat16 rounding of the library (svlf_to_bf16, which uses the
same hardware conversion as the shading kernels' BF16 operands) against the
oracle's round-to-nearest-even on adversarial bit patterns: ties in both
parities, just below / above ties, subnormals, the largest finite values
(rounding up to infinity), infinities and signed zeros."""

import numpy as np
import pytest

from oracle.render import bf16_round

pytestmark = pytest.mark.gpu


def _patterns(seed=0):
    rng = np.random.default_rng(seed)
    hi = np.arange(1 << 16, dtype=np.uint32)                 # every sign/exponent/7-bit head
    lows = np.array([0x0000, 0x0001, 0x7FFF, 0x8000, 0x8001, 0xFFFF], np.uint32)
    pats = (hi[:, None] << 16 | lows[None, :]).ravel()
    pats = np.concatenate([pats, rng.integers(0, 1 << 32, 1 << 20, dtype=np.uint64).astype(np.uint32)])
    keep = (pats & 0x7FFFFFFF) <= 0x7F800000                 # no NaNs
    return pats[keep]


def test_to_bf16_matches_round_to_nearest_even(gpu_lib):
    import torch
    pats = _patterns()
    x = pats.view(np.float32)
    with np.errstate(over="ignore"):                       # values rounding to infinity
        exp = np.float32(bf16_round(x.astype(np.float64))).view(np.uint32) >> 16
    src = torch.from_numpy(x.copy()).cuda()
    dst = torch.empty(src.shape, dtype=torch.int16, device="cuda")
    gpu_lib.to_bf16(src, dst)
    torch.cuda.synchronize()
    got = dst.cpu().numpy().view(np.uint16).astype(np.uint32)
    bad = np.nonzero(got != exp)[0]
    assert bad.size == 0, (f"{bad.size} of {x.size} differ, first input 0x{pats[bad[0]]:08x}: "
                           f"got 0x{got[bad[0]]:04x}, expected 0x{exp[bad[0]]:04x}")
