"""Pins of the Adam oracle: against torch's own Adam and SparseAdam (CPU,
independent implementations of the same published update), the closed form
of the first step, and the lazy-update invariants."""

import numpy as np
import pytest
import torch

from oracle.optim import adam, lazy_adam, touched_rows


def _table(seed, rows=40, cols=8, frac=0.4):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((rows, cols))
    g = rng.standard_normal((rows, cols))
    g[rng.uniform(size=rows) > frac] = 0.0
    return rng, p, g


def test_dense_matches_torch_adam_over_steps():
    rng, p0, _ = _table(0)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in range(1, 6):
        g = rng.standard_normal(p0.shape)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = adam(p, g, m, v, t, lr=1e-2)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14)


def test_lazy_matches_torch_sparse_adam_over_steps():
    rng, p0, _ = _table(1)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SparseAdam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in range(1, 6):
        _, _, g = _table(100 + t)
        idx = np.nonzero(touched_rows(g))[0]
        # torch's sparse gradient lists the touched rows; its step count is
        # per parameter tensor, i.e. the global step here
        tp.grad = torch.sparse_coo_tensor(torch.tensor(idx)[None, :], torch.tensor(g[idx]),
                                          size=p0.shape)
        # torch's SparseAdam uses Kingma & Ba's "efficient" ordering,
        # lr*sqrt(1-b2^t)/(1-b1^t) * m / (sqrt(v) + eps'), which is the update
        # above with eps' = eps * sqrt(1 - b2^t)
        opt.param_groups[0]["eps"] = 1e-8 * np.sqrt(1.0 - 0.999 ** t)
        opt.step()
        p, m, v = lazy_adam(p, g, m, v, t, lr=1e-2)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14)


def test_first_step_closed_form():
    # m_hat = g and v_hat = g^2 at t = 1, so the step is lr * g / (|g| + eps)
    g = np.array([[2.0, -0.5, 1e-3, 0.0]])
    p, m, v = adam(np.zeros_like(g), g, np.zeros_like(g), np.zeros_like(g), 1, lr=0.1, eps=1e-8)
    np.testing.assert_allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_lazy_invariants():
    rng, p0, g = _table(2)
    m0 = rng.uniform(-1, 1, p0.shape)
    v0 = rng.uniform(0, 1, p0.shape)
    p, m, v = lazy_adam(p0, g, m0, v0, 7)
    rows = touched_rows(g)
    assert 0 < rows.sum() < rows.size
    # untouched rows keep parameters and moments exactly
    assert np.array_equal(p[~rows], p0[~rows]) and np.array_equal(m[~rows], m0[~rows])
    assert np.array_equal(v[~rows], v0[~rows])
    # touched rows take the dense step, including their zero entries
    pd, md, vd = adam(p0, g, m0, v0, 7)
    assert np.array_equal(p[rows], pd[rows]) and np.array_equal(m[rows], md[rows])
    # a touched row with a zero entry still decays that entry's moments
    r = np.nonzero(rows)[0][0]
    gz = g.copy()
    gz[r, 0] = 0.0
    _, mz, _ = lazy_adam(p0, gz, m0, v0, 7)
    assert mz[r, 0] == pytest.approx(0.9 * m0[r, 0])
    # every row touched: lazy == dense
    gfull = g + (g == 0) * 0.5
    pl, _, _ = lazy_adam(p0, gfull, m0, v0, 3)
    pd, _, _ = adam(p0, gfull, m0, v0, 3)
    assert np.array_equal(pl, pd)
