"""Adam (Kingma & Ba, the optimiser SVLF trains with, section 4.5) in FP64,
dense and lazy (row-sparse).

TEST INFRASTRUCTURE ONLY (see the package header).

Dense Adam, one step t >= 1 with gradient g:
    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Lazy Adam applies that step only to the rows of a [rows][row_len] table
whose gradient row has a nonzero entry; every other row keeps its
parameters and both moments.  The bias corrections use the global step t.
"""

from __future__ import annotations

import numpy as np


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Returns the updated (p, m, v) as new FP64 arrays."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def touched_rows(g):
    """Rows of a 2-D gradient table with at least one nonzero entry."""
    return np.any(np.asarray(g) != 0, axis=1)


def lazy_adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam on the touched rows only; returns new FP64 (p, m, v)."""
    p = np.array(p, np.float64)
    m = np.array(m, np.float64)
    v = np.array(v, np.float64)
    rows = touched_rows(g)
    if rows.any():
        p[rows], m[rows], v[rows] = adam(p[rows], np.asarray(g, np.float64)[rows], m[rows], v[rows],
                                         t, lr, b1, b2, eps)
    return p, m, v
