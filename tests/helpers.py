"""Shared test helpers: fixture loading and crafted occupancy grids."""

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def f32(v):
    return np.float32(float(v))


def crafted_occupancy(kind, depth, seed=0):
    n = 1 << depth
    cells = np.array(list(itertools.product(range(n), repeat=3)), np.int64)
    if kind == "full":
        return cells
    if kind == "checker":
        return cells[(cells.sum(axis=1) % 2) == 0]
    if kind == "empty":
        return cells[:0]
    if kind == "single":
        rng = np.random.default_rng(seed)
        return cells[rng.integers(0, cells.shape[0], 1)]
    if kind.startswith("random"):
        frac = float(kind[6:]) / 100.0
        rng = np.random.default_rng(seed)
        return cells[rng.random(cells.shape[0]) < frac]
    raise KeyError(kind)


def golden_case_arrays(case):
    o = np.array([[f32(v) for v in case["o"]]], np.float32)
    d = np.array([[f32(v) for v in case["d"]]], np.float32)
    return o, d


def random_rays(rng, n, inside_frac=0.25, axis_frac=0.1):
    """Rays from a sphere of radius 3 towards random points of the cube,
    plus rays starting inside the cube and some axis-parallel ones."""
    v = rng.standard_normal((n, 3))
    o = 3.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
    tgt = rng.uniform(-0.9, 0.9, (n, 3))
    n_in = int(n * inside_frac)
    o[:n_in] = rng.uniform(-0.95, 0.95, (n_in, 3))
    d = tgt - o
    d[:n_in] = rng.standard_normal((n_in, 3))
    n_ax = int(n * axis_frac)
    if n_ax:
        sel = rng.choice(n, n_ax, replace=False)
        ax = rng.integers(0, 3, n_ax)
        keep = np.zeros((n_ax, 3))
        keep[np.arange(n_ax), ax] = 1.0
        d[sel] = d[sel] * keep
        d[sel[np.all(d[sel] == 0, axis=1)], 0] = 1.0
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
