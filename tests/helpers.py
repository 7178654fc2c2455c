"""Independent numpy evaluators used by the tests (no code shared with the
oracle or the GPU library): power series and Bernstein polynomials evaluated
from their definitions, and the plain forward pass of a ReLU network."""
import itertools
from math import comb  # noqa: F401  (re-exported for tests)

import numpy as np


def multi_indices(n, d):
    return np.array(list(itertools.product(range(d + 1), repeat=n)), dtype=np.int64).reshape(-1, n)


def power_eval(n, d, a, t):
    """sum_K a_K t^K at points t [m, n]."""
    K = multi_indices(n, d)
    t = np.atleast_2d(t)
    mon = np.prod(t[:, None, :] ** K[None, :, :], axis=2)
    return mon @ np.asarray(a)


def bern_basis(n, d, t):
    K = multi_indices(n, d)
    t = np.atleast_2d(t)
    C = np.array([[comb(d, int(k)) for k in row] for row in K], dtype=np.float64)
    return np.prod(C[None] * t[:, None, :] ** K[None] * (1 - t[:, None, :]) ** (d - K[None]), axis=2)


def bern_eval(n, d, b, t):
    """sum_K b_K Ber_{K,d}(t) at points t [m, n] (Def. 1 in t = normalised box coordinate)."""
    return bern_basis(n, d, t) @ np.asarray(b)


def forward(Ws, bs, x):
    """Pre-activations of every layer for inputs x [m, n]; returns list (one per layer)."""
    z = np.atleast_2d(x)
    pres = []
    for i, (W, b) in enumerate(zip(Ws, bs)):
        p = z @ W.T + b
        pres.append(p)
        z = np.maximum(p, 0.0)
    return pres


def box_points(lo, hi, m, rng, grid=None):
    """Corners + random points (+ optional full grid) of a box."""
    n = lo.shape[0]
    corners = np.array(list(itertools.product([0.0, 1.0], repeat=n)))
    pts = [corners, rng.random((m, n))]
    if grid:
        g = np.linspace(0, 1, grid)
        pts.append(np.stack(np.meshgrid(*[g] * n, indexing="ij"), -1).reshape(-1, n))
    t = np.concatenate(pts)
    return t, lo + t * (hi - lo)


def poisoned_workspace(torch, net, n_boxes, **opts):
    """A device workspace for bern_bounds filled with 0xFF bytes (NaN in FP32
    and FP64): a kernel that reads scratch it did not write first turns the
    bounds into NaN instead of silently reusing a previous run's values."""
    total, _ = net.workspace_size(n_boxes, **opts)
    return torch.full((total + 256,), 255, dtype=torch.uint8, device="cuda:0")
