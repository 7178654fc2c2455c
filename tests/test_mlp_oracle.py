"""Pins of the predictor's FP64 MLP oracle: analytic gradients against central
finite differences of the loss, and the loss's closed form at zero output
weights (uniform softmax: log 4)."""
import numpy as np

from oracle import mlp_oracle as M


def _params(rng):
    P = np.zeros(M.N_PARAMS)
    P[slice(*M.OFF["mean"])] = rng.standard_normal(8) * 0.1
    P[slice(*M.OFF["std"])] = 0.5 + rng.random(8)
    for k, s in (("W1", 0.5), ("b1", 0.1), ("W2", 0.2), ("b2", 0.1), ("W3", 0.3), ("b3", 0.1)):
        a, b = M.OFF[k]
        P[a:b] = rng.standard_normal(b - a) * s
    return P


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = _params(rng)
    X = rng.standard_normal((40, 8))
    y = rng.integers(0, 4, 40)
    G = M.grad(P, X, y)
    idx = np.concatenate([rng.choice(np.arange(16, M.N_PARAMS), 60, replace=False), [M.N_PARAMS - 1]])
    for i in idx:
        h = 1e-6
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (M.loss(Pp, X, y) - M.loss(Pm, X, y)) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, G[i])
    assert np.all(G[:16] == 0.0)


def test_uniform_softmax_loss():
    rng = np.random.default_rng(1)
    P = _params(rng)
    P[slice(*M.OFF["W3"])] = 0.0
    P[slice(*M.OFF["b3"])] = 0.0
    X = rng.standard_normal((10, 8))
    assert M.loss(P, X, rng.integers(0, 4, 10)) == np.log(4.0)
