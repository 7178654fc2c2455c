"""FP64 CPU oracle of the degree predictor's MLP (test infrastructure only).

Plain numpy forward and backward of the 8 -> 64 -> 64 -> 4 ReLU network with
a mean softmax cross-entropy loss, in the parameter layout the library uses:
mean[8], std[8], W1[64][8], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].
The GPU training kernels are checked against these gradients; these gradients
are checked against central finite differences of the loss.
"""
import numpy as np

F, H, C = 8, 64, 4
OFF = {}
_o = 0
for name, size in (("mean", F), ("std", F), ("W1", H * F), ("b1", H), ("W2", H * H), ("b2", H), ("W3", C * H),
                   ("b3", C)):
    OFF[name] = (_o, _o + size)
    _o += size
N_PARAMS = _o


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    g = {k: P[a:b] for k, (a, b) in OFF.items()}
    g["W1"] = g["W1"].reshape(H, F)
    g["W2"] = g["W2"].reshape(H, H)
    g["W3"] = g["W3"].reshape(C, H)
    return g


def forward(P, X):
    p = unpack(P)
    Xn = (np.asarray(X, np.float64) - p["mean"]) / p["std"]
    a1 = Xn @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, (Xn, a1, h1, a2, h2)


def loss(P, X, y):
    z, _ = forward(P, X)
    m = z.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z - m).sum(axis=1)) + m[:, 0]
    return float(np.mean(lse - z[np.arange(len(y)), y]))


def grad(P, X, y):
    """Gradient of `loss` w.r.t. every parameter (zero for mean/std)."""
    p = unpack(P)
    N = len(y)
    z, (Xn, a1, h1, a2, h2) = forward(P, X)
    e = np.exp(z - z.max(axis=1, keepdims=True))
    sm = e / e.sum(axis=1, keepdims=True)
    dz = sm.copy()
    dz[np.arange(N), y] -= 1.0
    dz /= N
    gW3 = dz.T @ h2
    gb3 = dz.sum(0)
    dh2 = (dz @ p["W3"]) * (a2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0)
    gW1 = dh1.T @ Xn
    gb1 = dh1.sum(0)
    G = np.zeros(N_PARAMS)
    for k, v in (("W1", gW1), ("b1", gb1), ("W2", gW2), ("b2", gb2), ("W3", gW3), ("b3", gb3)):
        a, b = OFF[k]
        G[a:b] = v.ravel()
    return G
