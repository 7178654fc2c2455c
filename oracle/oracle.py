"""Python access to the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module. It wraps ``liboracle.so`` built from
``bernnn_oracle.c`` with ctypes and converts numpy arrays; no arithmetic of the
method happens here.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_d = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int)
_pi8 = ctypes.POINTER(ctypes.c_int8)
_ll = ctypes.c_longlong


def _builder():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_oracle_build", os.path.join(HERE, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def use_native():
    """Switch to a copy of the oracle compiled with -O3 -march=native on this
    host (built now; the same source). Must be called before the first use."""
    global _LIB
    if _LIB is not None and getattr(_LIB, "_native", False):
        return
    if _LIB is not None:
        raise RuntimeError("the oracle library is already loaded")
    _builder().build_native()
    lib(native=True)


def lib(native=False):
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle_native.so" if native else "liboracle.so")
        if not os.path.exists(path):
            _builder().build()
        L = ctypes.CDLL(path)
        L._native = native
        L.orc_binom.restype = _d
        L.orc_binom.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_tsize.restype = _ll
        L.orc_tsize.argtypes = [ctypes.c_int, ctypes.c_int]
        for name in ("orc_prod", "orc_prod_bern", "orc_sum_bern"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int, _pd, _pd]
        L.orc_elevate.restype = ctypes.c_int
        L.orc_elevate.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int, _pd]
        L.orc_pow_bern.restype = ctypes.c_int
        L.orc_pow_bern.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int, _pd]
        L.orc_power_to_bern.restype = ctypes.c_int
        L.orc_power_to_bern.argtypes = [ctypes.c_int, ctypes.c_int, _pd, _pd]
        L.orc_bern_eval.restype = _d
        L.orc_bern_eval.argtypes = [ctypes.c_int, ctypes.c_int, _pd, _pd]
        L.orc_relu_bern_coefs.restype = None
        L.orc_relu_bern_coefs.argtypes = [_d, _d, ctypes.c_int, _pd]
        L.orc_bern_to_power_1d.restype = None
        L.orc_bern_to_power_1d.argtypes = [ctypes.c_int, _pd, _pd]
        L.orc_bern_eval_1d.restype = _d
        L.orc_bern_eval_1d.argtypes = [ctypes.c_int, _pd, _d]
        L.orc_relu_poly.restype = None
        L.orc_relu_poly.argtypes = [_d, _d, ctypes.c_int, _pd, _pd]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        L.orc_network.restype = ctypes.c_int
        L.orc_network.argtypes = [ctypes.c_int, _pi, _pd, _pd, _pd, _pd, ctypes.c_int, _pi8,
                                  _pd, _pd, _pd, _pd, _pd, _pi, _pd, _pd, _ll, _pi8, ctypes.c_int]
        L.orc_ls_affine.restype = None
        L.orc_ls_affine.argtypes = [ctypes.c_int, ctypes.c_int, _pd, _pd]
        L.orc_linearize.restype = None
        L.orc_linearize.argtypes = [ctypes.c_int, ctypes.c_int, _pd, ctypes.c_int, _pd]
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(_pd)


def _c(a, dt=np.float64):
    return np.ascontiguousarray(a, dtype=dt)


class OracleError(RuntimeError):
    pass


def _check(st):
    if st != 0:
        raise OracleError(f"oracle status {st}")


def binom(n, k):
    return lib().orc_binom(n, k)


def tsize(n, d):
    return lib().orc_tsize(n, d)


def prod(n, da, A, db, B):
    A, B = _c(A), _c(B)
    out = np.zeros(tsize(n, da + db))
    _check(lib().orc_prod(n, da, _p(A), db, _p(B), _p(out)))
    return out


def prod_bern(n, da, A, db, B):
    A, B = _c(A), _c(B)
    out = np.zeros(tsize(n, da + db))
    _check(lib().orc_prod_bern(n, da, _p(A), db, _p(B), _p(out)))
    return out


def sum_bern(n, da, A, db, B):
    A, B = _c(A), _c(B)
    out = np.zeros(tsize(n, max(da, db)))
    _check(lib().orc_sum_bern(n, da, _p(A), db, _p(B), _p(out)))
    return out


def elevate(n, d, A, e):
    A = _c(A)
    out = np.zeros(tsize(n, e))
    _check(lib().orc_elevate(n, d, _p(A), e, _p(out)))
    return out


def pow_bern(n, d, A, i):
    A = _c(A)
    out = np.zeros(max(tsize(n, i * d), 1))
    _check(lib().orc_pow_bern(n, d, _p(A), i, _p(out)))
    return out


def power_to_bern(n, d, a):
    a = _c(a)
    out = np.zeros(tsize(n, d))
    _check(lib().orc_power_to_bern(n, d, _p(a), _p(out)))
    return out


def bern_eval(n, d, B, t):
    B, t = _c(B), _c(t)
    return lib().orc_bern_eval(n, d, _p(B), _p(t))


def relu_bern_coefs(lo, hi, L):
    out = np.zeros(L + 1)
    lib().orc_relu_bern_coefs(lo, hi, L, _p(out))
    return out


def bern_to_power_1d(L, b):
    b = _c(b)
    out = np.zeros(L + 1)
    lib().orc_bern_to_power_1d(L, _p(b), _p(out))
    return out


def bern_eval_1d(L, b, u):
    b = _c(b)
    return lib().orc_bern_eval_1d(L, _p(b), u)


def relu_poly(lo, hi, L):
    c = np.zeros(L + 1)
    e = np.zeros(1)
    lib().orc_relu_poly(lo, hi, L, _p(c), _p(e))
    return c, float(e[0])


def set_threads(t):
    lib().orc_set_threads(int(t))


def get_threads():
    return lib().orc_get_threads()


def ls_affine(n, d, B):
    """Least-squares affine fit of the Bernstein control net of B (degree d):
    beta[0] + sum_a beta[1+a] (t_a - 1/2)."""
    B = _c(B)
    beta = np.zeros(n + 1)
    lib().orc_ls_affine(n, d, _p(B), _p(beta))
    return beta


def linearize(n, d, P, sign):
    """Degree-1 Bernstein tensor of the linear fallback of P (sign +1: upper,
    -1: lower)."""
    P = _c(P)
    out = np.zeros(tsize(n, 1))
    lib().orc_linearize(n, d, _p(P), int(sign), _p(out))
    return out


def network(Ws, bs, box_lo, box_hi, L=2, plan=None, want_polys=False, lin=0):
    """Bounds of one box (Problem 1). ``Ws``/``bs`` are lists of per-layer
    arrays (W^(i) of shape h_i x h_{i-1}). Returns a dict with the hidden
    pre-activation bounds, output bounds, relative volume, output degree, the
    per-neuron degree actually used and (optionally) the output Bernstein
    tensors. ``lin`` > 0 linearises every lin-th hidden layer's post
    polynomials."""
    H = len(Ws)
    widths = np.array([Ws[0].shape[1]] + [w.shape[0] for w in Ws], dtype=np.int32)
    n = int(widths[0])
    W = _c(np.concatenate([np.asarray(w, dtype=np.float64).ravel() for w in Ws]))
    b = _c(np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in bs]))
    lo_, hi_ = _c(box_lo), _c(box_hi)
    nh = int(widths[1:H].sum())
    o = int(widths[H])
    nlo, nhi = np.zeros(max(nh, 1)), np.zeros(max(nh, 1))
    olo, ohi, rv = np.zeros(o), np.zeros(o), np.zeros(o)
    deg = np.zeros(1, dtype=np.int32)
    used = np.zeros(max(nh, 1), dtype=np.int8)
    planp = None
    if plan is not None:
        plan = _c(plan, np.int8)
        planp = plan.ctypes.data_as(_pi8)
    cap = 0
    oU = oL = None
    if want_polys:
        # capacity for the largest degree this call can reach
        Lmax = L if plan is None else max(1, int(plan.max()))
        dmax = Lmax ** (H - 1) if lin == 0 else Lmax ** max(1, min(H - 1, lin))
        cap = o * tsize(n, dmax)
        oU, oL = np.zeros(cap), np.zeros(cap)
    st = lib().orc_network(H, widths.ctypes.data_as(_pi), _p(W), _p(b), _p(lo_), _p(hi_), int(L), planp,
                           _p(nlo), _p(nhi), _p(olo), _p(ohi), _p(rv), deg.ctypes.data_as(_pi),
                           _p(oU) if oU is not None else None, _p(oL) if oL is not None else None,
                           cap, used.ctypes.data_as(_pi8), int(lin))
    _check(st)
    res = dict(neuron_lo=nlo[:nh], neuron_hi=nhi[:nh], out_lo=olo, out_hi=ohi, rel_vol=rv,
               out_deg=int(deg[0]), used_plan=used[:nh])
    if want_polys:
        c = tsize(n, res["out_deg"])
        res["out_U"] = oU[: o * c].reshape(o, c)
        res["out_L"] = oL[: o * c].reshape(o, c)
    return res


def network_boxes(Ws, bs, box_lo, box_hi, L=2, plan=None):
    """``network`` over many boxes; returns stacked arrays."""
    box_lo = np.atleast_2d(box_lo)
    box_hi = np.atleast_2d(box_hi)
    res = []
    for i in range(box_lo.shape[0]):
        res.append(network(Ws, bs, box_lo[i], box_hi[i], L=L,
                           plan=None if plan is None else plan[i]))
    return {k: np.stack([r[k] for r in res]) for k in ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "rel_vol")}
