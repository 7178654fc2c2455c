"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a value the
paper prints, a closed form, a mathematical identity evaluated at points with
independent numpy code, a textbook special case, or brute-force sampling of
the network. None of these needs a GPU.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2211_14438_amd import workloads as wl
from tests import helpers as H

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


# ----------------------------------------------------------- ReLU approximant

def test_table1_relu_area():
    """Table 1: area between over- and under-approximant on [-6,10] is
    (hi-lo) * B(0) (Prop. 2 shift is constant); the paper prints one decimal."""
    for L, area in _golden("table1_relu_area.txt"):
        _, e = orc.relu_poly(-6.0, 10.0, int(L))
        assert round(16.0 * e, 1) == pytest.approx(area, abs=1e-12)
    c, e = orc.relu_poly(-6.0, 10.0, 2)
    assert np.allclose(c, [0.0, 4.0, 6.0], atol=1e-14)
    assert e == pytest.approx(2.34375, abs=1e-15)


@pytest.mark.parametrize("lo,hi", [(-6.0, 10.0), (-1.0, 0.3), (-0.01, 5.0), (-3.0, 3.0)])
@pytest.mark.parametrize("L", [1, 2, 3, 5, 8])
def test_relu_over_under_invariants(lo, hi, L):
    """Prop. 1 (B >= sigma), Prop. 2 (B - B(0) <= sigma, max error at 0),
    interpolation at the ends, and power form == Bernstein form (Step 2)."""
    c, e = orc.relu_poly(lo, hi, L)
    b = orc.relu_bern_coefs(lo, hi, L)
    y = np.unique(np.concatenate([np.linspace(lo, hi, 2001), [0.0]]))
    u = (y - lo) / (hi - lo)
    # power series in u, evaluated with numpy's polyval (independent of the Bernstein form)
    Bp = np.polynomial.polynomial.polyval(u, c)
    Bb = np.array([sum(b[k] * H.comb(L, k) * uu ** k * (1 - uu) ** (L - k) for k in range(L + 1)) for uu in u])
    assert np.allclose(Bp, Bb, rtol=0, atol=1e-12 * max(1.0, hi))
    sig = np.maximum(y, 0.0)
    assert np.all(Bp >= sig - 1e-12)
    assert np.all(Bp - e <= sig + 1e-12)
    assert Bp[0] == pytest.approx(0.0, abs=1e-12)
    assert Bp[-1] == pytest.approx(hi, abs=1e-12)
    err = Bp - sig
    assert err.max() == pytest.approx(e, abs=1e-9 * max(1.0, hi))
    assert np.all(err[y < 0] <= e + 1e-12) and np.all(err[y > 0] <= e + 1e-12)


def test_relu_monotone_in_order():
    """B_{L+1} <= B_L pointwise (sigma convex), and the Table 1 area sequence
    16*B(0) = 60, 37.5, 28.125, 16.90, 12.15 for L = 1, 2, 3, 8, 16."""
    y = np.linspace(-6, 10, 801)
    prev = None
    for L in range(1, 17):
        b = orc.relu_bern_coefs(-6.0, 10.0, L)
        u = (y + 6) / 16
        B = sum(b[k] * H.comb(L, k) * u ** k * (1 - u) ** (L - k) for k in range(L + 1))
        if prev is not None:
            assert np.all(B <= prev + 1e-11)
        prev = B
    areas = {L: 16 * orc.relu_poly(-6.0, 10.0, L)[1] for L in (1, 2, 3, 8, 16)}
    assert areas[1] == pytest.approx(60.0, abs=1e-12)
    assert areas[2] == pytest.approx(37.5, abs=1e-12)
    assert areas[3] == pytest.approx(28.125, abs=1e-12)
    assert areas[8] == pytest.approx(16.8979, abs=1e-4)
    assert areas[16] == pytest.approx(12.1524, abs=1e-4)


def test_bern_to_power_point_evaluation():
    rng = np.random.default_rng(7)
    for L in (1, 2, 4, 7):
        b = rng.standard_normal(L + 1)
        c = orc.bern_to_power_1d(L, b)
        for u in rng.random(20):
            ref = sum(b[k] * H.comb(L, k) * u ** k * (1 - u) ** (L - k) for k in range(L + 1))
            assert np.polynomial.polynomial.polyval(u, c) == pytest.approx(ref, abs=1e-12)


# ------------------------------------------------------- basis change (Def. 2)

@pytest.mark.parametrize("n,d", [(1, 4), (2, 3), (3, 2), (4, 2), (2, 8)])
def test_power_to_bern_identities(n, d):
    rng = np.random.default_rng(n * 10 + d)
    a = rng.standard_normal(orc.tsize(n, d))
    b = orc.power_to_bern(n, d, a)
    t = rng.random((50, n))
    # same polynomial: Bernstein evaluation == power evaluation (independent numpy code)
    assert np.allclose(H.bern_eval(n, d, b, t), H.power_eval(n, d, a, t), atol=1e-11)
    # range enclosure (Def. 2)
    p = H.power_eval(n, d, a, rng.random((2000, n)))
    assert p.min() >= b.min() - 1e-12 and p.max() <= b.max() + 1e-12
    # end (corner) coefficients equal the polynomial at the box corners
    K = H.multi_indices(n, d)
    for idx, k in enumerate(K):
        if np.all((k == 0) | (k == d)):
            assert b[idx] == pytest.approx(H.power_eval(n, d, a, (k / d)[None])[0], abs=1e-11)


def test_power_to_bern_special_cases():
    n, d = 3, 4
    C = orc.tsize(n, d)
    K = H.multi_indices(n, d)
    a = np.zeros(C); a[0] = 2.5
    assert np.allclose(orc.power_to_bern(n, d, a), 2.5)               # constant
    for i in range(n):                                                # linear precision
        a = np.zeros(C)
        a[np.flatnonzero((K.sum(1) == 1) & (K[:, i] == 1))[0]] = 1.0
        assert np.allclose(orc.power_to_bern(n, d, a), K[:, i] / d)
    a = np.zeros(C); a[-1] = 1.0                                       # t^(d,...,d)
    b = orc.power_to_bern(n, d, a)
    assert b[-1] == 1.0 and np.allclose(b[:-1], 0.0)


# --------------------------------------------- Section 4 products and sums

def test_prod_point_evaluation():
    rng = np.random.default_rng(3)
    for n, da, db in [(1, 3, 2), (2, 2, 2), (3, 1, 2), (2, 4, 1)]:
        A = rng.standard_normal(orc.tsize(n, da)); B = rng.standard_normal(orc.tsize(n, db))
        t = rng.random((30, n))
        P = orc.prod(n, da, A, db, B)
        assert np.allclose(H.power_eval(n, da + db, P, t), H.power_eval(n, da, A, t) * H.power_eval(n, db, B, t),
                           rtol=1e-12, atol=1e-12)
        PB = orc.prod_bern(n, da, A, db, B)
        assert np.allclose(H.bern_eval(n, da + db, PB, t), H.bern_eval(n, da, A, t) * H.bern_eval(n, db, B, t),
                           rtol=1e-12, atol=1e-12)
        # Prop. 3 on Bernstein tensors equals the basis change of the power product
        a1 = rng.standard_normal(orc.tsize(n, da)); a2 = rng.standard_normal(orc.tsize(n, db))
        lhs = orc.prod_bern(n, da, orc.power_to_bern(n, da, a1), db, orc.power_to_bern(n, db, a2))
        rhs = orc.power_to_bern(n, da + db, orc.prod(n, da, a1, db, a2))
        assert np.allclose(lhs, rhs, atol=1e-12)


def test_pow_and_sum_bern_point_evaluation():
    rng = np.random.default_rng(4)
    n, d = 2, 2
    A = rng.standard_normal(orc.tsize(n, d)); B = rng.standard_normal(orc.tsize(n, 3))
    t = rng.random((30, n))
    for i in range(4):
        P = orc.pow_bern(n, d, A, i)
        assert np.allclose(H.bern_eval(n, i * d, P[: orc.tsize(n, i * d)], t), H.bern_eval(n, d, A, t) ** i,
                           atol=1e-12)
    S = orc.sum_bern(n, d, A, 3, B)
    assert np.allclose(H.bern_eval(n, 3, S, t), H.bern_eval(n, d, A, t) + H.bern_eval(n, 3, B, t), atol=1e-12)


def test_elevation_nesting_and_zero_pad():
    rng = np.random.default_rng(5)
    n, d = 3, 2
    a = rng.standard_normal(orc.tsize(n, d))
    b = orc.power_to_bern(n, d, a)
    lo, hi = b.min(), b.max()
    t = rng.random((20, n))
    for e in (3, 4, 6):
        be = orc.elevate(n, d, b, e)
        assert np.allclose(H.bern_eval(n, e, be, t), H.bern_eval(n, d, b, t), atol=1e-12)
        assert be.min() >= lo - 1e-12 and be.max() <= hi + 1e-12     # elevation nests
        # power-basis zero pad to degree e == Prop. 4 elevation
        pad = np.zeros((e + 1,) * n)
        pad[(slice(0, d + 1),) * n] = a.reshape((d + 1,) * n)
        assert np.allclose(orc.power_to_bern(n, e, pad.ravel()), be, atol=1e-12)


# --------------------------------------------------------- whole network

def _affine_range(a0, a):
    return a0 + np.minimum(a, 0).sum(), a0 + np.maximum(a, 0).sum()


def _linear_symbolic(Ws, bs, lo, hi):
    """Independent L = 1 propagator on affine forms in t (the linear
    relaxation Prop. 1 says degree 1 reduces to)."""
    n = lo.shape[0]
    w = hi - lo
    U = np.concatenate([lo[:, None], np.diag(w)], axis=1)   # x_i = lo_i + w_i t_i
    Lw = U.copy()
    hid = []
    for i, (W, b) in enumerate(zip(Ws, bs)):
        Wp, Wm = np.maximum(W, 0), np.minimum(W, 0)
        Uh = Wp @ U + Wm @ Lw; Uh[:, 0] += b
        Lh = Wp @ Lw + Wm @ U; Lh[:, 0] += b
        if i == len(Ws) - 1:
            olo = np.array([_affine_range(r[0], r[1:])[0] for r in Lh])
            ohi = np.array([_affine_range(r[0], r[1:])[1] for r in Uh])
            return hid, olo, ohi
        U2, L2 = np.zeros_like(Uh), np.zeros_like(Lh)
        for j in range(W.shape[0]):
            l = _affine_range(Lh[j, 0], Lh[j, 1:])[0]
            h = _affine_range(Uh[j, 0], Uh[j, 1:])[1]
            hid.append((l, h))
            if h <= 0:
                continue
            if l >= 0:
                U2[j], L2[j] = Uh[j], Lh[j]
                continue
            lam = h / (h - l)
            U2[j] = lam * Uh[j]; U2[j, 0] -= lam * l
            L2[j] = lam * Lh[j]
        U, Lw = U2, L2


@pytest.mark.parametrize("seed", range(6))
def test_L1_equals_linear_symbolic_propagation(seed):
    case = wl.random_net_case([3, 6, 5, 2], seed=50 + seed)
    r = orc.network(case.Ws, case.bs, case.box_lo[0], case.box_hi[0], L=1)
    hid, olo, ohi = _linear_symbolic(case.Ws, case.bs, case.box_lo[0], case.box_hi[0])
    assert np.allclose(r["neuron_lo"], [h[0] for h in hid], atol=1e-12)
    assert np.allclose(r["neuron_hi"], [h[1] for h in hid], atol=1e-12)
    assert np.allclose(r["out_lo"], olo, atol=1e-12) and np.allclose(r["out_hi"], ohi, atol=1e-12)
    assert r["out_deg"] == 1


def test_worked_example():
    for s, olo, ohi in _golden("worked_example_1neuron.txt"):
        r = orc.network([np.array([[1.0]]), np.array([[s]])], [np.zeros(1), np.zeros(1)],
                        np.array([-6.0]), np.array([10.0]), L=2, want_polys=True)
        assert r["out_lo"][0] == pytest.approx(olo, abs=1e-14)
        assert r["out_hi"][0] == pytest.approx(ohi, abs=1e-14)
    r = orc.network([np.array([[1.0]]), np.array([[1.0]])], [np.zeros(1), np.zeros(1)],
                    np.array([-6.0]), np.array([10.0]), L=2, want_polys=True)
    assert np.allclose(r["out_U"][0], [0, 2, 10]) and np.allclose(r["out_L"][0], [-2.34375, -0.34375, 7.65625])


def test_layer1_bounds_exact():
    case = wl.cfg2()
    r = orc.network(case.Ws, case.bs, case.box_lo[0], case.box_hi[0], L=2)
    W, b = case.Ws[0], case.bs[0]
    lo, hi = case.box_lo[0], case.box_hi[0]
    ex_lo = b + np.minimum(W * lo, W * hi).sum(1)
    ex_hi = b + np.maximum(W * lo, W * hi).sum(1)
    assert np.allclose(r["neuron_lo"][:20], ex_lo, atol=1e-14)
    assert np.allclose(r["neuron_hi"][:20], ex_hi, atol=1e-14)


def test_affine_and_all_stable_are_exact():
    rng = np.random.default_rng(9)
    lo, hi = np.array([-1.0, 0.0, 0.5]), np.array([0.5, 2.0, 1.0])
    W = rng.standard_normal((4, 3))
    b = rng.standard_normal(4)
    r = orc.network([W], [b], lo, hi, L=2)                                    # H = 1
    assert np.allclose(r["out_lo"], b + np.minimum(W * lo, W * hi).sum(1), atol=1e-13)
    assert np.allclose(r["out_hi"], b + np.maximum(W * lo, W * hi).sum(1), atol=1e-13)
    W1 = np.abs(rng.standard_normal((5, 3))); b1 = np.full(5, 10.0)           # every hidden neuron active
    W2 = rng.standard_normal((2, 5)); b2 = rng.standard_normal(2)
    r = orc.network([W1, W2], [b1, b2], lo, hi, L=3)
    We, be = W2 @ W1, W2 @ b1 + b2
    assert np.allclose(r["out_lo"], be + np.minimum(We * lo, We * hi).sum(1), atol=1e-12)
    assert np.allclose(r["out_hi"], be + np.maximum(We * lo, We * hi).sum(1), atol=1e-12)
    assert np.all(r["used_plan"] == -1)


def _check_sound(case, res, i_box, rng, grid=None, polys=True):
    lo, hi = case.box_lo[i_box], case.box_hi[i_box]
    t, x = H.box_points(lo, hi, 3000, rng, grid=grid)
    pres = H.forward(case.Ws, case.bs, x)
    hidden = np.concatenate(pres[:-1], axis=1) if len(pres) > 1 else np.zeros((x.shape[0], 0))
    tol = 1e-9
    assert np.all(hidden >= res["neuron_lo"] - tol) and np.all(hidden <= res["neuron_hi"] + tol)
    out = pres[-1]
    assert np.all(out >= res["out_lo"] - tol) and np.all(out <= res["out_hi"] + tol)
    if polys and "out_U" in res:
        n, d = case.n, res["out_deg"]
        Bt = H.bern_basis(n, d, t)
        U = Bt @ res["out_U"].T
        L = Bt @ res["out_L"].T
        assert np.all(L <= out + tol) and np.all(out <= U + tol)


def test_bruteforce_tiny_net_grid():
    """Every sample of a 101x101 grid (+ corners + random points) of the tiny
    network lies inside every reported bound, and the output polynomials
    enclose the network pointwise."""
    case = wl.cfg1()
    r = orc.network(case.Ws, case.bs, case.box_lo[0], case.box_hi[0], L=2, want_polys=True)
    _check_sound(case, r, 0, np.random.default_rng(0), grid=101)
    assert r["out_deg"] == 4


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("L", [1, 2, 3])
def test_bruteforce_random_nets(seed, L):
    case = wl.random_net_case([3, 8, 6, 2], seed=seed, n_boxes=2)
    for i in range(case.n_boxes):
        r = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=L, want_polys=True)
        _check_sound(case, r, i, np.random.default_rng(seed))
        assert r["out_deg"] == L ** 2


@pytest.mark.parametrize("seed", range(4))
def test_bruteforce_given_plans(seed):
    """Any per-neuron plan (degrees 1..3 and the linear fallback, code 0)
    yields sound bounds."""
    case = wl.random_net_case([3, 8, 6, 2], seed=20 + seed, n_boxes=2)
    rng = np.random.default_rng(seed)
    for i in range(case.n_boxes):
        plan = rng.integers(0, 4, size=case.n_hidden).astype(np.int8)
        r = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], plan=plan, want_polys=True)
        _check_sound(case, r, i, rng)


def test_fallback_everywhere_is_degree_one():
    case = wl.random_net_case([2, 6, 6, 1], seed=77, half_width=1.0)
    plan = np.zeros(case.n_hidden, dtype=np.int8)
    r = orc.network(case.Ws, case.bs, case.box_lo[0], case.box_hi[0], plan=plan, want_polys=True)
    assert r["out_deg"] <= 1
    _check_sound(case, r, 0, np.random.default_rng(1))


def test_given_uniform_plan_equals_plain_when_all_unstable():
    """With every hidden neuron unstable, a plan giving every neuron degree L
    is the plain rule."""
    Ws, bs = wl.make_net([2, 6, 4, 1], 11, law="uniform5")
    lo, hi = np.array([-1.0, -1.0]), np.array([1.0, 1.0])
    for L in (2, 3):
        rp = orc.network(Ws, bs, lo, hi, L=L)
        if not np.all(rp["used_plan"] == L):
            continue
        rg = orc.network(Ws, bs, lo, hi, plan=np.full(10, L, dtype=np.int8))
        for k in ("neuron_lo", "neuron_hi", "out_lo", "out_hi"):
            assert np.array_equal(rp[k], rg[k])


@pytest.mark.parametrize("L,H_", [(2, 3), (2, 4), (3, 3)])
def test_output_degree_law(L, H_):
    widths = [2] + [4] * (H_ - 1) + [1]
    case = wl.random_net_case(widths, seed=3)
    r = orc.network(case.Ws, case.bs, case.box_lo[0], case.box_hi[0], L=L)
    assert r["out_deg"] == L ** (H_ - 1)


def test_relative_volume_closed_form():
    """Relative volume (Section 6) from the Bernstein coefficients equals the
    exact integral of U - L by tensor Gauss-Legendre quadrature."""
    case = wl.random_net_case([2, 5, 4, 1], seed=8, half_width=0.8)
    r = orc.network(case.Ws, case.bs, case.box_lo[0], case.box_hi[0], L=2, want_polys=True)
    d = r["out_deg"]
    x, w = np.polynomial.legendre.leggauss(d + 1)
    x, w = (x + 1) / 2, w / 2
    T = np.stack(np.meshgrid(x, x, indexing="ij"), -1).reshape(-1, 2)
    Wq = np.outer(w, w).ravel()
    Bt = H.bern_basis(2, d, T)
    integral = Wq @ (Bt @ (r["out_U"][0] - r["out_L"][0]))
    assert r["rel_vol"][0] == pytest.approx(integral, rel=1e-12)


def test_invalid_inputs_rejected():
    Ws, bs = wl.make_net([2, 3, 1], 1)
    with pytest.raises(orc.OracleError):
        orc.network(Ws, bs, np.array([1.0, 0.0]), np.array([0.0, 1.0]), L=2)
    with pytest.raises(orc.OracleError):
        orc.network(Ws, bs, np.array([0.0, 0.0]), np.array([1.0, 1.0]), L=0)
    with pytest.raises(orc.OracleError):
        orc.network(Ws, bs, np.array([0.0, np.nan]), np.array([1.0, 1.0]), L=2)


def test_paper_fig4_weak_sanity():
    """Parity unpinned: 50 random [2,20,20,1] nets with U[-5,5] weights on
    [-1,1]^2 (Fig. 4 setting; the paper's seeds and precision are unknown).
    Median relative volume must be within a factor 2 of the paper's medians
    and decrease with L. Catches gross misreadings only."""
    paper = {2: 1823.96, 3: 1524.99, 4: 1348.26}
    med = {}
    for L in paper:
        v = []
        for s in range(50):
            Ws, bs = wl.make_net([2, 20, 20, 1], 1000 + s, law="uniform5")
            v.append(orc.network(Ws, bs, np.array([-1.0, -1.0]), np.array([1.0, 1.0]), L=L)["rel_vol"][0])
        med[L] = float(np.median(v))
        assert paper[L] / 2 < med[L] < paper[L] * 2
    assert med[2] > med[3] > med[4]
