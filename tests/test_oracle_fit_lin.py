"""Pins of the oracle's linear fallback (reading R9: least-squares affine fit
of the Bernstein control net plus the extreme remainder) and of the periodic
linearisation Lin (Section 5.4, reading R13), against things other than the
oracle itself: numpy's least-squares solver on the control net, affine
functions the fit must reproduce exactly (linear precision of the Bernstein
form), a hand-worked example, the reduction at L = 1, the degree law and
brute-force sampling of the network."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2211_14438_amd import workloads as wl
from tests import helpers as H

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(n, d):
    """Control-net abscissae K/d of a degree-d tensor, last variable fastest."""
    K = np.array(list(itertools.product(range(d + 1), repeat=n)), dtype=np.float64).reshape(-1, n)
    return K / d


def _lstsq_line(n, d, B):
    """The least-squares affine function of the control net {(K/d, B_K)},
    solved by numpy: l(t) = beta0 + sum_a beta_a (t_a - 1/2)."""
    X = np.hstack([np.ones((B.size, 1)), _grid(n, d) - 0.5])
    beta, *_ = np.linalg.lstsq(X, B, rcond=None)
    return beta


CASES = [(1, 1), (1, 3), (2, 2), (3, 2), (2, 4), (4, 1), (3, 3), (6, 2)]


@pytest.mark.parametrize("n,d", CASES)
def test_fit_is_the_least_squares_solution(n, d):
    rng = np.random.default_rng(10 * n + d)
    for _ in range(3):
        B = rng.standard_normal((d + 1) ** n) * rng.uniform(0.1, 10.0)
        ref = _lstsq_line(n, d, B)
        got = orc.ls_affine(n, d, B)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(B).max()


@pytest.mark.parametrize("n,d", CASES)
def test_linearisation_adds_the_extreme_remainder(n, d):
    """Upper: l + max_K (B_K - l(K/d)); lower: l + min; written as a degree-1
    Bernstein tensor, whose coefficients are the values at the box corners."""
    rng = np.random.default_rng(7 * n + d)
    B = rng.standard_normal((d + 1) ** n)
    beta = _lstsq_line(n, d, B)
    line = lambda t: beta[0] + (t - 0.5) @ beta[1:]  # noqa: E731
    rem = B - line(_grid(n, d))
    corners = _grid(n, 1)
    for sign, ext in ((+1, rem.max()), (-1, rem.min())):
        got = orc.linearize(n, d, B, sign)
        assert np.max(np.abs(got - (line(corners) + ext))) <= 1e-12 * np.abs(B).max()


@pytest.mark.parametrize("n,d", CASES)
def test_linearisation_reproduces_affine_functions(n, d):
    """By linear precision the control net of an affine f at degree d is
    f(K/d): the fit is f itself and the remainder zero, for either sign."""
    rng = np.random.default_rng(3 * n + d)
    a0, a = rng.standard_normal(), rng.standard_normal(n)
    B = a0 + _grid(n, d) @ a
    want = a0 + _grid(n, 1) @ a
    for sign in (+1, -1):
        assert np.max(np.abs(orc.linearize(n, d, B, sign) - want)) <= 1e-13 * (abs(a0) + np.abs(a).sum())


@pytest.mark.parametrize("n,d", [(1, 4), (2, 3), (3, 2)])
def test_linearisation_encloses_the_polynomial(n, d):
    """Def. 2 applied to P - l: the upper line lies above the polynomial and
    the lower one below it, at sampled points."""
    rng = np.random.default_rng(n + 5 * d)
    B = rng.standard_normal((d + 1) ** n)
    t = rng.random((3000, n))
    p = H.bern_eval(n, d, B, t)
    up = H.bern_eval(n, 1, orc.linearize(n, d, B, +1), t)
    lo = H.bern_eval(n, 1, orc.linearize(n, d, B, -1), t)
    assert np.all(up >= p - 1e-12) and np.all(lo <= p + 1e-12)


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


def test_lin_worked_example():
    for s, olo, ohi in _golden("worked_example_lin.txt"):
        Ws = [np.array([[1.0]]), np.array([[s]])]
        bs = [np.array([0.0]), np.array([0.0])]
        r = orc.network(Ws, bs, np.array([-6.0]), np.array([10.0]), L=2, lin=1)
        assert r["out_lo"][0] == pytest.approx(olo, abs=1e-12)
        assert r["out_hi"][0] == pytest.approx(ohi, abs=1e-12)
        assert r["out_deg"] == 1
        # without Lin: the worked example of the plain method
        r0 = orc.network(Ws, bs, np.array([-6.0]), np.array([10.0]), L=2, lin=0)
        assert r0["out_lo"][0] == pytest.approx(-2.34375 if s > 0 else -10.0, abs=1e-12)


@pytest.mark.parametrize("lin", [1, 2])
def test_lin_changes_nothing_at_order_one(lin):
    """L = 1 keeps every post polynomial affine (degree 1), so its
    linearisation is itself: the bounds equal those without Lin."""
    case = wl.random_net_case([3, 6, 5, 4, 2], seed=17, n_boxes=3)
    for i in range(case.n_boxes):
        a = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=1, lin=0)
        b = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=1, lin=lin)
        for k in ("neuron_lo", "neuron_hi", "out_lo", "out_hi"):
            scale = np.maximum(np.abs(a[k]), 1.0)
            assert np.max(np.abs(a[k] - b[k]) / scale) <= 1e-12, k


@pytest.mark.parametrize("L,lin,H_hidden", [(2, 1, 3), (2, 2, 3), (3, 2, 2), (2, 3, 3), (3, 1, 1)])
def test_lin_degree_law(L, lin, H_hidden):
    """The output polynomials carry degree L^((H-1) mod Lin) (1 when the last
    hidden layer is linearised)."""
    widths = [2] + [4] * H_hidden + [1]
    case = wl.random_net_case(widths, seed=5, n_boxes=1)
    r = orc.network(case.Ws, case.bs, case.box_lo[0], case.box_hi[0], L=L, lin=lin)
    assert r["out_deg"] == L ** (H_hidden % lin)


@pytest.mark.parametrize("L,lin", [(2, 1), (2, 2), (3, 1), (4, 2)])
def test_lin_bounds_are_sound_by_sampling(L, lin):
    case = wl.random_net_case([2, 6, 6, 6, 2], seed=23 + L + lin, n_boxes=2, half_width=0.6)
    rng = np.random.default_rng(9)
    for i in range(case.n_boxes):
        r = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=L, lin=lin)
        _, x = H.box_points(case.box_lo[i], case.box_hi[i], 4000, rng, grid=41)
        pres = H.forward(case.Ws, case.bs, x)
        hid = np.concatenate(pres[:-1], axis=1)
        assert np.all(hid >= r["neuron_lo"] - 1e-9) and np.all(hid <= r["neuron_hi"] + 1e-9)
        assert np.all(pres[-1] >= r["out_lo"] - 1e-9) and np.all(pres[-1] <= r["out_hi"] + 1e-9)


def test_lin_layers_before_the_first_linearisation_are_unchanged():
    """Lin acts after hidden layer Lin: every pre-activation bound up to and
    including that layer is the plain method's."""
    case = wl.random_net_case([3, 5, 5, 5, 2], seed=31, n_boxes=2)
    for i in range(case.n_boxes):
        a = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=2, lin=0)
        b = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=2, lin=2)
        assert np.array_equal(a["neuron_lo"][:10], b["neuron_lo"][:10])
        assert np.array_equal(a["neuron_hi"][:10], b["neuron_hi"][:10])
