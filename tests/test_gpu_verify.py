"""Branch and bound (bern_verify) decisions against the FP64 oracle: every
decided box of the decision log is re-bounded by the oracle one box at a
time. A box verified for "output <= threshold" must be verified by the
oracle's bounds too, a violating box violating (FP32 padded bounds contain
the oracle's, so the oracle's decision follows; in FP64 mode the bounds match
the oracle's within 1e-9 and decisions agree away from the threshold), and
the logged boxes partition the input box."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2211_14438_amd import workloads as wl
from tests import helpers as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_14438_amd import bernnn as B  # noqa: E402


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_verify_decisions_match_oracle(precision):
    case = wl.random_net_case([2, 8, 8, 1], seed=91, n_boxes=1, half_width=0.5)
    net = B.Net(case.Ws, case.bs)
    g = np.linspace(0.0, 1.0, 101)
    t = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    x = case.box_lo[0] + t * (case.box_hi[0] - case.box_lo[0])
    f = H.forward(case.Ws, case.bs, x)[-1][:, 0]
    tau = float(np.median(f))
    r = B.verify(net, case.box_lo, case.box_hi, 0, tau, max_rounds=8, max_boxes=4096, precision=precision,
                 log_cap=20000)
    net.close()
    log = r["log"]
    st = log["status"]
    print({k: r[k] for k in ("verified", "violated", "undecided", "rounds", "boxes_bounded")}, "logged", st.size,
          flush=True)
    assert (st == 1).any() and (st == -1).any()
    # the logged boxes partition the input box
    vol = np.prod(log["hi"] - log["lo"], axis=1).sum()
    assert abs(vol - np.prod(case.box_hi[0] - case.box_lo[0])) <= 1e-12 * vol
    rng = np.random.default_rng(3)
    pick = []
    for s in (1, -1, 0):
        idx = np.nonzero((st == s) & np.isfinite(log["out_lo"]))[0]
        pick += list(rng.choice(idx, size=min(12, idx.size), replace=False))
    for k in pick:
        o = orc.network(case.Ws, case.bs, log["lo"][k], log["hi"][k], L=2)
        olo, ohi = o["out_lo"][0], o["out_hi"][0]
        glo, ghi = log["out_lo"][k], log["out_hi"][k]
        scale = max(abs(olo), abs(ohi), ohi - olo, 1e-12)
        if precision == "fp32":
            assert glo <= olo and ghi >= ohi, k
            assert (olo - glo) <= 1e-4 * scale and (ghi - ohi) <= 1e-4 * scale, k
        else:
            assert abs(glo - olo) <= 1e-9 * scale and abs(ghi - ohi) <= 1e-9 * scale, k
        if st[k] == 1:
            assert ohi <= tau + (1e-9 * scale if precision == "fp64" else 0.0), k
        elif st[k] == -1:
            assert olo > tau - (1e-9 * scale if precision == "fp64" else 0.0), k
        else:
            assert olo <= tau + 1e-9 * scale and ohi > tau - 1e-9 * scale, k


def _host_rounds(net, lo, hi, k, tau, max_rounds, max_boxes, precision):
    """The same branch and bound with the rounds driven from the host: each
    round bounds the pending boxes with bounds_host, decides them and
    bisects the open ones (widest dimension, lowest index on ties) in box
    order; returns the fractions and the decision log."""
    total = np.prod(hi - lo, axis=1).sum()
    frac = dict(verified=0.0, violated=0.0, undecided=0.0)
    log = dict(lo=[], hi=[], out_lo=[], out_hi=[], status=[])
    for rnd in range(max_rounds):
        r = B.bounds_host(net, lo, hi, precision=precision)
        blo, bhi = r["out_lo"][:, k], r["out_hi"][:, k]
        st = np.where(bhi <= tau, 1, np.where(blo > tau, -1, 0)).astype(np.int8)
        vol = np.prod(hi - lo, axis=1) / total
        frac["verified"] += vol[st == 1].sum()
        frac["violated"] += vol[st == -1].sum()
        op = np.nonzero(st == 0)[0]
        split = rnd + 1 < max_rounds and 2 * op.size <= max_boxes
        for b in np.nonzero(st != 0)[0]:
            for key, v in (("lo", lo[b]), ("hi", hi[b]), ("out_lo", blo[b]), ("out_hi", bhi[b]), ("status", st[b])):
                log[key].append(v)
        if not split:
            frac["undecided"] += vol[op].sum()
            for b in op:
                for key, v in (("lo", lo[b]), ("hi", hi[b]), ("out_lo", blo[b]), ("out_hi", bhi[b]), ("status", 0)):
                    log[key].append(v)
            break
        w = np.argmax(hi[op] - lo[op], axis=1)
        mid = 0.5 * (lo[op, w] + hi[op, w])
        nlo = np.repeat(lo[op], 2, axis=0)
        nhi = np.repeat(hi[op], 2, axis=0)
        nhi[0::2][np.arange(op.size), w] = mid
        nlo[1::2][np.arange(op.size), w] = mid
        lo, hi = nlo, nhi
        if op.size == 0:
            break
    return frac, {key: np.array(v) for key, v in log.items()}


@pytest.mark.parametrize("precision,max_boxes", [("fp64", 4096), ("fp32", 300)])
def test_verify_device_rounds_match_host_rounds(precision, max_boxes):
    """The device-resident rounds decide, bisect and log exactly as rounds
    driven from the host over bounds_host do (the boxes bit for bit, the
    fractions up to summation order), also when max_boxes stops the
    splitting early (300)."""
    case = wl.random_net_case([3, 10, 10, 2], seed=17, n_boxes=3, half_width=0.4)
    net = B.Net(case.Ws, case.bs)
    x = case.box_lo[0] + np.random.default_rng(5).random((2000, 3)) * (case.box_hi[0] - case.box_lo[0])
    tau = float(np.median(H.forward(case.Ws, case.bs, x)[-1][:, 1]))
    r = B.verify(net, case.box_lo, case.box_hi, 1, tau, max_rounds=7, max_boxes=max_boxes, precision=precision,
                 log_cap=100000)
    frac, log = _host_rounds(net, case.box_lo.copy(), case.box_hi.copy(), 1, tau, 7, max_boxes, precision)
    net.close()
    print({k: r[k] for k in ("verified", "violated", "undecided", "rounds", "boxes_bounded")}, flush=True)
    for key in ("verified", "violated", "undecided"):
        assert abs(r[key] - frac[key]) <= 1e-12, (key, r[key], frac[key])
    assert r["log"]["status"].size == log["status"].size
    for key in ("lo", "hi", "out_lo", "out_hi", "status"):
        assert np.array_equal(r["log"][key], log[key]), key
