"""GPU tests of the box-batch scheduler's launch forms: graph capture and
replay of the plain rule, and the kernel-variant autotuner. Every result is
checked against the eager path (bitwise where the arithmetic order is the
same) and against the FP64 oracle (same tolerance as the parity tests:
|g - o| <= 1e-9 max(|o|, hi_o - lo_o))."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2211_14438_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_14438_amd import bernnn as B  # noqa: E402

DEV = "cuda:0"
KEYS = ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "used_plan")


def _np(r):
    torch.cuda.synchronize()
    return {k: r[k].cpu().numpy().copy() for k in KEYS}


def _oracle_close(case, g, L=2, tol=1e-9):
    for i in range(case.n_boxes):
        o = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=L)
        for k in ("out_lo", "out_hi"):
            scale = np.maximum(np.maximum(np.abs(o[k]), o["out_hi"] - o["out_lo"]), 1e-300)
            assert np.max(np.abs(g[k][i] - o[k]) / scale) <= tol, (i, k)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_match_eager(precision):
    case = wl.random_net_case([4, 12, 12, 3], seed=41, n_boxes=12)
    print(f"case {case.name} {precision}", flush=True)
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    kw = dict(L=2, precision=precision, sched="batched")
    eager = _np(B.bounds(net, lo, hi, **kw))
    g = B.bounds(net, lo, hi, graph=True, **kw)  # capture + first launch
    first = _np(g)
    for k in KEYS:
        assert np.array_equal(first[k], eager[k], equal_nan=True), k
    outputs = {k: g[k] for k in KEYS}
    ws = g["workspace"]
    rng = np.random.default_rng(7)
    for rep in range(3):
        # new boxes in the same input tensors, eager work in between, then a replay
        c = rng.uniform(-1, 1, size=case.box_lo.shape)
        w = rng.uniform(0.05, 0.4, size=(case.n_boxes, 1))
        lo.copy_(torch.tensor(c - w, device=DEV))
        hi.copy_(torch.tensor(c + w, device=DEV))
        ref = _np(B.bounds(net, lo, hi, **kw))
        rr = _np(B.bounds(net, lo, hi, graph=True, outputs=outputs, workspace=ws, **kw))
        for k in KEYS:
            assert np.array_equal(rr[k], ref[k], equal_nan=True), (rep, k)
    net.close()


def test_autotune_variants_agree_with_oracle():
    case = wl.random_net_case([3, 24, 24, 4], seed=43, n_boxes=6)
    print(f"case {case.name}", flush=True)
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    kw = dict(L=2, precision="fp64", sched="batched")
    base = _np(B.bounds(net, lo, hi, **kw))
    _oracle_close(case, base)
    variants = B.tune_variants()
    assert len(variants) == 4 and all(v >= 2 for v in variants)
    for q, nv in enumerate(variants):
        for v in range(nv):
            choice = [0] * len(variants)
            choice[q] = v
            B.tune_set(net, choice)
            assert B.tune_get(net) == choice
            r = _np(B.bounds(net, lo, hi, **kw))
            if q in (0, 1):  # affine-kernel tiles: same summation order, same bits
                for k in KEYS:
                    assert np.array_equal(r[k], base[k]), (q, v, k)
            else:
                _oracle_close(case, r)
    with pytest.raises(B.BernError):
        B.tune_set(net, [99, 0, 0, 0])
    B.tune_set(net, [0, 0, 0, 0])
    choice, ms = B.autotune(net, lo, hi, reps=2, **kw)
    assert all(0 <= c < nv for c, nv in zip(choice, variants)) and ms > 0
    assert B.tune_get(net) == choice
    _oracle_close(case, _np(B.bounds(net, lo, hi, **kw)))
    net.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grouped_compositions_match_one_item_per_wave(precision):
    """With many items (at least 65,536 per launch) the scatter and square
    compositions take groups of items per wave, their jobs built at once and
    each loaded ahead of the previous one's stores; the same boxes in waves
    small enough for one item per wave give the same bounds bit for bit (a
    per-neuron plan of orders 1 and 2 and the linear fallback, so both
    kernels run)."""
    case = wl.random_net_case([6, 64, 64, 4], seed=23, n_boxes=512)
    print(f"case {case.name} {precision}", flush=True)
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    plan = np.random.default_rng(4).integers(0, 3, size=(case.n_boxes, case.n_hidden)).astype(np.int8)
    kw = dict(L=2, precision=precision, sched="batched", plan="given", degree_plan=torch.tensor(plan, device=DEV))
    grouped = _np(B.bounds(net, lo, hi, **kw))  # one wave: 512 x 64 x 2 items
    single = _np(B.bounds(net, lo, hi, max_wave=128, **kw))  # 16,384 items per wave
    used = grouped["used_plan"][:, :case.n_hidden]
    assert (used == 1).any() and (used == 2).any() and (used == -2).any()
    for k in KEYS:
        assert np.array_equal(grouped[k], single[k], equal_nan=True), k
    net.close()
