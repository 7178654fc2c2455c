"""Full-size runs of the measured workloads, in the launch configuration
bench.py times (batched waves, FP32 padded), checked on 16 seeded boxes each
against the FP64 oracle (one box at a time) and on every box by properties
that hold at any size: sampled network values inside the reported bounds
(soundness, no slack) and per-neuron bounds ordered lo <= hi.

FP32 tolerance (as in the parity tests): each GPU interval contains the
oracle's and is at most 1e-4 * max(|o|, hi_o - lo_o) wider per side."""
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
from paper_2211_14438_amd import predictor as PR  # noqa: E402

DEV = "cuda:0"
KEYS = ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "used_plan")


def _run(case, **kw):
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    ws = H.poisoned_workspace(torch, net, case.n_boxes, L=case.L, precision="fp32", sched="batched",
                              **{k: v for k, v in kw.items() if k in ("plan", "pred")})
    r = B.bounds(net, lo, hi, L=case.L, precision="fp32", sched="batched", workspace=ws, **kw)
    torch.cuda.synchronize()
    out = {k: r[k].cpu().numpy() for k in KEYS}
    net.close()
    return out


def _check_box_fp32(g, i, o, nh):
    for k_lo, k_hi, n in (("neuron_lo", "neuron_hi", nh), ("out_lo", "out_hi", None)):
        glo, ghi = g[k_lo][i][:n], g[k_hi][i][:n]
        olo, ohi = o[k_lo][:n], o[k_hi][:n]
        scale = np.maximum(np.maximum(np.abs(olo), np.abs(ohi)), ohi - olo)
        scale = np.where(scale > 0, scale, 1.0)
        assert np.all(glo <= olo + 1e-12 * scale) and np.all(ghi >= ohi - 1e-12 * scale), k_lo
        assert np.max((olo - glo) / scale) <= 1e-4 and np.max((ghi - ohi) / scale) <= 1e-4, k_lo


def _check_sound_all(case, g, m=400, seed=0):
    """FP32 padded bounds are rigorous: every sampled value of every box lies
    inside them, with no slack."""
    rng = np.random.default_rng(seed)
    nh = case.n_hidden
    assert np.all(g["neuron_lo"][:, :nh] <= g["neuron_hi"][:, :nh]) and np.all(g["out_lo"] <= g["out_hi"])
    for i in range(case.n_boxes):
        _, x = H.box_points(case.box_lo[i], case.box_hi[i], m, rng)
        pres = H.forward(case.Ws, case.bs, x)
        hid = np.concatenate(pres[:-1], axis=1)
        assert np.all(hid >= g["neuron_lo"][i][:nh]) and np.all(hid <= g["neuron_hi"][i][:nh]), i
        assert np.all(pres[-1] >= g["out_lo"][i]) and np.all(pres[-1] <= g["out_hi"][i]), i


def _sample(case, k=16, seed=0):
    """k seeded box indices of the workload (first and last included)."""
    rest = np.random.default_rng(seed).choice(np.arange(1, case.n_boxes - 1), size=k - 2, replace=False)
    return [0] + sorted(int(i) for i in rest) + [case.n_boxes - 1]


def test_learned_workload_full_size():
    case = wl.cfg5()  # 1024 boxes, [6,64,64,64,4], L = 2
    print(f"case {case.name}", flush=True)
    pred = PR.load_predictor()
    g = _run(case, plan="learned", pred=pred)
    pred.close()
    _check_sound_all(case, g, m=200)
    used = g["used_plan"]
    for i in _sample(case, seed=5):  # sampled boxes against the oracle under the plan the GPU took
        plan = np.where(used[i] >= 1, used[i], np.where(used[i] == -2, 0, 1)).astype(np.int8)
        o = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=case.L, plan=plan)
        assert np.array_equal(used[i], o["used_plan"]), i
        _check_box_fp32(g, i, o, case.n_hidden)


def test_batched_plain_workload_full_size():
    case = wl.cfg4()  # 256 boxes, [8,100,100,10], L = 2
    print(f"case {case.name}", flush=True)
    g = _run(case)
    _check_sound_all(case, g, m=100)
    for i in _sample(case, seed=4):
        o = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=case.L)
        _check_box_fp32(g, i, o, case.n_hidden)


def test_given_plan_workload_full_size():
    case = wl.cfg3()  # 1024 cells of [-1,1]^6, [6,50,50,4], L = 3, codes from {1,2,3}
    print(f"case {case.name}", flush=True)
    g = _run(case, plan="given", degree_plan=torch.tensor(case.plan, dtype=torch.int8, device=DEV))
    _check_sound_all(case, g, m=100)
    for i in _sample(case, seed=3):
        o = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=case.L, plan=case.plan[i])
        assert np.array_equal(g["used_plan"][i], o["used_plan"]), i
        _check_box_fp32(g, i, o, case.n_hidden)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_degenerate_boxes(precision):
    """Boxes of zero width along some or all axes (the polynomials lose those
    variables; a point box makes every neuron stable), next to ordinary ones."""
    case = wl.random_net_case([3, 9, 7, 2], seed=91, n_boxes=5)
    lo, hi = case.box_lo.copy(), case.box_hi.copy()
    hi[0] = lo[0]              # a point
    hi[1, 0] = lo[1, 0]        # one flat axis
    hi[2, :2] = lo[2, :2]      # two flat axes
    case.box_lo, case.box_hi = lo, hi
    net = B.Net(case.Ws, case.bs)
    r = B.bounds(net, torch.tensor(lo, device=DEV), torch.tensor(hi, device=DEV), L=2, precision=precision,
                 sched="batched")
    torch.cuda.synchronize()
    g = {k: r[k].cpu().numpy() for k in KEYS}
    net.close()
    for i in range(case.n_boxes):
        o = orc.network(case.Ws, case.bs, lo[i], hi[i], L=2)
        if precision == "fp64":
            for k in ("out_lo", "out_hi"):
                scale = np.maximum(np.maximum(np.abs(o[k]), o["out_hi"] - o["out_lo"]), 1e-12)
                assert np.max(np.abs(g[k][i] - o[k]) / scale) <= 1e-9, (i, k)
        else:
            _check_box_fp32(g, i, o, case.n_hidden)
    # a point box: the bounds enclose the network's value there
    v = H.forward(case.Ws, case.bs, lo[0][None, :])[-1][0]
    assert np.all(g["out_lo"][0] <= v + 1e-9) and np.all(g["out_hi"][0] >= v - 1e-9)


def test_tree_readoff_without_block_fixed_indices():
    """Output tensors beyond one block's LDS (n = 7, degree 4: 78,125 Bernstein
    coefficients) for 8,800 tensors: the tree read-off then fixes no index per
    block (every block folds from the stored coefficients and refolds them
    round by round). Sampled boxes against the oracle, every box for
    soundness."""
    case = wl.random_net_case([7, 5, 5, 4], seed=93, n_boxes=1100)
    print(f"case {case.name}", flush=True)
    g = _run(case)
    _check_sound_all(case, g, m=40)
    for i in (0, 549, 1099):
        o = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=case.L)
        _check_box_fp32(g, i, o, case.n_hidden)
