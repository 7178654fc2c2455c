"""Per-neuron plans (given codes, the learned predictor) run as one captured
graph: a classification kernel lists, per hidden layer, the boxes of every
(pre degree, post degree) class the rules can give, and each class is
launched with its box count read from device memory, so the wave needs no
host round trip.

Bar: bit-for-bit equality of every output (neuron and output bounds, the
plan used, the counters) with the eager run, whose classes are read back to
the host once per hidden layer; on poisoned workspaces, over several replays
of one graph with other device work, workspace poisoning and eager calls in
between. A configuration with more classes than the device path takes runs
eagerly under opts.graph and says so in its statistics."""
import numpy as np
import pytest

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


def _setup(case, plan, codes=None):
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    kw = {}
    if plan == "given":
        kw["degree_plan"] = torch.tensor(codes, dtype=torch.int8, device=DEV)
    return net, lo, hi, kw


def _outputs(net, nb):
    nh = max(net.n_hidden, 1)
    return dict(neuron_lo=torch.empty((nb, nh), dtype=torch.float64, device=DEV),
                neuron_hi=torch.empty((nb, nh), dtype=torch.float64, device=DEV),
                out_lo=torch.empty((nb, net.n_out), dtype=torch.float64, device=DEV),
                out_hi=torch.empty((nb, net.n_out), dtype=torch.float64, device=DEV),
                used_plan=torch.empty((nb, nh), dtype=torch.int8, device=DEV))


def _host(r, counters=None):
    out = {k: r[k].cpu().numpy().copy() for k in KEYS}
    if counters is not None:
        out["counters"] = counters.cpu().numpy().copy()
    return out


def _same(a, b, what):
    for k in a:
        x, y = a[k], b[k]
        if x.dtype.kind == "f":
            # NaN-aware bit equality: the bytes must agree
            same = x.view(np.uint64) == y.view(np.uint64)
        else:
            same = x == y
        assert same.all(), (what, k, int((~same).sum()))


def _compare(case, plan, precision, L, codes=None, pred=None, lin=0, counters=False, replays=3,
             expect_device=True, max_wave=0):
    print(f"case {case.name} plan={plan} {precision} L={L} lin={lin} counters={counters}", flush=True)
    net, lo, hi, kw = _setup(case, plan, codes)
    nb = case.n_boxes
    opts = dict(L=L, precision=precision, plan=plan, sched="batched", lin=lin, pred=pred, max_wave=max_wave, **kw)
    cnt_e = torch.zeros(len(B.COUNTERS), dtype=torch.int64, device=DEV) if counters else None
    cnt_g = torch.zeros(len(B.COUNTERS), dtype=torch.int64, device=DEV) if counters else None
    ws_e = H.poisoned_workspace(torch, net, nb, L=L, precision=precision, plan=plan, sched="batched", lin=lin,
                                pred=pred, max_wave=max_wave)
    r = B.bounds(net, lo, hi, workspace=ws_e, counters=cnt_e, **opts)
    torch.cuda.synchronize()
    assert r["stats"]["graph"] == 0 and r["stats"]["device_classes"] == 0
    eager = _host(r, cnt_e)
    assert np.isfinite(eager["out_lo"]).all() and np.isfinite(eager["out_hi"]).all()

    ws_g = H.poisoned_workspace(torch, net, nb, L=L, precision=precision, plan=plan, sched="batched", lin=lin,
                                pred=pred, max_wave=max_wave)
    outs = _outputs(net, nb)
    for rep in range(replays):
        # other device work between replays: the graph's workspace poisoned
        # again, its outputs cleared, and an eager call on its own workspace
        ws_g.fill_(255)
        for v in outs.values():
            v.fill_(-7)
        if cnt_g is not None:
            cnt_g.fill_(-1)
        g = B.bounds(net, lo, hi, workspace=ws_g, outputs=outs, graph=True, counters=cnt_g, **opts)
        st = g["stats"]
        assert st["graph"] == (1 if expect_device else 0), st
        assert st["device_classes"] == (1 if expect_device else 0), st
        x = torch.randn(4096, device=DEV)
        (x @ x).item()
        e2 = B.bounds(net, lo, hi, workspace=ws_e, **opts)
        torch.cuda.synchronize()
        _same(eager, _host(g, cnt_g), f"replay {rep}")
        _same({k: eager[k] for k in KEYS}, _host(e2), f"eager {rep}")
        print(f"  replay {rep}: bit-identical", flush=True)
    net.close()


def test_graph_given_codes_cfg3_shape():
    case = wl.cfg3(n_keep=128)
    _compare(case, "given", "fp32", 3, codes=case.plan)


def test_graph_given_codes_fp64_with_fallback():
    case = wl.random_net_case([4, 24, 24, 2], 41, n_boxes=96, L=2)
    codes = wl.degree_draws(case.n_boxes, 48, 77, choices=(0, 1, 2))
    _compare(case, "given", "fp64", 2, codes=codes)


def test_graph_learned_cfg5_shape_counters():
    case = wl.cfg5(n_boxes=256)
    pred = PR.load_predictor()
    _compare(case, "learned", "fp32", 2, pred=pred, counters=True)
    pred.close()


def test_graph_learned_fp64_waves():
    # several waves, one graph per call replaying every wave's launches
    case = wl.cfg5(n_boxes=200)
    pred = PR.load_predictor()
    _compare(case, "learned", "fp64", 2, pred=pred, max_wave=64)
    pred.close()


def test_graph_learned_lin():
    case = wl.cfg5(n_boxes=128)
    pred = PR.load_predictor()
    _compare(case, "learned", "fp32", 2, pred=pred, lin=1)
    pred.close()


def test_graph_given_lin2():
    case = wl.random_net_case([3, 16, 16, 16, 2], 23, n_boxes=64, L=2)
    codes = wl.degree_draws(case.n_boxes, 48, 78, choices=(0, 1, 2, 3))
    _compare(case, "given", "fp32", 2, codes=codes, lin=2)


def test_graph_too_many_classes_runs_eagerly():
    # given codes up to 8 over four hidden layers: more (pre, post) pairs
    # than the device path launches, so the call stays on host classes
    case = wl.random_net_case([2, 8, 8, 8, 8, 1], 31, n_boxes=16, L=2)
    codes = wl.degree_draws(case.n_boxes, 32, 79, choices=(1, 2))
    _compare(case, "given", "fp32", 2, codes=codes, expect_device=False, replays=2)
