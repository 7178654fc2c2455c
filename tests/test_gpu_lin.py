"""GPU parity of the periodic linearisation option (the Lin parameter of
Section 5.4, reading R13) against the FP64 oracle, through the C ABI.

Bar: FP64 within 1e-9 relative (|g - o| <= 1e-9 max(|o|, hi_o - lo_o)); FP32
padded within 1e-4 relative, every GPU interval containing the oracle's,
and every sampled network value inside the padded bounds (no slack)."""
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

DEV = "cuda:0"
KEYS = ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "used_plan")


def _gpu(case, **kw):
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    if "degree_plan" in kw and kw["degree_plan"] is not None:
        kw["degree_plan"] = torch.tensor(kw["degree_plan"], dtype=torch.int8, device=DEV)
    ws = H.poisoned_workspace(torch, net, case.n_boxes, **{k: v for k, v in kw.items() if k != "degree_plan"})
    r = B.bounds(net, lo, hi, workspace=ws, **kw)
    torch.cuda.synchronize()
    out = {k: r[k].cpu().numpy() for k in KEYS}
    out["stats"] = r["stats"]
    net.close()
    return out


def _oracle(case, L, lin, plan=None):
    rs = [orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=L, lin=lin,
                      plan=None if plan is None else plan[i]) for i in range(case.n_boxes)]
    o = {k: np.stack([r[k] for r in rs]) for k in ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "used_plan")}
    o["out_deg"] = max(r["out_deg"] for r in rs)
    return o


def _rel(g, o, lo, hi):
    scale = np.maximum(np.abs(o), hi - lo)
    return np.abs(g - o) / np.where(scale > 0, scale, 1.0)


def _check(g, o, nh, precision):
    tol = 1e-9 if precision == "fp64" else 1e-4
    pairs = [("out_lo", "out_hi", None)] + ([("neuron_lo", "neuron_hi", nh)] if nh else [])
    for klo, khi, m in pairs:
        olo, ohi = o[klo][:, :m], o[khi][:, :m]
        for k, ov in ((klo, olo), (khi, ohi)):
            e = _rel(g[k][:, :m], ov, olo, ohi)
            print(f"  {k}: max rel err {e.max():.2e}", flush=True)
            assert e.max() <= tol, (k, e.max())
        if precision == "fp32":
            assert np.all(g[klo][:, :m] <= olo) and np.all(g[khi][:, :m] >= ohi), klo


def _sound(case, g, precision, m=3000, seed=0):
    """Sampled network values inside the bounds: FP32 padded bounds are
    rigorous (no slack); FP64 mode is not (as in the paper), so a value at a
    box corner may cross its exact bound by rounding: 1e-9 slack there."""
    rng = np.random.default_rng(seed)
    nh = case.n_hidden
    tol = 0.0 if precision == "fp32" else 1e-9
    for i in range(case.n_boxes):
        _, x = H.box_points(case.box_lo[i], case.box_hi[i], m, rng)
        pres = H.forward(case.Ws, case.bs, x)
        hid = np.concatenate(pres[:-1], axis=1)
        assert np.all(hid >= g["neuron_lo"][i][:nh] - tol) and np.all(hid <= g["neuron_hi"][i][:nh] + tol), i
        assert np.all(pres[-1] >= g["out_lo"][i] - tol) and np.all(pres[-1] <= g["out_hi"][i] + tol), i


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lin", [1, 2])
def test_lin_cfg2_shape(precision, lin):
    """The [4,20,20,20,2] workload (one box, L = 2) with Lin = 1 and 2."""
    case = wl.cfg2()
    print(f"case {case.name} lin {lin} {precision}", flush=True)
    g = _gpu(case, L=2, precision=precision, lin=lin)
    o = _oracle(case, 2, lin)
    _check(g, o, case.n_hidden, precision)
    assert g["stats"]["out_degree"] == o["out_deg"] == 2 ** (3 % lin)
    assert g["stats"]["lin_layers"] == 3 // lin
    _sound(case, g, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("L,lin", [(2, 1), (3, 1), (4, 1), (2, 2), (2, 3)])
def test_lin_random_nets_batched(precision, L, lin):
    case = wl.random_net_case([3, 7, 6, 5, 2], seed=50 + 7 * L + lin, n_boxes=5)
    print(f"case {case.name} L {L} lin {lin} {precision}", flush=True)
    g = _gpu(case, L=L, precision=precision, lin=lin, sched="batched")
    o = _oracle(case, L, lin)
    _check(g, o, case.n_hidden, precision)
    if precision == "fp32":
        _sound(case, g, precision, seed=L + lin)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_lin_given_plans_uneven_degrees(precision):
    """Per-neuron codes (0..3, so fallback, orders 1-3 and stable neurons):
    boxes reach the Lin layer at different degrees, several classes are
    linearised, then every box continues at degree 1."""
    case = wl.random_net_case([3, 8, 7, 6, 2], seed=64, n_boxes=8)
    plan = np.random.default_rng(4).integers(0, 4, size=(case.n_boxes, case.n_hidden)).astype(np.int8)
    plan[::3] = 1
    print(f"case {case.name} given {precision}", flush=True)
    g = _gpu(case, L=2, precision=precision, lin=2, sched="batched", plan="given", degree_plan=plan)
    # the rule each neuron took (codes above the layer's cap are lowered) as
    # the plan the oracle runs
    used = g["used_plan"][:, :case.n_hidden]
    taken = np.where(used >= 1, used, np.where(used == -2, 0, 1)).astype(np.int8)
    assert np.all((used < 1) | (used <= plan))
    o = _oracle(case, 2, 2, plan=taken)
    assert np.array_equal(used, o["used_plan"])
    _check(g, o, case.n_hidden, precision)
    _sound(case, g, precision, seed=5)


def test_lin_schedules_and_graph_agree():
    """Per-box, batched, smaller waves and graph replays of a Lin run give the
    same bits."""
    case = wl.random_net_case([4, 9, 9, 9, 3], seed=71, n_boxes=7)
    print(f"case {case.name}", flush=True)
    a = _gpu(case, L=2, precision="fp32", lin=2, sched="batched")
    b = _gpu(case, L=2, precision="fp32", lin=2, sched="per_box")
    c = _gpu(case, L=2, precision="fp32", lin=2, sched="batched", max_wave=3)
    for k in KEYS:
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    kw = dict(L=2, precision="fp32", lin=2, sched="batched")
    r = B.bounds(net, lo, hi, graph=True, **kw)
    outs = {k: r[k] for k in KEYS}
    for rep in range(3):
        B.bounds(net, lo, hi, graph=True, outputs=outs, workspace=r["workspace"], **kw)
        torch.cuda.synchronize()
        for k in KEYS:
            assert np.array_equal(outs[k].cpu().numpy(), a[k]), (rep, k)
    net.close()


def test_lin_output_polys_and_volume():
    """With Lin the output polynomials have the degree the oracle gives them,
    and their relative volume matches the oracle's."""
    case = wl.random_net_case([3, 6, 5, 4, 2], seed=93, n_boxes=3)
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    r = B.rel_volume(net, lo, hi, L=2, precision="fp64", lin=2)
    p = B.output_polys(net, lo, hi, 2, L=2, precision="fp64", lin=2)
    torch.cuda.synchronize()
    vol = r["rel_vol"].cpu().numpy()
    U = p["U"].cpu().numpy()
    net.close()
    for i in range(case.n_boxes):
        o = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=2, lin=2, want_polys=True)
        assert o["out_deg"] == 2
        for j in range(2):
            scale = max(abs(o["rel_vol"][j]), o["out_hi"][j] - o["out_lo"][j])
            assert abs(vol[i, j] - o["rel_vol"][j]) <= 1e-9 * scale
            bu = orc.power_to_bern(case.n, 2, U[i, j])
            assert np.max(np.abs(bu - o["out_U"][j])) <= 1e-9 * np.abs(o["out_U"][j]).max()
