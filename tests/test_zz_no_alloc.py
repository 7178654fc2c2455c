"""bern_bounds_noalloc (bern_bounds on the library's own per-GPU scratch
array, for callers that cannot allocate) against bern_bounds with a caller
workspace, through the C ABI: two calls in a row on the same GPU, the second
with fewer boxes, each bitwise equal to bern_bounds (same kernels and
summation order) and so within the parity bar of the FP64 oracle (1e-9
relative in FP64; FP32 padded: within 1e-4 and containing the oracle's
interval). The learned plan runs there with its degree classes listed on
the device, bitwise equal to bern_bounds with host classes. Also the
documented refusals."""
import ctypes

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


def _oracle_close(case, g, i, L, lin, precision):
    o = orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=L, lin=lin)
    for klo, khi in (("out_lo", "out_hi"), ("neuron_lo", "neuron_hi")):
        olo, ohi = o[klo], o[khi]
        glo, ghi = g[klo][i][:olo.size], g[khi][i][:ohi.size]
        scale = np.maximum(np.maximum(np.abs(olo), np.abs(ohi)), ohi - olo)
        scale = np.where(scale > 0, scale, 1.0)
        tol = 1e-9 if precision == "fp64" else 1e-4
        assert np.max(np.abs(glo - olo) / scale) <= tol and np.max(np.abs(ghi - ohi) / scale) <= tol
        if precision == "fp32":
            assert np.all(glo <= olo) and np.all(ghi >= ohi)


@pytest.mark.parametrize("precision,lin", [("fp64", 0), ("fp32", 0), ("fp32", 2)])
def test_noalloc_matches_bounds_twice(precision, lin):
    case = wl.random_net_case([4, 12, 10, 9, 3], seed=123, n_boxes=40)
    print(f"case {case.name} {precision} lin {lin}", flush=True)
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    kw = dict(L=2, precision=precision, lin=lin)
    # builds the network's index tables for these options
    ref = B.bounds(net, lo, hi, sched="batched", **kw)
    torch.cuda.synchronize()
    ref = {k: ref[k].cpu().numpy() for k in KEYS}
    for nb in (40, 13):  # the second call on fewer boxes reuses the same scratch
        r = B.bounds_noalloc(net, lo[:nb], hi[:nb], **kw)
        torch.cuda.synchronize()
        g = {k: r[k].cpu().numpy() for k in KEYS}
        for k in KEYS:
            assert np.array_equal(g[k], ref[k][:nb]), (nb, k)
        assert r["stats"]["n_waves"] >= 1
        for i in (0, nb - 1):
            _oracle_close(case, g, i, 2, lin, precision)
    net.close()


@pytest.mark.parametrize("precision,lin", [("fp32", 0), ("fp64", 0), ("fp32", 1)])
def test_noalloc_learned_plan_matches_bounds_twice(precision, lin):
    """The learned plan on the scratch array: its degree classes listed on the
    device (no host staging), bitwise equal to bern_bounds with host classes."""
    from paper_2211_14438_amd import predictor as PR
    case = wl.cfg5(n_boxes=48)
    print(f"case {case.name} learned {precision} lin {lin}", flush=True)
    net = B.Net(case.Ws, case.bs)
    pred = PR.load_predictor()
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    kw = dict(L=2, precision=precision, lin=lin, plan="learned", pred=pred)
    B.bounds(net, lo, hi, sched="batched", graph=True, **kw)  # builds every class's index tables
    ref = B.bounds(net, lo, hi, sched="batched", **kw)  # host classes
    torch.cuda.synchronize()
    assert ref["stats"]["device_classes"] == 0
    ref = {k: ref[k].cpu().numpy() for k in KEYS}
    for nb in (48, 17):
        r = B.bounds_noalloc(net, lo[:nb], hi[:nb], **kw)
        torch.cuda.synchronize()
        assert r["stats"]["device_classes"] == 1
        g = {k: r[k].cpu().numpy() for k in KEYS}
        for k in KEYS:
            assert np.array_equal(g[k], ref[k][:nb]), (nb, k)
    pred.close()
    net.close()


def test_noalloc_refusals():
    case = wl.random_net_case([3, 6, 5, 2], seed=9, n_boxes=2)
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    # tables not built on this fresh network
    with pytest.raises(B.BernError) as ei:
        B.bounds_noalloc(net, lo, hi, L=3)
    assert ei.value.status == -1 and "not built" in str(ei.value)
    B.bounds(net, lo, hi, L=3)
    torch.cuda.synchronize()
    B.bounds_noalloc(net, lo, hi, L=3)
    torch.cuda.synchronize()
    # another plan
    L_ = B.lib()
    o = B.make_opts(L=3, plan="given")
    out = torch.empty((2, 2), dtype=torch.float64, device=DEV)
    st = L_.bern_bounds_noalloc(net.handle, ctypes.byref(o), 2, B._ptr(lo), B._ptr(hi), None, None, B._ptr(out),
                                B._ptr(out), None, None, None)
    assert st == -1 and b"plain rule" in L_.bern_last_error()
    net.close()
    # one box beyond the scratch: 8 inputs, order 2, three hidden layers of
    # 200 (each pre-activation arena alone holds 200 x 2 x C(16, 8) FP64
    # coefficients, 41 MB)
    big = wl.random_net_case([8, 200, 200, 200, 1], seed=3, n_boxes=1)
    net = B.Net(big.Ws, big.bs)
    _, one = net.workspace_size(1, L=2)
    assert one > B.NOALLOC_SCRATCH_BYTES
    lo = torch.tensor(big.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(big.box_hi, dtype=torch.float64, device=DEV)
    with pytest.raises(B.BernError) as ei:
        B.bounds_noalloc(net, lo, hi, L=2)
    assert ei.value.status == -5
    net.close()
