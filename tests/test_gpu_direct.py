"""The direct read-offs (a lane per Bernstein-digit prefix, folds in
registers): degree-2 tensors of every layer at n = 4..8 and output tensors
of degree 3 and 4 at n = 5, 6, against the FP64 oracle (FP64 within 1e-9,
FP32 padded within 1e-4 and containing the oracle's bounds), and against the
tree read-off they replace (same bounds up to rounding)."""
import numpy as np
import pytest

from paper_2211_14438_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2211_14438_amd import bernnn as B  # noqa: E402
from tests.test_gpu_parity import _assert_fp32, _assert_parity, _oracle, _rel_err  # noqa: E402

DEV = "cuda:0"


def _bounds(case, L, precision, tune=None):
    net = B.Net(case.Ws, case.bs)
    if tune is not None:
        B.tune_set(net, tune)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=DEV)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=DEV)
    r = B.bounds(net, lo, hi, L=L, precision=precision, sched="batched")
    torch.cuda.synchronize()
    out = {k: r[k].cpu().numpy() for k in ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "used_plan")}
    net.close()
    return out


CASES = [([4, 6, 2], 2, 3),        # output degree 2, n = 4
         ([5, 6, 5, 2], 2, 3),     # hidden degree 2 and output degree 4, n = 5
         ([6, 5, 5, 2], 2, 3),     # the same at n = 6
         ([6, 7, 2], 3, 3),        # output degree 3, n = 6
         ([7, 5, 4, 1], 2, 2),     # hidden degree 2 at n = 7 (one round variable)
         ([8, 5, 4, 1], 2, 2)]     # hidden degree 2 at n = 8 (two round variables)


@pytest.mark.parametrize("widths,L,nb", CASES, ids=lambda v: "-".join(map(str, v)) if isinstance(v, list) else str(v))
def test_direct_readoffs_match_oracle(widths, L, nb):
    case = wl.random_net_case(widths, seed=500 + sum(widths), n_boxes=nb, half_width=0.4, L=L)
    print(f"case {widths} L={L}", flush=True)
    o = _oracle(case, L=L)
    g64 = _bounds(case, L, "fp64")
    _assert_parity(g64, o, 1e-9, case.n_hidden)
    g32 = _bounds(case, L, "fp32")
    _assert_fp32(g32, o, case.n_hidden)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_direct_equals_tree_up_to_rounding(precision):
    """The autotuner's read-off variant 3 keeps the tree: both give the same
    bounds up to rounding (1e-12 of the interval in FP64; FP32 padded bounds
    differ by the pads' own rounding terms only) and the same rules."""
    case = wl.random_net_case([6, 9, 9, 3], seed=77, n_boxes=6, half_width=0.3)
    d = _bounds(case, 2, precision)
    t = _bounds(case, 2, precision, tune=[0, 0, 0, 3])
    tol = 1e-12 if precision == "fp64" else 1e-9
    nh = case.n_hidden
    for k in ("neuron_lo", "neuron_hi"):
        assert _rel_err(d[k][:, :nh], t[k][:, :nh], t["neuron_lo"][:, :nh], t["neuron_hi"][:, :nh]).max() <= tol, k
    for k in ("out_lo", "out_hi"):
        assert _rel_err(d[k], t[k], t["out_lo"], t["out_hi"]).max() <= tol, k
    assert np.array_equal(d["used_plan"], t["used_plan"])
