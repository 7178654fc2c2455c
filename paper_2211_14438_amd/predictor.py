"""Learned degree proposal: records, teacher labels, GPU training.

The predictor (an MLP 8 -> 64 -> 64 -> 4, see include/bernnn.h) chooses, per
unstable neuron, the order of its Bernstein ReLU approximant (1, 2, 3) or the
linear fallback (class 0). Every choice yields sound bounds; the choice only
trades output-bound width for work.

Training data come from the method's own GPU runs on training networks (the
architecture of the learned workload, other seeds, boxes of the same law).
A box's tensors are stored at the largest degree of each layer's neurons,
while the composition and the next affine map work per neuron (composed
neurons carry full tensors, order-1, fallback and active ones only their own
prefix). The teacher therefore decides in two measured levels:
  1. per box and hidden layer, the layer's top class, over every
     combination of one class per layer from {order 3, order 2, order 1,
     fallback} (orders are lowered on the device where the plain degree cap
     does not allow them);
  2. within each such layer, a fraction of its unstable neurons -- those
     with the least downstream effect (sensitivity times interval width
     times the ReLU band gap of Prop. 2 between the top class and the one
     below) -- drop one class below the top; the fraction comes from measured
     plans as well.
Each box then takes, from every measured plan of both levels, the cheapest
(run time shared over the boxes) subject to the mean output width staying
within the budget, by a Lagrange multiplier on the width. Every unstable
neuron is labelled with its own class in the chosen plan; its features are
recorded from a run under that plan, so that they match what the predictor
sees when it drives the plan itself. The MLP is trained on these labels by bern_pred_train (the library's
FP32 HIP forward/backward/Adam kernels); inference inside the bounds
pipeline is BF16. The library then raises, per box and layer, the classes
below the layer's top class (bern_opts.no_raise = 0); measured on the
held-out network this is tighter than keeping every predicted class, at
about the same run time (the evaluation reports both).
"""
import json
import math
import os
import time

import numpy as np

from . import bernnn as B
from . import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "predictor_params.bin")


# --------------------------------------------------------------- teacher

def _relu_band(u0, c):
    """Height of the band of the order-c approximant on [lo, hi] relative to
    w = hi - lo, as a function of u0 = -lo/w: B_c(0)/w with the Bernstein
    coefficients sigma(lo + w k/c) (eq. bernpolcoeff2) evaluated at u0."""
    u0 = np.asarray(u0, dtype=np.float64)
    val = np.zeros_like(u0)
    for k in range(c + 1):
        bk = np.maximum(-u0 + k / c, 0.0)  # sigma(lo + w k/c) / w
        val += bk * math.comb(c, k) * u0 ** k * (1.0 - u0) ** (c - k)
    return val


def teacher_labels(feat, n, width, mu, cap_deg=None):
    """Teacher classes (0 fallback, 1..3 order) for feature rows `feat` [N, 8]
    of unstable neurons; `width` [N] = the plain output width of each row's
    box; `cap_deg` [N] optional largest allowed post degree."""
    u0 = np.clip(feat[:, 0], 0.0, 1.0)
    D = np.rint(np.exp(feat[:, 3]) - 1.0)
    sw = np.exp(feat[:, 5])              # s * w
    spread = np.maximum(feat[:, 6], 0.0)  # remainder spread / w
    lam = 1.0 - u0                       # hi / w
    gaps = np.stack([_relu_band(u0, 1) + lam * spread, _relu_band(u0, 1), _relu_band(u0, 2), _relu_band(u0, 3)], 1)
    degs = np.stack([np.ones_like(D), D, 2 * D, 3 * D], 1)
    cost = n * np.log((degs + 1.0) / (D[:, None] + 1.0))
    score = cost + mu * gaps * sw[:, None] / np.maximum(width, 1e-12)[:, None]
    if cap_deg is not None:
        score = np.where(degs <= cap_deg[:, None], score, np.inf)
    return np.argmin(score, axis=1).astype(np.int8)


def consistency(codes, used, widths):
    """The library's cost-neutral raise of learned classes (per box and
    hidden layer): with any unstable neuron at order >= 2, lower classes are
    raised to 2; else with any at order 1, fallbacks are raised to 1.
    `codes` [boxes, nh] classes, `used` [boxes, nh] rule of the plain run
    (only unstable entries, == 2 there, are considered)."""
    out = codes.copy()
    col = 0
    for h in widths[1:-1]:
        blk = out[:, col:col + h]
        uns = used[:, col:col + h] == 2
        top = np.where(uns, blk, -1).max(axis=1)
        raise2 = uns & (top[:, None] >= 2) & (blk < 2)
        raise1 = uns & (top[:, None] == 1) & (blk == 0)
        blk[raise2] = 2
        blk[raise1] = 1
        col += h
    return out


# --------------------------------------------------------------- records

def collect(case, precision="fp32", max_wave=0):
    """One plain run of `case` with feature export. Returns (features
    [boxes, nh, 8], used rule [boxes, nh], output width per box [boxes],
    pre degree per hidden neuron [nh], layer index per hidden neuron [nh])."""
    import torch
    net = B.Net(case.Ws, case.bs)
    dev = "cuda"
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=dev)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=dev)
    feat = torch.zeros((case.n_boxes, case.n_hidden, 8), dtype=torch.float32, device=dev)
    r = B.bounds(net, lo, hi, L=case.L, precision=precision, sched="batched", features=feat, max_wave=max_wave,
                 workspace=_workspace(net, case.n_boxes, L=case.L, precision=precision))
    torch.cuda.synchronize()
    width = (r["out_hi"] - r["out_lo"]).mean(dim=1).cpu().numpy()
    out = feat.cpu().numpy(), r["used_plan"].cpu().numpy(), width
    net.close()
    return out


def _workspace(net, n_boxes, frac=0.5, **kw):
    import torch
    total, one = net.workspace_size(n_boxes, sched="batched", **kw)
    free, _ = torch.cuda.mem_get_info()
    size = int(min(total, max(one, frac * free)))
    return torch.empty(size + 256, dtype=torch.uint8, device="cuda")


def post_cap(case):
    """Largest post degree (plain rule at order L) per hidden neuron column."""
    caps = []
    for i in range(1, len(case.widths) - 1):
        caps += [case.L ** i] * case.widths[i]
    return np.asarray(caps, dtype=np.float64)


# --------------------------------------------------------------- training

def train(X, y, path=DEFAULT_PARAMS, epochs=40, batch=8192, lr=3e-3, seed=0, meta=None, log=print):
    """Train the MLP on the GPU (bern_pred_train) and write the predictor
    file. Returns (Predictor, per-epoch mean losses)."""
    pred, losses = B.pred_train(X, y, path=path, epochs=epochs, batch=batch, lr=lr, seed=seed,
                                meta=None if meta is None else json.dumps(meta))
    if log:
        log("epoch losses: " + " ".join(f"{v:.4f}" for v in losses[:: max(1, len(losses) // 8)]) +
            f" ... {losses[-1]:.4f}")
    return pred, losses


def load_predictor(path=DEFAULT_PARAMS):
    """The trained predictor on the current device (bern_pred_load)."""
    return B.Predictor.load(path)


# --------------------------------------------------------------- pipeline

def training_cases(n_nets=4, n_boxes=1024):
    """Networks of the learned workload's architecture on seeds other than the
    evaluation net's, with boxes of the same distribution."""
    cases = []
    for k in range(n_nets):
        c = wl.cfg5(n_boxes=n_boxes, net_seed=1105 + 1000 * k)
        lo, hi = wl.boxes_centred(6, n_boxes, 2205 + 1000 * k, half_width=0.05)
        c.box_lo, c.box_hi = lo, hi
        cases.append(c)
    return cases


def run_given(case, codes, precision="fp32"):
    import torch
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device="cuda")
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device="cuda")
    pl = torch.tensor(codes, dtype=torch.int8, device="cuda")
    ws = _workspace(net, case.n_boxes, L=case.L, precision=precision, plan="given")
    B.bounds(net, lo, hi, L=case.L, precision=precision, sched="batched", plan="given", degree_plan=pl, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = B.bounds(net, lo, hi, L=case.L, precision=precision, sched="batched", plan="given", degree_plan=pl,
                 workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    w = (r["out_hi"] - r["out_lo"]).mean().item()
    net.close()
    return w, dt


def layer_combos(n_layers, classes=(3, 2, 1, 0)):
    import itertools
    return list(itertools.product(classes, repeat=n_layers))


def combo_codes(case, combo):
    codes = np.empty((case.n_boxes, case.n_hidden), np.int8)
    col = 0
    for li, h in enumerate(case.widths[1:-1]):
        codes[:, col:col + h] = combo[li]
        col += h
    return codes


def run_plan(case, codes, precision="fp32", features=False, reps=1):
    """GIVEN-plan run: per-box output widths, time of the last repetition,
    and (optionally) the exported features and rules."""
    import torch
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device="cuda")
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device="cuda")
    pl = torch.tensor(codes, dtype=torch.int8, device="cuda")
    ws = _workspace(net, case.n_boxes, L=case.L, precision=precision, plan="given")
    feat = torch.zeros((case.n_boxes, case.n_hidden, 8), dtype=torch.float32, device="cuda") if features else None
    dt = 0.0
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = B.bounds(net, lo, hi, L=case.L, precision=precision, sched="batched", plan="given", degree_plan=pl,
                     workspace=ws, features=feat)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    width = (r["out_hi"] - r["out_lo"]).mean(dim=1).cpu().numpy()
    out = dict(width=width, time=dt, used=r["used_plan"].cpu().numpy())
    if features:
        out["features"] = feat.cpu().numpy()
    net.close()
    return out


def _lagrange_pick(t, dw, budget):
    """Per box, argmin_k t[k] + lam * dw[b, k] with the smallest lam whose
    mean width increase stays within `budget` (t [K] time shares, dw [B, K]
    width increases relative to the plain mean width)."""
    nb = dw.shape[0]

    def pick(lam):
        return np.argmin(t[None, :] + lam * dw, axis=1)

    lo_l, hi_l = 0.0, 1.0
    while (dw[np.arange(nb), pick(hi_l)].mean() > budget) and hi_l < 1e12:
        hi_l *= 4.0
    for _ in range(60):
        mid = 0.5 * (lo_l + hi_l)
        if dw[np.arange(nb), pick(mid)].mean() > budget:
            lo_l = mid
        else:
            hi_l = mid
    return pick(hi_l)


def measured_teacher(case, budget, log=print):
    """Level 1: per box, one top class per hidden layer, chosen from measured
    runs of every combination (a plan with that class for all of a layer's
    neurons): minimise run time subject to the mean output width staying
    within (1 + budget) of the plain rule's. Returns (choice per box,
    combos, per-combo results, the plain run)."""
    nl = len(case.widths) - 2
    combos = layer_combos(nl)
    res = [run_plan(case, combo_codes(case, cb)) for cb in combos]
    base = run_plan(case, np.full((case.n_boxes, case.n_hidden), case.L, np.int8))
    nb = case.n_boxes
    t = np.array([r["time"] for r in res]) / nb
    dw = np.stack([r["width"] - base["width"] for r in res], 1) / base["width"].mean()
    choice = _lagrange_pick(t, dw, budget)
    for k, cb in enumerate(combos):
        if (choice == k).sum():
            log(f"  combo {cb}: time {res[k]['time'] * 1e3:.1f} ms  width x{res[k]['width'].mean() / base['width'].mean():.4f}"
                f"  chosen by {(choice == k).sum()} boxes")
    return choice, combos, res, base


def demote(case, codes, feat, used, q):
    """Level 2 candidate: in every box and hidden layer whose top class is k
    >= 1, the fraction q of its unstable neurons with the smallest downstream
    effect drop to class k - 1 (order 1 drops to the fallback). Effect =
    downstream sensitivity x interval width x the band gap (Prop. 2 heights)
    between the lower class and k."""
    out = codes.copy()
    u0 = np.clip(feat[..., 0], 0.0, 1.0)
    sw = np.exp(feat[..., 5])
    spread = np.maximum(feat[..., 6], 0.0)
    band = {c: _relu_band(u0, c) for c in (1, 2, 3)}
    band[0] = band[1] + (1.0 - u0) * spread
    col = 0
    for h in case.widths[1:-1]:
        blk = out[:, col:col + h]
        uns = (used[:, col:col + h] >= 1) | (used[:, col:col + h] == -2)
        top = blk[:, 0].astype(int)  # level-1 plans hold one class per layer
        for b in np.nonzero((top >= 1) & uns.any(axis=1))[0]:
            k = int(top[b])
            idx = np.nonzero(uns[b])[0]
            m = int(np.floor(q * idx.size))
            if m == 0:
                continue
            gap = band[k - 1][b, col + idx] - band[k][b, col + idx]
            eff = sw[b, col + idx] * gap
            drop = idx[np.argsort(eff, kind="stable")[:m]]
            blk[b, drop] = k - 1
        col += h
    return out


def refine(case, variants, fractions, res1, base, budget, log=print):
    """Level 2: the demotion variants of each box's level-1 plan, measured,
    and one final pick per box over every measured plan -- the level-1
    combinations (res1) and these variants -- within the full width budget.
    Returns the per-box index into combinations + variants."""
    res2 = [run_plan(case, v) for v in variants]
    res = list(res1) + res2
    t = np.array([r["time"] for r in res]) / case.n_boxes
    dw = np.stack([r["width"] - base["width"] for r in res], 1) / base["width"].mean()
    choice = _lagrange_pick(t, dw, budget)
    k1 = len(res1)
    for k, q in enumerate(fractions):
        log(f"  demote {q:.2f}: time {res2[k]['time'] * 1e3:.1f} ms  width x{res2[k]['width'].mean() / base['width'].mean():.4f}"
            f"  chosen by {(choice == k1 + k).sum()} boxes")
    return choice


def evaluate(pred, case=None, precision="fp32", log=print):
    """The learned plan (with the per-layer raise, and without it) against
    the batched plain rule, a fixed order 1 and the linear fallback for every
    unstable neuron, all batched, on the held-out evaluation network."""
    import torch
    case = case or wl.cfg5()
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device="cuda")
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device="cuda")
    shape = (case.n_boxes, case.n_hidden)
    forms = (("plain", dict(plan="plain")),
             ("learned", dict(plan="learned", pred=pred)),
             ("learned_no_raise", dict(plan="learned", pred=pred, no_raise=True)),
             ("fixed1", dict(plan="given", degree_plan=torch.full(shape, 1, dtype=torch.int8, device="cuda"))),
             ("fallback", dict(plan="given", degree_plan=torch.full(shape, 0, dtype=torch.int8, device="cuda"))))
    out = {}
    for name, kw in forms:
        ws = _workspace(net, case.n_boxes, L=case.L, precision=precision,
                        **{k: v for k, v in kw.items() if k not in ("degree_plan", "no_raise")})
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = B.bounds(net, lo, hi, L=case.L, precision=precision, sched="batched", workspace=ws, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        used = r["used_plan"].cpu().numpy().ravel()
        out[name] = dict(time=dt, width=float((r["out_hi"] - r["out_lo"]).mean().item()),
                         rules={k: int((used == v).sum()) for k, v in (("inactive", 0), ("active", -1),
                                                                        ("fallback", -2), ("order1", 1),
                                                                        ("order2", 2), ("order3", 3))})
        del ws
    res = dict(detail=out)
    for name in ("learned", "learned_no_raise", "fixed1", "fallback"):
        res[name] = dict(width_ratio=out[name]["width"] / out["plain"]["width"],
                         speedup=out["plain"]["time"] / out[name]["time"])
        log(f"eval net: {name} width x{res[name]['width_ratio']:.4f}, speedup over batched plain "
            f"x{res[name]['speedup']:.2f}")
    net.close()
    return res


def main(argv=None):
    import argparse
    import torch
    ap = argparse.ArgumentParser(description="collect records, label them by measured plans, train the predictor")
    ap.add_argument("--out", default=DEFAULT_PARAMS)
    ap.add_argument("--nets", type=int, default=8)
    ap.add_argument("--boxes", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--budget", type=float, default=0.08, help="mean output-width increase the teacher may spend")
    ap.add_argument("--report", default=None)
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, flush=True)
    report = dict(budget=args.budget, nets=[])
    Xs, ys = [], []
    for ci, c in enumerate(training_cases(args.nets, args.boxes)):
        t0 = time.perf_counter()
        choice, combos, res, base = measured_teacher(c, args.budget, log=log)
        combo_plans = [combo_codes(c, cb) for cb in combos]
        codes1 = np.stack([combo_plans[k][b] for b, k in enumerate(choice)])
        run1 = run_plan(c, codes1, features=True)
        fracs = (0.25, 0.5, 0.75)
        variants = [demote(c, codes1, run1["features"], run1["used"], q) for q in fracs]
        pick = refine(c, variants, fracs, res, base, args.budget, log=log)
        plans = combo_plans + variants
        codes = np.stack([plans[k][b] for b, k in enumerate(pick)])
        run = run_plan(c, codes, features=True)
        used, feat = run["used"], run["features"]
        mask = (used >= 1) | (used == -2)  # unstable neurons (any order or the fallback)
        X = feat[mask]
        # label: the class the library applied (orders lowered under the degree cap)
        y = np.where(used[mask] == -2, 0, used[mask]).astype(np.int8)
        Xs.append(X)
        ys.append(y)
        entry = dict(net=ci, records=int(X.shape[0]), width_ratio=float(run["width"].mean() / base["width"].mean()),
                     speedup=float(base["time"] / run["time"]), label_counts=np.bincount(y, minlength=4).tolist(),
                     seconds=time.perf_counter() - t0)
        report["nets"].append(entry)
        log(f"net {ci}: teacher plan width x{entry['width_ratio']:.4f} speedup x{entry['speedup']:.2f}, "
            f"{entry['records']} records, labels {entry['label_counts']}")
    X = np.concatenate(Xs).astype(np.float32)
    y = np.concatenate(ys).astype(np.int8)
    report["records"] = int(X.shape[0])
    report["label_counts"] = np.bincount(y, minlength=4).tolist()
    pred, losses = train(X, y, path=args.out, epochs=args.epochs,
                         meta=dict(records=int(X.shape[0]), budget=args.budget, classes=report["label_counts"]),
                         log=log)
    report["losses"] = [float(v) for v in losses]
    # accuracy per class of the BF16 inference arithmetic, on the training records
    P = torch.tensor(read_params(args.out), device="cuda")
    cls, _ = B.mlp_classify(P, torch.tensor(X, device="cuda"), bf16=True)
    cls = cls.cpu().numpy()
    report["train_accuracy_bf16"] = float((cls == y).mean())
    report["per_class_accuracy_bf16"] = [float((cls[y == c] == c).mean()) if (y == c).any() else None
                                         for c in range(4)]
    log(f"saved {args.out}: accuracy {report['train_accuracy_bf16']:.4f}, per class "
        f"{report['per_class_accuracy_bf16']}")
    report["eval"] = evaluate(pred, log=log)
    pred.close()
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)


def read_params(path=DEFAULT_PARAMS):
    """The parameter vector of a predictor file (format of bern_pred_load),
    for tests and reports."""
    with open(path, "rb") as fh:
        head = fh.read(16)
        assert head[:8] == b"BERNPRED"
        n = int(np.frombuffer(head[12:16], dtype="<u4")[0])
        return np.frombuffer(fh.read(4 * n), dtype="<f4").astype(np.float32)


if __name__ == "__main__":
    main()
