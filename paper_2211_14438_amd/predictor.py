"""Learned degree proposal: records, teacher labels, GPU training.

The predictor (an MLP 8 -> 64 -> 64 -> 4, see include/bernnn.h) chooses, per
unstable neuron, the order of its Bernstein ReLU approximant (1, 2, 3) or the
linear fallback (class 0). Every choice yields sound bounds; the choice only
trades output-bound width for tensor size.

Training data come from the method's own GPU runs on training networks (the
architecture of the learned workload, other seeds, boxes of the same law).
A box's tensors are stored at the largest degree of each layer's neurons, so
the decisions that pay are per box and layer. The teacher measures them: it
runs every combination of one class per hidden layer (order 2, order 1,
linear fallback for all unstable neurons of that layer) as a given plan, and
picks for each box the cheapest combination (by measured run time) whose
output-bound width for that box stays within (1 + budget) times the plain
width. Every unstable neuron is labelled with its layer's class in the chosen
combination; its features are recorded from a run under the chosen plans, so
that they match what the predictor sees when it drives the plan itself. The
MLP is trained to reproduce these labels with the library's own FP32 HIP
forward/backward/Adam kernels; inference inside the bounds pipeline is BF16.
A simpler per-neuron teacher (band height of each class, Prop. 2, times the
neuron's downstream sensitivity, against tensor growth) is kept as a
reference.
"""
import json
import math
import os
import time

import numpy as np

from . import bernnn as B
from . import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "predictor_params.npz")


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

def train(X, y, mean, std, epochs=30, batch=8192, lr=3e-3, seed=0, log=print):
    """Train the MLP on the GPU with the library's kernels. X [N, 8] float32,
    y [N] int8 classes. Returns the parameter vector (numpy float32)."""
    import torch
    rng = np.random.default_rng(seed)
    P = np.zeros(B.N_PARAMS, dtype=np.float32)
    F, H, C = 8, 64, 4
    o = 0
    P[o:o + F] = mean; o += F
    P[o:o + F] = std; o += F
    P[o:o + H * F] = rng.standard_normal(H * F) * np.sqrt(2.0 / F); o += H * F + H
    P[o:o + H * H] = rng.standard_normal(H * H) * np.sqrt(2.0 / H); o += H * H + H
    P[o:o + C * H] = rng.standard_normal(C * H) * np.sqrt(1.0 / H)
    dev = "cuda"
    Pd = torch.tensor(P, device=dev)
    m = torch.zeros_like(Pd)
    v = torch.zeros_like(Pd)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    yd = torch.tensor(y, dtype=torch.int8, device=dev)
    N = X.shape[0]
    scratch = torch.empty(B.lib().bern_mlp_backward_scratch(batch), dtype=torch.uint8, device=dev)
    step = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(N), device=dev)
        tot = 0.0
        nb = 0
        for s0 in range(0, N - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            G, loss = B.mlp_backward(Pd, Xd[idx], yd[idx], scratch=scratch)
            step += 1
            B.mlp_adam(Pd, G, m, v, step, lr * (0.5 * (1 + math.cos(math.pi * ep / epochs))))
            tot += float(loss.item())
            nb += 1
        if log and (ep % 5 == 0 or ep == epochs - 1):
            cls, _ = B.mlp_classify(Pd, Xd, bf16=True)
            acc = float((cls == yd).float().mean().item())
            log(f"epoch {ep}: loss {tot / max(nb, 1):.4f}  bf16 accuracy {acc:.4f}")
    return Pd.cpu().numpy()


def save(path, P, meta):
    np.savez(path, params=np.asarray(P, np.float32), meta=json.dumps(meta))


def load(path=DEFAULT_PARAMS):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(str(z["meta"]))


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


def layer_combos(n_layers, classes=(2, 1, 0)):
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


def measured_teacher(case, budget, log=print):
    """Per box, one combination of per-layer classes, chosen from measured
    runs: minimise total run time subject to the mean output width staying
    within (1 + budget) of the plain rule's. Solved by a Lagrange multiplier
    on the width: box b takes argmin_k t_k / B + lam * (w_bk - w_b0) / mean(w_0),
    with lam bisected to meet the budget. Returns (choice per box, combos,
    per-combo results)."""
    nl = len(case.widths) - 2
    combos = layer_combos(nl)
    res = [run_plan(case, combo_codes(case, cb)) for cb in combos]
    k0 = combos.index((2,) * nl)
    base = res[k0]
    nb = case.n_boxes
    t = np.array([r["time"] for r in res]) / nb                      # [K] time share per box
    dw = np.stack([r["width"] - base["width"] for r in res], 1) / base["width"].mean()  # [B, K]

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
    choice = pick(hi_l)
    for k, cb in enumerate(combos):
        log(f"  combo {cb}: time {res[k]['time'] * 1e3:.1f} ms  width x{res[k]['width'].mean() / base['width'].mean():.4f}"
            f"  chosen by {(choice == k).sum()} boxes")
    return choice, combos, res


def evaluate(P, case=None, precision="fp32", log=print):
    """Learned plan against the plain rule (both batched) on the held-out
    evaluation network: output-width ratio and speedup."""
    import torch
    case = case or wl.cfg5()
    pred = B.Predictor(P)
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device="cuda")
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device="cuda")
    out = {}
    for name, kw in (("plain", dict(plan="plain")), ("learned", dict(plan="learned", pred=pred))):
        ws = _workspace(net, case.n_boxes, L=case.L, precision=precision, **kw)
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = B.bounds(net, lo, hi, L=case.L, precision=precision, sched="batched", workspace=ws, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        out[name] = dict(time=dt, width=float((r["out_hi"] - r["out_lo"]).mean().item()),
                         used=np.bincount(r["used_plan"].cpu().numpy().ravel() + 2, minlength=12).tolist())
        del ws
    res = dict(width_ratio=out["learned"]["width"] / out["plain"]["width"],
               speedup=out["plain"]["time"] / out["learned"]["time"], detail=out)
    log(f"eval net: learned width x{res['width_ratio']:.4f}, speedup x{res['speedup']:.2f} (batched plain "
        f"{out['plain']['time'] * 1e3:.1f} ms, learned {out['learned']['time'] * 1e3:.1f} ms)")
    net.close()
    pred.close()
    return res


def main(argv=None):
    import argparse
    import torch
    ap = argparse.ArgumentParser(description="collect records, label them by measured plans, train the predictor")
    ap.add_argument("--out", default=DEFAULT_PARAMS)
    ap.add_argument("--nets", type=int, default=2)
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
        choice, combos, res = measured_teacher(c, args.budget, log=log)
        nl = len(c.widths) - 2
        codes = np.stack([combo_codes(c, combos[k])[b] for b, k in enumerate(choice)])
        run = run_plan(c, codes, features=True)
        base = res[combos.index((2,) * nl)]
        used, feat = run["used"], run["features"]
        mask = (used >= 1) | (used == -2)  # unstable neurons (any order or the fallback)
        X = feat[mask]
        y = codes[mask]
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
    mean = X.mean(0)
    std = X.std(0) + 1e-3
    P = train(X, y, mean, std, epochs=args.epochs, log=log)
    cls, _ = B.mlp_classify(torch.tensor(P, device="cuda"), torch.tensor(X, device="cuda"), bf16=True)
    report["train_accuracy_bf16"] = float((cls.cpu().numpy() == y).mean())
    save(args.out, P, dict(records=int(X.shape[0]), accuracy=report["train_accuracy_bf16"], budget=args.budget))
    log(f"saved {args.out}")
    report["eval"] = evaluate(P, log=log)
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
