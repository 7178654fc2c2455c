"""Benchmark of the bound-propagation hot path on one MI355X.

A step is one pass of the whole path (input encoding, every layer's affine
map, bounds read-off, ReLU approximant and composition, output bounds) over
one batch of synthetic input: all boxes of the workload. Inputs are resident
in HBM before the timed region starts. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bounded neurons/s on 1 GPU + output-bound width: plain vs batched+learned form"
# Peaks of one MI355X: HBM3E 8 TB/s; FP64 / non-packed FP32 FMA on the vector
# ALUs: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s.
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12

WORKLOADS = {
    "cfg1": dict(k=1, form="plain", sched="per_box", precision="fp64"),
    "cfg2": dict(k=2, form="plain", sched="per_box", precision="fp64"),
    "cfg2_fp32": dict(k=2, form="plain", sched="per_box", precision="fp32"),
    "cfg4": dict(k=4, form="plain", sched="batched", precision="fp32"),
}


def composed_flops(case, used, L):
    """Algorithmic FLOPs of the order-2 compositions: for every neuron-bound
    that is composed (unstable neuron, kind == 2), one symmetric square of its
    (D+1)^n-coefficient pre-activation tensor = (C^2 + C)/2 multiply-adds."""
    n = case.n
    widths = case.widths
    col = 0
    D = 1
    total = 0.0
    for i in range(1, len(widths) - 1):
        h = widths[i]
        C = (D + 1) ** n
        k2 = int((used[:, col:col + h] == 2).sum())
        total += k2 * 2 * (C * C + C)
        col += h
        D *= L
    return total


def cpu_baseline(case, budget_s=10.0):
    """The oracle, as it stands, on the host cores: repeated passes over boxes
    of the workload until about `budget_s` seconds of CPU work."""
    from oracle import oracle as orc
    t0 = time.perf_counter()
    boxes = 0
    reps = 0
    while True:
        for i in range(case.n_boxes):
            orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=case.L,
                        plan=None if case.plan is None else case.plan[i])
            boxes += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=boxes * case.bounded_neurons_per_box / dt, unit="neurons/s", cores=orc.get_threads(),
                kind="oracle",
                sample=f"{boxes} box evaluations of the workload ({reps} pass(es) over its {case.n_boxes} box(es)) "
                       f"in {dt:.1f} s, FP64 Bernstein-literal oracle")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the boxes of a workload are independent and this build "
              "measures one GPU's share; --gpus N > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_14438_amd import bernnn as B
    from paper_2211_14438_amd import workloads as wl

    spec = WORKLOADS[args.workload]
    case = wl.CONFIGS[spec["k"]]()
    dev = "cuda:0"
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=dev)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=dev)
    kw = dict(L=case.L, precision=spec["precision"], sched=spec["sched"])
    total, one = net.workspace_size(case.n_boxes, **kw)
    ws = torch.empty(total + 256, dtype=torch.uint8, device=dev)
    r = B.bounds(net, lo, hi, workspace=ws, **kw)
    outs = {k: r[k] for k in ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "used_plan")}
    for _ in range(args.warmup):
        B.bounds(net, lo, hi, workspace=ws, outputs=outs, **kw)
    torch.cuda.synchronize()

    B.prof_reset()
    B.prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.bounds(net, lo, hi, workspace=ws, outputs=outs, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B.prof_enable(False)
    prof = B.prof_read()
    B.prof_reset()

    dt = t1 - t0
    ms_step = dt / args.steps * 1e3
    neurons = case.n_boxes * case.bounded_neurons_per_box
    value = neurons * args.steps / dt
    used = outs["used_plan"].cpu().numpy()
    width = float((outs["out_hi"] - outs["out_lo"]).mean().item())

    # roofline of the dominant kernel class (largest summed duration)
    kernels = {}
    for name, (launches, ms, by) in prof.items():
        kernels[name] = dict(launches=launches, avg_us=ms / launches * 1e3, total_ms=ms)
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0]
    launches, ms, by = prof[dom]
    if dom == "compose_square":
        flops = composed_flops(case, used, case.L) * args.steps
        achieved = flops / (ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=PEAK_VALU_TFLOPS, unit="TFLOP/s",
                    frac=achieved / PEAK_VALU_TFLOPS, traffic=None, kernel=dom,
                    per_launch_flops=flops / launches, avg_launch_us=ms / launches * 1e3)
    else:
        achieved = by / (ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s", frac=achieved / PEAK_HBM_GBS,
                    traffic=None, kernel=dom, per_launch_bytes=by / launches, avg_launch_us=ms / launches * 1e3)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "neurons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if spec["precision"] == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": case.name, "boxes": case.n_boxes, "net": "-".join(map(str, case.widths)),
                   "L": case.L, "precision": spec["precision"], "form": f"{spec['form']} ({spec['sched']})"},
        "mean_output_width": width,
        "stable_neurons_skipped": int(((used == 0) | (used == -1)).sum()),
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
