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

# form: "plain" = the paper's rule at order L; "learned" = the degree
# predictor's plan (timed against the plain form on the same boxes).
WORKLOADS = {
    "cfg1": dict(k=1, form="plain", sched="per_box", precision="fp64"),
    "cfg2": dict(k=2, form="plain", sched="per_box", precision="fp64"),
    "cfg2_fp32": dict(k=2, form="plain", sched="per_box", precision="fp32"),
    "cfg3": dict(k=3, form="given", sched="batched", precision="fp32"),
    "cfg4": dict(k=4, form="plain", sched="batched", precision="fp32"),
    "cfg5": dict(k=5, form="learned", sched="batched", precision="fp32", plain_sched="per_box"),
    "cfg5_batched_plain": dict(k=5, form="plain", sched="batched", precision="fp32"),
}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, budget_s=20.0):
    """The oracle, as it stands (FP64, Bernstein-literal), built -O3
    -march=native on this host and timed on its cores: a seeded sample of the
    workload's boxes (boxes are independent), first with every OpenMP thread,
    then single-threaded, each leg within its share of `budget_s` seconds
    (at least one box). Per-box times give the median and spread; `value`
    scales the all-core median to the metric's unit."""
    from oracle import oracle as orc
    orc.use_native()
    all_threads = orc.get_threads()
    order = np.random.default_rng(1234).permutation(case.n_boxes)

    def leg(threads, budget, cap):
        orc.set_threads(threads)
        times = []
        t_all = time.perf_counter()
        for i in order[:cap]:
            t0 = time.perf_counter()
            orc.network(case.Ws, case.bs, case.box_lo[i], case.box_hi[i], L=case.L,
                        plan=None if case.plan is None else case.plan[i])
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_all >= budget:
                break
        return np.array(times)

    multi = leg(all_threads, 0.6 * budget_s, 32)
    single = leg(1, 0.4 * budget_s, 32)
    orc.set_threads(all_threads)
    per_box = case.bounded_neurons_per_box

    def summary(t, threads):
        return dict(value=per_box / float(np.median(t)), threads=threads, boxes=int(t.size),
                    median_box_s=float(np.median(t)), min_box_s=float(t.min()), max_box_s=float(t.max()))

    m, s1 = summary(multi, all_threads), summary(single, 1)
    return dict(value=m["value"], unit="neurons/s", cores=all_threads, kind="oracle",
                sample=(f"{m['boxes']} seeded boxes of the workload's {case.n_boxes} with {all_threads} threads "
                        f"(median {m['median_box_s']:.3f} s per box), {s1['boxes']} single-threaded (median "
                        f"{s1['median_box_s']:.3f} s); FP64 Bernstein-literal oracle, gcc -O3 -march=native"),
                single_thread=s1, all_core=m, nproc=os.cpu_count(), cpu_model=_cpu_model())


def _ssize(n, D):
    from math import comb
    return comb(n + D, n) if D >= 0 else 0


def executed_work(case, used, L, plain, elem):
    """Executed work of one pass in the composition and affine-map classes,
    from the rule each hidden neuron took (used_plan) and the degrees that
    follow from them: per box, a hidden layer's post degree is the largest of
    its neurons' (inactive 0, active D, fallback 1, order k: k D; the plain
    rule stores every neuron at L D). Square compositions (order 2) sum every
    index pair of the stored coefficients once (S (S + 1) / 2 FMAs per bound,
    S = C(n + D, n)); orders k >= 3 take k - 1 Horner products of the
    (D, m D) tables; the affine map multiplies each live input coefficient by
    every output row twice (midpoint and radius). Bytes: tensors read and
    written. Returns {class: (flops, bytes)}."""
    n, widths = case.n, case.widths
    nb = used.shape[0]
    D = np.ones(nb, dtype=np.int64)
    sq_f = sq_b = hz_f = gm_f = gm_b = 0.0
    col = 0
    for i in range(1, len(widths) - 1):
        h, hn = widths[i], widths[i + 1]
        k = used[:, col:col + h].astype(np.int64)
        deg = np.where(k == 0, 0, np.where(k == -1, D[:, None], np.where(k == -2, 1, k * D[:, None])))
        Dout = np.full(nb, L, np.int64) * D if plain else deg.max(axis=1)
        for d in np.unique(D):
            rows = D == d
            S = _ssize(n, int(d))
            n2 = int((k[rows] == 2).sum())
            sq_f += 2.0 * 2 * n2 * S * (S + 1) / 2
            sq_b += 2 * n2 * elem * (S + _ssize(n, 2 * int(d)))
            for order in range(3, 9):
                no = int((k[rows] == order).sum())
                if no:
                    hz_f += 2.0 * 2 * no * sum(S * _ssize(n, m * int(d)) for m in range(1, order))
        for b in range(nb):
            so = _ssize(n, int(Dout[b]))
            si = _ssize(n, int(D[b]))
            sm = _ssize(n, int(min(D[b], Dout[b])))
            kb = k[b]
            live = so * int((kb >= 2).sum()) + sm * int(((kb == 1) | (kb == -2)).sum()) + si * int((kb == -1).sum())
            gm_f += 2.0 * 2 * hn * live
            gm_b += elem * (2 * live + 2 * hn * so)
        D = Dout
        col += h
    return {"compose_square": (sq_f, sq_b), "compose_horner": (hz_f, 0.0), "gemm": (gm_f, gm_b)}


def verify_demo(torch):
    """Branch and bound (bern_verify) of the property "output <= its sampled
    median" on a network of Fig. 4's shape ([2,20,20,1], weights and biases
    U[-5,5]) over [-1,1]^2, FP32 padded, L = 2: the input-volume fractions
    verified, violated and left undecided after 12 rounds, and the fraction
    decided per second of the call (host time, bounds of every round
    included)."""
    from paper_2211_14438_amd import bernnn as B
    from paper_2211_14438_amd import workloads as wl
    Ws, bs = wl.make_net([2, 20, 20, 1], 1000, law="uniform5")
    net = B.Net(Ws, bs)
    g = np.linspace(-1.0, 1.0, 201)
    x = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    z = x
    for i, (W, b) in enumerate(zip(Ws, bs)):
        z = z @ W.T + b
        if i < len(Ws) - 1:
            z = np.maximum(z, 0.0)
    tau = float(np.median(z[:, 0]))
    lo, hi = np.array([[-1.0, -1.0]]), np.array([[1.0, 1.0]])
    B.verify(net, lo, hi, 0, tau, max_rounds=2, precision="fp32")  # warm-up: tables, first allocations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = B.verify(net, lo, hi, 0, tau, max_rounds=12, max_boxes=1 << 16, precision="fp32")
    dt = time.perf_counter() - t0
    net.close()
    decided = r["verified"] + r["violated"]
    return dict(net="2-20-20-1 U[-5,5]", property="output <= sampled median", rounds=r["rounds"],
                verified=r["verified"], violated=r["violated"], undecided=r["undecided"],
                boxes_bounded=r["boxes_bounded"], seconds=dt, decided_fraction_per_s=decided / dt,
                verified_fraction_per_s=r["verified"] / dt)


# The paper's Section 6.1 medians (50 random networks, weights and biases
# U[-5,5], box [-1,1]^n, L = 2 unless stated; one NVIDIA RTX 2080 Ti and
# PyTorch): seconds per network, and relative volumes where printed.
PAPER_SWEEPS = {
    "fig4_L": {"shape": [2, 20, 20, 1], "values": {2: (1.29, 1823.96), 3: (1.70, 1524.99), 4: (2.44, 1348.26),
                                                   5: (3.47, 1248.37), 6: (5.11, 1173.46)}},
    "fig5_n": {"values": {2: 1.17, 3: 1.34, 4: 1.54, 5: 1.759, 6: 2.79, 7: 3.36, 8: 6.56}},
    "fig6_Ne": {"values": {10: 0.45, 20: 1.22, 40: 3.87, 60: 8.48, 80: 14.64, 100: 18.25}},
    "fig7_depth": {"values": {1: 0.28, 2: 1.27, 3: 2.291, 4: 3.23, 5: 4.25}},
}


def sweeps(torch, nets=50):
    """The shapes of Figs. 4-7 on this GPU: per shape, `nets` seeded random
    networks (U[-5,5] weights and biases), one box [-1,1]^n, the plain rule
    in FP64 one box per launch sequence (the paper's setting): median time of
    one bound computation (HIP-synchronised wall time after a warm-up run)
    and median relative volume, printed one JSON line per figure beside the
    paper's medians."""
    from paper_2211_14438_amd import bernnn as B
    from paper_2211_14438_amd import workloads as wl
    figs = {
        "fig4_L": [([2, 20, 20, 1], L) for L in (2, 3, 4, 5, 6)],
        "fig5_n": [([n, 20, 20, 1], 2) for n in range(2, 9)],
        "fig6_Ne": [([2, Ne, Ne, 1], 2) for Ne in (10, 20, 40, 60, 80, 100)],
        "fig7_depth": [([2] + [20] * d + [1], 2) for d in range(1, 6)],
    }
    for fig, cases in figs.items():
        rows = []
        for widths, L in cases:
            n = widths[0]
            lo = torch.full((1, n), -1.0, dtype=torch.float64, device="cuda:0")
            hi = torch.full((1, n), 1.0, dtype=torch.float64, device="cuda:0")
            ts, vs = [], []
            for s in range(nets):
                Ws, bs = wl.make_net(widths, 1000 + s, law="uniform5")
                net = B.Net(Ws, bs)
                B.rel_volume(net, lo, hi, L=L, precision="fp64", sched="per_box")  # tables, buffers
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = B.rel_volume(net, lo, hi, L=L, precision="fp64", sched="per_box")
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                vs.append(float(r["rel_vol"][0, 0]))
                net.close()
            key = {"fig4_L": L, "fig5_n": n, "fig6_Ne": widths[1], "fig7_depth": len(widths) - 2}[fig]
            paper = PAPER_SWEEPS[fig]["values"].get(key)
            rows.append(dict(shape=widths, L=L, median_s=float(np.median(ts)),
                             neurons_per_s=sum(widths[1:]) / float(np.median(ts)),
                             median_rel_volume=float(np.median(vs)),
                             paper_median_s=paper[0] if isinstance(paper, tuple) else paper,
                             paper_median_rel_volume=paper[1] if isinstance(paper, tuple) else None))
        print(json.dumps({"sweep": fig, "nets": nets, "precision": "fp64", "rows": rows}), flush=True)


def roof(flops, bytes_, ms, peak_flops):
    """Roofline of a class by the intensity of its executed work: the FP64
    vector roof above the ridge point, the HBM roof below it."""
    ridge = peak_flops * 1e12 / (PEAK_HBM_GBS * 1e9)
    if flops > 0 and (bytes_ <= 0 or flops / bytes_ > ridge):
        a = flops / (ms * 1e-3) / 1e12
        return dict(bound="alu", achieved=a, peak=peak_flops, unit="TFLOP/s", frac=a / peak_flops,
                    intensity=flops / bytes_ if bytes_ > 0 else None)
    a = bytes_ / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=a, peak=PEAK_HBM_GBS, unit="GB/s", frac=a / PEAK_HBM_GBS,
                intensity=flops / bytes_ if bytes_ > 0 else None)


def measured_traffic(workload, cls):
    """HBM bytes per launch of kernel class `cls` on `workload`, from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary under profiles/ (scaled by the
    copy calibration recorded there), or None when there is none or when the
    kernel sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("TRAFFIC "):
            continue
        rec = json.loads(line[len("TRAFFIC "):])
        if rec.get("class") != cls:
            continue
        h = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, "paper_2211_14438_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != rec["source_sha256_16"]:
            return None
        return rec["hbm_bytes_per_launch"]
    return None


def copy_calibration(torch, nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of `nbytes` bytes, `reps` times: the
    HBM byte counters read on it give the factor between counted and moved
    bytes (it moves 2 * nbytes per launch: one read, one write)."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": reps,
                      "GB_per_s": 2 * nbytes / dt / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg5", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-plain", action="store_true", help="do not time the plain form (profiling runs)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in kernel variants")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of kernel-variant choices per device architecture, shape and options: a stored "
                         "choice is applied instead of autotuning, a new search's choice is stored")
    ap.add_argument("--tune", default=None,
                    help="comma-separated kernel variants to use instead of autotuning (profiling runs)")
    ap.add_argument("--eager", action="store_true",
                    help="launch eagerly; by default batched runs replay their launch sequence as one captured "
                         "graph (per-neuron plans with their degree classes listed on the device)")
    ap.add_argument("--sweep", action="store_true",
                    help="only time the network shapes of the paper's Figs. 4-7 (one JSON line per figure)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain device copy of 1 GiB (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the boxes of a workload are independent, so one GPU's share "
              "is what is measured; --gpus N > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.sweep:
        sweeps(torch)
        return
    from paper_2211_14438_amd import bernnn as B
    from paper_2211_14438_amd import workloads as wl

    spec = WORKLOADS[args.workload]
    case = wl.CONFIGS[spec["k"]]()
    dev = "cuda:0"
    net = B.Net(case.Ws, case.bs)
    lo = torch.tensor(case.box_lo, dtype=torch.float64, device=dev)
    hi = torch.tensor(case.box_hi, dtype=torch.float64, device=dev)
    free, _ = torch.cuda.mem_get_info()

    def setup(form, sched):
        kw = dict(L=case.L, precision=spec["precision"], sched=sched)
        if form == "learned":
            from paper_2211_14438_amd import predictor as PR
            kw.update(plan="learned", pred=PR.load_predictor())
        elif form == "given":
            kw.update(plan="given", degree_plan=torch.tensor(case.plan, dtype=torch.int8, device=dev))
        total, one = net.workspace_size(case.n_boxes, **{k: v for k, v in kw.items() if k != "degree_plan"})
        size = int(min(total, max(one, 0.45 * free)))
        kw["workspace"] = torch.empty(size + 256, dtype=torch.uint8, device=dev)
        r = B.bounds(net, lo, hi, **kw)
        kw["outputs"] = {k: r[k] for k in ("neuron_lo", "neuron_hi", "out_lo", "out_hi", "used_plan")}
        if sched == "batched" and not args.eager:
            kw["graph"] = True
        return kw

    def autotune(kw):
        # one-time setup, outside the timed region: kernel variants for this net and workload,
        # each timed over about 10 ms of passes (2 to 16) so that short passes are not picked on noise
        tkw = {k: v for k, v in kw.items() if k not in ("graph",)}
        t0 = time.perf_counter()
        B.bounds(net, lo, hi, **tkw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.bounds(net, lo, hi, **tkw)
        torch.cuda.synchronize()
        reps = int(min(16, max(2, round(0.010 / max(time.perf_counter() - t1, 1e-6)))))
        if args.tune_cache:
            from paper_2211_14438_amd import tune_cache as TC
            arch = torch.cuda.get_device_properties(0).gcnArchName
            choice, tms, cached = TC.tuned(net, case.widths, lo, hi, args.tune_cache, arch, reps=reps, **tkw)
            return dict(choice=choice, seconds=time.perf_counter() - t0, ms_per_pass=tms, cached=cached, reps=reps)
        choice, tms = B.autotune(net, lo, hi, reps=reps, **tkw)
        return dict(choice=choice, seconds=time.perf_counter() - t0, ms_per_pass=tms, reps=reps)

    def timed(kw, steps, profile):
        for _ in range(args.warmup):
            B.bounds(net, lo, hi, **kw)
        torch.cuda.synchronize()
        if profile:
            B.prof_reset()
            B.prof_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            B.bounds(net, lo, hi, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = None
        if profile:
            B.prof_enable(False)
            prof = B.prof_read()
            B.prof_reset()
        return dt, prof

    kw = setup(spec["form"], spec["sched"])
    if args.tune:
        B.tune_set(net, [int(v) for v in args.tune.split(",")])
        tuned = dict(choice=B.tune_get(net), seconds=0.0, ms_per_pass=None, fixed=True)
    else:
        tuned = None if args.no_autotune else autotune(kw)
    graph = bool(kw.get("graph"))
    # the timed region that gives `value` runs without per-launch events; the
    # kernel classes are then timed over the same number of steps with a pair
    # of HIP events around every launch (eagerly when graphs are replayed)
    dt_graph, _ = timed(kw, args.steps, False)
    eager_kw = {k: v for k, v in kw.items() if k != "graph"}
    st = B.bounds(net, lo, hi, **kw)["stats"]
    dt_eager = timed(eager_kw, args.steps, False)[0] if graph else dt_graph
    # `value`: the faster of the two launch forms of the same work, both
    # reported under "launch"
    dt = min(dt_graph, dt_eager)
    form = "graph" if graph and dt_graph <= dt_eager else "eager"
    _, prof = timed(eager_kw, args.steps, True)
    outs = kw["outputs"]
    ms_step = dt / args.steps * 1e3
    neurons = case.n_boxes * case.bounded_neurons_per_box
    value = neurons * args.steps / dt
    used = outs["used_plan"].cpu().numpy()
    width = float((outs["out_hi"] - outs["out_lo"]).mean().item())
    plain_line = None
    plain_batched = None
    if spec["form"] != "plain" and not args.skip_plain:
        del kw
        torch.cuda.empty_cache()
        psteps = max(1, min(args.steps, 3))
        lines = {}
        for psched in sorted({spec.get("plain_sched", "batched"), "batched"}):
            pkw = setup("plain", psched)
            pdt, _ = timed(pkw, psteps, False)
            if pkw.get("graph"):  # the faster launch form, as for `value`
                pdt = min(pdt, timed({k: v for k, v in pkw.items() if k != "graph"}, psteps, False)[0])
            pw = float((pkw["outputs"]["out_hi"] - pkw["outputs"]["out_lo"]).mean().item())
            lines[psched] = dict(form=f"plain order-{case.L} ({psched})", value=neurons * psteps / pdt,
                                 ms_per_step=pdt / psteps * 1e3, mean_output_width=pw)
            del pkw
            torch.cuda.empty_cache()
        plain_line = lines[spec.get("plain_sched", "batched")]
        plain_batched = lines["batched"]

    # roofline of the dominant kernel class (largest summed duration), from
    # the work its kernels execute as the library counts it per launch (the
    # tree read-off: its folds, expansions, lane tiles and extrema; bytes:
    # stored tensors read, bounds and rules written): the FP64 vector roof
    # when that work's flops per byte exceed the ridge point, else HBM. The
    # read-off's arithmetic is FP64 in both precision modes.
    kernels = {}
    for name, (launches, ms, by, fl) in prof.items():
        kernels[name] = dict(launches=launches, avg_us=ms / launches * 1e3, total_ms=ms)
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0]
    launches, ms, by, fl = prof[dom]
    roofline = roof(fl / launches, by / launches, ms / launches, PEAK_VALU_TFLOPS)
    roofline.update(traffic=measured_traffic(case.name, dom), kernel=dom, per_launch_flops=fl / launches,
                    per_launch_bytes=by / launches, avg_launch_us=ms / launches * 1e3)
    # the composition and affine-map classes: executed work of the timed
    # passes from the rules the neurons took, over the classes' event times
    classes = {}
    if used is not None:
        elem = 8 if spec["precision"] == "fp64" else 4
        work = executed_work(case, used[:, :case.n_hidden], case.L, spec["form"] == "plain", elem)
        for cls, (wf, wb) in work.items():
            if cls in prof and wf > 0:
                n_, ms_, _, _ = prof[cls]
                classes[cls] = roof(wf * args.steps / n_, wb * args.steps / n_, ms_ / n_, PEAK_VALU_TFLOPS)
                classes[cls].update(avg_launch_us=ms_ / n_ * 1e3, launches=n_)

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
        "roofline": roofline,
        "class_rooflines": classes,
        "kernels": kernels,
    }
    if tuned is not None:
        line["autotune"] = tuned
    line["kernel_timing"] = ("per-launch HIP events over a second timed region of the same steps" +
                             (", launched eagerly (value: one captured graph per pass)" if graph else ""))
    line["launch"] = dict(value_from=form, graph=bool(st["graph"]), device_classes=bool(st["device_classes"]),
                          eager_ms_per_step=dt_eager / args.steps * 1e3,
                          graph_ms_per_step=dt_graph / args.steps * 1e3 if graph else None)
    if plain_line is not None:
        line["plain"] = plain_line
        line["speedup_vs_plain"] = value / plain_line["value"]
        line["width_ratio_vs_plain"] = width / plain_line["mean_output_width"]
        line["plain_batched"] = plain_batched
        line["speedup_vs_batched_plain"] = value / plain_batched["value"]
        line["width_ratio_vs_batched_plain"] = width / plain_batched["mean_output_width"]
    if not args.skip_plain:
        line["verify"] = verify_demo(torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
