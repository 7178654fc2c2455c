"""Kernel-variant choices kept across processes.

bern_autotune stores its choice in the network handle only, so every process
would search again. This module keeps the choices in a JSON file keyed by
the device architecture, the network's layer widths and the options that
change which kernels run (order, precision, plan, schedule, Lin, box count),
and applies a stored choice instead of searching when the key matches.
"""
import json
import os

from . import bernnn as B

_KEY_OPTS = ("L", "precision", "plan", "sched", "lin", "max_wave")


def cache_key(arch, widths, n_boxes, **opts):
    """The key of one workload: architecture, widths, box count and the
    options that select kernels (others, such as buffers and streams, do not
    enter)."""
    parts = [str(arch), "-".join(str(int(w)) for w in widths), f"boxes={int(n_boxes)}"]
    for k in _KEY_OPTS:
        if k in opts and opts[k] is not None:
            parts.append(f"{k}={opts[k]}")
    return "|".join(parts)


def load(path):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data if isinstance(data, dict) else {}


def store(path, key, choice, ms):
    data = load(path)
    data[key] = {"choice": [int(v) for v in choice], "ms_per_pass": float(ms)}
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(net, widths, box_lo, box_hi, path, arch, reps=3, **opts):
    """Apply the cached choice for this workload if `path` holds one (after
    checking it names a valid variant of every parameter), else run the
    autotuner and store its choice. Returns (choice, ms per pass or None,
    True when taken from the cache)."""
    key = cache_key(arch, widths, box_lo.shape[0], **opts)
    hit = load(path).get(key)
    if hit:
        choice = hit.get("choice", [])
        variants = B.tune_variants()
        if len(choice) == len(variants) and all(0 <= c < v for c, v in zip(choice, variants)):
            B.tune_set(net, choice)
            return choice, hit.get("ms_per_pass"), True
    choice, ms = B.autotune(net, box_lo, box_hi, reps=reps, **opts)
    store(path, key, choice, ms)
    return choice, ms, False
