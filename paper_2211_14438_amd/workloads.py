"""Seeded synthetic workloads: networks, input boxes and per-neuron degree draws.

This module holds random-number draws only, none of the bound-propagation
arithmetic, so that the GPU library and the CPU oracle can be fed identical
inputs. Every array is FP64 and comes from ``numpy.random.default_rng(seed)``.

Shapes follow the five workloads the project measures (the paper's random
networks are fully connected ReLU nets over an input hyperrectangle,
Section 2.1; its Section 6 draws weights from U[-5,5], the workloads here use
N(0, 1/fan_in) for weights and biases, and U[-5,5] is kept as an option).
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Workload:
    name: str
    widths: List[int]                 # n, h_1, ..., h_H
    Ws: List[np.ndarray]              # W^(i), h_i x h_{i-1}
    bs: List[np.ndarray]              # b^(i), h_i
    box_lo: np.ndarray                # [n_boxes, n]
    box_hi: np.ndarray                # [n_boxes, n]
    L: int = 2                        # ReLU approximation order
    plan: Optional[np.ndarray] = None  # int8 [n_boxes, sum hidden] degree codes, or None
    precision: str = "fp64"
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.widths[0]

    @property
    def n_boxes(self):
        return self.box_lo.shape[0]

    @property
    def n_hidden(self):
        return int(sum(self.widths[1:-1]))

    @property
    def bounded_neurons_per_box(self):
        return int(sum(self.widths[1:]))

    def subset(self, idx):
        idx = np.asarray(idx)
        return Workload(self.name, self.widths, self.Ws, self.bs, self.box_lo[idx], self.box_hi[idx], self.L,
                        None if self.plan is None else self.plan[idx], self.precision, dict(self.meta))


def make_net(widths, seed, law="normal_fanin"):
    """Random fully connected ReLU network. ``normal_fanin``: W ~ N(0, 1/h_{i-1})
    and b with the same law; ``uniform5``: W, b ~ U[-5, 5] (the paper's law)."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for i in range(1, len(widths)):
        fan_in, h = widths[i - 1], widths[i]
        if law == "normal_fanin":
            W = rng.standard_normal((h, fan_in)) / np.sqrt(fan_in)
            b = rng.standard_normal(h) / np.sqrt(fan_in)
        elif law == "uniform5":
            W = rng.uniform(-5.0, 5.0, size=(h, fan_in))
            b = rng.uniform(-5.0, 5.0, size=h)
        else:
            raise ValueError(law)
        Ws.append(W)
        bs.append(b)
    return Ws, bs


def boxes_centred(n, n_boxes, seed, half_width=None, hw_range=None, centre_range=(-1.0, 1.0)):
    """Boxes with centres ~U[centre_range]^n and either a fixed half-width or
    one half-width per box drawn from U[hw_range]."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(centre_range[0], centre_range[1], size=(n_boxes, n))
    if half_width is not None:
        hw = np.full((n_boxes, 1), float(half_width))
    else:
        hw = rng.uniform(hw_range[0], hw_range[1], size=(n_boxes, 1))
    return c - hw, c + hw


def boxes_grid(n, splits, keep, seed, lo=-1.0, hi=1.0):
    """Uniform ``splits``-per-axis split of [lo,hi]^n; a seeded random subset of
    ``keep`` cells (as branch-and-bound refinement produces)."""
    rng = np.random.default_rng(seed)
    side = (hi - lo) / splits
    cells = np.stack(np.meshgrid(*[np.arange(splits)] * n, indexing="ij"), axis=-1).reshape(-1, n)
    pick = rng.permutation(cells.shape[0])[:keep]
    c = cells[pick].astype(np.float64)
    return lo + c * side, lo + (c + 1) * side


def degree_draws(n_boxes, n_hidden, seed, choices=(1, 2, 3)):
    rng = np.random.default_rng(seed)
    return rng.choice(np.asarray(choices, dtype=np.int8), size=(n_boxes, n_hidden)).astype(np.int8)


# The five measured workloads. Seeds: weights 100+k, boxes 200+k, degrees 300+k.
def cfg1():
    widths = [2, 5, 5, 1]
    Ws, bs = make_net(widths, 101)
    return Workload("tiny_2-5-5-1_L2_fp64", widths, Ws, bs, np.array([[-1.0, -1.0]]), np.array([[1.0, 1.0]]),
                    L=2, precision="fp64")


def cfg2():
    widths = [4, 20, 20, 20, 2]
    Ws, bs = make_net(widths, 102)
    lo, hi = boxes_centred(4, 1, 202, half_width=0.1)
    return Workload("plain_4-20-20-20-2_L2_1box", widths, Ws, bs, lo, hi, L=2, precision="fp64")


def cfg3(n_keep=1024):
    widths = [6, 50, 50, 4]
    Ws, bs = make_net(widths, 103)
    lo, hi = boxes_grid(6, 4, n_keep, 203)
    plan = degree_draws(lo.shape[0], 100, 303)
    return Workload("batched_6-50-50-4_1024cells_deg123", widths, Ws, bs, lo, hi, L=3, plan=plan,
                    precision="fp32")


def cfg4(n_boxes=256):
    widths = [8, 100, 100, 10]
    Ws, bs = make_net(widths, 104)
    lo, hi = boxes_centred(8, n_boxes, 204, hw_range=(0.02, 0.2))
    return Workload("batched_8-100-100-10_256boxes_L2", widths, Ws, bs, lo, hi, L=2, precision="fp32")


def cfg5(n_boxes=1024, net_seed=105):
    widths = [6, 64, 64, 64, 4]
    Ws, bs = make_net(widths, net_seed)
    lo, hi = boxes_centred(6, n_boxes, 205, half_width=0.05)
    return Workload("learned_6-64-64-64-4_1024boxes", widths, Ws, bs, lo, hi, L=2, precision="fp32")


CONFIGS = {1: cfg1, 2: cfg2, 3: cfg3, 4: cfg4, 5: cfg5}


def random_net_case(widths, seed, n_boxes=1, half_width=None, law="normal_fanin", L=2):
    """Small ad-hoc case for tests: network + boxes from one seed."""
    Ws, bs = make_net(widths, seed, law=law)
    if half_width is None:
        lo, hi = boxes_centred(widths[0], n_boxes, seed + 1, hw_range=(0.05, 0.6))
    else:
        lo, hi = boxes_centred(widths[0], n_boxes, seed + 1, half_width=half_width)
    return Workload(f"case_{'-'.join(map(str, widths))}_s{seed}", list(widths), Ws, bs, lo, hi, L=L)
