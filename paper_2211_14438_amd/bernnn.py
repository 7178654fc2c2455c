"""Thin Python binding of ``libbernnn.so`` (the C ABI declared in
``include/bernnn.h``).

Argument marshalling only: PyTorch provides device memory and the stream, every
step of the computation runs in the library's HIP kernels. There is no CPU
fallback: if the library is missing the import of this module's functions
raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbernnn.so")

BERN_OK = 0
FP64, FP32_PADDED = 0, 1
PLAN_PLAIN, PLAN_GIVEN, PLAN_LEARNED = 0, 1, 2
SCHED_PER_BOX, SCHED_BATCHED = 0, 1

_PREC = {"fp64": FP64, "fp32": FP32_PADDED, "fp32_padded": FP32_PADDED}
_PLAN = {"plain": PLAN_PLAIN, "given": PLAN_GIVEN, "learned": PLAN_LEARNED}
_SCHED = {"per_box": SCHED_PER_BOX, "batched": SCHED_BATCHED}

_vp = ctypes.c_void_p


class bern_opts(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("precision", ctypes.c_int32), ("plan", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("pred", ctypes.c_void_p), ("features", ctypes.c_void_p),
                ("max_wave", ctypes.c_int32), ("graph", ctypes.c_int32), ("lin", ctypes.c_int32),
                ("no_raise", ctypes.c_int32), ("mem_budget_bytes", ctypes.c_uint64), ("counters", ctypes.c_void_p)]


class bern_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("loss_out", ctypes.c_void_p), ("reserved", ctypes.c_int32 * 4)]


COUNTERS = ("hidden", "inactive", "active", "fallback", "order1", "order2", "order3up", "max_pad")


class bern_stats(ctypes.Structure):
    _fields_ = [("n_waves", ctypes.c_int32), ("boxes_per_wave", ctypes.c_int32), ("out_degree", ctypes.c_int32),
                ("lin_layers", ctypes.c_int32), ("workspace_used", ctypes.c_uint64),
                ("enqueue_ms", ctypes.c_double), ("graph", ctypes.c_int32), ("device_classes", ctypes.c_int32),
                ("reserved", ctypes.c_uint64 * 4)]


def _stats(st):
    return dict(n_waves=st.n_waves, boxes_per_wave=st.boxes_per_wave, out_degree=st.out_degree,
                lin_layers=st.lin_layers, workspace_used=st.workspace_used, enqueue_ms=st.enqueue_ms,
                graph=st.graph, device_classes=st.device_classes)


class bern_verify_result(ctypes.Structure):
    _fields_ = [("verified", ctypes.c_double), ("violated", ctypes.c_double), ("undecided", ctypes.c_double),
                ("rounds", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("boxes_bounded", ctypes.c_int64),
                ("undecided_boxes", ctypes.c_int64), ("log_cap", ctypes.c_int64), ("log_count", ctypes.c_int64),
                ("log_lo", ctypes.c_void_p), ("log_hi", ctypes.c_void_p), ("log_out_lo", ctypes.c_void_p),
                ("log_out_hi", ctypes.c_void_p), ("log_status", ctypes.c_void_p)]


class BernError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


_LIB = None


def lib():
    """Load the in-tree HIP library (raises if it was not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2211_14438_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.bern_status_str.restype = ctypes.c_char_p
    L.bern_status_str.argtypes = [i32]
    L.bern_last_error.restype = ctypes.c_char_p
    L.bern_last_error.argtypes = []
    L.bern_opts_default.restype = None
    L.bern_opts_default.argtypes = [ctypes.POINTER(bern_opts)]
    L.bern_net_create.restype = i32
    L.bern_net_create.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_vp)]
    L.bern_net_destroy.restype = None
    L.bern_net_destroy.argtypes = [_vp]
    for f in ("bern_net_inputs", "bern_net_hidden", "bern_net_outputs"):
        getattr(L, f).restype = i32
        getattr(L, f).argtypes = [_vp]
    L.bern_workspace_size.restype = i32
    L.bern_workspace_size.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.bern_bounds.restype = i32
    L.bern_bounds.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, sz,
                              _vp, ctypes.POINTER(bern_stats)]
    L.bern_output_polys.restype = i32
    L.bern_output_polys.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, _vp, _vp, _vp, i32, _vp, _vp, _vp, _vp, _vp,
                                    sz, _vp]
    L.bern_rel_volume.restype = i32
    L.bern_rel_volume.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, sz, _vp]
    L.bern_verify.restype = i32
    L.bern_verify.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, _vp, _vp, i32, ctypes.c_double, i32, i64,
                              ctypes.POINTER(bern_verify_result)]
    L.bern_bounds_noalloc.restype = i32
    L.bern_bounds_noalloc.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      ctypes.POINTER(bern_stats)]
    L.bern_bounds_host.restype = i32
    L.bern_bounds_host.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   ctypes.POINTER(bern_stats)]
    L.bern_basis_minmax_scratch.restype = sz
    L.bern_basis_minmax_scratch.argtypes = [i32, i32, i64]
    L.bern_basis_minmax.restype = i32
    L.bern_basis_minmax.argtypes = [i32, i32, i64, _vp, i32, _vp, _vp, _vp, _vp, _vp, sz, _vp]
    L.bern_poly_mul.restype = i32
    L.bern_poly_mul.argtypes = [i32, i32, i32, i64, _vp, _vp, _vp, i32, _vp]
    L.bern_relu_poly.restype = i32
    L.bern_relu_poly.argtypes = [i64, i32, _vp, _vp, _vp, _vp, _vp]
    L.bern_prof_enable.restype = i32
    L.bern_prof_enable.argtypes = [i32]
    L.bern_prof_reset.restype = i32
    L.bern_prof_reset.argtypes = []
    L.bern_prof_classes.restype = i32
    L.bern_prof_classes.argtypes = []
    L.bern_prof_name.restype = ctypes.c_char_p
    L.bern_prof_name.argtypes = [i32]
    L.bern_prof_read.restype = i32
    L.bern_prof_read.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    fp = ctypes.POINTER(ctypes.c_float)
    L.bern_pred_params.restype = i32
    L.bern_pred_params.argtypes = []
    L.bern_pred_create.restype = i32
    L.bern_pred_create.argtypes = [fp, i64, ctypes.POINTER(_vp)]
    L.bern_pred_destroy.restype = None
    L.bern_pred_destroy.argtypes = [_vp]
    L.bern_pred_load.restype = i32
    L.bern_pred_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(_vp)]
    L.bern_train_opts_default.restype = None
    L.bern_train_opts_default.argtypes = [ctypes.POINTER(bern_train_opts)]
    L.bern_pred_train.restype = i32
    L.bern_pred_train.argtypes = [_vp, _vp, i64, ctypes.POINTER(bern_train_opts), ctypes.c_char_p, ctypes.c_char_p,
                                  ctypes.POINTER(_vp)]
    L.bern_mlp_backward_scratch.restype = sz
    L.bern_mlp_backward_scratch.argtypes = [i64]
    L.bern_mlp_forward.restype = i32
    L.bern_mlp_forward.argtypes = [_vp, i64, _vp, _vp, i32, _vp]
    L.bern_mlp_backward.restype = i32
    L.bern_mlp_backward.argtypes = [_vp, i64, _vp, _vp, _vp, _vp, _vp, _vp]
    L.bern_mlp_adam.restype = i32
    L.bern_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, _vp]
    L.bern_tune_params.restype = i32
    L.bern_tune_params.argtypes = []
    L.bern_tune_variants.restype = i32
    L.bern_tune_variants.argtypes = [i32]
    L.bern_tune_get.restype = i32
    L.bern_tune_get.argtypes = [_vp, ctypes.POINTER(i32)]
    L.bern_tune_set.restype = i32
    L.bern_tune_set.argtypes = [_vp, ctypes.POINTER(i32)]
    L.bern_autotune.restype = i32
    L.bern_autotune.argtypes = [_vp, ctypes.POINTER(bern_opts), i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                sz, _vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    L.bern_mlp_classify.restype = i32
    L.bern_mlp_classify.argtypes = [_vp, i64, _vp, _vp, _vp, i32, _vp]
    _LIB = L
    return L


EXPORTED = ("bern_opts_default", "bern_net_create", "bern_net_destroy", "bern_net_inputs", "bern_net_hidden",
            "bern_net_outputs", "bern_workspace_size", "bern_bounds", "bern_basis_minmax_scratch",
            "bern_basis_minmax", "bern_poly_mul", "bern_relu_poly", "bern_status_str", "bern_last_error",
            "bern_prof_enable", "bern_prof_reset", "bern_prof_classes", "bern_prof_name", "bern_prof_read",
            "bern_pred_params", "bern_pred_create", "bern_pred_destroy", "bern_mlp_backward_scratch",
            "bern_mlp_forward", "bern_mlp_backward", "bern_mlp_adam", "bern_mlp_classify", "bern_tune_params",
            "bern_tune_variants", "bern_tune_get", "bern_tune_set", "bern_autotune", "bern_bounds_noalloc",
            "bern_pred_load", "bern_pred_train", "bern_train_opts_default")

NOALLOC_SCRATCH_BYTES = 64 << 20  # BERN_NOALLOC_SCRATCH_BYTES


def status_str(s):
    return lib().bern_status_str(int(s)).decode()


def _check(st):
    if st != BERN_OK:
        raise BernError(st, lib().bern_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_opts(L=2, precision="fp64", plan="plain", sched="per_box", max_wave=0, pred=None, features=None,
              graph=False, lin=0, mem_budget=0, counters=None, no_raise=False):
    o = bern_opts()
    lib().bern_opts_default(ctypes.byref(o))
    o.L = int(L)
    o.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    o.plan = _PLAN[plan] if isinstance(plan, str) else int(plan)
    o.sched = _SCHED[sched] if isinstance(sched, str) else int(sched)
    o.max_wave = int(max_wave)
    o.pred = None if pred is None else (pred.handle if isinstance(pred, Predictor) else pred)
    o.features = None if features is None else features.data_ptr()
    o.graph = 1 if graph else 0
    o.lin = int(lin)
    o.no_raise = 1 if no_raise else 0
    o.mem_budget_bytes = int(mem_budget)
    o.counters = None if counters is None else counters.data_ptr()
    return o


def read_counters(counters):
    """The bern_opts.counters entries of a finished call as a dict (the
    largest output pad decoded from its double bits)."""
    v = counters.cpu().numpy().astype(np.int64)
    d = {k: int(x) for k, x in zip(COUNTERS, v)}
    d["max_pad"] = float(np.array([v[7]], dtype=np.int64).view(np.float64)[0])
    return d


N_PARAMS = 5012


class Predictor:
    """Degree predictor on the current device (parameters copied at creation,
    or read from a predictor file with ``Predictor.load``)."""

    def __init__(self, params=None, handle=None):
        if handle is not None:
            self.handle = handle
            self.params = None
            return
        params = np.ascontiguousarray(params, dtype=np.float32)
        h = _vp()
        _check(lib().bern_pred_create(params.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), params.size,
                                      ctypes.byref(h)))
        self.handle = h
        self.params = params

    @classmethod
    def load(cls, path):
        h = _vp()
        _check(lib().bern_pred_load(os.fsencode(path), ctypes.byref(h)))
        return cls(handle=h)

    def close(self):
        if getattr(self, "handle", None):
            lib().bern_pred_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pred_train(X, y, path=None, epochs=40, batch=8192, lr=3e-3, seed=0, meta=None, want_predictor=True):
    """Train the degree predictor on host records (bern_pred_train): X
    [N, 8] float32 features, y [N] int8 classes. Writes ``path`` (if given)
    and returns (Predictor or None, per-epoch mean losses)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int8)
    t = bern_train_opts()
    lib().bern_train_opts_default(ctypes.byref(t))
    t.epochs, t.batch, t.lr, t.seed = int(epochs), int(batch), float(lr), int(seed)
    losses = np.zeros(int(epochs), dtype=np.float32)
    t.loss_out = losses.ctypes.data
    h = _vp()
    _check(lib().bern_pred_train(ctypes.c_void_p(X.ctypes.data), ctypes.c_void_p(y.ctypes.data), X.shape[0],
                                 ctypes.byref(t), None if path is None else os.fsencode(path),
                                 None if meta is None else meta.encode(),
                                 ctypes.byref(h) if want_predictor else None))
    return (Predictor(handle=h) if want_predictor else None), losses


def mlp_forward(P, X, bf16=False, stream=None):
    import torch
    N = X.shape[0]
    logits = torch.empty((N, 4), dtype=torch.float32, device=X.device)
    _check(lib().bern_mlp_forward(_ptr(P), N, _ptr(X.contiguous()), _ptr(logits), 1 if bf16 else 0, _stream(stream)))
    return logits


def mlp_backward(P, X, y, scratch=None, stream=None):
    import torch
    N = X.shape[0]
    G = torch.empty(N_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    if scratch is None:
        scratch = torch.empty(lib().bern_mlp_backward_scratch(N), dtype=torch.uint8, device=X.device)
    _check(lib().bern_mlp_backward(_ptr(P), N, _ptr(X.contiguous()), _ptr(y.contiguous()), _ptr(G), _ptr(loss),
                                   _ptr(scratch), _stream(stream)))
    return G, loss


def mlp_adam(P, G, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().bern_mlp_adam(_ptr(P), _ptr(G), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                               float(beta2), float(eps), _stream(stream)))


def mlp_classify(P, X, bf16=True, stream=None):
    import torch
    N = X.shape[0]
    logits = torch.empty((N, 4), dtype=torch.float32, device=X.device)
    cls = torch.empty(N, dtype=torch.int8, device=X.device)
    _check(lib().bern_mlp_classify(_ptr(P), N, _ptr(X.contiguous()), _ptr(logits), _ptr(cls), 1 if bf16 else 0,
                                   _stream(stream)))
    return cls, logits


class Net:
    """A network on the current HIP device (weights copied at creation)."""

    def __init__(self, Ws, bs):
        self.widths = [int(Ws[0].shape[1])] + [int(w.shape[0]) for w in Ws]
        self.H = len(Ws)
        W = np.ascontiguousarray(np.concatenate([np.asarray(w, np.float64).ravel() for w in Ws]))
        b = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64).ravel() for x in bs]))
        widths = (ctypes.c_int32 * (self.H + 1))(*self.widths)
        h = _vp()
        _check(lib().bern_net_create(self.H, widths, W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h)))
        self.handle = h
        self.n = self.widths[0]
        self.n_hidden = int(sum(self.widths[1:-1]))
        self.n_out = self.widths[-1]

    def close(self):
        if getattr(self, "handle", None):
            lib().bern_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self, n_boxes, **opt):
        o = make_opts(**opt)
        total, one = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().bern_workspace_size(self.handle, ctypes.byref(o), int(n_boxes), ctypes.byref(total),
                                         ctypes.byref(one)))
        return total.value, one.value


def _prepare(net, box_lo, box_hi, L, precision, plan, sched, degree_plan, max_wave, workspace, outputs, pred,
             features, graph, lin=0, mem_budget=0, counters=None, no_raise=False):
    import torch
    dev = box_lo.device
    assert box_lo.dtype == torch.float64 and box_hi.dtype == torch.float64
    box_lo = box_lo.contiguous()
    box_hi = box_hi.contiguous()
    nb = box_lo.shape[0]
    o = make_opts(L=L, precision=precision, plan=plan, sched=sched, max_wave=max_wave, pred=pred, features=features,
                  graph=graph, lin=lin, mem_budget=mem_budget, counters=counters, no_raise=no_raise)
    if outputs is None:
        nh = max(net.n_hidden, 1)
        outputs = dict(
            neuron_lo=torch.empty((nb, nh), dtype=torch.float64, device=dev),
            neuron_hi=torch.empty((nb, nh), dtype=torch.float64, device=dev),
            out_lo=torch.empty((nb, net.n_out), dtype=torch.float64, device=dev),
            out_hi=torch.empty((nb, net.n_out), dtype=torch.float64, device=dev),
            used_plan=torch.empty((nb, nh), dtype=torch.int8, device=dev),
        )
    if workspace is None:
        total, one = net.workspace_size(nb, L=L, precision=precision, plan=plan, sched=sched, max_wave=max_wave,
                                        pred=pred, lin=lin, mem_budget=mem_budget)
        workspace = torch.empty(total + 256, dtype=torch.uint8, device=dev)
    ws_ptr = workspace.data_ptr()
    pad = (-ws_ptr) % 256
    ws_bytes = workspace.numel() - pad
    if degree_plan is not None:
        degree_plan = degree_plan.contiguous()
    args = [net.handle, ctypes.byref(o), nb, _ptr(box_lo), _ptr(box_hi), _ptr(degree_plan),
            _ptr(outputs["neuron_lo"]), _ptr(outputs["neuron_hi"]), _ptr(outputs["out_lo"]), _ptr(outputs["out_hi"]),
            _ptr(outputs.get("used_plan")), ctypes.c_void_p(ws_ptr + pad), ws_bytes]
    # keep the tensors the pointers refer to alive for the call
    return args, dict(outputs), workspace, (o, box_lo, box_hi, degree_plan)


def bounds(net, box_lo, box_hi, L=2, precision="fp64", plan="plain", sched="per_box", degree_plan=None,
           max_wave=0, workspace=None, stream=None, outputs=None, pred=None, features=None, graph=False, lin=0,
           mem_budget=0, counters=None, no_raise=False):
    """Bounds of every box. ``box_lo``/``box_hi``: float64 CUDA tensors
    [n_boxes, n]. Returns a dict of CUDA tensors (neuron_lo/hi, out_lo/hi,
    used_plan) plus the run statistics. Enqueued on ``stream``. With
    ``graph`` the launch sequence is captured once and replayed as one graph
    launch; per-neuron plans then list their degree classes on the device."""
    args, res, workspace, keep = _prepare(net, box_lo, box_hi, L, precision, plan, sched, degree_plan, max_wave,
                                          workspace, outputs, pred, features, graph, lin, mem_budget, counters,
                                          no_raise)
    st = bern_stats()
    _check(lib().bern_bounds(*args, _stream(stream), ctypes.byref(st)))
    res["stats"] = _stats(st)
    res["workspace"] = workspace
    return res


def bounds_noalloc(net, box_lo, box_hi, L=2, precision="fp64", lin=0, outputs=None, stream=None, plan="plain",
                   pred=None):
    """``bounds`` of the plain rule or the learned plan without a workspace
    (bern_bounds_noalloc): the library's own per-GPU scratch array, no
    allocation by the library. Output tensors are allocated here unless
    ``outputs`` is given."""
    import torch
    dev = box_lo.device
    box_lo, box_hi = box_lo.contiguous(), box_hi.contiguous()
    nb = box_lo.shape[0]
    if outputs is None:
        nh = max(net.n_hidden, 1)
        outputs = dict(neuron_lo=torch.empty((nb, nh), dtype=torch.float64, device=dev),
                       neuron_hi=torch.empty((nb, nh), dtype=torch.float64, device=dev),
                       out_lo=torch.empty((nb, net.n_out), dtype=torch.float64, device=dev),
                       out_hi=torch.empty((nb, net.n_out), dtype=torch.float64, device=dev),
                       used_plan=torch.empty((nb, nh), dtype=torch.int8, device=dev))
    o = make_opts(L=L, precision=precision, plan=plan, sched="batched", lin=lin, pred=pred)
    st = bern_stats()
    _check(lib().bern_bounds_noalloc(net.handle, ctypes.byref(o), nb, _ptr(box_lo), _ptr(box_hi),
                                     _ptr(outputs["neuron_lo"]), _ptr(outputs["neuron_hi"]), _ptr(outputs["out_lo"]),
                                     _ptr(outputs["out_hi"]), _ptr(outputs.get("used_plan")), _stream(stream),
                                     ctypes.byref(st)))
    res = dict(outputs)
    res["stats"] = _stats(st)
    return res


def output_polys(net, box_lo, box_hi, degree, L=2, precision="fp64", plan="plain", sched="batched",
                 degree_plan=None, max_wave=0, pred=None, stream=None, lin=0):
    """The output polynomials of every box as dense power tensors in t at
    per-variable ``degree``: a dict with ``U`` and ``L`` (float64 CUDA
    tensors [n_boxes, n_out, (degree+1)^n]) and the output bounds
    ``out_lo``/``out_hi``. Asynchronous on ``stream``."""
    import torch
    args, res, workspace, keep = _prepare(net, box_lo, box_hi, L, precision, plan, sched, degree_plan, max_wave,
                                          None, None, pred, None, False, lin)
    nb, dev = box_lo.shape[0], box_lo.device
    C = (int(degree) + 1) ** net.n
    U = torch.empty((nb, net.n_out, C), dtype=torch.float64, device=dev)
    Lw = torch.empty((nb, net.n_out, C), dtype=torch.float64, device=dev)
    # args: handle, opts, nb, lo, hi, plan, neuron_lo, neuron_hi, out_lo, out_hi, used, ws, ws_bytes
    _check(lib().bern_output_polys(args[0], args[1], args[2], args[3], args[4], args[5], int(degree), _ptr(U),
                                   _ptr(Lw), args[8], args[9], args[11], args[12], _stream(stream)))
    return dict(U=U, L=Lw, out_lo=res["out_lo"], out_hi=res["out_hi"], workspace=workspace)


def rel_volume(net, box_lo, box_hi, L=2, precision="fp64", plan="plain", sched="batched", degree_plan=None,
               max_wave=0, pred=None, stream=None, lin=0):
    """Relative volume of the output set of every box (Section 6): a dict with
    ``rel_vol`` (float64 CUDA tensor [n_boxes, n_out]) and the output bounds
    ``out_lo``/``out_hi``. Asynchronous on ``stream``."""
    import torch
    args, res, workspace, keep = _prepare(net, box_lo, box_hi, L, precision, plan, sched, degree_plan, max_wave,
                                          None, None, pred, None, False, lin)
    vol = torch.empty((box_lo.shape[0], net.n_out), dtype=torch.float64, device=box_lo.device)
    # args: handle, opts, nb, lo, hi, plan, neuron_lo, neuron_hi, out_lo, out_hi, used, ws, ws_bytes
    _check(lib().bern_rel_volume(args[0], args[1], args[2], args[3], args[4], args[5], _ptr(vol), args[8], args[9],
                                 args[11], args[12], _stream(stream)))
    return dict(rel_vol=vol, out_lo=res["out_lo"], out_hi=res["out_hi"], workspace=workspace)


def verify(net, box_lo, box_hi, out_index, threshold, max_rounds=8, max_boxes=1 << 16, L=2, precision="fp64",
           plan="plain", sched="batched", pred=None, lin=0, log_cap=0):
    """Branch and bound for "output ``out_index`` <= ``threshold``" over host
    boxes (numpy [n_boxes, n]); returns the verified / violated / undecided
    volume fractions, the rounds run and the box counts, and with
    ``log_cap`` > 0 the decision log (boxes, output bounds, status)."""
    box_lo = np.ascontiguousarray(box_lo, dtype=np.float64)
    box_hi = np.ascontiguousarray(box_hi, dtype=np.float64)
    n = box_lo.shape[1]
    o = make_opts(L=L, precision=precision, plan=plan, sched=sched, pred=pred, lin=lin)
    r = bern_verify_result()
    logs = None
    if log_cap > 0:
        logs = dict(lo=np.zeros((log_cap, n)), hi=np.zeros((log_cap, n)), out_lo=np.zeros(log_cap),
                    out_hi=np.zeros(log_cap), status=np.zeros(log_cap, dtype=np.int8))
        r.log_cap = int(log_cap)
        r.log_lo, r.log_hi = logs["lo"].ctypes.data, logs["hi"].ctypes.data
        r.log_out_lo, r.log_out_hi = logs["out_lo"].ctypes.data, logs["out_hi"].ctypes.data
        r.log_status = logs["status"].ctypes.data
    _check(lib().bern_verify(net.handle, ctypes.byref(o), box_lo.shape[0], ctypes.c_void_p(box_lo.ctypes.data),
                             ctypes.c_void_p(box_hi.ctypes.data), int(out_index), float(threshold), int(max_rounds),
                             int(max_boxes), ctypes.byref(r)))
    out = dict(verified=r.verified, violated=r.violated, undecided=r.undecided, rounds=r.rounds,
               boxes_bounded=r.boxes_bounded, undecided_boxes=r.undecided_boxes)
    if logs is not None:
        k = int(r.log_count)
        out["log"] = {key: v[:k] for key, v in logs.items()}
    return out


def bounds_host(net, box_lo, box_hi, L=2, precision="fp64", plan="plain", sched="batched", degree_plan=None,
                max_wave=0, pred=None, lin=0, mem_budget=0):
    """``bounds`` on host arrays (numpy float64 [n_boxes, n]), synchronous:
    the library allocates and frees the device buffers itself. Returns a dict
    of numpy arrays (neuron_lo/hi, out_lo/hi, used_plan) and the run
    statistics."""
    box_lo = np.ascontiguousarray(box_lo, dtype=np.float64)
    box_hi = np.ascontiguousarray(box_hi, dtype=np.float64)
    nb = box_lo.shape[0]
    nh = max(net.n_hidden, 1)
    o = make_opts(L=L, precision=precision, plan=plan, sched=sched, max_wave=max_wave, pred=pred, lin=lin,
                  mem_budget=mem_budget)
    res = dict(neuron_lo=np.empty((nb, nh)), neuron_hi=np.empty((nb, nh)), out_lo=np.empty((nb, net.n_out)),
               out_hi=np.empty((nb, net.n_out)), used_plan=np.empty((nb, nh), dtype=np.int8))
    dp = None if degree_plan is None else np.ascontiguousarray(degree_plan, dtype=np.int8)
    vp = lambda a: None if a is None else ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    st = bern_stats()
    _check(lib().bern_bounds_host(net.handle, ctypes.byref(o), nb, vp(box_lo), vp(box_hi), vp(dp),
                                  vp(res["neuron_lo"]), vp(res["neuron_hi"]), vp(res["out_lo"]), vp(res["out_hi"]),
                                  vp(res["used_plan"]), ctypes.byref(st)))
    res["stats"] = _stats(st)
    return res


def autotune(net, box_lo, box_hi, reps=3, L=2, precision="fp64", plan="plain", sched="batched", degree_plan=None,
             max_wave=0, workspace=None, stream=None, outputs=None, pred=None, lin=0):
    """Pick the fastest kernel variants for this network and workload (stored
    in the network handle). Returns (choice list, mean ms per run)."""
    args, res, workspace, keep = _prepare(net, box_lo, box_hi, L, precision, plan, sched, degree_plan, max_wave,
                                          workspace, outputs, pred, None, False, lin)
    L_ = lib()
    k = L_.bern_tune_params()
    choice = (ctypes.c_int32 * k)()
    ms = ctypes.c_float()
    _check(L_.bern_autotune(*args, _stream(stream), int(reps), choice, ctypes.byref(ms)))
    return list(choice), ms.value


def tune_get(net):
    L_ = lib()
    choice = (ctypes.c_int32 * L_.bern_tune_params())()
    _check(L_.bern_tune_get(net.handle, choice))
    return list(choice)


def tune_set(net, choice):
    L_ = lib()
    c = (ctypes.c_int32 * L_.bern_tune_params())(*[int(v) for v in choice])
    _check(L_.bern_tune_set(net.handle, c))


def tune_variants():
    L_ = lib()
    return [L_.bern_tune_variants(q) for q in range(L_.bern_tune_params())]


def prof_enable(on=True):
    _check(lib().bern_prof_enable(1 if on else 0))


def prof_reset():
    _check(lib().bern_prof_reset())


def prof_read():
    """{kernel class: (launches, total ms, algorithmic bytes, algorithmic
    flops)} of the launches recorded since the last reset (waits for them)."""
    L = lib()
    out = {}
    for c in range(L.bern_prof_classes()):
        n, ms, by, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(L.bern_prof_read(c, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl)))
        if n.value:
            out[L.bern_prof_name(c).decode()] = (n.value, ms.value, by.value, fl.value)
    return out


def basis_minmax(coef, n, D, want_bern=False, stream=None):
    """Step-level basis change + enclosure for a [count, (D+1)^n] tensor."""
    import torch
    coef = coef.contiguous()
    count = coef.shape[0]
    dev = coef.device
    mn = torch.empty(count, dtype=torch.float64, device=dev)
    mx = torch.empty(count, dtype=torch.float64, device=dev)
    l1 = torch.empty(count, dtype=torch.float64, device=dev)
    bern = torch.empty(coef.shape, dtype=torch.float64, device=dev) if want_bern else None
    _check(lib().bern_basis_minmax(n, D, count, _ptr(coef), 1 if coef.dtype == torch.float64 else 0, _ptr(bern),
                                   _ptr(mn), _ptr(mx), _ptr(l1), None, 0, _stream(stream)))
    return dict(min=mn, max=mx, l1=l1, bern=bern)


def poly_mul(A, B, n, da, db, stream=None):
    import torch
    A = A.contiguous()
    B = A if B is None else B.contiguous()
    count = A.shape[0]
    out = torch.empty((count, (da + db + 1) ** n), dtype=A.dtype, device=A.device)
    _check(lib().bern_poly_mul(n, da, db, count, _ptr(A), _ptr(B), _ptr(out), 1 if A.dtype == torch.float64 else 0,
                               _stream(stream)))
    return out


def relu_poly(lo, hi, L, stream=None):
    import torch
    count = lo.shape[0]
    c = torch.empty((count, L + 1), dtype=torch.float64, device=lo.device)
    e = torch.empty(count, dtype=torch.float64, device=lo.device)
    _check(lib().bern_relu_poly(count, L, _ptr(lo.contiguous()), _ptr(hi.contiguous()), _ptr(c), _ptr(e),
                                _stream(stream)))
    return c, e
