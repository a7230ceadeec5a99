"""Thin Python binding of libedm (include/edm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libedm.so``.  Tensors must be CUDA (HIP) tensors of the stated dtype and
C-contiguous; work is enqueued on torch's current stream of the tensor's
device.  There is no fallback: if ``libedm.so`` is missing or fails to load,
every call raises.

Functions mirror the C ABI names: ``edm_embed``, ``edm_knn``, ``edm_lookup``,
``edm_simplex_sweep``, ``edm_ccm`` (plus ``Context`` for the edm_ctx calls).
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libedm.so")

EDM_OK = 0
EDM_E_ARG = -1
EDM_E_SHORT = -2
EDM_E_HIP = -3
EDM_E_NOMEM = -4
EDM_E_NONFINITE = -5
EDM_FORM_PLAIN = 0
EDM_FORM_CHOSEN = 1
EDM_FORM_BATCHED = 2
EDM_FORM_TWO_KERNEL = 3
E_MAX = 20
K_MAX = 32
L_MAX = 32768

NET_KW = 7
NET_CLASSES = 20
NET_C_MAX = 64

EXPORTS = (
    "edm_ctx_create", "edm_ctx_set_form", "edm_sync", "edm_last_error",
    "edm_ctx_destroy", "edm_embed", "edm_knn", "edm_lookup",
    "edm_simplex_sweep", "edm_ccm", "edm_sweep_ccm",
    "edm_net_param_count", "edm_net_forward", "edm_net_forward_bf16", "edm_net_loss_grad",
    "edm_net_adam",
    "edm_select_E",
    "edm_tune_default", "edm_ccm_plan_create", "edm_ccm_plan_run", "edm_ccm_plan_destroy",
    "edm_ctx_set_timing", "edm_ctx_timing", "edm_ctx_set_exclusion_radius", "edm_ccm_subsample",
    "edm_simplex_sweep_noalloc", "edm_ceilings",
)

# kernel families of edm_ctx_timing (include/edm.h, EDM_KF_*)
KERNEL_FAMILIES = ("exact_scan", "batched_scan", "filter_prep", "filter_scan", "tables_from_sweep",
                   "lookup", "finalize", "other", "distances", "row_topk", "group", "plan")


class Tune(ctypes.Structure):
    """Launch shapes of a batched CCM plan (edm_tune)."""
    _fields_ = [("tables_wg_per_cu", ctypes.c_int32), ("lookup_wg_per_cu", ctypes.c_int32),
                ("lookup_targets", ctypes.c_int32), ("filter_stride", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class EdmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libedm error {code}: {msg}")
        self.code = code


_lib = None
_lib_lock = threading.Lock()

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def load_library(path: str = LIB_PATH):
    """Load libedm.so and declare its signatures (no GPU needed to load)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2105_12301_amd.build`")
        lib = ctypes.CDLL(path)
        lib.edm_ctx_create.argtypes = [ctypes.POINTER(_p), _p]
        lib.edm_ctx_set_form.argtypes = [_p, ctypes.c_int]
        lib.edm_sync.argtypes = [_p]
        lib.edm_last_error.argtypes = [_p]
        lib.edm_last_error.restype = ctypes.c_char_p
        lib.edm_ctx_destroy.argtypes = [_p]
        lib.edm_ctx_destroy.restype = None
        lib.edm_embed.argtypes = [_p, _p, _i64, _i32, _i32, _p]
        lib.edm_knn.argtypes = [_p, _p, _i64, _i32, _i32, _i32, _i32, _p, _p, _p]
        lib.edm_lookup.argtypes = [_p, _p, _p, _i64, _i32, _i32, _i32, _i32, _p, _i64, _i64, _p, _p]
        lib.edm_simplex_sweep.argtypes = [_p, _p, _p, _i64, _i64, _i32, _i32, _i32, _p, _p]
        lib.edm_ccm.argtypes = [_p, _p, _p, _i64, _i64, _p, _p, _i64, _i64, _p, _i32, _i32, _p]
        lib.edm_sweep_ccm.argtypes = [_p, _p, _p, _i64, _i64, _i32, _i32, _p, _p, _p]
        lib.edm_net_param_count.argtypes = [_i32]
        lib.edm_net_param_count.restype = _i64
        lib.edm_net_forward.argtypes = [_p, _p, _i32, _p, _i64, _i64, _i64, _p]
        lib.edm_net_forward_bf16.argtypes = [_p, _p, _i32, _p, _i64, _i64, _i64, _p]
        lib.edm_net_loss_grad.argtypes = [_p, _p, _i32, _p, _p, _i64, _i64, _i64, _p, _p]
        lib.edm_net_adam.argtypes = [_p, _p, _p, _p, _p, _i64, _i32, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float]
        lib.edm_select_E.argtypes = [_p, _p, _p, _i64, _i64, _i32, _i32, _i32, _p, _i32,
                                     ctypes.c_float, _p, _p, ctypes.POINTER(_i64)]
        lib.edm_tune_default.argtypes = [ctypes.POINTER(Tune)]
        lib.edm_tune_default.restype = None
        lib.edm_ccm_plan_create.argtypes = [_p, _p, _i64, _i64, _p, _i64, _i64, _p, _i32,
                                            ctypes.POINTER(Tune), ctypes.POINTER(_p)]
        lib.edm_ccm_plan_run.argtypes = [_p, _p, _p, _p, _p]
        lib.edm_ctx_set_timing.argtypes = [_p, ctypes.c_int]
        lib.edm_ctx_timing.argtypes = [_p, _p, _p]
        lib.edm_ctx_set_exclusion_radius.argtypes = [_p, _i32]
        lib.edm_ceilings.argtypes = [_p, _p, _p, _p]
        lib.edm_simplex_sweep_noalloc.argtypes = [_p, _p, _p, _i64, _i64, _i32, _i32, _i32, _p, _p]
        lib.edm_ccm_subsample.argtypes = [_p, _p, _i64, _p, _i64, _i64, _i32, _i32, _i32, _p, _p,
                                          _i64, _p, _p]
        lib.edm_ccm_plan_destroy.argtypes = [_p, _p]
        lib.edm_ccm_plan_destroy.restype = None
        for name in EXPORTS:
            if name not in ("edm_last_error", "edm_ctx_destroy", "edm_net_param_count",
                            "edm_tune_default", "edm_ccm_plan_destroy"):
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
        return lib


def _check(rc: int, ctx_handle=None):
    if rc != EDM_OK:
        lib = load_library()
        msg = lib.edm_last_error(ctx_handle).decode(errors="replace")
        raise EdmError(rc, msg)


def _dev_ptr(t, dtype, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _host_i64(a, n, name):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    if arr.shape != (n,):
        raise ValueError(f"{name} must have shape ({n},)")
    return arr


class Context:
    """An edm_ctx bound to a torch stream (default: the current stream)."""

    def __init__(self, device=None, stream=None, form: int = EDM_FORM_PLAIN):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libedm needs a HIP GPU; none is visible")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _check(lib.edm_ctx_create(ctypes.byref(h), ctypes.c_void_p(self.stream.cuda_stream)))
        self._h = h
        self.set_form(form)

    @property
    def handle(self):
        return self._h

    def set_form(self, form: int):
        _check(load_library().edm_ctx_set_form(self._h, int(form)), self._h)
        self.form = int(form)

    def set_exclusion_radius(self, r: int):
        """Exclusion radius of the neighbour search (edm_ctx_set_exclusion_radius)."""
        _check(load_library().edm_ctx_set_exclusion_radius(self._h, int(r)), self._h)
        self.excl = int(r)

    def sync(self):
        _check(load_library().edm_sync(self._h), self._h)

    def set_timing(self, on: bool = True):
        """Time every kernel launch by family (edm_ctx_set_timing); clears totals."""
        _check(load_library().edm_ctx_set_timing(self._h, int(bool(on))), self._h)

    def timing(self):
        """{family: (ms, launches)} recorded since the last call (edm_ctx_timing)."""
        n = len(KERNEL_FAMILIES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(load_library().edm_ctx_timing(self._h, ctypes.cast(ms, _p), ctypes.cast(cnt, _p)), self._h)
        return {f: (float(ms[i]), int(cnt[i])) for i, f in enumerate(KERNEL_FAMILIES)}

    def ceilings(self):
        """Measured device ceilings (edm_ceilings): HBM GB/s, BF16 MFMA TFLOP/s,
        float32 VALU T ops/s."""
        v = [ctypes.c_double(0.0) for _ in range(3)]
        _check(load_library().edm_ceilings(self._h, *[ctypes.byref(x) for x in v]), self._h)
        return {"hbm_copy_GBps": v[0].value, "mfma_bf16_TFLOPs": v[1].value, "valu_fp32_Tops": v[2].value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().edm_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_default = {}


def default_context(device=None) -> Context:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    stream = torch.cuda.current_stream(dev)
    key = (dev, stream.cuda_stream)
    ctx = _default.get(key)
    if ctx is None:
        ctx = Context(device=dev, stream=stream)
        _default[key] = ctx
    return ctx


def n_query(L: int, E: int, tau: int, Tp: int) -> int:
    return int(L) - (int(E) - 1) * int(tau) - int(Tp)


def edm_embed(x, E: int, tau: int = 1, out=None, ctx: Context | None = None):
    ctx = ctx or default_context(x.device)
    L = x.shape[0]
    n = L - (E - 1) * tau
    if out is None:
        out = torch.empty((max(n, 0), E), dtype=torch.float32, device=x.device)
    _check(load_library().edm_embed(ctx.handle, _dev_ptr(x, torch.float32, "x"), L, E, tau,
                                    _dev_ptr(out, torch.float32, "out")), ctx.handle)
    return out


def edm_knn(x, E: int, tau: int = 1, Tp: int = 0, k: int = 0, want_dist=True, want_w=True,
            ctx: Context | None = None):
    """Returns (idx int32 [nq][k], dist float32 or None, w float32 or None)."""
    ctx = ctx or default_context(x.device)
    L = x.shape[0]
    kk = k if k else E + 1
    nq = max(n_query(L, E, tau, Tp), 0)
    idx = torch.empty((nq, kk), dtype=torch.int32, device=x.device)
    dist = torch.empty((nq, kk), dtype=torch.float32, device=x.device) if want_dist else None
    w = torch.empty((nq, kk), dtype=torch.float32, device=x.device) if want_w else None
    _check(load_library().edm_knn(ctx.handle, _dev_ptr(x, torch.float32, "x"), L, E, tau, Tp, k,
                                  _dev_ptr(idx, torch.int32, "idx"),
                                  _dev_ptr(dist, torch.float32, "dist"),
                                  _dev_ptr(w, torch.float32, "w")), ctx.handle)
    return idx, dist, w


def edm_lookup(idx, w, Y, E: int, tau: int = 1, Tp: int = 0, want_pred=False, want_rho=True,
               ctx: Context | None = None):
    """Returns (pred float32 [N][nq] or None, rho float32 [N] or None)."""
    ctx = ctx or default_context(Y.device)
    nq, k = idx.shape
    if Y.dim() == 1:
        Y = Y.unsqueeze(0)
    N, ldy = Y.shape
    pred = torch.empty((N, nq), dtype=torch.float32, device=Y.device) if want_pred else None
    rho = torch.empty((N,), dtype=torch.float32, device=Y.device) if want_rho else None
    _check(load_library().edm_lookup(ctx.handle, _dev_ptr(idx, torch.int32, "idx"),
                                     _dev_ptr(w, torch.float32, "w"), nq, k, E, tau, Tp,
                                     _dev_ptr(Y, torch.float32, "Y"), N, ldy,
                                     _dev_ptr(pred, torch.float32, "pred"),
                                     _dev_ptr(rho, torch.float32, "rho")), ctx.handle)
    return pred, rho


def edm_simplex_sweep(X, lengths=None, E_max: int = E_MAX, tau: int = 1, Tp: int = 1,
                      ctx: Context | None = None):
    """Returns (rho float32 [N][E_max], E_opt int32 [N])."""
    ctx = ctx or default_context(X.device)
    N, ldx = X.shape
    L = _host_i64(np.full(N, ldx) if lengths is None else lengths, N, "lengths")
    rho = torch.empty((N, E_max), dtype=torch.float32, device=X.device)
    E_opt = torch.empty((N,), dtype=torch.int32, device=X.device)
    _check(load_library().edm_simplex_sweep(
        ctx.handle, _dev_ptr(X, torch.float32, "X"), L.ctypes.data_as(_p), N, ldx, E_max, tau, Tp,
        _dev_ptr(rho, torch.float32, "rho"), _dev_ptr(E_opt, torch.int32, "E_opt")), ctx.handle)
    return rho, E_opt


def edm_ccm(X, E_tgt, Y=None, Lx=None, Ly=None, tau: int = 1, Tp: int = 0, rho=None,
            ctx: Context | None = None):
    """All-to-all CCM; returns rho float32 [Nl][Nt] (rho[i][j]: library i, target j)."""
    ctx = ctx or default_context(X.device)
    if Y is None:
        Y = X
        if Ly is None:
            Ly = Lx
    Nl, ldx = X.shape
    Nt, ldy = Y.shape
    Lx = _host_i64(np.full(Nl, ldx) if Lx is None else Lx, Nl, "Lx")
    Ly = _host_i64(np.full(Nt, ldy) if Ly is None else Ly, Nt, "Ly")
    if rho is None:
        rho = torch.empty((Nl, Nt), dtype=torch.float32, device=X.device)
    _check(load_library().edm_ccm(
        ctx.handle, _dev_ptr(X, torch.float32, "X"), Lx.ctypes.data_as(_p), Nl, ldx,
        _dev_ptr(Y, torch.float32, "Y"), Ly.ctypes.data_as(_p), Nt, ldy,
        _dev_ptr(E_tgt, torch.int32, "E_tgt"), tau, Tp, _dev_ptr(rho, torch.float32, "rho")),
        ctx.handle)
    return rho


def edm_sweep_ccm(X, lengths=None, E_max: int = E_MAX, tau: int = 1, rho=None,
                  ctx: Context | None = None, rho_sweep=None, E_opt=None):
    """E sweep (Tp = 1) then all-to-all CCM of the same series at the targets'
    E* (Tp = 0).  Returns (rho_sweep [N][E_max], E_opt [N], rho [N][N]);
    rho_sweep, E_opt and rho may be given (preallocated outputs)."""
    ctx = ctx or default_context(X.device)
    N, ldx = X.shape
    L = _host_i64(np.full(N, ldx) if lengths is None else lengths, N, "lengths")
    rho_s = rho_sweep if rho_sweep is not None else torch.empty((N, E_max), dtype=torch.float32,
                                                                device=X.device)
    if E_opt is None:
        E_opt = torch.empty((N,), dtype=torch.int32, device=X.device)
    if rho is None:
        rho = torch.empty((N, N), dtype=torch.float32, device=X.device)
    _check(load_library().edm_sweep_ccm(
        ctx.handle, _dev_ptr(X, torch.float32, "X"), L.ctypes.data_as(_p), N, ldx, E_max, tau,
        _dev_ptr(rho_s, torch.float32, "rho_sweep"), _dev_ptr(E_opt, torch.int32, "E_opt"),
        _dev_ptr(rho, torch.float32, "rho")), ctx.handle)
    return rho_s, E_opt, rho


def edm_ccm_subsample(x, Y, E: int, sets, tau: int = 1, Tp: int = 0, want_idx=False,
                      ctx: Context | None = None):
    """Cross map of library x on subsamples (the convergence test).
    sets: sequence of S ascending int index arrays (candidate points).
    Returns (rho float32 [S][Nt], idx int32 [S][nq][k] or None)."""
    ctx = ctx or default_context(x.device)
    if Y.dim() == 1:
        Y = Y.unsqueeze(0)
    L = x.shape[0]
    Nt, ldy = Y.shape
    S = len(sets)
    off = np.zeros(S + 1, dtype=np.int64)
    for s, c in enumerate(sets):
        off[s + 1] = off[s] + len(c)
    flat = (np.concatenate([np.asarray(c, dtype=np.int32) for c in sets]) if S and off[-1]
            else np.zeros(1, dtype=np.int32))
    flat = np.ascontiguousarray(flat, dtype=np.int32)
    nq = max(n_query(L, E, tau, Tp), 0)
    rho = torch.empty((S, Nt), dtype=torch.float32, device=x.device)
    idx = torch.empty((S, nq, E + 1), dtype=torch.int32, device=x.device) if want_idx else None
    _check(load_library().edm_ccm_subsample(
        ctx.handle, _dev_ptr(x, torch.float32, "x"), L, _dev_ptr(Y, torch.float32, "Y"), Nt, ldy,
        E, tau, Tp, flat.ctypes.data_as(_p), off.ctypes.data_as(_p), S,
        _dev_ptr(idx, torch.int32, "idx"), _dev_ptr(rho, torch.float32, "rho")), ctx.handle)
    return rho, idx


# ---------------------------------------------------------------- surrogate --
def edm_net_param_count(C: int) -> int:
    n = load_library().edm_net_param_count(int(C))
    if n < 0:
        raise EdmError(EDM_E_ARG, "C must be in 1..64")
    return int(n)


def edm_net_forward(params, C: int, X, logits=None, ctx: Context | None = None):
    """logits float32 [B][20] of the surrogate network for series X [B][L]."""
    ctx = ctx or default_context(X.device)
    B, L = X.shape
    if logits is None:
        logits = torch.empty((B, NET_CLASSES), dtype=torch.float32, device=X.device)
    _check(load_library().edm_net_forward(ctx.handle, _dev_ptr(params, torch.float32, "params"), C,
                                          _dev_ptr(X, torch.float32, "X"), B, L, X.stride(0),
                                          _dev_ptr(logits, torch.float32, "logits")), ctx.handle)
    return logits


def edm_net_forward_bf16(params, C: int, X, logits=None, ctx: Context | None = None):
    """Inference logits float32 [B][20] with the C -> C convolutions on BF16
    matrix cores (C = 32 or 64)."""
    ctx = ctx or default_context(X.device)
    B, L = X.shape
    if logits is None:
        logits = torch.empty((B, NET_CLASSES), dtype=torch.float32, device=X.device)
    _check(load_library().edm_net_forward_bf16(ctx.handle, _dev_ptr(params, torch.float32, "params"), C,
                                               _dev_ptr(X, torch.float32, "X"), B, L, X.stride(0),
                                               _dev_ptr(logits, torch.float32, "logits")), ctx.handle)
    return logits


def edm_net_loss_grad(params, C: int, X, labels, grad=None, loss=None, ctx: Context | None = None):
    """(loss float32 [1], grad float32 [P]) of the mean cross-entropy."""
    ctx = ctx or default_context(X.device)
    B, L = X.shape
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty((1,), dtype=torch.float32, device=X.device)
    _check(load_library().edm_net_loss_grad(ctx.handle, _dev_ptr(params, torch.float32, "params"), C,
                                            _dev_ptr(X, torch.float32, "X"),
                                            _dev_ptr(labels, torch.int32, "labels"), B, L, X.stride(0),
                                            _dev_ptr(loss, torch.float32, "loss"),
                                            _dev_ptr(grad, torch.float32, "grad")), ctx.handle)
    return loss, grad


def edm_net_adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
                 ctx: Context | None = None):
    ctx = ctx or default_context(params.device)
    _check(load_library().edm_net_adam(ctx.handle, _dev_ptr(params, torch.float32, "params"),
                                       _dev_ptr(grad, torch.float32, "grad"),
                                       _dev_ptr(m, torch.float32, "m"), _dev_ptr(v, torch.float32, "v"),
                                       params.numel(), int(step), float(lr), float(beta1),
                                       float(beta2), float(eps)), ctx.handle)


def edm_select_E(X, logits, lengths=None, E_max: int = E_MAX, tau: int = 1, Tp: int = 1,
                 m_top: int = 2, min_conf: float = 0.0, ctx: Context | None = None):
    """(rho float32 [N][E_max], E_opt int32 [N], n_fallback) from the network's logits."""
    ctx = ctx or default_context(X.device)
    N, ldx = X.shape
    L = _host_i64(np.full(N, ldx) if lengths is None else lengths, N, "lengths")
    rho = torch.empty((N, E_max), dtype=torch.float32, device=X.device)
    E_opt = torch.empty((N,), dtype=torch.int32, device=X.device)
    nfb = ctypes.c_int64(0)
    _check(load_library().edm_select_E(
        ctx.handle, _dev_ptr(X, torch.float32, "X"), L.ctypes.data_as(_p), N, ldx, E_max, tau, Tp,
        _dev_ptr(logits, torch.float32, "logits"), int(m_top), float(min_conf),
        _dev_ptr(rho, torch.float32, "rho"), _dev_ptr(E_opt, torch.int32, "E_opt"),
        ctypes.byref(nfb)), ctx.handle)
    return rho, E_opt, int(nfb.value)


# ---------------------------------------------------------------- plan ------
def default_tune() -> Tune:
    t = Tune()
    load_library().edm_tune_default(ctypes.byref(t))
    return t


class CcmPlan:
    """Batched all-to-all CCM over libraries of uneven length (edm_ccm_plan_*).

    Built once from host lengths and target E values; ``run`` replays a
    captured HIP graph when the context's stream is not the legacy default
    stream."""

    def __init__(self, Lx, Ly, E_tgt, ldx: int, ldy: int, Tp: int = 0, tune: Tune | None = None,
                 ctx: Context | None = None):
        self.ctx = ctx or default_context()
        self.Lx = _host_i64(Lx, len(Lx), "Lx")
        self.Ly = _host_i64(Ly, len(Ly), "Ly")
        E = np.ascontiguousarray(np.asarray(E_tgt.cpu() if isinstance(E_tgt, torch.Tensor) else E_tgt,
                                            dtype=np.int32))
        self.Nl, self.Nt = len(self.Lx), len(self.Ly)
        h = ctypes.c_void_p()
        _check(load_library().edm_ccm_plan_create(
            self.ctx.handle, self.Lx.ctypes.data_as(_p), self.Nl, int(ldx), self.Ly.ctypes.data_as(_p),
            self.Nt, int(ldy), E.ctypes.data_as(_p), int(Tp), ctypes.byref(tune) if tune else None,
            ctypes.byref(h)), self.ctx.handle)
        self._h = h

    def run(self, X, Y=None, rho=None):
        Y = X if Y is None else Y
        if rho is None:
            rho = torch.empty((self.Nl, self.Nt), dtype=torch.float32, device=X.device)
        _check(load_library().edm_ccm_plan_run(self.ctx.handle, self._h, _dev_ptr(X, torch.float32, "X"),
                                               _dev_ptr(Y, torch.float32, "Y"),
                                               _dev_ptr(rho, torch.float32, "rho")), self.ctx.handle)
        return rho

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().edm_ccm_plan_destroy(self.ctx.handle, self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
