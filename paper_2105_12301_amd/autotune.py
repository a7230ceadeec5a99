"""Autotuner for the batched CCM plan (edm_tune): launch shapes and, in the
chosen form, the matrix-core filter's first-pass tile stride.

Candidates are timed on a sample of libraries spread over the length range
(every target kept), each on a fresh plan whose graph is captured by a first
run; the fastest replay wins.  The search is coordinate-wise: the launch
shapes with the filter's default stride, then the winner with each stride.  Results are cached in a JSON file (path from
EDM_AUTOTUNE_CACHE, default ~/.cache/edm_autotune.json) keyed by the device
name and a coarse shape class of the workload.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import edm

CANDIDATES = [
    dict(tables_wg_per_cu=t, lookup_wg_per_cu=l, lookup_targets=T, filter_stride=0)
    for t in (0, 1, 2) for l in (0, 4) for T in (4, 8, 16)
]
FILTER_STRIDES = (1, 2, 4, 8)


def _cache_path():
    return os.environ.get("EDM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "edm_autotune.json"))


def shape_key(Lx, Ly, E, form: int = 0):
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    Lx = np.asarray(Lx)
    return (f"{dev}|Nl~{2 ** int(np.log2(max(len(Lx), 1)))}|Nt~{2 ** int(np.log2(max(len(Ly), 1)))}"
            f"|Lmax~{int(np.ceil(Lx.max() / 1000))}k|Emax={int(np.max(E))}|form={int(form)}")


def make_tune(d) -> edm.Tune:
    t = edm.Tune()
    for k, v in d.items():
        setattr(t, k, int(v))
    return t


def autotune(X, Lx, Y, Ly, E, Tp: int = 0, ctx=None, sample: int = 48, reps: int = 2,
             use_cache: bool = True, log=None):
    """Return (best Tune, {candidate: ms}) for this workload shape and the
    context's form (the chosen form's plan runs other table kernels)."""
    ctx = ctx or edm.default_context(X.device)
    key = shape_key(Lx, Ly, E, getattr(ctx, "form", 0))
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return make_tune(cache[key]["tune"]), cache[key].get("times", {})
    Lx = np.asarray(Lx)
    order = np.argsort(-Lx, kind="stable")
    pick = order[np.linspace(0, len(order) - 1, min(sample, len(order))).astype(int)]
    Xs = X.index_select(0, torch.from_numpy(pick).to(X.device)).contiguous()
    rho = torch.empty((len(pick), Y.shape[0]), dtype=torch.float32, device=X.device)
    times = {}

    def name_of(c):
        return ",".join(f"{k}={v}" for k, v in c.items())

    def time_one(cand):
        plan = edm.CcmPlan(Lx[pick], Ly, E, Xs.shape[1], Y.shape[1], Tp=Tp, tune=make_tune(cand), ctx=ctx)
        plan.run(Xs, Y, rho)  # capture
        ctx.sync()
        best = float("inf")
        for _ in range(reps):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(ctx.stream)
            plan.run(Xs, Y, rho)
            ev1.record(ctx.stream)
            ev1.synchronize()
            best = min(best, ev0.elapsed_time(ev1))
        plan.close()
        times[name_of(cand)] = best
        if log:
            log(f"  {name_of(cand)}: {best:.2f} ms")

    for cand in CANDIDATES:
        time_one(cand)
    win = min(CANDIDATES, key=lambda c: times[name_of(c)])
    if getattr(ctx, "form", 0) == edm.EDM_FORM_CHOSEN:
        strided = [dict(win, filter_stride=f) for f in FILTER_STRIDES]
        for cand in strided:
            time_one(cand)
        win = min([win] + strided, key=lambda c: times[name_of(c)])
    if use_cache:
        cache[key] = {"tune": win, "times": times}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return make_tune(win), times
