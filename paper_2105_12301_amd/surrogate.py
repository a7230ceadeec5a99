"""Learned embedding-dimension surrogate: training loop and E selection.

The network, its loss, gradients and Adam updates run in libedm's kernels
(``edm_net_*``); this module only orders minibatches.  Labels are the E* that
the simplex sweep selects (``edm_simplex_sweep``), and selection keeps the
sweep as verifier and fallback: the network proposes its ``m_top`` most likely
E values, the simplex skill is evaluated at those only, and series whose top
probability is below ``min_conf`` get the full sweep (``edm_select_E``).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import edm, synth


class Surrogate:
    def __init__(self, C: int = 64, seed: int = 0, device=None, ctx: edm.Context | None = None):
        self.C = int(C)
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.ctx = ctx or edm.default_context(self.device)
        self.params = torch.from_numpy(synth.net_init_params(self.C, seed=seed)).to(self.device)
        assert self.params.numel() == edm.edm_net_param_count(self.C)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0

    def train(self, X, labels, epochs: int = 5, batch: int = 256, lr: float = 1e-3, seed: int = 0,
              log=None):
        """Adam on the mean cross-entropy; X float32 [N][L] (device), labels int32 [N] in 1..20."""
        N = X.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        loss = torch.empty((1,), dtype=torch.float32, device=self.device)
        history = []
        for ep in range(epochs):
            perm = torch.randperm(N, generator=g).to(self.device)
            tot, nb, t0 = 0.0, 0, time.perf_counter()
            for b0 in range(0, N - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                xb = X.index_select(0, idx).contiguous()
                yb = labels.index_select(0, idx).contiguous()
                edm.edm_net_loss_grad(self.params, self.C, xb, yb, grad=self.grad, loss=loss, ctx=self.ctx)
                self.step += 1
                edm.edm_net_adam(self.params, self.grad, self.m, self.v, self.step, lr, ctx=self.ctx)
                tot += float(loss)  # one sync per batch keeps the log honest
                nb += 1
            history.append((tot / max(nb, 1), time.perf_counter() - t0))
            if log:
                log(f"epoch {ep}: loss {history[-1][0]:.4f} ({history[-1][1]:.2f} s)")
        return history

    def logits(self, X, batch: int = 1024, bf16: bool | None = None):
        """Inference logits; BF16 matrix-core convolutions when C allows it
        (bf16=None), else float32 (training always runs in float32)."""
        if bf16 is None:
            bf16 = self.C in (32, 64)
        fwd = edm.edm_net_forward_bf16 if bf16 else edm.edm_net_forward
        out = torch.empty((X.shape[0], edm.NET_CLASSES), dtype=torch.float32, device=X.device)
        for b0 in range(0, X.shape[0], batch):
            xb = X[b0:b0 + batch]
            fwd(self.params, self.C, xb, logits=out[b0:b0 + batch], ctx=self.ctx)
        return out

    def select_E(self, X, E_max: int = 20, Tp: int = 1, m_top: int = 2, min_conf: float = 0.0,
                 lengths=None):
        """Network-proposed, sweep-verified E per series: (rho, E_opt, n_fallback)."""
        return edm.edm_select_E(X, self.logits(X), lengths=lengths, E_max=E_max, Tp=Tp,
                                m_top=m_top, min_conf=min_conf, ctx=self.ctx)

    def calibrate(self, X, rho_sweep, m_top: int = 3, max_loss: float = 0.01) -> float:
        """Confidence threshold for the fallback, chosen on held-out series.

        X: held-out series (device), rho_sweep: their full-sweep skill
        [N][20] (edm_simplex_sweep).  A series whose top softmax probability
        is at least c keeps the best of its m_top proposed E, losing
        max(rho) - max(rho at the proposals); below c it takes the full sweep
        and loses nothing.  Returns the smallest c (a probability) for which no
        held-out series loses more than max_loss."""
        lg = self.logits(X).double().cpu().numpy()
        rs = rho_sweep.double().cpu().numpy()
        lg = lg - lg.max(axis=1, keepdims=True)
        p = np.exp(lg)
        conf = p.max(axis=1) / p.sum(axis=1)
        top = np.argsort(-lg, axis=1, kind="stable")[:, :m_top]
        best = np.nanmax(np.where(np.isnan(rs), -np.inf, rs), axis=1)
        got = np.take_along_axis(np.where(np.isnan(rs), -np.inf, rs), top, axis=1).max(axis=1)
        loss = best - got
        order = np.argsort(conf)
        # suffix maximum of the loss over series at least as confident
        suf = np.maximum.accumulate(loss[order][::-1])[::-1]
        ok = np.nonzero(suf <= max_loss)[0]
        if ok.size == 0:
            return 1.0
        c = float(conf[order][ok[0]])
        return min(1.0, c)

    def accuracy(self, X, labels):
        pred = self.logits(X).argmax(dim=1).to(torch.int32) + 1
        return float((pred == labels).float().mean())
