"""What the trained surrogate gains over the method without it.

Labels are the plain sweep's E* (E = 1..20, Tp = 1).  The network is trained
on the GPU by the library's own kernels; on held-out series its top-m
proposals are verified by the simplex skill (edm_select_E), and the sweep
judges the result: the E-selection time against the full sweep, and the rho
lost where the verified E is not the sweep's E*.  A frequency prior (the m
most common training labels for every series) is the no-network reference.
With the confidence fallback calibrated on held-out training series, the
least confident series take the full sweep and the worst loss shrinks.
"""
import time

import numpy as np
import pytest

from paper_2105_12301_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.slow
def test_surrogate_gain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_12301_amd import edm
    from paper_2105_12301_amd.surrogate import Surrogate

    N_tr, N_te, L, m_top = 6000, 2000, 1500, 3
    X, fam = synth.surrogate_mix(seed=5, N=N_tr + N_te, L=L)
    Xd = torch.from_numpy(X).cuda()
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    rho_s, E_s = edm.edm_simplex_sweep(Xd, E_max=20, Tp=1, ctx=ctx)
    ctx.sync()
    sur = Surrogate(C=64, seed=0, ctx=ctx)
    n_val = 1000  # held out of training, for the fallback's calibration
    hist = sur.train(Xd[:N_tr - n_val], E_s[:N_tr - n_val], epochs=6, batch=128, lr=2e-3,
                     log=lambda m: print(m, flush=True))
    assert hist[-1][0] < hist[0][0]
    Xte, Ete = Xd[N_tr:].contiguous(), E_s[N_tr:].contiguous()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs_te, es_te = edm.edm_simplex_sweep(Xte, E_max=20, Tp=1, ctx=ctx)
    ctx.sync()
    t_sweep = time.perf_counter() - t0
    t0 = time.perf_counter()
    r_sel, e_sel, nfb = sur.select_E(Xte, m_top=m_top)
    ctx.sync()
    t_sel = time.perf_counter() - t0

    rs = rs_te.cpu().numpy().astype(np.float64)
    best = np.nanmax(rs, axis=1)
    es = e_sel.cpu().numpy()
    got = rs[np.arange(N_te), es - 1]
    loss_net = best - got

    # no-network reference: the m most frequent training labels for everyone
    counts = np.bincount(E_s[:N_tr - n_val].cpu().numpy(), minlength=21)[1:]
    prior = np.argsort(-counts, kind="stable")[:m_top] + 1
    got_prior = np.nanmax(rs[:, prior - 1], axis=1)
    loss_prior = best - got_prior

    acc = sur.accuracy(Xte, Ete)
    exact = float(np.mean(es == Ete.cpu().numpy()))
    print(f"sweep {t_sweep*1e3:.1f} ms, surrogate+verify {t_sel*1e3:.1f} ms "
          f"({t_sweep / t_sel:.2f}x); top-1 acc {acc:.3f}; verified E == E* {exact:.3f}; "
          f"mean rho loss net {loss_net.mean():.2e} (max {loss_net.max():.2e}), "
          f"prior {loss_prior.mean():.2e} (max {loss_prior.max():.2e}); fallback {nfb}")
    assert np.all(loss_net >= -1e-7)
    assert loss_net.mean() < loss_prior.mean()
    assert exact > 0.5
    assert t_sel < t_sweep

    # the confidence fallback: min_conf chosen on the held-out series so that
    # none of them loses more than 0.01 of rho, then used on the test set
    min_conf = sur.calibrate(Xd[N_tr - n_val:N_tr].contiguous(), rho_s[N_tr - n_val:N_tr].contiguous(),
                             m_top=m_top, max_loss=0.01)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, e_fb, nfb_fb = sur.select_E(Xte, m_top=m_top, min_conf=min_conf)
    ctx.sync()
    t_fb = time.perf_counter() - t0
    loss_fb = best - rs[np.arange(N_te), e_fb.cpu().numpy() - 1]
    print(f"fallback at min_conf {min_conf:.3f}: {nfb_fb} of {N_te} series take the full sweep; "
          f"{t_fb*1e3:.1f} ms ({t_sweep / t_fb:.2f}x); rho loss mean {loss_fb.mean():.2e} "
          f"max {loss_fb.max():.2e} (without: max {loss_net.max():.2e})")
    assert 0 < nfb_fb < N_te
    assert np.all(loss_fb >= -1e-7)
    assert loss_fb.max() <= loss_net.max() and loss_fb.mean() <= loss_net.mean()
    assert t_fb < t_sweep
