"""Parity at the real shapes of the benchmark workloads, through the C ABI.

* calcium-like 10000 x 2000 (the headline step): the chosen form's fused
  sweep + full cross map against the plain form bit for bit, and against the
  oracle on sampled series (sweep rho and E* with the near-tie rule), on a
  parity subset of libraries x targets (rho), and on sampled kNN rows;
* spike trains 4096 x L ~ U{1000..20000} with E given (the batched plan):
  the chosen-form plan against the plain form bit for bit, and the oracle on
  the shortest and a median library x 16 targets in two E buckets;
* surrogate mix 100000 x 1500 (the learned-E workload): network-proposed,
  sweep-verified E for every series, then library rows 0..15 against all
  100000 targets; the oracle checks the selection on sampled series and rho
  on 8 libraries x 32 targets at the selected E.

Bar: rho within 1e-5 of the float64 oracle, tables bit-identical, forms
bit-identical to each other.
"""
import time

import numpy as np
import pytest

from oracle import edm_oracle as O
from paper_2105_12301_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5


@pytest.fixture(scope="module")
def edm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_12301_amd import edm as _edm

    _edm.load_library()
    return _edm


def bits(a):
    return np.ascontiguousarray(a).view(np.int32)


def check_E(E_gpu, rho_o, E_o):
    """E* equal to the oracle's, or a near tie of the oracle's rho."""
    for eg, ro, eo in zip(E_gpu, rho_o, E_o):
        if eg != eo:
            assert eg >= 1 and abs(ro[eg - 1] - ro[eo - 1]) < 2e-5, (eg, eo)


def test_calcium_full_shape(edm):
    t0 = time.perf_counter()
    X, group = synth.calcium_like(seed=4)
    print(f"calcium data {time.perf_counter() - t0:.1f} s", flush=True)
    N, L = X.shape
    Xd = torch.from_numpy(X).cuda()
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    rs, Es, rho = edm.edm_sweep_ccm(Xd, E_max=20, ctx=ctx)
    ctx.set_form(edm.EDM_FORM_PLAIN)
    rs_p, Es_p = edm.edm_simplex_sweep(Xd, E_max=20, ctx=ctx)
    rho_p = edm.edm_ccm(Xd, Es_p, ctx=ctx)
    ctx.sync()
    assert torch.equal(rs.view(torch.int32), rs_p.view(torch.int32))
    assert torch.equal(Es, Es_p)
    assert torch.equal(rho.view(torch.int32), rho_p.view(torch.int32))
    rs_h, Es_h = rs.cpu().numpy(), Es.cpu().numpy()
    # parity subset: 8 libraries sharing two latent drivers and 8 others x
    # 16 targets (driven ones and random)
    rng = np.random.default_rng(4)
    driven = [np.nonzero(group == g)[0][:4] for g in (0, 1)]
    others = rng.choice(np.nonzero(group < 0)[0], size=8, replace=False)
    libs = np.sort(np.r_[driven[0], driven[1], others])
    tgts = np.sort(np.r_[driven[0][::-1], driven[1][::-1],
                         rng.choice(np.setdiff1d(np.arange(N), libs), size=8, replace=False)])
    # sweep of 4 target series against the oracle
    sw = tgts[::4]
    ro, Eo = O.simplex_sweep(X[sw], np.full(len(sw), L), 20)
    np.testing.assert_allclose(rs_h[sw], ro, rtol=0, atol=RHO_TOL)
    check_E(Es_h[sw], ro, Eo)
    # rho of the subset at the GPU's E* (frozen and shared with the oracle)
    lib8 = libs[::2]
    rc = O.ccm(X, np.full(N, L), X, np.full(N, L), Es_h, lib_rows=lib8, tgt_cols=tgts)
    g = rho.cpu().numpy()[np.ix_(lib8, tgts)]
    assert np.array_equal(np.isnan(g), np.isnan(rc))
    np.testing.assert_allclose(g, rc, rtol=0, atol=RHO_TOL)
    # kNN rows of two libraries at two E in use, chosen and plain forms
    rows = np.r_[0, 1, 255, 256, 1990, np.random.default_rng(1).integers(0, 1990, 12)]
    for i in libs[:2]:
        for E in sorted(set(Es_h[tgts].tolist()))[:2]:
            oi, _ = O.knn_rows(X[i], E, 1, 0, rows)
            for form in (edm.EDM_FORM_CHOSEN, edm.EDM_FORM_PLAIN):
                ctx.set_form(form)
                idx, _, _ = edm.edm_knn(Xd[i].contiguous(), E, 1, 0, want_dist=False, want_w=False, ctx=ctx)
                ctx.sync()
                np.testing.assert_array_equal(idx.cpu().numpy()[rows], oi)
    ctx.close()


def test_uneven_plan_full_shape(edm):
    t0 = time.perf_counter()
    X, lens, E = synth.spike_trains(seed=3)
    print(f"spike data {time.perf_counter() - t0:.1f} s", flush=True)
    N = X.shape[0]
    Xd, Ed = torch.from_numpy(X).cuda(), torch.from_numpy(E).cuda()
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    plan = edm.CcmPlan(lens, lens, E, X.shape[1], X.shape[1], ctx=ctx)
    rho = plan.run(Xd, Xd)
    ctx.set_form(edm.EDM_FORM_PLAIN)
    rho_p = edm.edm_ccm(Xd, Ed, Lx=lens, Ly=lens, ctx=ctx)
    ctx.sync()
    assert torch.equal(rho.view(torch.int32), rho_p.view(torch.int32))
    g = rho.cpu().numpy()
    plan.close()
    order = np.argsort(lens, kind="stable")
    rng = np.random.default_rng(3)
    # the shortest, the median, and the shortest library beyond 14336 samples
    # (the filter reads its samples from global memory there)
    long_i = next(k for k in order if lens[k] > 14336)
    for i in (order[0], order[N // 2], long_i):
        defined = np.nonzero(lens >= lens[i])[0]
        Es = np.unique(E[defined])
        pick = rng.choice(Es[Es >= 5], size=1)[0], rng.choice(Es[Es < 5], size=1)[0]
        cols = np.sort(np.r_[rng.choice(defined[E[defined] == pick[0]], 8, replace=False),
                             rng.choice(defined[E[defined] == pick[1]], 8, replace=False)])
        rc = O.ccm(X[i:i + 1, :lens[i]], [lens[i]], X, lens, E, tgt_cols=cols)[0]
        np.testing.assert_allclose(g[i, cols], rc, rtol=0, atol=RHO_TOL)
        undefined = np.nonzero(lens < lens[i])[0]
        assert np.all(np.isnan(g[i, undefined]))
    ctx.close()


def test_learned_selection_full_shape(edm):
    from paper_2105_12301_amd.surrogate import Surrogate

    t0 = time.perf_counter()
    X, _ = synth.surrogate_mix(seed=6, N=100000, L=1500)
    print(f"surrogate data {time.perf_counter() - t0:.1f} s", flush=True)
    N, L = X.shape
    Xd = torch.from_numpy(X).cuda()
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    sur = Surrogate(C=64, seed=0, ctx=ctx)
    # a briefly trained network (its quality does not matter for parity)
    _, Etr = edm.edm_simplex_sweep(Xd[:4096].contiguous(), E_max=20, ctx=ctx)
    sur.train(Xd[:4096].contiguous(), Etr, epochs=1, batch=256, lr=2e-3)
    logits = sur.logits(Xd)
    rs, Es, nfb = edm.edm_select_E(Xd, logits, E_max=20, m_top=3, min_conf=0.5, ctx=ctx)
    lib = Xd[:16].contiguous()
    rho = edm.edm_ccm(lib, Es, Y=Xd, ctx=ctx)
    ctx.sync()
    Es_h, rs_h, lg = Es.cpu().numpy(), rs.cpu().numpy(), logits.cpu().numpy()
    # selection on sampled series: the best oracle rho among the network's
    # top-3 proposals (or all E where the top probability is below 0.5)
    sample = np.random.default_rng(6).choice(N, 6, replace=False)
    for s in sample:
        z = lg[s].astype(np.float64)
        p = np.exp(z - z.max())
        p /= p.sum()
        cand = (np.arange(1, 21) if p.max() < 0.5
                else np.argsort(-z, kind="stable")[:3] + 1)
        ro = np.full(20, np.nan)
        for E in cand:
            ro[E - 1] = O.simplex_rho(X[s], X[s], int(E), 1, 1)
        np.testing.assert_allclose(rs_h[s][cand - 1], ro[cand - 1], rtol=0, atol=RHO_TOL)
        check_E([Es_h[s]], [ro], [O.select_E(ro)])
    # rho of 8 libraries x 32 targets at the selected E
    tg = np.sort(np.random.default_rng(7).choice(N, 32, replace=False))
    lib8 = np.arange(0, 16, 2)
    rc = O.ccm(X[:16], np.full(16, L), X, np.full(N, L), Es_h, lib_rows=lib8, tgt_cols=tg)
    np.testing.assert_allclose(rho.cpu().numpy()[np.ix_(lib8, tg)], rc, rtol=0, atol=RHO_TOL)
    ctx.close()
