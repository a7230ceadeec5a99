"""Exclusion radius and library subsampling (the convergence test of CCM)
through the C ABI, against the oracle.

Bar: neighbour tables bit-identical to the oracle; weights to 1e-6; rho
within 1e-5 absolute of the float64 oracle; NaN where the oracle has NaN.
"""
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


@pytest.fixture()
def ctx(edm):
    c = edm.Context(device=0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def levels(L, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 4, size=L) * 0.25).astype(np.float32)


def logistic(L=800, s=0):
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=4, L=L)
    return X[s].copy()


EXCL_CASES = [
    # name, series, E, tau, Tp, k, r
    ("ramp E3 r1", synth.ramp(150), 3, 1, 0, 0, 1),
    ("ramp E1 r5", synth.ramp(120), 1, 1, 1, 0, 5),
    ("logistic E4 r5", logistic(), 4, 1, 1, 0, 5),
    ("logistic E9 r2 Tp0", logistic(s=3), 9, 1, 0, 0, 2),
    ("ties E2 r3", levels(300, 2), 2, 1, 1, 0, 3),
    ("tau2 E5 r1", logistic(s=5), 5, 2, 1, 0, 1),
    ("k5 E2 r4", logistic(s=6), 2, 1, 0, 5, 4),
    ("tight r", logistic(24, 2), 2, 1, 0, 0, 9),   # nq - 1 - 2r = 23 - 1 - 18 = 4 >= k = 3
    ("r0", logistic(s=1), 3, 1, 1, 0, 0),
]


@pytest.mark.parametrize("case", EXCL_CASES, ids=[c[0] for c in EXCL_CASES])
def test_knn_exclusion_radius(edm, ctx, case):
    _, x, E, tau, Tp, k, r = case
    oi, _ = O.knn(x, E, tau, Tp, k, excl=r)
    _, W = O.weights(x, oi, E, tau)
    ctx.set_exclusion_radius(r)
    for form in (edm.EDM_FORM_PLAIN, edm.EDM_FORM_TWO_KERNEL, edm.EDM_FORM_CHOSEN):
        ctx.set_form(form)
        idx, _, w = edm.edm_knn(dev(x), E, tau, Tp, k, want_dist=False, ctx=ctx)
        ctx.sync()
        np.testing.assert_array_equal(idx.cpu().numpy(), oi)
        np.testing.assert_allclose(w.cpu().numpy(), W, rtol=0, atol=1e-6)


def test_knn_exclusion_too_short(edm, ctx):
    ctx.set_exclusion_radius(10)
    with pytest.raises(edm.EdmError) as ei:
        edm.edm_knn(dev(logistic(24, 2)), 2, 1, 0, ctx=ctx)   # 23 - 1 - 20 < 3
    assert ei.value.code == edm.EDM_E_SHORT
    with pytest.raises(edm.EdmError):
        ctx.set_exclusion_radius(-1)


def test_sweep_and_ccm_exclusion_radius(edm, ctx):
    X, _, _ = synth.logistic_network(seed=8, N=6, L=500)
    lens = np.array([500, 470, 60, 333, 500, 47], dtype=np.int64)
    r = 3
    ro, Eo = O.simplex_sweep(X, lens, 10, excl=r)
    Xd = dev(X)
    ctx.set_exclusion_radius(r)
    for form in (edm.EDM_FORM_PLAIN, edm.EDM_FORM_CHOSEN, edm.EDM_FORM_TWO_KERNEL):
        ctx.set_form(form)
        rs, Es = edm.edm_simplex_sweep(Xd, lengths=lens, E_max=10, ctx=ctx)
        ctx.sync()
        g = rs.cpu().numpy()
        assert np.array_equal(np.isnan(g), np.isnan(ro))
        np.testing.assert_allclose(g, ro, rtol=0, atol=RHO_TOL)
        E_tgt = dev(Eo.astype(np.int32))
        rho = edm.edm_ccm(Xd, E_tgt, Lx=lens, Ly=lens, ctx=ctx)
        ctx.sync()
        rc = O.ccm(X, lens, X, lens, Eo, excl=r)
        gc = rho.cpu().numpy()
        assert np.array_equal(np.isnan(gc), np.isnan(rc))
        np.testing.assert_allclose(gc, rc, rtol=0, atol=RHO_TOL)
    # the fused pipeline honours the radius too (it takes the per-E path)
    ctx.set_form(edm.EDM_FORM_CHOSEN)
    X8, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=2, L=400)
    rs, Es, rho = edm.edm_sweep_ccm(dev(X8), E_max=6, ctx=ctx)
    ctx.sync()
    ro8, Eo8 = O.simplex_sweep(X8, np.full(4, 400), 6, excl=r)
    np.testing.assert_allclose(rs.cpu().numpy(), ro8, rtol=0, atol=RHO_TOL)
    E_g = Es.cpu().numpy()
    rc8 = O.ccm(X8, np.full(4, 400), X8, np.full(4, 400), E_g, excl=r)
    np.testing.assert_allclose(rho.cpu().numpy(), rc8, rtol=0, atol=RHO_TOL)


def test_plan_rejects_exclusion_radius(edm, ctx):
    ctx.set_exclusion_radius(2)
    with pytest.raises(edm.EdmError) as ei:
        edm.CcmPlan(np.full(4, 300), np.full(4, 300), np.full(4, 3, dtype=np.int32), 300, 300, ctx=ctx)
    assert ei.value.code == edm.EDM_E_ARG


SUB_CASES = [
    # name, (x, y), E, tau, Tp, sizes, samples, r
    ("logistic E2", 0, 2, 1, 0, (8, 40, 200, 597), 3, 0),
    ("logistic E3 r2", 2, 3, 1, 0, (20, 150), 2, 2),
    ("logistic E5 Tp1", 4, 5, 1, 1, (30, 400), 2, 0),
    ("logistic E4 tau2", 6, 4, 2, 0, (50,), 3, 1),
]


@pytest.mark.parametrize("case", SUB_CASES, ids=[c[0] for c in SUB_CASES])
def test_ccm_subsample(edm, ctx, case):
    _, s, E, tau, Tp, sizes, ns, r = case
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=4, L=600)
    x, y = X[s + 1], X[s]          # library: the response; target: its driver
    m = O.n_embedded(600, E, tau) - Tp
    subs = synth.library_subsets(seed=11 + s, m=m, sizes=sizes, n_samples=ns)
    sets = [row for a in subs for row in a]
    ctx.set_exclusion_radius(r)
    rho, idx = edm.edm_ccm_subsample(dev(x), dev(np.stack([y, x])), E, sets, tau, Tp, want_idx=True, ctx=ctx)
    ctx.sync()
    g = rho.cpu().numpy()
    gi = idx.cpu().numpy()
    ro = np.stack([O.ccm_subsample(x, y, E, tau, Tp, sets, excl=r),
                   O.ccm_subsample(x, x, E, tau, Tp, sets, excl=r)], axis=1)
    np.testing.assert_allclose(g, ro, rtol=0, atol=RHO_TOL)
    for si in range(0, len(sets), max(1, len(sets) // 3)):
        oi, _ = O.knn_subset(x, E, tau, Tp, sets[si], excl=r)
        np.testing.assert_array_equal(gi[si], oi)


def test_subsample_full_set_is_the_full_table(edm, ctx):
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=4, L=700)
    x, y = X[3], X[2]
    E = 3
    m = 700 - (E - 1)
    rho, idx = edm.edm_ccm_subsample(dev(x), dev(y), E, [np.arange(m)], want_idx=True, ctx=ctx)
    fi, _, fw = edm.edm_knn(dev(x), E, 1, 0, want_dist=False, ctx=ctx)
    _, fr = edm.edm_lookup(fi, fw, dev(y), E, ctx=ctx)
    ctx.sync()
    np.testing.assert_array_equal(idx.cpu().numpy()[0], fi.cpu().numpy())
    assert rho.cpu().numpy()[0, 0].view(np.int32) == fr.cpu().numpy()[0].view(np.int32)


def test_subsample_convergence_direction(edm, ctx):
    # coupled logistic maps: cross-map skill of the driver from the response
    # library rises with the library size (the convergence criterion), and
    # the other direction stays far lower; per-subsample rho as the oracle's
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=1, L=600)
    x, y = X[1], X[0]
    E, m = 2, 599
    sizes = (12, 50, 200, m)
    subs = synth.library_subsets(3, m, sizes, 6)
    sets = [row for a in subs for row in a]
    rho, _ = edm.edm_ccm_subsample(dev(x), dev(y), E, sets, ctx=ctx)
    rev, _ = edm.edm_ccm_subsample(dev(y), dev(x), E, sets, ctx=ctx)
    ctx.sync()
    g = rho.cpu().numpy()[:, 0]
    o = O.ccm_subsample(x, y, E, 1, 0, sets)
    np.testing.assert_allclose(g, o, rtol=0, atol=RHO_TOL)
    means = g.reshape(len(sizes), 6).mean(axis=1)
    assert np.all(np.diff(means) > 0), means
    assert rev.cpu().numpy().reshape(len(sizes), 6).mean(axis=1).max() < means[-1] - 0.2


def test_subsample_errors(edm, ctx):
    x = dev(logistic(200))
    with pytest.raises(edm.EdmError) as ei:
        edm.edm_ccm_subsample(x, x, 2, [np.array([5, 3, 9, 11, 20])], ctx=ctx)
    assert ei.value.code == edm.EDM_E_ARG
    with pytest.raises(edm.EdmError) as ei:
        edm.edm_ccm_subsample(x, x, 2, [np.array([1, 2, 3])], ctx=ctx)
    assert ei.value.code == edm.EDM_E_SHORT
    with pytest.raises(edm.EdmError) as ei:
        edm.edm_ccm_subsample(x, x, 2, [np.array([1, 2, 3, 400])], ctx=ctx)
    assert ei.value.code == edm.EDM_E_ARG
