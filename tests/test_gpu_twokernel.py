"""The paper's two-kernel kNN (Section 3.3: Algorithm 1 writes the distance
matrix, Algorithm 2 selects each row's k smallest) through the C ABI
(EDM_FORM_TWO_KERNEL).

Bar: index tables bit-identical to the oracle; distances, weights, sweep rho
and CCM rho bit-identical to the fused plain form (the same float32 keys and
the same float64 epilogue in the same order), hence within the oracle's
tolerances too.
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


@pytest.fixture(scope="module")
def ctx(edm):
    c = edm.Context(device=0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def levels(L, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 4, size=L) * 0.25).astype(np.float32)


def logistic(L=1000, s=0):
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=4, L=L)
    return X[s].copy()


def bits(t):
    return t.cpu().numpy().view(np.int32)


CASES = [
    # name, series, E, tau, Tp, k
    ("E1", logistic(), 1, 1, 1, 0),
    ("E2 Tp0", logistic(s=1), 2, 1, 0, 0),
    ("E5", logistic(s=3), 5, 1, 1, 0),
    ("E20", logistic(700, 2), 20, 1, 1, 0),
    ("ties E1", levels(300, 1), 1, 1, 1, 0),
    ("ties E4", levels(500, 3), 4, 1, 1, 0),
    ("tiled E6", synth.tiled_period(11 * 12, 11, 2), 6, 1, 0, 0),
    ("tau3 E5 ties", levels(400, 5), 5, 3, 0, 0),
    ("k1", logistic(s=4), 3, 1, 1, 1),
    ("k32 E4", logistic(400, 1), 4, 1, 1, 32),
    ("nq=k+2", logistic(7, 1), 2, 1, 1, 0),
    ("nq=65", logistic(67, 1), 2, 1, 1, 0),
    ("nq=257", logistic(260, 3), 3, 1, 1, 0),
    ("nq=321 (ldd pad)", logistic(325, 4), 4, 1, 0, 0),
    ("ramp E3", synth.ramp(200), 3, 1, 0, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_two_kernel_table(edm, ctx, case):
    _, x, E, tau, Tp, k = case
    ctx.set_form(edm.EDM_FORM_TWO_KERNEL)
    idx, dist, w = edm.edm_knn(dev(x), E, tau, Tp, k, ctx=ctx)
    ctx.set_form(edm.EDM_FORM_PLAIN)
    pi, pd, pw = edm.edm_knn(dev(x), E, tau, Tp, k, ctx=ctx)
    ctx.sync()
    oi, _ = O.knn(x, E, tau, Tp, k)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(bits(dist), bits(pd))
    np.testing.assert_array_equal(bits(w), bits(pw))
    _, W = O.weights(x, oi, E, tau)
    np.testing.assert_allclose(w.cpu().numpy(), W, rtol=0, atol=1e-6)


def test_two_kernel_long_series_passes(edm, ctx):
    # One library's matrix above the 2 GiB pass size (m = 24000: 2.3 GB), so
    # every library is its own pass; sampled rows against the oracle.
    X = synth.logistic_network(seed=3, N=4, L=24002)[0][:3].copy()
    ctx.set_form(edm.EDM_FORM_TWO_KERNEL)
    E_tgt = torch.full((3,), 3, dtype=torch.int32, device="cuda")
    rho2 = edm.edm_ccm(dev(X), E_tgt, ctx=ctx)
    idx, _, w = edm.edm_knn(dev(X[1]), 3, 1, 0, ctx=ctx)
    ctx.set_form(edm.EDM_FORM_PLAIN)
    rho1 = edm.edm_ccm(dev(X), E_tgt, ctx=ctx)
    ctx.sync()
    np.testing.assert_array_equal(bits(rho2), bits(rho1))
    m = idx.shape[0]
    rows = np.unique(np.r_[0, 1, 255, 256, m - 2, m - 1, np.random.default_rng(0).integers(0, m, 24)])
    oi, _ = O.knn_rows(X[1], 3, 1, 0, rows)
    np.testing.assert_array_equal(idx.cpu().numpy()[rows], oi)
    _, W = O.weights(X[1], oi, 3, 1, rows=rows)
    np.testing.assert_allclose(w.cpu().numpy()[rows], W, rtol=0, atol=1e-6)


def test_two_kernel_sweep_and_ccm_bitwise(edm, ctx):
    # Uneven lengths (the shortest feasible at E_max among them), several
    # libraries per pass; bit-identical to the fused plain form, and the
    # oracle within tolerance.
    X, _, _ = synth.logistic_network(seed=5, N=10, L=700)
    lens = np.array([700, 650, 41, 512, 700, 300, 257, 699, 23, 640], dtype=np.int64)
    Xd = dev(X)
    out = {}
    for form in (edm.EDM_FORM_TWO_KERNEL, edm.EDM_FORM_PLAIN):
        ctx.set_form(form)
        rs, Es = edm.edm_simplex_sweep(Xd, lengths=lens, E_max=12, ctx=ctx)
        rho = edm.edm_ccm(Xd, Es, Lx=lens, Ly=lens, ctx=ctx)
        ctx.sync()
        out[form] = (rs, Es, rho)
    a, b = out[edm.EDM_FORM_TWO_KERNEL], out[edm.EDM_FORM_PLAIN]
    np.testing.assert_array_equal(bits(a[0]), bits(b[0]))
    np.testing.assert_array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
    np.testing.assert_array_equal(bits(a[2]), bits(b[2]))
    ro, Eo = O.simplex_sweep(X, lens, 12)
    np.testing.assert_allclose(a[0].cpu().numpy(), ro, rtol=0, atol=RHO_TOL)
    E_g = a[1].cpu().numpy()
    rc = O.ccm(X, lens, X, lens, E_g)
    g = a[2].cpu().numpy()
    assert np.array_equal(np.isnan(g), np.isnan(rc))
    np.testing.assert_allclose(g, rc, rtol=0, atol=RHO_TOL)


def test_two_kernel_sweep_ccm_call(edm, ctx):
    # edm_sweep_ccm in the two-kernel form (sweep, then the cross map at E*).
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=4, L=1000)
    Xd = dev(X)
    out = {}
    for form in (edm.EDM_FORM_TWO_KERNEL, edm.EDM_FORM_CHOSEN):
        ctx.set_form(form)
        out[form] = edm.edm_sweep_ccm(Xd, E_max=10, ctx=ctx)
        ctx.sync()
    for u, v in zip(out[edm.EDM_FORM_TWO_KERNEL], out[edm.EDM_FORM_CHOSEN]):
        np.testing.assert_array_equal(u.cpu().numpy().view(np.int32), v.cpu().numpy().view(np.int32))
    ctx.set_form(edm.EDM_FORM_PLAIN)
