"""The HIP path (through the C ABI) against the hand-worked examples of
tests/golden/: exact neighbour tables, distances and weights to float32
rounding, predictions and rho within 1e-5, in every form (an exclusion radius
routes the scans through the exact per-E kernels whatever the form)."""
import numpy as np
import pytest

from golden_io import load

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = load()
TOL = 1e-5


@pytest.fixture(scope="module")
def edm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_12301_amd import edm as _edm

    _edm.load_library()
    return _edm


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("form", [0, 1, 2, 3])
@pytest.mark.parametrize("name", sorted(n for n in CASES
                                         if "idx" in CASES[n] and "subset" not in CASES[n]))
def test_worked_example(edm, name, form):
    c = CASES[name]
    ctx = edm.Context(device=0, form=form)
    ctx.set_exclusion_radius(c.get("excl", 0))
    try:
        x, y = dev(c["x"]), dev(c["y"])
        idx, dist, w = edm.edm_knn(x, c["E"], c["tau"], c["Tp"], c["k"], ctx=ctx)
        assert np.array_equal(idx.cpu().numpy(), c["idx"].astype(np.int32))
        assert np.allclose(dist.cpu().numpy(), np.sqrt(c["key"]), rtol=1e-6, atol=0)
        assert np.allclose(w.cpu().numpy(), c["w"], rtol=0, atol=1e-6)
        pred, rho = edm.edm_lookup(idx, w, y, c["E"], c["tau"], c["Tp"], want_pred=True,
                                   ctx=ctx)
        assert np.allclose(pred.cpu().numpy()[0], c["pred"], rtol=0, atol=TOL)
        assert abs(float(rho.cpu()[0]) - c["rho"][0]) < TOL
        if c["k"] == c["E"] + 1:
            r = edm.edm_ccm(x[None, :], dev([c["E"]], np.int32), Y=y[None, :],
                            tau=c["tau"], Tp=c["Tp"], ctx=ctx)
            assert abs(float(r.cpu()[0, 0]) - c["rho"][0]) < TOL
    finally:
        ctx.close()


@pytest.mark.parametrize("name", sorted(n for n in CASES if "subset" in CASES[n]))
def test_worked_subsample(edm, name):
    c = CASES[name]
    ctx = edm.Context(device=0)
    ctx.set_exclusion_radius(c.get("excl", 0))
    try:
        rho, idx = edm.edm_ccm_subsample(dev(c["x"]), dev(c["y"]), c["E"],
                                         [c["subset"].astype(np.int32)], tau=c["tau"],
                                         Tp=c["Tp"], want_idx=True, ctx=ctx)
        assert np.array_equal(idx.cpu().numpy()[0], c["idx"].astype(np.int32))
        assert abs(float(rho.cpu()[0, 0]) - c["rho"][0]) < TOL
    finally:
        ctx.close()


@pytest.mark.parametrize("form", [0, 1, 2, 3])
def test_worked_sweep(edm, form):
    c = CASES["S"]
    ctx = edm.Context(device=0, form=form)
    try:
        x = dev(c["x"])
        for E in (1, 3):
            idx, _, _ = edm.edm_knn(x, E, c["tau"], c["Tp"], ctx=ctx)
            assert np.array_equal(idx.cpu().numpy(), c[f"idx_E{E}"].astype(np.int32)), E
        rho, E_opt = edm.edm_simplex_sweep(x[None, :], E_max=c["E_max"], tau=c["tau"],
                                           Tp=c["Tp"], ctx=ctx)
        got, want = rho.cpu().numpy()[0].astype(np.float64), c["rho_sweep"]
        assert np.array_equal(np.isnan(got), np.isnan(want))
        ok = ~np.isnan(want)
        assert np.allclose(got[ok], want[ok], rtol=0, atol=TOL)
        assert int(E_opt.cpu()[0]) == c["E_opt"]
    finally:
        ctx.close()
