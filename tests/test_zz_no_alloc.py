"""The allocation-free sweep entry point (edm_simplex_sweep_noalloc), called
through the C ABI, against edm_simplex_sweep in the plain form: bit-identical
rho and E*, on two calls in a row (the second smaller, so the static scratch
holds the first call's data), uneven lengths, and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_2105_12301_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def edm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_12301_amd import edm as _edm

    _edm.load_library()
    return _edm


def noalloc(edm, ctx, X, lens, E_max, Tp=1):
    N, ldx = X.shape
    L = np.ascontiguousarray(lens, dtype=np.int64)
    rho = torch.full((N, E_max), -7.0, dtype=torch.float32, device="cuda")
    E_opt = torch.full((N,), -7, dtype=torch.int32, device="cuda")
    rc = edm.load_library().edm_simplex_sweep_noalloc(
        ctx.handle, ctypes.c_void_p(X.data_ptr()), L.ctypes.data_as(ctypes.c_void_p), N, ldx, E_max,
        1, Tp, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(E_opt.data_ptr()))
    return rc, rho, E_opt


def reference(edm, ctx, X, lens, E_max, Tp=1):
    ctx.set_form(edm.EDM_FORM_PLAIN)
    return edm.edm_simplex_sweep(X, lengths=lens, E_max=E_max, Tp=Tp, ctx=ctx)


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_noalloc_sweep_matches_two_calls(edm):
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    X1, _, _ = synth.logistic_network(seed=12, N=96, L=1500)
    X1 = torch.from_numpy(X1).cuda()
    lens1 = np.full(96, 1500)
    X2, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=4, L=700)
    X2 = torch.from_numpy(X2).cuda()
    lens2 = np.array([700, 650, 80, 700, 512, 41, 699, 300])
    rc1, r1, e1 = noalloc(edm, ctx, X1, lens1, 20)
    rc2, r2, e2 = noalloc(edm, ctx, X2, lens2, 12)   # smaller, uneven lengths
    assert rc1 == edm.EDM_OK and rc2 == edm.EDM_OK
    ctx.sync()
    ref1 = reference(edm, ctx, X1, lens1, 20)
    ref2 = reference(edm, ctx, X2, lens2, 12)
    ctx.sync()
    assert same(r1, ref1[0]) and torch.equal(e1, ref1[1])
    assert same(r2, ref2[0]) and torch.equal(e2, ref2[1])
    # the first input again, after the smaller call, still matches
    rc3, r3, e3 = noalloc(edm, ctx, X1, lens1, 20)
    ctx.sync()
    assert rc3 == edm.EDM_OK and same(r3, ref1[0]) and torch.equal(e3, ref1[1])
    ctx.close()


def test_noalloc_exclusion_radius_and_limit(edm):
    ctx = edm.Context(device=0)
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=2, L=400)
    X = torch.from_numpy(X).cuda()
    lens = np.full(4, 400)
    ctx.set_exclusion_radius(3)
    rc, r, e = noalloc(edm, ctx, X, lens, 8)
    assert rc == edm.EDM_OK
    ref = edm.edm_simplex_sweep(X, lengths=lens, E_max=8, ctx=ctx)
    ctx.sync()
    assert same(r, ref[0]) and torch.equal(e, ref[1])
    # 8 N + 48 N E_max ceil(L/256) bytes above 64 MiB: refused, nothing written
    ctx.set_exclusion_radius(0)
    big = torch.zeros((4096, 8192), dtype=torch.float32, device="cuda")
    rc, r, e = noalloc(edm, ctx, big, np.full(4096, 8192), 20)
    assert rc == edm.EDM_E_NOMEM
    assert b"static" in edm.load_library().edm_last_error(ctx.handle)
    ctx.sync()
    assert torch.all(r == -7.0) and torch.all(e == -7)
    ctx.close()
