"""Surrogate network kernels (through the C ABI) against the float64 oracle,
and the network-driven E selection against the plain sweep."""
import numpy as np
import pytest

from oracle import net_oracle as NO
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


@pytest.fixture(scope="module")
def ctx(edm):
    c = edm.Context(device=0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def case(C, L, B, seed):
    rng = np.random.default_rng(seed)
    theta = synth.net_init_params(C, seed=seed).astype(np.float64)
    theta += rng.normal(scale=0.05, size=theta.size)
    theta = theta.astype(np.float32)
    X = rng.normal(size=(B, L)).astype(np.float32)
    y = rng.integers(1, 21, size=B).astype(np.int32)
    return theta, X, y


@pytest.mark.parametrize("C,L,B", [(8, 64, 5), (8, 131, 3), (64, 300, 3), (16, 1500, 2)])
def test_forward_logits(edm, ctx, C, L, B):
    theta, X, _ = case(C, L, B, C + L)
    lg = edm.edm_net_forward(dev(theta), C, dev(X), ctx=ctx)
    ctx.sync()
    ref, _ = NO.forward(theta.astype(np.float64), X, C)
    np.testing.assert_allclose(lg.cpu().numpy(), ref, rtol=1e-4, atol=1e-5)


@pytest.mark.parametrize("C,L,B", [(64, 300, 3), (64, 1500, 2), (32, 257, 3), (64, 5, 2)])
def test_forward_bf16_logits(edm, ctx, C, L, B):
    # BF16 inference form against the oracle's emulation of it (weights and
    # C->C inputs rounded to BF16, exact products, float64 sums).  The GPU sums
    # in FP32 and rounds its own FP32 activations, so a value sitting on a
    # BF16 rounding boundary may round the other way: the bar is 1e-3 of the
    # logit scale, against ~1e-2 for the BF16-vs-float64 difference itself.
    theta, X, _ = case(C, L, B, 3 * C + L)
    lg = edm.edm_net_forward_bf16(dev(theta), C, dev(X), ctx=ctx)
    ctx.sync()
    got = lg.cpu().numpy()
    emu = NO.forward_bf16(theta.astype(np.float64), X, C)
    ref, _ = NO.forward(theta.astype(np.float64), X, C)
    scale = max(1.0, float(np.abs(ref).max()))
    assert np.abs(got - emu).max() <= 1e-3 * scale
    assert np.abs(got - ref).max() <= 3e-2 * scale


def test_forward_bf16_rejects_other_widths(edm, ctx):
    theta, X, _ = case(16, 64, 2, 1)
    with pytest.raises(edm.EdmError):
        edm.edm_net_forward_bf16(dev(theta), 16, dev(X), ctx=ctx)


@pytest.mark.parametrize("C,L,B", [(8, 64, 5), (8, 200, 4), (64, 300, 3)])
def test_loss_and_gradients(edm, ctx, C, L, B):
    theta, X, y = case(C, L, B, 7 * C + L)
    loss, grad = edm.edm_net_loss_grad(dev(theta), C, dev(X), dev(y), ctx=ctx)
    ctx.sync()
    rl, rg = NO.loss_and_grads(theta.astype(np.float64), X, y, C)
    assert abs(float(loss) - rl) <= 1e-5 * max(1.0, abs(rl))
    g = grad.cpu().numpy()
    scale = np.abs(rg).max()
    np.testing.assert_allclose(g, rg, rtol=1e-4, atol=1e-5 * scale)


def test_gradients_deterministic(edm, ctx):
    theta, X, y = case(16, 400, 8, 3)
    _, g1 = edm.edm_net_loss_grad(dev(theta), 16, dev(X), dev(y), ctx=ctx)
    _, g2 = edm.edm_net_loss_grad(dev(theta), 16, dev(X), dev(y), ctx=ctx)
    ctx.sync()
    assert torch.equal(g1, g2)


def test_adam_step(edm, ctx):
    rng = np.random.default_rng(4)
    n = 1000
    p, g = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m, v = rng.normal(size=n).astype(np.float32) * 0.1, np.abs(rng.normal(size=n)).astype(np.float32) * 0.1
    P, G, M, V = dev(p), dev(g), dev(m), dev(v)
    edm.edm_net_adam(P, G, M, V, 3, 1e-3, ctx=ctx)
    ctx.sync()
    # the hyper-parameters cross the ABI as float32: give the oracle the same values
    f32 = lambda a: float(np.float32(a))  # noqa: E731
    rp, rm, rv = NO.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                              v.astype(np.float64), 3, f32(1e-3), b1=f32(0.9), b2=f32(0.999),
                              eps=f32(1e-8))
    np.testing.assert_allclose(P.cpu().numpy(), rp, rtol=0, atol=1e-6)
    np.testing.assert_allclose(M.cpu().numpy(), rm, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(V.cpu().numpy(), rv, rtol=1e-6, atol=1e-7)


def test_select_all_candidates_equals_sweep(edm, ctx):
    X, _ = synth.surrogate_mix(seed=11, N=24, L=500)
    Xd = dev(X)
    logits = torch.zeros((24, 20), dtype=torch.float32, device="cuda")
    rs, es = edm.edm_simplex_sweep(Xd, E_max=20, ctx=ctx)
    r1, e1, nfb = edm.edm_select_E(Xd, logits, E_max=20, m_top=20, ctx=ctx)
    r2, e2, nfb2 = edm.edm_select_E(Xd, logits, E_max=20, m_top=1, min_conf=1.0, ctx=ctx)
    ctx.sync()
    assert torch.equal(rs.view(torch.int32), r1.view(torch.int32)) and torch.equal(es, e1)
    assert torch.equal(rs.view(torch.int32), r2.view(torch.int32)) and torch.equal(es, e2)
    assert nfb == 0 and nfb2 == 24


def test_select_top1_evaluates_only_the_proposal(edm, ctx):
    X, _ = synth.surrogate_mix(seed=12, N=16, L=400)
    Xd = dev(X)
    prop = np.arange(16) % 20 + 1
    logits = np.full((16, 20), -5.0, np.float32)
    logits[np.arange(16), prop - 1] = 5.0
    rs, _ = edm.edm_simplex_sweep(Xd, E_max=20, ctx=ctx)
    r, e, nfb = edm.edm_select_E(Xd, dev(logits), E_max=20, m_top=1, min_conf=0.5, ctx=ctx)
    ctx.sync()
    r, e, rs = r.cpu().numpy(), e.cpu().numpy(), rs.cpu().numpy()
    assert nfb == 0 and np.array_equal(e, prop)
    for s in range(16):
        assert np.array_equal(np.isnan(r[s]), np.arange(1, 21) != prop[s])
        assert r[s, prop[s] - 1] == rs[s, prop[s] - 1]


@pytest.mark.parametrize("form", ["chosen", "batched"])
def test_select_mixed_fallback_batched_form(edm, form):
    # Even series get one confident proposal; odd series uniform logits, below
    # min_conf, so they take the full sweep, which the batched forms run on
    # packed rows (uneven lengths) and scatter back.
    N = 40
    X, _ = synth.surrogate_mix(seed=13, N=N, L=700)
    lens = np.random.default_rng(13).integers(300, 701, size=N)
    Xd = dev(X)
    prop = np.arange(N) % 20 + 1
    logits = np.zeros((N, 20), np.float32)
    ev = np.arange(0, N, 2)
    logits[ev, prop[ev] - 1] = 8.0
    c = edm.Context(device=0, form=getattr(edm, f"EDM_FORM_{form.upper()}"))
    rs, es = edm.edm_simplex_sweep(Xd, lengths=lens, E_max=20, ctx=c)
    r, e, nfb = edm.edm_select_E(Xd, dev(logits), lengths=lens, E_max=20, m_top=1, min_conf=0.5, ctx=c)
    c.sync()
    r, e, rs, es = r.cpu().numpy(), e.cpu().numpy(), rs.cpu().numpy(), es.cpu().numpy()
    c.close()
    assert nfb == N // 2
    for s in range(N):
        if s % 2:
            assert np.array_equal(r[s].view(np.int32), rs[s].view(np.int32)) and e[s] == es[s]
        else:
            assert np.array_equal(np.isnan(r[s]), np.arange(1, 21) != prop[s])
            assert r[s, prop[s] - 1] == rs[s, prop[s] - 1] and e[s] == prop[s]
