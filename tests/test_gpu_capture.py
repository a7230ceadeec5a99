"""The fused pipeline (edm_sweep_ccm, chosen form) groups its targets by E on
the device, so with equal lengths a call has no host transfer and no
synchronisation: it is captured in a HIP graph and replayed.  Every replay,
with the program's own eager work and synchronisations between replays,
must equal the uncaptured call bit for bit."""
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


def bits(t):
    return t.view(torch.int32)


def test_sweep_ccm_graph_replays(edm):
    X, _, _ = synth.logistic_network(seed=9, N=48, L=900)
    Xd = torch.from_numpy(X).cuda()
    X2 = torch.from_numpy(synth.logistic_network(seed=10, N=48, L=900)[0]).cuda()
    N = X.shape[0]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = edm.Context(device=0, stream=s, form=edm.EDM_FORM_CHOSEN)
        rs = torch.empty((N, 20), dtype=torch.float32, device="cuda")
        Es = torch.empty((N,), dtype=torch.int32, device="cuda")
        rho = torch.empty((N, N), dtype=torch.float32, device="cuda")
        # eager reference (also grows the workspace before the capture)
        ref = [t.clone() for t in edm.edm_sweep_ccm(Xd, E_max=20, ctx=ctx)]
        ctx.sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        edm.edm_sweep_ccm(Xd, E_max=20, rho=rho, rho_sweep=rs, E_opt=Es, ctx=ctx)
    for rep in range(3):
        with torch.cuda.stream(s):
            rs.fill_(-1.0)
            Es.fill_(-1)
            rho.fill_(-1.0)
            other = edm.edm_sweep_ccm(X2, E_max=20, ctx=ctx)  # eager work in between
            ctx.sync()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bits(rs), bits(ref[0])), rep
        assert torch.equal(Es, ref[1]), rep
        assert torch.equal(bits(rho), bits(ref[2])), rep
        assert other[2].isfinite().any()
    with torch.cuda.stream(s):
        ctx.close()


def test_sweep_ccm_device_grouping_matches_plain(edm):
    # E* spread over many buckets, including empty ones and E = 0 (too short):
    # the device-grouped cross map equals the plain sweep + edm_ccm.
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=4, L=600)
    Xl, _, _ = synth.logistic_network(seed=11, N=24, L=600)
    Xa = np.concatenate([X, Xl], axis=0)
    lens = np.full(Xa.shape[0], 600)
    lens[3] = 30
    lens[17] = 12           # too short for any E at k = E + 1 with Tp = 1
    Xd = torch.from_numpy(Xa).cuda()
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    a = edm.edm_sweep_ccm(Xd, lengths=lens, E_max=20, ctx=ctx)
    ctx.set_form(edm.EDM_FORM_PLAIN)
    rs, Es = edm.edm_simplex_sweep(Xd, lengths=lens, E_max=20, ctx=ctx)
    rho = edm.edm_ccm(Xd, Es, Lx=lens, Ly=lens, ctx=ctx)
    ctx.sync()
    assert torch.equal(bits(a[0]), bits(rs))
    assert torch.equal(a[1], Es)
    assert torch.equal(bits(a[2]), bits(rho))
    ctx.close()
