"""Batched CCM plan (persistent launches, graph replay) against edm_ccm and the
oracle, on libraries of uneven length with per-target E."""
import numpy as np
import pytest

from oracle import edm_oracle as O
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
def side():
    s = torch.cuda.Stream()  # default priority; graphs cannot capture the legacy stream
    return s


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


TUNES = [dict(tables_wg_per_cu=0, lookup_wg_per_cu=0, lookup_targets=4),
         dict(tables_wg_per_cu=1, lookup_wg_per_cu=4, lookup_targets=2),
         dict(tables_wg_per_cu=2, lookup_wg_per_cu=8, lookup_targets=1)]


@pytest.mark.parametrize("tune", TUNES, ids=["grid", "persistent-1", "persistent-2"])
@pytest.mark.parametrize("limit", [None, 4 << 20])
def test_plan_equals_ccm_bitwise(edm, side, tune, limit, monkeypatch):
    if limit:
        monkeypatch.setenv("EDM_WORKSPACE_LIMIT", str(limit))
    from paper_2105_12301_amd.autotune import make_tune
    X, lens, E = synth.spike_trains(seed=21, N=48, L_min=150, L_max=1400)
    E[5] = 0
    with torch.cuda.stream(side):
        ctx = edm.Context(device=0, stream=side)
        Xd = dev(X)
        ref = edm.edm_ccm(Xd, dev(E), Lx=lens, Ly=lens, ctx=ctx)
        plan = edm.CcmPlan(lens, lens, E, X.shape[1], X.shape[1], tune=make_tune(tune), ctx=ctx)
        r1 = plan.run(Xd).clone()   # captures the graph
        r2 = plan.run(Xd).clone()   # replays it
        ctx.sync()
        assert torch.equal(ref.view(torch.int32), r1.view(torch.int32))
        assert torch.equal(r1.view(torch.int32), r2.view(torch.int32))
        plan.close()
        ctx.close()


@pytest.mark.parametrize("form", ["plain", "chosen"])
def test_plan_full_target_tiles_bitwise(edm, side, form):
    # Few E values, so each E bucket holds ~20 targets: lookup items stage 16
    # targets, every wave makes several table passes (4 targets a pass, 2 at
    # E = 20), and each group of 16 libraries of mixed length skips the
    # targets shorter than a library.
    from paper_2105_12301_amd.autotune import make_tune
    X, lens, _ = synth.spike_trains(seed=24, N=64, L_min=150, L_max=1400)
    E = np.random.default_rng(24).choice(np.array([3, 6, 20], np.int32), size=len(lens))
    with torch.cuda.stream(side):
        ctx = edm.Context(device=0, stream=side, form=edm.EDM_FORM_PLAIN)
        Xd = dev(X)
        ref = edm.edm_ccm(Xd, dev(E), Lx=lens, Ly=lens, ctx=ctx)
        if form == "chosen":
            ctx.set_form(edm.EDM_FORM_CHOSEN)
        tune = make_tune(dict(tables_wg_per_cu=0, lookup_wg_per_cu=4, lookup_targets=16))
        plan = edm.CcmPlan(lens, lens, E, X.shape[1], X.shape[1], tune=tune, ctx=ctx)
        r1 = plan.run(Xd).clone()
        r2 = plan.run(Xd).clone()
        ctx.sync()
        assert torch.isfinite(ref).sum().item() > 1000
        assert torch.equal(ref.view(torch.int32), r1.view(torch.int32))
        assert torch.equal(r1.view(torch.int32), r2.view(torch.int32))
        plan.close()
        ctx.close()


@pytest.mark.parametrize("tune", TUNES[:2], ids=["grid", "persistent-1"])
def test_chosen_plan_equals_plain_ccm_bitwise(edm, side, tune):
    # In the chosen form the plan's tables for E >= 5 come from the matrix-core
    # filter for libraries up to 14336 samples and from the exact scan for
    # longer ones; every rho must equal the plain form's bit for bit.
    from paper_2105_12301_amd.autotune import make_tune
    X, lens, E = synth.spike_trains(seed=22, N=40, L_min=150, L_max=1400)
    Xw = np.zeros((X.shape[0] + 2, 14400), np.float32)
    Xw[:X.shape[0], :X.shape[1]] = X
    long_x, _, _ = synth.logistic_network(seed=23, N=4, L=14400)
    Xw[-2:] = long_x[:2]
    lens = np.concatenate([lens, [14336, 14400]]).astype(np.int64)
    E = np.concatenate([E, [7, 12]]).astype(np.int32)
    E[3] = 0
    with torch.cuda.stream(side):
        ctx = edm.Context(device=0, stream=side, form=edm.EDM_FORM_PLAIN)
        Xd = dev(Xw)
        ref = edm.edm_ccm(Xd, dev(E), Lx=lens, Ly=lens, ctx=ctx)
        ctx.set_form(edm.EDM_FORM_CHOSEN)
        plan = edm.CcmPlan(lens, lens, E, Xw.shape[1], Xw.shape[1], tune=make_tune(tune), ctx=ctx)
        r1 = plan.run(Xd).clone()
        r2 = plan.run(Xd).clone()
        ctx.sync()
        assert torch.equal(ref.view(torch.int32), r1.view(torch.int32))
        assert torch.equal(r1.view(torch.int32), r2.view(torch.int32))
        plan.close()
        ctx.close()


@pytest.mark.parametrize("stride", [1, 3, 8])
def test_chosen_plan_filter_stride_bitwise(edm, side, stride):
    # The filter's first-pass tile stride (a tune field) changes only how
    # tight the first bounds are: every rho equals the plain form's bit for
    # bit, for series both shorter and longer than 4096 samples.
    from paper_2105_12301_amd.autotune import make_tune
    X, lens, E = synth.spike_trains(seed=24, N=24, L_min=300, L_max=6000)
    E = np.where(E < 5, E + 8, E).astype(np.int32)   # every pair through the filter
    with torch.cuda.stream(side):
        ctx = edm.Context(device=0, stream=side, form=edm.EDM_FORM_PLAIN)
        Xd = dev(X)
        ref = edm.edm_ccm(Xd, dev(E), Lx=lens, Ly=lens, ctx=ctx)
        ctx.set_form(edm.EDM_FORM_CHOSEN)
        tune = make_tune(dict(TUNES[0], filter_stride=stride))
        plan = edm.CcmPlan(lens, lens, E, X.shape[1], X.shape[1], tune=tune, ctx=ctx)
        r1 = plan.run(Xd).clone()
        ctx.sync()
        assert torch.equal(ref.view(torch.int32), r1.view(torch.int32))
        plan.close()
        ctx.close()


def test_plan_rejects_filter_stride_out_of_range(edm):
    from paper_2105_12301_amd.autotune import make_tune
    X, lens, E = synth.spike_trains(seed=25, N=8, L_min=300, L_max=600)
    ctx = edm.Context(device=0)
    with pytest.raises(edm.EdmError):
        edm.CcmPlan(lens, lens, E, X.shape[1], X.shape[1], tune=make_tune(dict(TUNES[0], filter_stride=9)), ctx=ctx)
    ctx.close()


def test_plan_matches_oracle_and_default_stream(edm):
    X, lens, E = synth.spike_trains(seed=22, N=20, L_min=200, L_max=900)
    ctx = edm.Context(device=0)   # legacy stream: enqueued without a graph
    plan = edm.CcmPlan(lens, lens, E, X.shape[1], X.shape[1], ctx=ctx)
    r = plan.run(dev(X))
    ctx.sync()
    ro = O.ccm(X, lens, X, lens, E, lib_rows=[0, 7, 19])
    g = r.cpu().numpy()[[0, 7, 19]]
    assert np.array_equal(np.isnan(g), np.isnan(ro))
    assert np.nanmax(np.abs(g - ro)) <= 1e-5
    plan.close()


def test_autotune_picks_a_candidate(edm, side, tmp_path, monkeypatch):
    monkeypatch.setenv("EDM_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    from paper_2105_12301_amd import autotune
    X, lens, E = synth.spike_trains(seed=23, N=32, L_min=300, L_max=1200)
    with torch.cuda.stream(side):
        ctx = edm.Context(device=0, stream=side)
        Xd = dev(X)
        t, times = autotune.autotune(Xd, lens, Xd, lens, E, ctx=ctx, sample=8, reps=1)
        assert len(times) == len(autotune.CANDIDATES)
        t2, _ = autotune.autotune(Xd, lens, Xd, lens, E, ctx=ctx, sample=8, reps=1)   # cached
        assert t.as_dict() == t2.as_dict()
        # chosen form: the filter's first-pass stride is searched as well
        ctx.set_form(edm.EDM_FORM_CHOSEN)
        t3, times3 = autotune.autotune(Xd, lens, Xd, lens, E, ctx=ctx, sample=8, reps=1)
        assert len(times3) == len(autotune.CANDIDATES) + len(autotune.FILTER_STRIDES)
        assert t3.filter_stride in (0,) + autotune.FILTER_STRIDES
        ctx.close()
