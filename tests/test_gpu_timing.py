"""Kernel timing through the C ABI (edm_ctx_set_timing / edm_ctx_timing):
launches are attributed to their kernel families and the totals clear."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_12301_amd import edm, synth

pytestmark = pytest.mark.gpu


def test_timing_attributes_launches_to_families():
    X, _, _ = synth.logistic_network(seed=2, N=16, L=600)
    Xd = torch.from_numpy(X).cuda()
    ctx = edm.Context(device=0, form=edm.EDM_FORM_CHOSEN)
    ctx.set_timing(True)
    edm.edm_sweep_ccm(Xd, E_max=8, ctx=ctx)
    t = ctx.timing()
    for fam in ("batched_scan", "filter_prep", "filter_scan", "finalize", "lookup"):
        ms, n = t[fam]
        assert n >= 1 and ms > 0.0, (fam, t[fam])
    assert t["exact_scan"][1] == 0
    again = ctx.timing()  # cleared by the previous read
    assert all(n == 0 for _, n in again.values())
    ctx.set_form(edm.EDM_FORM_PLAIN)
    edm.edm_simplex_sweep(Xd, E_max=8, ctx=ctx)
    t = ctx.timing()
    assert t["exact_scan"][1] == 8 and t["exact_scan"][0] > 0.0
    ctx.set_timing(False)
    edm.edm_simplex_sweep(Xd, E_max=8, ctx=ctx)
    assert all(n == 0 for _, n in ctx.timing().values())
    ctx.close()


def test_ceilings_are_plausible():
    ctx = edm.Context(device=0)
    c = ctx.ceilings()
    # a streaming copy reaches a sizeable share of the 8 TB/s HBM, the matrix
    # cores a sizeable share of the 2.5 PFLOP/s BF16 peak; neither exceeds it
    assert 1000.0 < c["hbm_copy_GBps"] <= 8000.0, c
    assert 500.0 < c["mfma_bf16_TFLOPs"] <= 2500.0, c
    assert 5.0 < c["valu_fp32_Tops"] <= 157.3, c
    ctx.close()
