"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/edm.h declares, and rejects invalid arguments on the host before any
device work (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2105_12301_amd import edm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NULL = None
P = ctypes.c_void_p(256)  # a non-NULL stand-in; never dereferenced by validation


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "edm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(edm_[A-Za-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(edm.LIB_PATH):
        pytest.skip("libedm.so not built (run __graft_entry__.build())")
    return edm.load_library()


def test_header_declares_the_five_calls():
    names = declared_symbols()
    for n in ("edm_embed", "edm_knn", "edm_lookup", "edm_simplex_sweep", "edm_ccm"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert set(names) == set(edm.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_exported_with_c_linkage():
    out = os.popen(f"nm -D --defined-only {edm.LIB_PATH}").read()
    for n in declared_symbols():
        assert re.search(rf"\bT {n}$", out, re.M), n


def err(lib):
    return lib.edm_last_error(None).decode()


def test_knn_validation(lib):
    assert lib.edm_knn(NULL, P, 100, 0, 1, 0, 0, P, NULL, NULL) == edm.EDM_E_ARG
    assert lib.edm_knn(NULL, P, 100, 21, 1, 0, 0, P, NULL, NULL) == edm.EDM_E_ARG
    assert lib.edm_knn(NULL, P, 100, 2, 0, 0, 0, P, NULL, NULL) == edm.EDM_E_ARG
    assert lib.edm_knn(NULL, P, 100, 2, 1, -1, 0, P, NULL, NULL) == edm.EDM_E_ARG
    assert lib.edm_knn(NULL, P, 100, 2, 1, 0, 33, P, NULL, NULL) == edm.EDM_E_ARG
    assert lib.edm_knn(NULL, NULL, 100, 2, 1, 0, 0, P, NULL, NULL) == edm.EDM_E_ARG
    assert lib.edm_knn(NULL, P, 100, 2, 1, 0, 0, NULL, NULL, NULL) == edm.EDM_E_ARG
    assert lib.edm_knn(NULL, P, 40000, 2, 1, 0, 0, P, NULL, NULL) == edm.EDM_E_ARG
    # L = 6, E = 3, Tp = 1: nq = 3, needs nq - 1 >= 4
    assert lib.edm_knn(NULL, P, 6, 3, 1, 1, 0, P, NULL, NULL) == edm.EDM_E_SHORT
    assert "too short" in err(lib)
    # boundary: nq - 1 == k is accepted (then fails only on the NULL context)
    assert lib.edm_knn(NULL, P, 8, 3, 1, 1, 0, P, NULL, NULL) == edm.EDM_E_ARG
    assert "context" in err(lib)


def test_lookup_validation(lib):
    f = lib.edm_lookup
    assert f(NULL, P, P, 100, 3, 2, 1, 0, P, 4, 101, NULL, NULL) == edm.EDM_E_ARG  # nothing to do
    assert f(NULL, P, P, 100, 3, 2, 1, 0, P, 4, 100, NULL, P) == edm.EDM_E_ARG     # ldy too short
    assert f(NULL, P, P, 3, 3, 2, 1, 0, P, 4, 101, NULL, P) == edm.EDM_E_SHORT
    assert f(NULL, P, P, 100, 0, 2, 1, 0, P, 4, 101, NULL, P) == edm.EDM_E_ARG
    assert f(NULL, P, P, 100, 3, 2, 1, 0, P, 4, 101, NULL, P) == edm.EDM_E_ARG     # NULL ctx
    assert "context" in err(lib)


def test_sweep_and_ccm_validation(lib):
    L = (ctypes.c_int64 * 2)(100, 100)
    Lbad = (ctypes.c_int64 * 2)(100, 101)
    s = lib.edm_simplex_sweep
    assert s(NULL, P, L, 2, 100, 0, 1, 1, P, P) == edm.EDM_E_ARG
    assert s(NULL, P, L, 2, 100, 21, 1, 1, P, P) == edm.EDM_E_ARG
    assert s(NULL, P, Lbad, 2, 100, 10, 1, 1, P, P) == edm.EDM_E_ARG
    assert s(NULL, P, L, 2, 100, 10, 1, 1, P, P) == edm.EDM_E_ARG  # NULL ctx
    c = lib.edm_ccm
    assert c(NULL, P, L, 2, 100, P, Lbad, 2, 100, P, 1, 0, P) == edm.EDM_E_ARG
    assert c(NULL, P, L, 2, 100, P, L, 2, 100, NULL, 1, 0, P) == edm.EDM_E_ARG
    assert c(NULL, P, L, 2, 100, P, L, 2, 100, P, 0, 0, P) == edm.EDM_E_ARG
    assert c(NULL, P, L, 2, 100, P, L, 2, 100, P, 1, 0, P) == edm.EDM_E_ARG  # NULL ctx


def test_ctx_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.edm_ctx_create(ctypes.byref(h), NULL) == edm.EDM_E_HIP
    assert not h.value


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2105_12301_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), f
                assert "oracle" not in text.lower(), f"{f} mentions the oracle"


def test_net_validation(lib):
    assert lib.edm_net_param_count(64) == 7 * 64 + 64 + 2 * (64 * 64 * 7 + 64) + 20 * 64 + 20
    assert lib.edm_net_param_count(0) < 0 and lib.edm_net_param_count(65) < 0
    f = lib.edm_net_forward
    assert f(NULL, P, 0, P, 4, 100, 100, P) == edm.EDM_E_ARG        # C = 0
    assert f(NULL, P, 8, P, 4, 100, 99, P) == edm.EDM_E_ARG         # ldx < L
    assert f(NULL, P, 8, P, 4, 100, 100, NULL) == edm.EDM_E_ARG     # no logits
    assert f(NULL, P, 8, P, 4, 100, 100, P) == edm.EDM_E_ARG        # NULL ctx
    g = lib.edm_net_loss_grad
    assert g(NULL, P, 8, P, NULL, 4, 100, 100, P, P) == edm.EDM_E_ARG
    a = lib.edm_net_adam
    assert a(NULL, P, P, P, P, 10, 0, 1e-3, 0.9, 0.999, 1e-8) == edm.EDM_E_ARG   # step 0
    assert a(NULL, P, P, P, P, 10, 1, 1e-3, 1.0, 0.999, 1e-8) == edm.EDM_E_ARG   # beta1 = 1
    L = (ctypes.c_int64 * 2)(100, 100)
    s = lib.edm_select_E
    nfb = ctypes.c_int64()
    assert s(NULL, P, L, 2, 100, 20, 1, 1, P, 0, 0.0, P, P, ctypes.byref(nfb)) == edm.EDM_E_ARG
    assert s(NULL, P, L, 2, 100, 20, 1, 1, P, 2, 1.5, P, P, ctypes.byref(nfb)) == edm.EDM_E_ARG
    assert s(NULL, P, L, 2, 100, 20, 1, 1, NULL, 2, 0.5, P, P, ctypes.byref(nfb)) == edm.EDM_E_ARG


def test_kernel_family_names_follow_the_header():
    src = open(os.path.join(ROOT, "include", "edm.h")).read()
    fams = dict((int(v), k) for k, v in re.findall(r"\bEDM_KF_([A-Z_]+)\s*=\s*(\d+)", src))
    count = fams.pop(max(fams))
    assert count == "COUNT" and len(fams) == len(edm.KERNEL_FAMILIES)
    for i, name in enumerate(edm.KERNEL_FAMILIES):
        assert fams[i].lower() == name, (i, fams[i], name)


def test_timing_calls_reject_null_context(lib):
    assert lib.edm_ctx_set_timing(NULL, 1) == edm.EDM_E_ARG
    assert lib.edm_ctx_timing(NULL, NULL, NULL) == edm.EDM_E_ARG
