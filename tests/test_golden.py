"""The oracle against the hand-worked examples of tests/golden/ (CPU).

The fixtures were worked out by hand from Section 2.1 steps 1-4 and
Algorithms 1-3 (exact integer neighbour tables and squared distances, closed-
form weights), so they pin the oracle to something other than itself: a
transposed embedding, a wrong horizon offset, a tie broken the other way, a
dropped normalisation, a wrong Pearson term, an exclusion window off by one or
a subsample that leaks other candidates each changes a stored value.
"""
import numpy as np
import pytest

from golden_io import load
from oracle import edm_oracle as O

CASES = load()
TABLES = sorted(n for n in CASES if "idx" in CASES[n])


def table(c):
    x = c["x"].astype(np.float32)
    if "subset" in c:
        return O.knn_subset(x, c["E"], c["tau"], c["Tp"], c["subset"].astype(np.int64), c["k"],
                            excl=c.get("excl", 0))
    return O.knn(x, c["E"], c["tau"], c["Tp"], c["k"], excl=c.get("excl", 0))


@pytest.mark.parametrize("name", TABLES)
def test_table_and_keys(name):
    c = CASES[name]
    idx, key = table(c)
    assert np.array_equal(idx, c["idx"].astype(np.int32))
    assert np.array_equal(key, c["key"].astype(np.float32))


@pytest.mark.parametrize("name", TABLES)
def test_weights_prediction_rho(name):
    c = CASES[name]
    x = c["x"].astype(np.float32)
    idx = c["idx"].astype(np.int64)
    D, w = O.weights(x, idx, c["E"], c["tau"])
    assert np.allclose(D, np.sqrt(c["key"]), rtol=0, atol=1e-15)
    assert np.allclose(w, c["w"], rtol=0, atol=1e-15)
    pred, obs = O.lookup(idx, w, c["y"], c["E"], c["tau"], c["Tp"])
    assert np.array_equal(obs, c["obs"])
    assert np.allclose(pred, c["pred"], rtol=0, atol=1e-13)
    assert abs(O.pearson(obs, pred) - c["rho"][0]) < 1e-13
    if "subset" in c:
        r = O.ccm_subsample(x, c["y"], c["E"], c["tau"], c["Tp"], [c["subset"].astype(np.int64)],
                            c["k"], excl=c.get("excl", 0))[0]
    else:
        r = O.simplex_rho(x, c["y"], c["E"], c["tau"], c["Tp"], c["k"], excl=c.get("excl", 0))
    assert abs(r - c["rho"][0]) < 1e-13


@pytest.mark.parametrize("name", ["A", "A_excl1"])
def test_ccm_pair(name):
    # The cross map of Section 3.4 with the target's E equal to the case's E
    # reaches the same pair: library x, target y (k = E + 1 in these cases).
    c = CASES[name]
    assert c["k"] == c["E"] + 1
    X = c["x"][None, :].astype(np.float32)
    Y = c["y"][None, :].astype(np.float32)
    L = np.array([X.shape[1]])
    rho = O.ccm(X, L, Y, L, np.array([c["E"]]), tau=c["tau"], Tp=c["Tp"], excl=c.get("excl", 0))
    assert abs(rho[0, 0] - c["rho"][0]) < 1e-13


def test_full_subset_is_case_A():
    # The subsample of every candidate is the plain table (case A).
    c = CASES["A"]
    x = c["x"].astype(np.float32)
    idx, _ = O.knn_subset(x, c["E"], c["tau"], c["Tp"], np.arange(6), c["k"])
    assert np.array_equal(idx, c["idx"].astype(np.int32))


def test_sweep():
    # Section 2.1: E chosen by simplex self-prediction; case S worked by hand.
    c = CASES["S"]
    x = c["x"].astype(np.float32)
    for E in (1, 3):
        idx, _ = O.knn(x, E, c["tau"], c["Tp"])
        assert np.array_equal(idx, c[f"idx_E{E}"].astype(np.int32)), E
    for E in (1, 2, 3):
        idx, _ = O.knn(x, E, c["tau"], c["Tp"])
        _, w = O.weights(x, idx, E, c["tau"])
        pred, _ = O.lookup(idx, w, x, E, c["tau"], c["Tp"])
        assert np.allclose(pred, c[f"pred_E{E}"], rtol=0, atol=1e-13), E
    rho, E_opt = O.simplex_sweep(x[None, :], np.array([x.size]), c["E_max"], c["tau"], c["Tp"])
    want = c["rho_sweep"]
    assert np.array_equal(np.isnan(rho[0]), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.allclose(rho[0][ok], want[ok], rtol=0, atol=1e-13)
    assert int(E_opt[0]) == c["E_opt"]
