"""Plain CPU oracle for all-to-all convergent cross mapping (CCM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
run this module: only the test suite, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path and imports nothing
from the package next to it.

What it computes follows the kEDM paper (Takahashi et al., "kEDM: A
Performance-portable Implementation of Empirical Dynamic Modeling using
Kokkos", PEARC '21):

* Section 2.1, step 1 (time-delay embedding),
* Section 2.1, step 2 (E+1 nearest neighbours, Euclidean distance),
* Section 2.1, step 3 (simplex lookup with exponential weights, first
  component of the prediction),
* Section 2.1, step 4 (Pearson correlation as the skill),
* Section 2.1, closing paragraph (steps repeated for every pair; the
  neighbour table is built once per library and reused for every target),
* Section 3.3.1, Algorithm 1 (squared distance accumulated over the E lags),
* Section 3.3.2, Algorithm 2 (the k smallest entries of each row),
* Section 3.4, Algorithm 3 (weighted sum of gathered target values) and the
  grouping of targets by their optimal embedding dimension.

Precision: the neighbour *ranking key* is evaluated in float32 exactly as
Algorithm 1 writes it (lags in ascending order, a separate rounding after every
subtraction, multiplication and addition, no fused multiply-add); everything
else (distances used for weights, weights, predictions, correlation) is float64.
numpy's float32 ufuncs perform exactly these IEEE operations one at a time.

Readings of points the paper leaves open (each is also listed in the design
notes):

* Orientation: point p has coordinates v_p[j] = X[p + j*tau], j = 0..E-1, and
  time stamp t(p) = p + (E-1)*tau (its newest sample).  This is the same point
  set as the backward-lag form of step 1 and the forward form of Algorithm 1.
* Horizon Tp: queries and candidate neighbours are both p in [0, n - Tp), with
  n = L - (E-1)*tau, so every neighbour's future value Y[t(q) + Tp] exists.
  The observation at query p is O(p) = Y[t(p) + Tp].
* Self exclusion: q = p is never a neighbour.  An optional exclusion radius
  r >= 0 (a Theiler window, which the paper does not use; default 0) also
  removes every candidate with |q - p| <= r; a call needs at least k
  candidates for every query, m - 1 - 2 r >= k.
* Ranking uses the float32 squared key; ties are broken by the lower index q.
* Weights: d_min = min_i D_i over all k neighbours.  When d_min = 0 the exact
  limit of exp(-D_i/d_min) is used: weight 1 where D_i = 0, else 0.
* Correlation: population Pearson over the query points; NaN when either
  series is constant.
* E selection (sweep): the smallest E whose rho is the largest non-NaN value;
  0 when no E is feasible.
* Uneven lengths: pair (library i, target j) is defined iff L_j >= L_i, and the
  target is read on the library's time axis [0, L_i).  Undefined pairs are NaN.
* Library subsampling (the convergence test of CCM, which Section 2.1 builds
  on but the paper does not run): a library of size l is a set of l distinct
  embedded points drawn at random by the caller; every query point p of the
  whole series is predicted from its k nearest neighbours inside that set
  (p itself and its exclusion window barred), and rho is taken over all query
  points.  The random sets are inputs, not drawn here.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "n_embedded",
    "embed",
    "knn_keys",
    "knn",
    "knn_rows",
    "weights",
    "lookup",
    "pearson",
    "simplex_rho",
    "simplex_sweep",
    "select_E",
    "ccm",
    "knn_subset",
    "ccm_subsample",
]


def n_embedded(L: int, E: int, tau: int) -> int:
    """Number of embedded points of a length-L series (Section 2.1, step 1)."""
    return int(L) - (int(E) - 1) * int(tau)


def embed(x, E: int, tau: int) -> np.ndarray:
    """Time-delay embedding, Section 2.1 step 1: out[p][j] = x[p + j*tau]."""
    x = np.asarray(x, dtype=np.float32)
    n = n_embedded(x.shape[0], E, tau)
    if E < 1 or tau < 1 or n < 1:
        raise ValueError("series too short for this embedding")
    out = np.empty((n, E), dtype=np.float32)
    for j in range(E):
        out[:, j] = x[j * tau: j * tau + n]
    return out


def knn_keys(x, E: int, tau: int, Tp: int, rows=None) -> np.ndarray:
    """Float32 squared-distance keys, Algorithm 1.

    Returns K[p][q] for p in ``rows`` (default: every query) and every
    candidate q in [0, n - Tp).  The sum runs over the lags in ascending order
    with a rounding after each operation, in float32.
    """
    v = embed(x, E, tau)
    m = v.shape[0] - Tp
    if rows is None:
        rows = np.arange(m)
    rows = np.asarray(rows)
    acc = np.zeros((rows.size, m), dtype=np.float32)
    for j in range(E):
        d = v[rows, j][:, None] - v[:m, j][None, :]   # float32, rounded
        acc = acc + d * d                              # float32, rounded twice
    return acc


def knn(x, E: int, tau: int, Tp: int, k: int = 0, block: int = 512, excl: int = 0):
    """All k-nearest-neighbour table of one library, Section 2.1 step 2.

    For every query p in [0, n - Tp): the k candidates q in [0, n - Tp) with
    |q - p| > excl (excl = 0: q != p) and the smallest (key, q), in ascending
    order (Algorithm 2's result).  k = 0 means k = E + 1.  Returns
    (idx int32 [nq][k], key float32 [nq][k]).
    """
    n = n_embedded(len(x), E, tau)
    return knn_rows(x, E, tau, Tp, np.arange(max(n - Tp, 0)), k, block, excl)


def knn_rows(x, E: int, tau: int, Tp: int, rows, k: int = 0, block: int = 512, excl: int = 0):
    """The rows ``rows`` of the table of ``knn`` (same definition), for
    checking sampled query points of long series."""
    if k == 0:
        k = E + 1
    n = n_embedded(len(x), E, tau)
    m = n - Tp
    if E < 1 or tau < 1 or Tp < 0 or k < 1 or excl < 0 or m - 1 - 2 * excl < k:
        raise ValueError("not enough points for k neighbours")
    rows = np.asarray(rows, dtype=np.int64)
    idx = np.empty((rows.size, k), dtype=np.int32)
    key = np.empty((rows.size, k), dtype=np.float32)
    allq = np.arange(m)
    for b0 in range(0, rows.size, block):
        blk = rows[b0:b0 + block]
        K = knn_keys(x, E, tau, Tp, blk)
        for r, p in enumerate(blk):
            cand = allq[np.abs(allq - p) > excl]         # self (and its window) excluded
            ck = K[r, cand]
            order = np.argsort(ck, kind="stable")[:k]   # ties keep lower q first
            idx[b0 + r] = cand[order]
            key[b0 + r] = ck[order]
    return idx, key


def weights(x, idx, E: int, tau: int, rows=None):
    """Simplex weights, Section 2.1 step 3, in float64.

    D_i = ||v_p - v_{q_i}|| from the float32 samples widened to float64,
    w_i = exp(-D_i / min_i D_i), normalised to sum to 1 ("Normalize D_k" in
    Algorithm 2).  Row r of ``idx`` belongs to query ``rows[r]`` (default: r).
    Returns (D [nq][k], wbar [nq][k]).
    """
    v = embed(x, E, tau).astype(np.float64)
    idx = np.asarray(idx)
    m, k = idx.shape
    rows = np.arange(m) if rows is None else np.asarray(rows)
    D = np.empty((m, k), dtype=np.float64)
    W = np.empty((m, k), dtype=np.float64)
    for r in range(m):
        diff = v[idx[r]] - v[rows[r]][None, :]
        D[r] = np.sqrt((diff * diff).sum(axis=1))
        dmin = D[r].min()
        if dmin > 0.0:
            w = np.exp(-D[r] / dmin)
        else:
            w = (D[r] == 0.0).astype(np.float64)
        W[r] = w / w.sum()
    return D, W


def lookup(idx, wbar, y, E: int, tau: int, Tp: int):
    """Simplex projection of target y through a library's table.

    Section 2.1 step 3 / Algorithm 3: Yhat(p) = sum_i wbar_i * y[t(q_i) + Tp],
    with t(q) = q + (E-1)*tau, i.e. the first component of the weighted
    neighbour combination.  Returns (Yhat [nq], O [nq]) with O(p) = y[t(p)+Tp].
    """
    y = np.asarray(y, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    m = idx.shape[0]
    off = (E - 1) * tau + Tp
    yhat = (np.asarray(wbar, dtype=np.float64) * y[idx + off]).sum(axis=1)
    obs = y[np.arange(m) + off]
    return yhat, obs


def pearson(a, b) -> float:
    """Population Pearson correlation, Section 2.1 step 4, two-pass float64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size < 2 or np.all(a == a[0]) or np.all(b == b[0]):
        return float("nan")
    da = a - a.mean()
    db = b - b.mean()
    return float((da * db).sum() / np.sqrt((da * da).sum() * (db * db).sum()))


def simplex_rho(x, y, E: int, tau: int, Tp: int, k: int = 0, excl: int = 0) -> float:
    """rho of predicting target y from library x (steps 1-4 for one pair)."""
    idx, _ = knn(x, E, tau, Tp, k, excl=excl)
    _, wbar = weights(x, idx, E, tau)
    yhat, obs = lookup(idx, wbar, y, E, tau, Tp)
    return pearson(obs, yhat)


def _feasible(L: int, E: int, tau: int, Tp: int, k: int, excl: int = 0) -> bool:
    return n_embedded(L, E, tau) - Tp - 1 - 2 * excl >= k


def select_E(rho_row) -> int:
    """Smallest E (1-based) attaining the largest non-NaN rho; 0 if none."""
    best, best_e = -np.inf, 0
    for e, r in enumerate(rho_row, start=1):
        if not np.isnan(r) and r > best:
            best, best_e = r, e
    return best_e


def simplex_sweep(X, lengths, E_max: int, tau: int = 1, Tp: int = 1, excl: int = 0):
    """Simplex E sweep: each series predicts itself Tp steps ahead.

    For E = 1..E_max the library and the target are the same series (Section
    2.1 step 1 leaves E to be determined empirically; Section 3.4 uses each
    target's optimal E).  Returns (rho float64 [N][E_max] with NaN where the
    series is too short, E_opt int32 [N]).
    """
    X = np.asarray(X, dtype=np.float32)
    N = X.shape[0]
    rho = np.full((N, E_max), np.nan)
    E_opt = np.zeros(N, dtype=np.int32)
    for s in range(N):
        L = int(lengths[s])
        x = X[s, :L]
        for E in range(1, E_max + 1):
            if _feasible(L, E, tau, Tp, E + 1, excl):
                rho[s, E - 1] = simplex_rho(x, x, E, tau, Tp, excl=excl)
        E_opt[s] = select_E(rho[s])
    return rho, E_opt


def ccm(X, Lx, Y, Ly, E_tgt, tau: int = 1, Tp: int = 0, lib_rows=None,
        tgt_cols=None, excl: int = 0):
    """All-to-all CCM, Section 2.1 (pairwise) and Section 3.4.

    rho[i][j] is the skill of predicting target Y_j from library X_i embedded
    at the target's optimal dimension E_tgt[j].  The library's table for a
    given E is built once and reused for every target of that E.  Returns
    rho float64 [len(lib_rows)][len(tgt_cols)] (NaN for undefined pairs).
    """
    X = np.asarray(X, dtype=np.float32)
    Y = np.asarray(Y, dtype=np.float32)
    lib_rows = np.arange(X.shape[0]) if lib_rows is None else np.asarray(lib_rows)
    tgt_cols = np.arange(Y.shape[0]) if tgt_cols is None else np.asarray(tgt_cols)
    rho = np.full((lib_rows.size, tgt_cols.size), np.nan)
    for a, i in enumerate(lib_rows):
        L = int(Lx[i])
        x = X[i, :L]
        tables = {}
        for b, j in enumerate(tgt_cols):
            E = int(E_tgt[j])
            if E < 1 or int(Ly[j]) < L or not _feasible(L, E, tau, Tp, E + 1, excl):
                continue
            if E not in tables:
                idx, _ = knn(x, E, tau, Tp, excl=excl)
                _, wbar = weights(x, idx, E, tau)
                tables[E] = (idx, wbar)
            idx, wbar = tables[E]
            yhat, obs = lookup(idx, wbar, Y[j, :L], E, tau, Tp)
            rho[a, b] = pearson(obs, yhat)
    return rho


def knn_subset(x, E: int, tau: int, Tp: int, cand, k: int = 0, excl: int = 0):
    """Neighbour table of every query p in [0, n - Tp) with the candidates
    restricted to the set ``cand`` (distinct indices in [0, n - Tp)): the k
    smallest (key, q) over q in cand with |q - p| > excl, ascending (Section
    2.1 step 2 on a library subsample).  Returns (idx int32 [nq][k], key
    float32 [nq][k])."""
    if k == 0:
        k = E + 1
    n = n_embedded(len(x), E, tau)
    m = n - Tp
    cand = np.unique(np.asarray(cand, dtype=np.int64))
    if cand.size and (cand[0] < 0 or cand[-1] >= m):
        raise ValueError("candidate index outside [0, n - Tp)")
    if cand.size - (2 * excl + 1) < k:
        raise ValueError("library subset too small for k neighbours")
    K = knn_keys(x, E, tau, Tp)
    idx = np.empty((m, k), dtype=np.int32)
    key = np.empty((m, k), dtype=np.float32)
    for p in range(m):
        c = cand[np.abs(cand - p) > excl]
        ck = K[p, c]
        order = np.argsort(ck, kind="stable")[:k]   # cand ascending: ties keep lower q first
        idx[p] = c[order]
        key[p] = ck[order]
    return idx, key


def ccm_subsample(x, y, E: int, tau: int, Tp: int, subsets, k: int = 0, excl: int = 0):
    """Cross-map skill of target y from library x for each library subsample
    (one row of ``subsets`` each): table from knn_subset, then the weights,
    lookup and Pearson of Section 2.1 steps 3-4 over every query point.
    Returns rho float64 [len(subsets)]."""
    out = np.empty(len(subsets))
    for s, cand in enumerate(subsets):
        idx, _ = knn_subset(x, E, tau, Tp, cand, k, excl)
        _, wbar = weights(x, idx, E, tau)
        yhat, obs = lookup(idx, wbar, y, E, tau, Tp)
        out[s] = pearson(obs, yhat)
    return out
