"""The matrix-core filter's margin, checked on the CPU.

The chosen form evaluates, per (query p, candidate q), the BF16 product chain
    e = s N_E(q) - 2 G_E(p, q) - T,   T = kth - s N_E(p) + 2^-90  (s = 1 - 2^-12)
with -T carried as a BF16 pair rounded down (so the chain subtracts at least
T) and skips q when e is not negative.  That is safe iff e < 0 whenever the
exact float32 key K(p, q) is at most kth (such a candidate could enter the
list).  This emulates the filter's arithmetic exactly where it is exact (BF16
splits, BF16 products, the norms, the threshold pair) and the FP32
accumulation of the matrix core in several summation orders, then checks the
sign for every pair of small series chosen to stress it, with kth equal to
the pair's own key (the tightest case) and larger.  The accumulation order
inside the hardware is not specified, hence the several orders; the margin
leaves a factor of three over the worst-case bound for any order.
"""
import numpy as np
import pytest

from paper_2105_12301_amd import synth

S = np.float32(1.0 - 2.0 ** -12)
FLOOR = np.float32(2.0 ** -90)
BIG = np.float32(2.0 ** 120)


def bf16(v):
    """Round float32 to the nearest BF16 (ties to even), returned as float32."""
    u = np.asarray(v, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16_down(v):
    """Round float32 to BF16 toward -inf, returned as float32."""
    u = np.asarray(v, np.float32).view(np.uint32).astype(np.uint64)
    t = u >> 16
    t = np.where(((u >> 31) & 1).astype(bool) & ((u & 0xFFFF) != 0), t + 1, t)
    return (t << 16).astype(np.uint32).view(np.float32)


def split(v):
    v = np.asarray(v, np.float32)
    hi = bf16(v)
    lo = bf16((v - hi).astype(np.float32))
    return hi, lo


def canonical_keys(x, E, m):
    """Exact float32 key of Algorithm 1 (lag order, one rounding per op)."""
    K = np.zeros((m, m), np.float32)
    for j in range(E):
        a = x[j:j + m]
        d = (a[:, None] - a[None, :]).astype(np.float32)
        K = (K + (d * d).astype(np.float32)).astype(np.float32)
    return K


def norms(b, E, m):
    s = np.zeros(m, np.float32)
    for j in range(E):
        s = (s + (b[j:j + m] * b[j:j + m]).astype(np.float32)).astype(np.float32)
    hi, lo = split((S * s).astype(np.float32))
    return hi, lo


def accumulate(terms, order):
    """Float32 sum of the term arrays (list of [m][m]) in a given order."""
    if order == "reverse":
        terms = terms[::-1]
    elif order == "shuffle":
        rng = np.random.default_rng(0)
        terms = [terms[i] for i in rng.permutation(len(terms))]
    if order == "pairwise":
        while len(terms) > 1:
            nxt = [(terms[i] + terms[i + 1]).astype(np.float32) for i in range(0, len(terms) - 1, 2)]
            if len(terms) % 2:
                nxt.append(terms[-1])
            terms = nxt
        return terms[0]
    acc = np.zeros_like(terms[0])
    for t in terms:
        acc = (acc + t).astype(np.float32)
    return acc


def threshold_terms(kth, vp, m):
    """-T as the BF16 pair of the threshold slot, [q][p] broadcast."""
    T = np.minimum(((kth - vp[None, :]).astype(np.float32) + FLOOR).astype(np.float32), BIG)
    u = (-T).astype(np.float32)
    hi = bf16(u)
    lo = bf16_down((u - hi).astype(np.float32))
    return [np.broadcast_to(hi, (m, m)).astype(np.float32), np.broadcast_to(lo, (m, m)).astype(np.float32)]


def filter_estimate(x, E, m, order, kth=None):
    mu = np.float32(np.mean(x.astype(np.float64)))
    b = (x - mu).astype(np.float32)
    hi, lo = split(b)
    nqh, nql = norms(b, E, m)
    terms = []
    for j in range(E):
        ah, al = hi[j:j + m], lo[j:j + m]          # candidates q (rows)
        bh, bl = (-2 * hi[j:j + m]).astype(np.float32), (-2 * lo[j:j + m]).astype(np.float32)
        terms.append((ah[:, None] * bh[None, :]).astype(np.float32))  # [q][p]
        terms.append((ah[:, None] * bl[None, :]).astype(np.float32))
        terms.append((al[:, None] * bh[None, :]).astype(np.float32))
    terms.append(np.repeat(nqh[:, None], m, axis=1))
    terms.append(np.repeat(nql[:, None], m, axis=1))
    vp = (nqh + nql).astype(np.float32)                # the query side's s N_E(p)
    if kth is not None:                                # kth[q][p]
        terms += threshold_terms(kth, vp, m)
    D = accumulate(terms, order)
    return D, vp


def cases():
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=2, L=260)
    C, _ = synth.calcium_like(seed=4, N=6, L=260, n_latent=1, per_latent=3)
    yield "logistic", X[0]
    yield "calcium", C[1]
    yield "offset", (X[1] + np.float32(1000.0)).astype(np.float32)
    yield "tiled", synth.tiled_period(260, 13, 5)
    yield "big", (X[2] * np.float32(3e15)).astype(np.float32)
    yield "small", (X[3] * np.float32(1e-12)).astype(np.float32)
    rng = np.random.default_rng(3)
    yield "levels", (rng.integers(0, 3, 260) * 0.5).astype(np.float32)
    yield "heavy", rng.standard_t(2, 260).astype(np.float32)


@pytest.mark.parametrize("E", [5, 8, 9, 12, 16, 20])
@pytest.mark.parametrize("order", ["forward", "reverse", "pairwise", "shuffle"])
def test_filter_never_drops_a_closer_candidate(E, order):
    for name, x in cases():
        m = len(x) - E + 1
        K = canonical_keys(x, E, m)                     # [p][q], symmetric
        for scale in (1.0, 1.0 + 2.0 ** -20, 3.0, 1e6, np.inf):
            kth = (np.full_like(K, np.inf) if np.isinf(scale)          # list not full yet
                   else (K.T * np.float32(scale)).astype(np.float32))  # [q][p], >= the pair's key
            e, _ = filter_estimate(x, E, m, order, kth)
            bad = ~np.signbit(e)
            np.fill_diagonal(bad, False)
            assert not bad.any(), (name, E, order, scale, int(bad.sum()))


def test_margin_is_tight_enough_to_filter():
    # On chaotic data the filter rejects most candidates of a settled list:
    # with kth the 21st smallest exact key per query, few pass.
    X, _ = synth.coupled_logistic_pairs(seed=1, n_pairs=2, L=600)
    x, E = X[0], 20
    m = len(x) - E + 1
    K = canonical_keys(x, E, m)
    np.fill_diagonal(K, np.inf)
    kth = np.sort(K, axis=1)[:, E]
    e, _ = filter_estimate(x, E, m, "forward", np.broadcast_to(kth[None, :], (m, m)))
    passed = np.signbit(e).sum(axis=0)
    assert np.median(passed) <= 2 * (E + 1)
