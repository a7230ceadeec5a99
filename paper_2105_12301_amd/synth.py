"""Seeded synthetic time-series generators.

These stand in for the neural and gene-expression recordings the kEDM paper
evaluates on (Section 4.3, Table 1), which are not available here.  Every
generator draws from ``numpy.random.default_rng(seed)`` (PCG64), integrates in
float64, stores float32 series in a row-major ``[N][L]`` array and asserts the
result is finite.

This module holds no part of the EDM method itself (no embedding, neighbour
search, lookup or correlation): it only produces inputs.  It is the one module
shared by both sides of every comparison in the tests and the benchmark.

Workloads (sizes are the defaults; tests pass smaller ones):

* ``coupled_logistic_pairs`` -- small case: 8 logistic series in 4 independent
  driver -> response pairs, x' = x (3.8 - 3.8 x - beta y), beta ~ U[0.02, 0.1].
* ``logistic_network`` -- 1024 series, each driven by 3 distinct random others
  through the mean coupling (1/3) sum beta_ij y_j, beta ~ U[0, 0.1], plus
  N(0, 0.01^2) observation noise, L = 5000.
* ``spike_trains`` -- AR(1)-filtered Poisson spike counts (rate ~ U[0.5, 5] Hz
  sampled at 2 Hz, decay 0.9), z-scored, with uneven lengths L ~ U{1000..20000}
  and a per-series E ~ U{1..20}.
* ``calcium_like`` -- 10000 spike-derived series of length 2000, 20 % of them
  modulated by 20 shared latent logistic drivers.
* ``surrogate_mix`` -- logistic, Euler-integrated Lorenz x and AR(2) series of
  length 1500, z-scored, one third each.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter

__all__ = [
    "coupled_logistic_pairs",
    "logistic_network",
    "spike_trains",
    "calcium_like",
    "surrogate_mix",
    "zscore",
    "sine",
    "ramp",
    "tiled_period",
    "net_init_params",
    "library_subsets",
]


def _finite(a: np.ndarray) -> np.ndarray:
    assert np.all(np.isfinite(a)), "generator produced a non-finite value"
    return a


def zscore(x: np.ndarray) -> np.ndarray:
    """Row-wise z-score with the population standard deviation, in float64."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean(axis=-1, keepdims=True)
    sd = x.std(axis=-1, keepdims=True)
    sd = np.where(sd > 0, sd, 1.0)
    return (x - mu) / sd


def coupled_logistic_pairs(seed: int = 1, n_pairs: int = 4, L: int = 1000):
    """Driver -> response logistic-map pairs.

    Series 2m is autonomous, x' = 3.8 x (1 - x); series 2m+1 follows
    x' = x (3.8 - 3.8 x - beta * y) with y = series 2m and beta ~ U[0.02, 0.1].
    x0 ~ U[0.1, 0.9].  Returns (X float32 [2*n_pairs][L], beta [n_pairs]).
    """
    rng = np.random.default_rng(seed)
    N = 2 * n_pairs
    x0 = rng.uniform(0.1, 0.9, size=N)
    beta = rng.uniform(0.02, 0.1, size=n_pairs)
    X = np.empty((N, L), dtype=np.float64)
    X[:, 0] = x0
    for t in range(L - 1):
        drv = X[0::2, t]
        rsp = X[1::2, t]
        X[0::2, t + 1] = drv * (3.8 - 3.8 * drv)
        X[1::2, t + 1] = rsp * (3.8 - 3.8 * rsp - beta * drv)
    return _finite(X.astype(np.float32)), beta


def logistic_network(seed: int = 2, N: int = 1024, L: int = 5000,
                     n_drivers: int = 3, beta_max: float = 0.1,
                     noise: float = 0.01):
    """Sparse random network of coupled logistic maps plus observation noise.

    Each series i is driven by ``n_drivers`` distinct others j != i:
    x_i' = x_i (3.8 - 3.8 x_i - mean_j(beta_ij x_j)), beta_ij ~ U[0, beta_max].
    The mean (not the sum) keeps every x in (0, 0.95].  After integration
    N(0, noise^2) is added.  Returns (X float32 [N][L], drivers int [N][n_drivers],
    beta [N][n_drivers]).
    """
    rng = np.random.default_rng(seed)
    drivers = np.empty((N, n_drivers), dtype=np.int64)
    for i in range(N):
        others = rng.choice(N - 1, size=n_drivers, replace=False)
        drivers[i] = others + (others >= i)  # skip i itself
    beta = rng.uniform(0.0, beta_max, size=(N, n_drivers))
    x = rng.uniform(0.1, 0.9, size=N)
    X = np.empty((N, L), dtype=np.float64)
    for t in range(L):
        X[:, t] = x
        drive = (beta * x[drivers]).mean(axis=1)
        x = x * (3.8 - 3.8 * x - drive)
    X += rng.normal(0.0, noise, size=X.shape)
    return _finite(X.astype(np.float32)), drivers, beta


def _ar1_spikes(rng, lam, L, decay=0.9):
    """c_t = decay c_{t-1} + s_t, s_t ~ Poisson(lam_t), c_{-1} = 0."""
    s = rng.poisson(lam, size=L).astype(np.float64)
    return lfilter([1.0], [1.0, -decay], s)


def spike_trains(seed: int = 3, N: int = 4096, L_min: int = 1000,
                 L_max: int = 20000, fs: float = 2.0, E_max: int = 20):
    """AR(1)-filtered Poisson spike trains of uneven length, z-scored.

    rate_i ~ U[0.5, 5] Hz sampled at ``fs`` Hz (lambda_i = rate_i / fs per
    sample), decay 0.9, L_i ~ U{L_min..L_max}, E_i ~ U{1..E_max}.
    Returns (X float32 [N][max L] zero-padded, lengths int64 [N], E int32 [N]).
    """
    rng = np.random.default_rng(seed)
    lengths = rng.integers(L_min, L_max + 1, size=N).astype(np.int64)
    rates = rng.uniform(0.5, 5.0, size=N)
    E = rng.integers(1, E_max + 1, size=N).astype(np.int32)
    ld = int(lengths.max())
    X = np.zeros((N, ld), dtype=np.float32)
    for i in range(N):
        c = _ar1_spikes(rng, rates[i] / fs, int(lengths[i]))
        X[i, : lengths[i]] = zscore(c).astype(np.float32)
    return _finite(X), lengths, E


def calcium_like(seed: int = 4, N: int = 10000, L: int = 2000,
                 n_latent: int = 20, per_latent: int = 100, fs: float = 2.0):
    """Calcium-like spike-derived series, a fraction driven by latent maps.

    rate_i ~ U[0.5, 5] Hz at ``fs`` Hz.  ``n_latent`` logistic drivers
    (r = 3.8) each modulate ``per_latent`` series through
    lambda_t = lambda_i (0.5 + D_t).  Returns (X float32 [N][L] z-scored,
    group int [N] with -1 for undriven series).
    """
    rng = np.random.default_rng(seed)
    D = np.empty((n_latent, L), dtype=np.float64)
    d = rng.uniform(0.1, 0.9, size=n_latent)
    for t in range(L):
        D[:, t] = d
        d = 3.8 * d * (1.0 - d)
    group = np.full(N, -1, dtype=np.int64)
    driven = rng.choice(N, size=min(N, n_latent * per_latent), replace=False)
    group[driven] = np.arange(driven.size) % n_latent
    rates = rng.uniform(0.5, 5.0, size=N)
    X = np.empty((N, L), dtype=np.float32)
    for i in range(N):
        lam = np.full(L, rates[i] / fs)
        if group[i] >= 0:
            lam = lam * (0.5 + D[group[i]])
        X[i] = zscore(_ar1_spikes(rng, lam, L)).astype(np.float32)
    return _finite(X), group


def _logistic_batch(rng, M, L, burn=100):
    r = rng.uniform(3.6, 3.99, size=M)
    x = rng.uniform(0.1, 0.9, size=M)
    out = np.empty((M, L))
    for t in range(burn + L):
        if t >= burn:
            out[:, t - burn] = x
        x = r * x * (1.0 - x)
    return out


def _lorenz_x_batch(rng, M, L, dt=0.01, burn=1000):
    """Euler-integrated Lorenz (10, 28, 8/3); x sampled every ``stride`` steps."""
    stride = rng.integers(1, 11, size=M)
    s, rho, b = 10.0, 28.0, 8.0 / 3.0
    x = rng.normal(0.0, 1.0, size=M) + 1.0
    y = rng.normal(0.0, 1.0, size=M) + 1.0
    z = rng.normal(0.0, 1.0, size=M) + 20.0
    out = np.empty((M, L))
    rows = np.arange(M)
    for t in range(burn + L * int(stride.max())):
        k = t - burn
        if k >= 0:
            take = (k % stride == 0) & (k // stride < L)
            out[rows[take], (k // stride)[take]] = x[take]
        x, y, z = (x + dt * s * (y - x),
                   y + dt * (x * (rho - z) - y),
                   z + dt * (x * y - b * z))
    return out


def _ar2_batch(rng, M, L, burn=200):
    """AR(2) with phi drawn uniformly inside the stationarity triangle."""
    out = np.empty((M, L))
    for i in range(M):
        while True:
            p1 = rng.uniform(-2.0, 2.0)
            p2 = rng.uniform(-1.0, 1.0)
            if p2 + p1 < 0.98 and p2 - p1 < 0.98 and abs(p2) < 0.98:
                break
        e = rng.normal(0.0, 1.0, size=burn + L)
        out[i] = lfilter([1.0], [1.0, -p1, -p2], e)[burn:]
    return out


def surrogate_mix(seed: int = 5, N: int = 50000, L: int = 1500):
    """Logistic, Lorenz-x and AR(2) series in equal thirds, z-scored.

    Returns (X float32 [N][L], family int [N]: 0 logistic, 1 Lorenz, 2 AR(2)).
    """
    rng = np.random.default_rng(seed)
    fam = np.arange(N) % 3
    rng.shuffle(fam)
    X = np.empty((N, L), dtype=np.float32)
    for f, gen in ((0, _logistic_batch), (1, _lorenz_x_batch), (2, _ar2_batch)):
        sel = np.nonzero(fam == f)[0]
        if sel.size:
            X[sel] = zscore(gen(rng, sel.size, L)).astype(np.float32)
    return _finite(X), fam


def net_init_params(C: int, seed: int = 0, kw: int = 7, n_class: int = 20) -> np.ndarray:
    """Random initial parameters of the E surrogate network, flat float32.

    Layout w1[C][1][kw], b1[C], w2[C][C][kw], b2[C], w3[C][C][kw], b3[C],
    wo[n_class][C], bo[n_class]; weights ~ U(-sqrt(6/fan_in), +sqrt(6/fan_in)),
    biases zero.
    """
    rng = np.random.default_rng(seed)
    shapes = [(C, 1, kw), (C,), (C, C, kw), (C,), (C, C, kw), (C,), (n_class, C), (n_class,)]
    parts = []
    for shp in shapes:
        if len(shp) == 1:
            parts.append(np.zeros(shp))
        else:
            lim = np.sqrt(6.0 / int(np.prod(shp[1:])))
            parts.append(rng.uniform(-lim, lim, size=shp))
    return np.concatenate([q.ravel() for q in parts]).astype(np.float32)


def library_subsets(seed: int, m: int, sizes, n_samples: int) -> list:
    """Random library subsamples for a convergence run: for every size l in
    ``sizes``, ``n_samples`` sets of l distinct indices drawn uniformly from
    [0, m) without replacement, each sorted ascending.  Returns a list over
    sizes of int32 arrays [n_samples][l]."""
    rng = np.random.default_rng(seed)
    out = []
    for l in sizes:
        a = np.empty((n_samples, int(l)), dtype=np.int32)
        for s in range(n_samples):
            a[s] = np.sort(rng.choice(m, size=int(l), replace=False))
        out.append(a)
    return out


# --- closed-form fixtures used by the pins -------------------------------

def ramp(L: int) -> np.ndarray:
    """X[t] = t as float32 (exact for t < 2**24)."""
    return np.arange(L, dtype=np.float32)


def sine(L: int, period: float = 37.3, phase: float = 0.0) -> np.ndarray:
    t = np.arange(L, dtype=np.float64)
    return _finite(np.sin(2.0 * np.pi * t / period + phase).astype(np.float32))


def tiled_period(L: int, P: int, seed: int = 0) -> np.ndarray:
    """X[t] = base[t mod P] with base ~ U[0, 1) (float32)."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(0.0, 1.0, size=P).astype(np.float32)
    return base[np.arange(L) % P]
