"""Pins for the surrogate-network oracle: finite differences, a library
convolution, closed forms of the loss and of the first Adam step."""
import math

import numpy as np
import pytest
from scipy.signal import correlate

from oracle import net_oracle as N
from paper_2105_12301_amd import synth


def test_param_count_matches_layout():
    C = 64
    assert N.param_count(C) == 7 * C + C + C * C * 7 + C + C * C * 7 + C + 20 * C + 20
    theta = synth.net_init_params(C, seed=1)
    assert theta.size == N.param_count(C)
    p = N.unpack(theta, C)
    assert p["w2"].shape == (C, C, 7) and np.all(p["b3"] == 0)


def test_conv_same_against_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 20))
    w = rng.normal(size=(4, 3, 7))
    b = rng.normal(size=4)
    y = N.conv_same(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate(x[n, i], w[o, i], mode="same") for i in range(3))
            np.testing.assert_allclose(y[n, o], ref, rtol=1e-12, atol=1e-12)


def test_uniform_logits_loss_is_log20():
    C = 4
    theta = np.zeros(N.param_count(C))
    X = np.random.default_rng(1).normal(size=(5, 30))
    assert abs(N.loss(theta, X, [1, 5, 20, 3, 7], C) - math.log(20.0)) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    C, L, B = 3, 16, 4
    rng = np.random.default_rng(seed)
    theta = synth.net_init_params(C, seed=seed).astype(np.float64)
    theta += rng.normal(scale=0.05, size=theta.size)   # non-zero biases too
    X = rng.normal(size=(B, L))
    y = rng.integers(1, 21, size=B)
    _, g = N.loss_and_grads(theta, X, y, C)
    h = 1e-6
    idx = np.unique(np.r_[np.arange(0, theta.size, 7), theta.size - 1, theta.size - 20])
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (N.loss(tp, X, y, C) - N.loss(tm, X, y, C)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(2)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = N.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3, eps=0.0)
    np.testing.assert_allclose(new, th - 1e-3 * np.sign(g), rtol=0, atol=1e-15)


def test_bf16_round_known_values():
    # BF16 keeps 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7
    # (ties to even -> 1), 1 + 3*2^-9 rounds up, negative values mirror, and
    # a value that is already BF16 is unchanged.
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8,
                  -(1.0 + 3 * 2.0 ** -9), 3.140625, 0.0, 2.0 ** -130])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -6,
                     -(1.0 + 2.0 ** -7), 3.140625, 0.0, 2.0 ** -130])
    np.testing.assert_array_equal(N.bf16_round(x), want)
    r = np.random.default_rng(0).normal(size=1000)
    rel = np.abs(N.bf16_round(r) - r) / np.abs(r)
    assert rel.max() <= 2.0 ** -8


def test_bf16_forward_close_to_float64():
    # The BF16 inference form moves logits only by the rounding of weights
    # and activations (relative 2^-8 each, partly averaging out over time).
    rng = np.random.default_rng(1)
    C, L, B = 8, 64, 4
    theta = rng.normal(scale=0.3, size=N.param_count(C))
    X = rng.normal(size=(B, L))
    ref, _ = N.forward(theta, X, C)
    got = N.forward_bf16(theta, X, C)
    assert np.max(np.abs(got - ref)) <= 0.02 * np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) > 0.0
