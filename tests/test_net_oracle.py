"""Pins for the surrogate-network oracle: finite differences, a library
convolution, closed forms of the loss and of the first Adam step."""
import math
from fractions import Fraction

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


def _bf16_exact(v: Fraction) -> Fraction:
    """Round an exact rational to the nearest BF16 value (8 significant bits,
    ties to even), written from the definition, without float bit tricks."""
    if v == 0:
        return Fraction(0)
    a = abs(v)
    e = 0
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    ulp = Fraction(2) ** (e - 7)
    n, r = divmod(a, ulp)
    n = int(n)
    if r > ulp / 2 or (r == ulp / 2 and n % 2 == 1):
        n += 1
    return (1 if v > 0 else -1) * n * ulp


# One-channel network whose only non-zero taps are the centre ones, so each
# layer is a scalar affine map per time step: every value below is an exact
# dyadic rational and BF16 rounding is the only rounding anywhere.
_FIX = dict(x=[1 + Fraction(11, 2048), Fraction(-1)],
            c1=Fraction(3, 2), b1=Fraction(0),
            c2=1 - Fraction(11, 1024), b2=Fraction(-40, 4096),
            c3=2 + Fraction(1, 256), b3=Fraction(0),
            wo=[1 + Fraction(1, 512), Fraction(2)], bo=[Fraction(0), Fraction(1, 4)])


def _scalar_net(f, round_l1=False, round_a1=True, round_w2=True, round_a2=True, round_w3=True,
                round_lin=False):
    R = lambda v, on: _bf16_exact(v) if on else v
    relu = lambda v: v if v > 0 else Fraction(0)
    a1 = [relu(R(x, round_l1) * R(f["c1"], round_l1) + f["b1"]) for x in f["x"]]
    a2 = [relu(R(a, round_a1) * R(f["c2"], round_w2) + f["b2"]) for a in a1]
    a3 = [relu(R(a, round_a2) * R(f["c3"], round_w3) + f["b3"]) for a in a2]
    g = R(sum(a3) / len(a3), round_lin)
    out = [R(w, round_lin) * g + b for w, b in zip(f["wo"], f["bo"])]
    return out + [Fraction(0)] * (N.NCLASS - len(out))


def test_bf16_forward_rounding_placement_exact():
    # The BF16 inference form rounds the inputs and weights of the two C -> C
    # convolutions only (they run on the matrix cores); layer 1, the sums,
    # biases, ReLU, pooling and the linear layer stay exact here.  Worked by
    # hand: a1 = 1.5 (1 + 11/2048) = 1.5 + 33/4096 -> bf16 1.5078125;
    # w2 = 1 - 11/1024 -> bf16 253/256; a2 = 193/128 * 253/256 - 40/4096
    # = 48509/32768 -> bf16 1.4765625; w3 = 2 + 1/256 -> bf16 2;
    # a3 = 2.953125 at t = 0 and 0 at t = 1 (ReLU of -1.5, then of -40/4096);
    # g = 1.4765625; logits = (1 + 1/512) g, 2 g + 1/4, then zeros.
    f = _FIX
    want = _scalar_net(f)
    assert want[0] == Fraction(1.4765625) * (1 + Fraction(1, 512))
    assert want[1] == Fraction(3.203125)
    C = 1
    p = {"w1": np.zeros((C, 1, N.KW)), "b1": np.zeros(C), "w2": np.zeros((C, C, N.KW)),
         "b2": np.zeros(C), "w3": np.zeros((C, C, N.KW)), "b3": np.zeros(C),
         "wo": np.zeros((N.NCLASS, C)), "bo": np.zeros(N.NCLASS)}
    h = N.KW // 2
    p["w1"][0, 0, h], p["b1"][0] = float(f["c1"]), float(f["b1"])
    p["w2"][0, 0, h], p["b2"][0] = float(f["c2"]), float(f["b2"])
    p["w3"][0, 0, h], p["b3"][0] = float(f["c3"]), float(f["b3"])
    p["wo"][:2, 0] = [float(v) for v in f["wo"]]
    p["bo"][:2] = [float(v) for v in f["bo"]]
    theta = N.pack(p, C)
    X = np.array([[float(v) for v in f["x"]]])
    got = N.forward_bf16(theta, X, C)[0]
    np.testing.assert_array_equal(got, np.array([float(v) for v in want]))
    # The fixture tells the placements apart: rounding layer 1 as well, or
    # the linear layer, or skipping any of the four roundings, changes a logit.
    for alt in (dict(round_l1=True), dict(round_a1=False), dict(round_w2=False),
                dict(round_a2=False), dict(round_w3=False), dict(round_lin=True)):
        assert _scalar_net(f, **alt) != want, alt
