"""Pins of the warm-start network oracle against calculus and definitions
(not against itself): finite differences, a shift identity, exactness on
quadratic sequences, bfloat16 rounding cases, Adam's first step."""
import math

import numpy as np
import pytest

import oracle.warmnet_oracle as N


def _rand_theta(rng, scale=0.3):
    return rng.normal(0.0, scale, N.param_count())


def test_param_count():
    assert N.param_count() == 7 * 32 * 5 + 32 + 2 * (32 * 32 * 5 + 32) + 32 * 5 + 1 == 11617


def test_backward_matches_central_differences():
    rng = np.random.default_rng(1)
    theta = _rand_theta(rng, 0.2)
    n = 11
    X = rng.normal(size=(N.CIN, n))
    t = rng.normal(size=n)

    exact = lambda a: a  # noqa: E731  (the chain rule, without the piecewise-constant rounding)

    def f(th):
        y, _ = N.forward(th, X, exact)
        return N.loss(y, X[1], t)

    y, acts = N.forward(theta, X, exact)
    g = N.backward(theta, acts, N.loss_dy(y, X[1], t), exact)
    idx = rng.choice(theta.size, 60, replace=False)
    # every layer's weights and biases among the probes
    offs = np.cumsum([0] + [co * ci * N.KS + co for ci, co in N.LAYERS])
    idx = np.concatenate([idx, offs[1:] - 1, offs[:-1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_one_tap_kernel_is_a_shift():
    rng = np.random.default_rng(2)
    a = rng.normal(size=(3, 9))
    for k in range(N.KS):
        W = np.zeros((1, 3, N.KS))
        W[0, 1, k] = 1.0
        out = N.conv(a, W, np.zeros(1))[0]
        shift = k - N.HALF
        ref = np.zeros(9)
        for p in range(9):
            q = p + shift
            if 0 <= q < 9:
                ref[p] = a[1, q]
        assert np.array_equal(out, ref), k


def test_quadratic_sequences_are_extrapolated_exactly():
    """u^j = a + b t_j + c t_j^2: the base prediction is u^{j+1} and the
    target vanishes; with zero parameters the prediction is the base."""
    rng = np.random.default_rng(3)
    n = 17
    a, b, c = rng.normal(size=(3, n))
    tau = 0.125
    U = [a + b * (k * tau) + c * (k * tau) ** 2 for k in range(4)]
    X, base, s = N.inputs(U[2], U[1], U[0], np.zeros(5))
    assert np.allclose(base, U[3], rtol=0, atol=1e-14)
    assert np.allclose(N.target(U[3], base, s), 0.0, atol=1e-12)
    # e2 = 2 c tau^2 exactly, so channel 1 has unit RMS
    assert math.isclose(float(np.sqrt(np.mean(X[1] ** 2))), 1.0, rel_tol=1e-12)
    zero = np.zeros(N.param_count())
    assert np.array_equal(N.predict(zero, U[2], U[1], U[0], np.zeros(5)), base)


def test_constant_history_has_unit_scale():
    u = np.linspace(0.0, 1.0, 8)
    X, base, s = N.inputs(u, u, u, np.zeros(5))
    assert s == 1.0 and np.array_equal(base, u) and not X[:2].any()


@pytest.mark.parametrize("x,expected", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                   # tie, rounds to even (last bit 0)
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),   # tie, rounds up to even
    (1.0 + 2.0 ** -8 + 2.0 ** -12, 1.0 + 2.0 ** -7),  # above the tie
    (-3.0, -3.0),
    (0.1, 0.10009765625),                     # 0x3DCD -> 0.10009765625
])
def test_bf16_rounding(x, expected):
    assert N.bf16_round(x) == expected


def test_adam_first_step_is_lr_sign():
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    lr = 1e-3
    new, m, v = N.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, lr, eps=1e-12)
    assert np.allclose(theta - new, lr * np.sign(g), rtol=1e-9, atol=0)


def test_level_features_by_hand():
    class P:  # alpha = 0.5: sigma = 0.75; n = 3 on [0, 1]: h = 0.25
        beta, alpha, a, b, n = 1.5, 0.5, 0.0, 1.0, 3
    f = N.level_features(P, 0, eta_j=2.0, gamma_j=-1.0, dplus_j=1.0, dminus_j=0.5)
    qg = 0.75 * -1.0 / (0.25 * 2.0)
    qp = 0.75 * 1.0 * 0.25 ** -1.5 / 2.0
    assert np.allclose(f, [0.5, 1.5, math.asinh(qg), math.log1p(qp), math.log1p(qp / 2)], rtol=1e-15)


def test_loss_of_zero_correction_is_one_and_derivative_by_differences():
    rng = np.random.default_rng(5)
    n = 9
    x1, t, y = rng.normal(size=(3, n))
    assert math.isclose(N.loss(np.zeros(n), x1, t), 1.0, rel_tol=1e-10)
    d = N.loss_dy(y, x1, t)
    h = 1e-7
    for p in range(n):
        e = np.zeros(n)
        e[p] = h
        fd = (N.loss(y + e, x1, t) - N.loss(y - e, x1, t)) / (2 * h)
        assert abs(fd - d[p]) <= 1e-6 * max(1.0, abs(fd))


def test_correction_vanishes_with_the_second_difference():
    """Where e2 = 0 (u fixed in time, e.g. at a Dirichlet boundary) the
    prediction is the extrapolation, whatever the parameters."""
    rng = np.random.default_rng(6)
    n = 12
    u = rng.normal(size=(3, n))
    u[:, :3] = 1.5  # the first three points constant in time
    theta = rng.normal(0, 0.3, N.param_count())
    x0 = N.predict(theta, u[2], u[1], u[0], rng.normal(size=5))
    base = 3.0 * (u[2] - u[1]) + u[0]
    assert np.array_equal(x0[:3], base[:3])
    assert not np.allclose(x0[3:], base[3:])


def test_rounded_network_is_the_exact_one_on_rounded_inputs():
    """With bfloat16 rounding, each layer computes what the exact network
    computes on that layer's (for the hidden layers, rounded) input, checked
    layer by layer; the output layer's weight gradient uses its input as is."""
    rng = np.random.default_rng(8)
    theta = N.weights_bf16(rng.normal(0, 0.3, N.param_count()))
    X = rng.normal(size=(N.CIN, 13))
    y, acts = N.forward(theta, X)
    layers = N.unpack(theta)
    for li, (W, b) in enumerate(layers):
        z = N.conv(N.bf16_round(acts[li]) if li in N.ROUNDED else acts[li], W, b)
        ref = np.tanh(z) if li < len(layers) - 1 else z
        assert np.array_equal(acts[li + 1], ref)
    dy = rng.normal(size=13)
    g = N.backward(theta, acts, dy)
    W3, _ = layers[3]
    a3 = np.zeros((32, 13 + 4))
    a3[:, 2:15] = acts[3]  # the output layer takes its input unrounded
    dW3 = np.stack([dy @ a3[:, k:k + 13].T for k in range(N.KS)], axis=-1)
    o3 = N.param_count() - (32 * N.KS + 1)
    assert np.allclose(g[o3:o3 + 32 * N.KS].reshape(1, 32, N.KS), dW3[None], rtol=1e-12, atol=0)
