"""Pins of the oracle's initial-guess network against the mathematics: a
brute-force convolution written with explicit lattice indices, translation
equivariance, central finite differences of the loss, and closed-form Adam
steps."""
import numpy as np
import pytest

from lattice_inputs import cnn_init_params, cnn_param_count
from oracle import cnn


def _brute_conv(inp, W, b, anti):
    nb, cin, Lt, Lx = inp.shape
    cout = W.shape[0]
    out = np.zeros((nb, cout, Lt, Lx))
    for n in range(nb):
        for co in range(cout):
            for t in range(Lt):
                for x in range(Lx):
                    acc = b[co]
                    for dt in range(3):
                        for dx in range(3):
                            tt, xx = t + dt - 1, x + dx - 1
                            sign = 1.0
                            if tt < 0 or tt >= Lt:
                                sign = -1.0 if anti else 1.0
                            tt %= Lt
                            xx %= Lx
                            for ci in range(cin):
                                acc += sign * W[co, ci, dt, dx] * inp[n, ci, tt, xx]
                    out[n, co, t, x] = acc
    return out


@pytest.mark.parametrize("anti", [True, False])
def test_conv_matches_brute_force(anti):
    rng = np.random.default_rng(1)
    inp = rng.standard_normal((2, 3, 4, 5))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    assert np.allclose(cnn.conv(inp, W, b, anti), _brute_conv(inp, W, b, anti), atol=1e-12)


def test_centre_identity_kernel_is_identity():
    rng = np.random.default_rng(2)
    inp = rng.standard_normal((1, 4, 6, 6))
    W = np.zeros((4, 4, 3, 3))
    W[:, :, 1, 1] = np.eye(4)
    b = np.arange(4.0)
    assert np.allclose(cnn.conv(inp, W, b, True), inp + b[None, :, None, None])


def test_channel_round_trip():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, 2 * 8 * 4)) + 1j * rng.standard_normal((3, 2 * 8 * 4))
    ch = cnn.complex_to_channels(v, 8, 4)
    # spin 1 of site (t=2, x=5) is dof (2*8+5)*2+1
    assert ch[1, 2, 2, 5] == v[1, (2 * 8 + 5) * 2 + 1].real
    assert ch[1, 3, 2, 5] == v[1, (2 * 8 + 5) * 2 + 1].imag
    assert np.array_equal(cnn.channels_to_complex(ch), v)


def _anti_translate_t(a):
    """(T a)[t] = a[t-1], with the slice that wraps round picking up a sign."""
    out = np.roll(a, 1, axis=-2)
    out[..., 0, :] *= -1.0
    return out


def test_translation_equivariance():
    rng = np.random.default_rng(4)
    theta = cnn_init_params(7)
    for k, p in enumerate(cnn.unpack(theta)):
        if p.ndim == 1:
            p[:] = rng.standard_normal(p.shape) * 0.1
    x = rng.standard_normal((2, 4, 6, 8))
    y, _ = cnn.forward(theta, x, anti=True)
    # periodic x: shifts commute with the network, biases included
    ys, _ = cnn.forward(theta, np.roll(x, 3, axis=-1), anti=True)
    assert np.allclose(ys, np.roll(y, 3, axis=-1), atol=1e-12)
    # periodic t
    yp, _ = cnn.forward(theta, x, anti=False)
    ysp, _ = cnn.forward(theta, np.roll(x, 2, axis=-2), anti=False)
    assert np.allclose(ysp, np.roll(yp, 2, axis=-2), atol=1e-12)
    # antiperiodic t: the sign-picking translation commutes with the
    # bias-free network (conv is linear and tanh is odd)
    theta0 = theta.copy()
    for p in cnn.unpack(theta0):
        if p.ndim == 1:
            p[:] = 0.0
    y0, _ = cnn.forward(theta0, x, anti=True)
    y0t, _ = cnn.forward(theta0, _anti_translate_t(x), anti=True)
    assert np.allclose(y0t, _anti_translate_t(y0), atol=1e-12)
    # ... and a bias breaks it (the test can fail)
    y1t, _ = cnn.forward(theta, _anti_translate_t(x), anti=True)
    assert not np.allclose(y1t, _anti_translate_t(y), atol=1e-6)


def test_param_count():
    assert cnn.n_params() == cnn_param_count() == 20736 + 100


@pytest.mark.parametrize("anti", [True, False])
def test_gradient_matches_central_differences(anti):
    rng = np.random.default_rng(5)
    widths = (4, 6, 5, 4)
    theta = cnn_init_params(11, widths)
    theta += 0.05 * rng.standard_normal(theta.shape)   # non-zero biases too
    x = rng.standard_normal((2, 4, 4, 6))
    tgt = rng.standard_normal((2, 4, 4, 6))
    loss, g = cnn.loss_and_grad(theta, x, tgt, anti, widths)
    h = 1e-6
    idx = rng.choice(theta.size, 40, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        lp, _ = cnn.loss_and_grad(theta + e, x, tgt, anti, widths)
        lm, _ = cnn.loss_and_grad(theta - e, x, tgt, anti, widths)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    # directional derivative along a random direction of all parameters
    d = rng.standard_normal(theta.shape)
    lp, _ = cnn.loss_and_grad(theta + h * d, x, tgt, anti, widths)
    lm, _ = cnn.loss_and_grad(theta - h * d, x, tgt, anti, widths)
    assert abs((lp - lm) / (2 * h) - g @ d) <= 1e-6 * max(1.0, abs(g @ d))


def test_loss_vanishes_at_target():
    rng = np.random.default_rng(6)
    theta = cnn_init_params(3)
    x = rng.standard_normal((2, 4, 4, 4))
    y, _ = cnn.forward(theta, x)
    loss, g = cnn.loss_and_grad(theta, x, y)
    assert loss == 0.0 and np.all(g == 0.0)


def test_loss_definition_on_zero_network():
    # all-zero parameters give y = 0, so every sample's relative error is 1
    theta = np.zeros(cnn.n_params())
    rng = np.random.default_rng(8)
    loss, _ = cnn.loss_and_grad(theta, rng.standard_normal((3, 4, 4, 4)),
                                rng.standard_normal((3, 4, 4, 4)))
    assert loss == pytest.approx(1.0, abs=1e-15)


def test_adam_constant_gradient_steps():
    # with a constant gradient g the bias-corrected moments are exactly g and
    # g^2, so every step moves each coordinate by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        theta_new, m, v = cnn.adam_step(theta, m, v, g, t, lr, eps=eps)
        step = lr * g / (np.abs(g) + eps)
        assert np.allclose(theta_new - theta, -step, rtol=1e-9, atol=1e-15)
        theta = theta_new


def test_adam_descends_a_quadratic():
    theta = np.array([3.0, -4.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 2001):
        theta, m, v = cnn.adam_step(theta, m, v, 2 * theta, t, 0.05)
    assert np.linalg.norm(theta) < 0.05
