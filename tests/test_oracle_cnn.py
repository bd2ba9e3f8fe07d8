"""Pins of the oracle's CNN (CPU only): convolution semantics by hand, gradients by central finite
differences, Adam against its published update rule written out for one scalar."""
import numpy as np

from oracle import cnn

SMALL = (3, 4, 4, 4, 1)


def test_parameter_count_of_the_network():
    assert cnn.n_params() == 19681
    assert cnn.n_params(SMALL) == 3 * 4 * 9 + 4 + 2 * (4 * 4 * 9 + 4) + 4 * 9 + 1


def test_conv_is_zero_padded_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(1, 1, 4, 5))
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 1, 1] = 1.0
    assert np.allclose(cnn.conv2d(x, W, np.zeros(1)), x)
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 2, 0] = 1.0                    # offset (v, u) = (+1, -1): picks x[y+1, x-1]
    out = cnn.conv2d(x, W, np.array([0.5]))
    assert out[0, 0, 1, 2] == x[0, 0, 2, 1] + 0.5
    assert out[0, 0, 3, 2] == 0.5          # y + 1 outside: zero padding
    assert out[0, 0, 1, 0] == 0.5          # x - 1 outside


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    theta = cnn.init_params(3, SMALL)
    theta[cnn.n_params(SMALL) - 1] = 0.1
    x = rng.normal(size=(2, 3, 5, 6))
    t = rng.normal(size=(2, 1, 5, 6))
    loss, g = cnn.loss_and_grad(theta, x, t, SMALL)
    assert np.isclose(loss, cnn.mse(cnn.forward(theta, x, SMALL)[0], t))
    h = 1e-6
    idx = rng.choice(theta.size, size=60, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (cnn.mse(cnn.forward(tp, x, SMALL)[0], t) - cnn.mse(cnn.forward(tm, x, SMALL)[0], t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_update_rule():
    theta, m, v = np.array([1.0]), np.array([0.0]), np.array([0.0])
    g = np.array([0.5])
    th1, m1, v1 = cnn.adam_step(theta, m, v, g, 1, 0.1)
    # first step: mhat = g, vhat = g^2, so the step is lr * g / (|g| + eps) = lr (up to eps)
    assert np.isclose(th1[0], 1.0 - 0.1 * 0.5 / (0.5 + 1e-8))
    assert np.isclose(m1[0], 0.05) and np.isclose(v1[0], 0.001 * 0.25)
