"""Pins of the surrogate network's FP64 oracle (CPU only).

The oracle's gradient is checked against central finite differences of its
own loss (an independent route: no chain rule), against a one-neuron network
differentiated by hand, and its Adam step against the closed form of the
first step; the BF16 rounding against exact bit patterns.
"""

import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_gradient_matches_finite_differences():
    widths = [3, 5, 4, 2]
    rng = np.random.default_rng(1)
    p = M.init_params(widths, seed=2) + 0.1 * rng.standard_normal(M.n_params(widths))
    X = rng.uniform(-1, 1, (7, 3))
    T = rng.uniform(-1, 1, (7, 2))
    _, g = M.loss_and_grad(p, widths, X, T)
    h = 1e-6
    fd = np.empty_like(p)
    for j in range(p.size):
        e = np.zeros_like(p)
        e[j] = h
        fd[j] = (M.loss_and_grad(p + e, widths, X, T)[0] - M.loss_and_grad(p - e, widths, X, T)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-8 * max(1.0, np.max(np.abs(fd)))


def test_one_neuron_network_by_hand():
    # y = w2 tanh(w1 x + b1) + b2, L = mean (y - t)^2
    w1, b1, w2, b2 = 0.7, -0.2, 1.3, 0.05
    x = np.array([[0.5], [-1.0], [2.0]])
    t = np.array([[0.1], [0.4], [-0.3]])
    p = np.array([w1, b1, w2, b2])
    loss, g = M.loss_and_grad(p, [1, 1, 1], x, t)
    a = np.tanh(w1 * x[:, 0] + b1)
    y = w2 * a + b2
    r = y - t[:, 0]
    n = len(r)
    assert abs(loss - np.mean(r ** 2)) < 1e-15
    dw1 = np.sum(2 * r / n * w2 * (1 - a ** 2) * x[:, 0])
    db1 = np.sum(2 * r / n * w2 * (1 - a ** 2))
    dw2 = np.sum(2 * r / n * a)
    db2 = np.sum(2 * r / n)
    np.testing.assert_allclose(g, [dw1, db1, dw2, db2], rtol=1e-14, atol=1e-16)


def test_zero_network_predicts_zero():
    widths = [5, 8, 8, 3]
    X = np.random.default_rng(3).uniform(-1, 1, (4, 5))
    T = np.random.default_rng(4).uniform(-1, 1, (4, 3))
    loss, g = M.loss_and_grad(np.zeros(M.n_params(widths)), widths, X, T)
    assert abs(loss - np.mean(T ** 2)) < 1e-15
    # only the output bias sees a gradient when every weight is zero
    W, b = M.unpack(g, widths)[-1]
    np.testing.assert_allclose(b, -2 * T.sum(axis=0) / T.size, rtol=1e-14)
    assert np.all(W == 0)


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.5, 1e-3, -2e2])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    p, m, v = M.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p, p0 - 0.01 * np.sign(g), rtol=0, atol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("x,bits", [(1.0, 0x3F80), (-2.0, 0xC000), (1.00390625, 0x3F80),    # tie -> even
                                    (1.01171875, 0x3F82), (3.140625, 0x4049), (1e-40, 0x0001)])
def test_bf16_rounding(x, bits):
    r = M.round_bf16(np.array([x]))[0]
    got = int(np.array([r], dtype=np.float32).view(np.uint32)[0] >> 16)
    assert got == bits, (x, hex(got))
