"""Pins of the FP64 reference of the learned initial guess (O3)."""
import numpy as np

from oracle import mlp_ref


def _theta(seed):
    rng = np.random.default_rng(seed)
    t = rng.normal(size=mlp_ref.NPARAM) * 0.3
    t[-1] = 1.0
    return t


def test_analytic_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    u = rng.uniform(0.2, 1.0, 64)
    for seed in (0, 1):
        th = _theta(seed)
        g = mlp_ref.grad(th, u, 0.6, 0.25)
        fd = mlp_ref.fd_grad(th, u, 0.6, 0.25)
        assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_quartic_collapse_equals_network():
    u = np.linspace(0.05, 1.0, 97)
    for seed in (2, 3):
        th = _theta(seed)
        c = mlp_ref.to_poly(th, 0.5, 0.3)
        y = mlp_ref.forward(th, u, 0.5, 0.3)
        yp = sum(c[k] * u ** k for k in range(5))
        np.testing.assert_allclose(yp, y, rtol=1e-10, atol=1e-10)


def test_single_unit_closed_form():
    """one live unit per layer: y = w3 (w2 (w1 z + b1)^2 + b2)^2 + b3"""
    W1, b1, W2, b2, W3, b3 = 0.7, -0.2, 1.3, 0.4, -0.9, 0.25
    th = np.zeros(mlp_ref.NPARAM)
    H = mlp_ref.H
    th[0], th[H] = W1, b1
    th[2 * H] = W2
    th[2 * H + H * H] = b2
    th[3 * H + H * H] = W3
    th[-1] = b3
    u = np.array([0.1, 0.5, 0.9])
    z = (u - 0.4) / 0.2
    want = W3 * (W2 * (W1 * z + b1) ** 2 + b2) ** 2 + b3
    np.testing.assert_allclose(mlp_ref.forward(th, u, 0.4, 0.2), want, rtol=1e-14)
    # with zero biases and unit weights the collapse is z^4 = ((u - m)/s)^4
    th2 = np.zeros(mlp_ref.NPARAM)
    th2[0], th2[2 * H], th2[3 * H + H * H] = 1.0, 1.0, 1.0
    c = mlp_ref.to_poly(th2, 0.0, 1.0)
    np.testing.assert_allclose(c, [0, 0, 0, 0, 1], atol=1e-15)


def test_loss_of_exact_guess_is_zero():
    """a network whose output is exactly 1/sqrt(u) at the samples has zero loss: one hidden
    path with z = u gives y = W3 u^4 + b3, and W3 = -256/255, b3 = 511/255 make y(1/4) = 2 and
    y(1) = 1"""
    H = mlp_ref.H
    u = np.array([0.25, 1.0])
    th = np.zeros(mlp_ref.NPARAM)
    th[0] = 1.0                       # W1[0]
    th[2 * H] = 1.0                   # W2[0][0]
    th[3 * H + H * H] = -256.0 / 255.0  # W3[0]
    th[-1] = 511.0 / 255.0            # b3
    np.testing.assert_allclose(mlp_ref.forward(th, u, 0.0, 1.0), [2.0, 1.0], rtol=1e-15)
    assert mlp_ref.loss(th, u, 0.0, 1.0) < 1e-30


def test_loss_is_the_mean_squared_relative_error():
    """the constant network y = 1 is exact at u = 1 and off by y sqrt(u) - 1 = -1/2 at u = 1/4:
    the loss is the mean of the squared relative errors, 1/8"""
    u = np.array([0.25, 1.0])
    th = np.zeros(mlp_ref.NPARAM)
    th[-1] = 1.0
    assert abs(mlp_ref.loss(th, u, 0.0, 1.0) - 0.125) < 1e-15
