"""Pins of the oracle's surrogate network and L-BFGS (no GPU).

Each check compares against something the oracle does not compute itself:
closed forms (GELU values, the first Adam step), central finite differences
of the loss, statistics of the uniform initialisation, and the known minima of
a quadratic and of the Rosenbrock function.
"""
import math

import numpy as np

from oracle import lbfgs, mlp


def test_gelu_closed_forms():
    # gelu(1) = Phi(1), the standard normal distribution function at 1
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([10.0]))[0] - 10.0) < 1e-15
    assert abs(mlp.gelu(np.array([-10.0]))[0]) < 1e-20
    # derivative against central differences
    z = np.linspace(-3, 3, 13)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(z))) < 1e-9


def test_loss_gradient_against_central_differences():
    n_in, width = 7, 5
    theta = mlp.init_params(n_in, width, seed=3).astype(np.float64)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((6, n_in))
    t = rng.standard_normal(6)
    loss, g = mlp.loss_grad(theta, X, t, n_in, width)
    h = 1e-6
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd = (mlp.loss_grad(theta + e, X, t, n_in, width)[0] - mlp.loss_grad(theta - e, X, t, n_in, width)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-8 * max(1.0, abs(g[i])), i


def test_initialisation_statistics():
    n_in, width = 400, 64
    theta = mlp.init_params(n_in, width, seed=11)
    assert theta.size == mlp.param_count(n_in, width) == width * n_in + width + width * width + width + width + 1
    W1 = theta[: width * n_in].astype(np.float64)
    bound = 1 / math.sqrt(n_in)
    assert np.all(np.abs(W1) <= bound)
    # uniform on [-b, b]: mean 0, variance b^2/3 (25600 draws: 5 sigma bands)
    n = W1.size
    assert abs(W1.mean()) < 5 * bound / math.sqrt(3 * n)
    assert abs(W1.var() / (bound * bound / 3) - 1) < 5 * math.sqrt(0.8 / n)
    # different seeds give different draws, the same seed the same ones
    assert np.array_equal(theta, mlp.init_params(n_in, width, seed=11))
    assert not np.array_equal(theta, mlp.init_params(n_in, width, seed=12))


def test_first_adam_step_is_a_signed_step():
    g = np.array([3.0, -0.5, 1e-3])
    theta, _, _ = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01, eps=0.0)
    assert np.allclose(theta, -0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_training_fits_a_linear_target():
    n_in, width = 5, 16
    rng = np.random.default_rng(1)
    X = rng.standard_normal((40, n_in))
    t = X @ rng.standard_normal(n_in) + 3.0
    theta, stats, losses = mlp.train(mlp.init_params(n_in, width, 2), X, t, n_in, width, 300, 1e-2)
    assert losses[-1] < 0.05 * losses[0]
    pred = mlp.predict(theta, X, n_in, width, stats)
    assert np.sqrt(np.mean((pred - t) ** 2)) < 0.3 * np.std(t)


def _quadratic(n, seed):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.standard_normal(n)
    return A, b, (lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b))


def _rosenbrock(x):
    f = np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)
    g = np.zeros_like(x)
    g[:-1] = -400.0 * x[:-1] * (x[1:] - x[:-1] ** 2) - 2.0 * (1 - x[:-1])
    g[1:] += 200.0 * (x[1:] - x[:-1] ** 2)
    return f, g


def test_lbfgs_quadratic_exact_minimiser():
    A, b, fg = _quadratic(20, 0)
    p = lbfgs.Params(max_iter=200, gtol=1e-10)
    res = lbfgs.minimize(fg, np.zeros(20), p)
    assert np.max(np.abs(res.x - np.linalg.solve(A, b))) < 1e-9


def test_lbfgs_rosenbrock():
    p = lbfgs.Params(max_iter=500, gtol=1e-8)
    res = lbfgs.minimize(_rosenbrock, np.array([-1.2, 1.0, -1.2, 1.0]), p)
    assert np.max(np.abs(res.x - 1.0)) < 1e-6
    # the energies of the accepted iterates never increase (Armijo)
    fs = [r[3] for r in res.records]
    assert all(b <= a + 1e-12 for a, b in zip(fs, fs[1:]))


def test_cubic_step_is_the_minimiser_of_a_cubic():
    # f(a) = (a - 0.3)^2 (a + 2): local minimum at a = 0.3
    f = lambda a: (a - 0.3) ** 2 * (a + 2)
    df = lambda a: 2 * (a - 0.3) * (a + 2) + (a - 0.3) ** 2
    a = lbfgs.cubic_step(0.0, f(0.0), df(0.0), 1.0, f(1.0), df(1.0))
    assert abs(a - 0.3) < 1e-12


def test_screening_with_exact_and_adversarial_predictors():
    """With the true function as predictor the screened search converges with
    fewer evaluations than the plain one; with its negative (an adversarial
    predictor) it still converges, through the plain fallback."""
    x0 = np.array([-1.2, 1.0, -1.2, 1.0])
    base = lbfgs.Params(max_iter=500, gtol=1e-8)
    plain = lbfgs.minimize(_rosenbrock, x0, base)
    feats = lambda x: x.copy()
    for sign in (1.0, -1.0):
        p = lbfgs.Params(max_iter=500, gtol=1e-8, sur_start=5, refit_every=10)
        res = lbfgs.minimize(_rosenbrock, x0, p, predictor=lambda X: [sign * _rosenbrock(x)[0] for x in X],
                             train=lambda dx, df: None, features=feats)
        assert np.max(np.abs(res.x - 1.0)) < 1e-6
        if sign > 0:
            assert any(r[2] for r in res.records)
            assert res.evals < plain.evals


def _kinked(x):
    """|x0 - 1| + 2 |x1 + 0.5| + 0.1 |x|^2: minimum 0.125 at (1, -0.5), where
    the gradient (sign(0) = 0) cannot meet the curvature test."""
    f = abs(x[0] - 1.0) + 2.0 * abs(x[1] + 0.5) + 0.1 * float(x @ x)
    g = np.array([np.sign(x[0] - 1.0), 2.0 * np.sign(x[1] + 0.5)]) + 0.2 * x
    return f, g


def test_lbfgs_kink_armijo_fallback():
    """f = |x - 1| has |f'| = 1 > c2 |f'(x0)| everywhere but at the kink, so no
    trial point meets the strong Wolfe conditions: the search takes its lowest
    Armijo point, which the cubic steps drive to the kink."""
    fg = lambda x: (abs(x[0] - 1.0), np.array([np.sign(x[0] - 1.0)]))
    res = lbfgs.minimize(fg, np.array([0.3]), lbfgs.Params(max_iter=5, gtol=1e-8))
    assert res.records and res.records[0][3] < 1e-9
    assert abs(res.x[0] - 1.0) < 1e-9


def test_lbfgs_kinked_minimum_with_history_reset():
    """On the two-kink function the run reaches the closed-form minimum 0.125
    at (1, -0.5) with f strictly decreasing, drops its history at least once
    (a failed search along the quasi-Newton direction) and ends when the search
    along -g fails at the minimum."""
    res = lbfgs.minimize(_kinked, np.array([0.3, 0.2]), lbfgs.Params(max_iter=100, gtol=1e-8))
    fs = [r[3] for r in res.records]
    assert all(b < a for a, b in zip(fs, fs[1:]))
    assert abs(res.f - 0.125) < 1e-12 and np.max(np.abs(res.x - [1.0, -0.5])) < 1e-9
    assert res.resets >= 1 and len(res.records) < 100
