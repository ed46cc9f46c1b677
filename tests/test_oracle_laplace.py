"""Pins for oracle/laplace.py (Gauss-Newton MAP and reduced Laplace samples).

* Linear surrogate: the posterior is Gaussian, J is quadratic and the Gauss-Newton
  Hessian is exact, so one full step lands on the closed-form posterior mean
  (I + A^T G^-1 A)^-1 A^T G^-1 (y - b) and the Laplace covariance is the closed-form
  posterior covariance.
* Nonlinear r = 1, 2: the MAP equals the maximiser of the log posterior found by brute
  force on a grid, and the gradient of J vanishes there.
* Planted mistake: with the printed (opposite) ppg sign the iteration misses the
  closed-form mean.
"""
import numpy as np
import pytest

from oracle import laplace, mcmc, network
from tests.test_oracle_mcmc import linear_problem, nonlinear_problem


def closed_form(prob, A, b):
    Gi = np.diag(1.0 / prob.noise_var)
    Sigma = np.linalg.inv(np.eye(A.shape[1]) + A.T @ Gi @ A)
    return Sigma @ A.T @ Gi @ (prob.y - b), Sigma


def test_linear_map_is_posterior_mean_in_one_step():
    prob, A, b = linear_problem(r=3, d_y=4)
    mu, Sigma = closed_form(prob, A, b)
    res = laplace.gauss_newton_map(prob, np.array([3.0, -2.0, 0.5]))
    assert res.converged and res.iters == 1
    np.testing.assert_allclose(res.x, mu, rtol=1e-12, atol=1e-12)


def test_linear_laplace_covariance_is_posterior_covariance():
    prob, A, b = linear_problem(r=3, d_y=4)
    mu, Sigma = closed_form(prob, A, b)
    S = laplace.laplace_samples(prob, mu, np.eye(3))   # rows: mu + L^-T e_c
    N = S - mu[None, :]
    np.testing.assert_allclose(N.T @ N, Sigma, rtol=1e-12, atol=1e-14)
    xi = np.random.default_rng(0).standard_normal((20000, 3))
    X = laplace.laplace_samples(prob, mu, xi)
    assert np.all(np.abs(np.cov(X.T) - Sigma) < 0.05 * np.sqrt(np.outer(np.diag(Sigma), np.diag(Sigma))))


def log_post(prob, pts):
    f, _ = network.forward(prob.layers, pts)
    phi = 0.5 * np.sum((prob.y - f[:, : prob.d_y]) ** 2 / prob.noise_var, axis=1)
    return -phi - 0.5 * np.sum(pts * pts, axis=1)


@pytest.mark.parametrize("r", [1, 2])
def test_nonlinear_map_matches_brute_force(r):
    prob = nonlinear_problem(r=r, d_out=2, dt=1.0, noise=0.5, seed=5)
    if r == 1:
        grid = np.linspace(-6, 6, 120001)[:, None]
        h = grid[1, 0] - grid[0, 0]
    else:
        g1 = np.linspace(-6, 6, 1201)
        X, Y = np.meshgrid(g1, g1, indexing="ij")
        grid = np.stack([X.ravel(), Y.ravel()], axis=1)
        h = g1[1] - g1[0]
    lp = log_post(prob, grid)
    best = grid[np.argmax(lp)]
    res = laplace.gauss_newton_map(prob, best + 0.3, iters=200)
    assert res.converged
    assert np.all(np.abs(res.x - best) <= 1.5 * h)
    c = mcmc.geometry(prob, res.x[None])
    assert np.linalg.norm(res.x + c.g[0]) < 1e-6   # J is flat to rounding within ~sqrt(eps)
    assert -res.J >= lp.max() - 1e-9


def test_printed_ppg_sign_misses_linear_mean(monkeypatch):
    prob, A, b = linear_problem(r=3, d_y=4)
    mu, _ = closed_form(prob, A, b)
    geometry = mcmc.geometry

    def flipped(p, x):
        c = geometry(p, x)
        c.g = -c.g
        return c

    monkeypatch.setattr(mcmc, "geometry", flipped)
    res = laplace.gauss_newton_map(prob, np.zeros(3), iters=5)
    assert np.linalg.norm(res.x - mu) > 1e-3 * (1 + np.linalg.norm(mu))
