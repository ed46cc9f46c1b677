"""Pins for the observation-space (dual) proposal noise of oracle/mcmc.py.

* The noise map (xi_1, xi_2) -> (I + H)^-1 (xi_1 + B^T xi_2) has covariance exactly
  (I + H)^-1, the law of the primal L^-T xi: checked as A A^T on the identity inputs.
* Linear surrogate: the dual chain is still the pCN of the Gaussian posterior
  (log rho == 0) and reproduces the closed-form posterior within MCSE.
* Zero likelihood: B = 0, the noise reduces to xi_1 (pCN, log rho == 0).
"""
import numpy as np

from oracle import mcmc
from tests.test_oracle_mcmc import linear_problem, nonlinear_problem


def test_dual_noise_covariance_is_exact():
    prob = nonlinear_problem(r=4, d_out=3, dt=0.7)
    prob.factor = "dual"
    r, dy = 4, prob.d_y
    n = r + dy
    x = np.tile(np.random.default_rng(1).standard_normal(r), (n, 1))
    cache = mcmc.geometry(prob, x)
    # x fixed: subtract the mean by proposing with zero noise
    mean = mcmc.propose(prob, x, cache, np.zeros((n, n)))
    A = (mcmc.propose(prob, x, cache, np.eye(n)) - mean).T / prob.beta   # r x (r + d_y)
    K = np.linalg.inv(np.eye(r) + cache.H[0])
    np.testing.assert_allclose(A @ A.T, K, rtol=1e-11, atol=1e-13)
    # the primal map gives the same covariance
    prob.factor = "primal"
    Ap = (mcmc.propose(prob, x[:r], mcmc.geometry(prob, x[:r]), np.eye(r)) - mean[:r]).T / prob.beta
    np.testing.assert_allclose(Ap @ Ap.T, K, rtol=1e-11, atol=1e-13)


def test_dual_linear_chain_matches_closed_form_posterior():
    prob, A, b = linear_problem(dt=0.5)
    prob.factor = "dual"
    C, N = 16, 3000
    x0 = np.random.default_rng(11).standard_normal((C, 3))
    st = mcmc.init_state(prob, x0)
    xs, _ = mcmc.run(prob, st, N)
    assert np.all(st.accepts == N)           # log rho == 0: every proposal accepted
    Gi = np.diag(1 / prob.noise_var)
    Sigma = np.linalg.inv(np.eye(3) + A.T @ Gi @ A)
    mu = Sigma @ A.T @ Gi @ (prob.y - b)
    X = xs[N // 5:].reshape(-1, 3)
    n_eff = X.shape[0] * (1 - prob.s) / (1 + prob.s)
    mcse = np.sqrt(np.diag(Sigma) / n_eff)
    assert np.all(np.abs(X.mean(0) - mu) < 4.5 * mcse)
    S = np.cov(X.T)
    assert np.all(np.abs(np.diag(S) - np.diag(Sigma)) < 5 * np.sqrt(2 / n_eff) * np.diag(Sigma))


def test_dual_zero_likelihood_is_pcn():
    prob = nonlinear_problem(dt=0.8)
    prob.factor = "dual"
    prob.noise_var = np.full(prob.d_y, np.inf)
    st = mcmc.init_state(prob, np.random.default_rng(2).standard_normal((6, 4)))
    rec = mcmc.transition(prob, st)
    np.testing.assert_allclose(rec.log_rho, 0.0, atol=1e-12)
