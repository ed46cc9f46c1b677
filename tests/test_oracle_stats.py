"""Pins for oracle/stats.py: the ESS% reading of eq. ess on processes with known
ESS (AR(1): (1 - phi)/(1 + phi); i.i.d.: 1), the Wasserstein MPSRF on chains with
equal and shifted laws, and the Rao-Blackwellised field moments against dense
covariance algebra."""
import numpy as np
import pytest

from oracle import prior, stats


def ar1(phi, n, n_c, dim=1, seed=0):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, n_c, dim))
    x[0] = rng.standard_normal((n_c, dim))
    e = rng.standard_normal((n, n_c, dim)) * np.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_ess_of_ar1(phi):
    tr = ar1(phi, 4000, 8, dim=3, seed=int(phi * 10))
    e = stats.ess_per_coordinate(tr)
    ref = (1 - phi) / (1 + phi)
    assert np.all(np.abs(e - ref) < 0.15 * ref + 0.02)


def test_ess_negative_correlation_truncates():
    tr = ar1(-0.5, 4000, 4, seed=3)
    e = stats.ess_per_coordinate(tr)
    assert np.all(e > 1.0)   # antithetic chains beat i.i.d. sampling


def test_within_between_definitions():
    rng = np.random.default_rng(1)
    s = rng.standard_normal((3, 50))
    w, v = stats.within_between(s)
    assert np.isclose(w, np.mean(np.var(s, axis=1, ddof=1)))
    B = 50 * np.var(s.mean(axis=1), ddof=1)
    assert np.isclose(v, 49 / 50 * w + (1 + 1 / 3) * B / 50)


def test_autocovariance_biased():
    c = np.array([1.0, 2.0, 4.0, 3.0])
    m = c.mean()
    ref = ((c[0] - m) * (c[1] - m) + (c[1] - m) * (c[2] - m) + (c[2] - m) * (c[3] - m)) / 4
    assert np.isclose(stats.autocovariance(c, 1), ref)


def test_wasserstein_mpsrf():
    same = ar1(0.3, 3000, 6, dim=3, seed=5)
    shifted = same.copy()
    shifted[:, :3] += 2.0
    a = stats.wasserstein_mpsrf(same)
    b = stats.wasserstein_mpsrf(shifted)
    assert 0 <= a < 0.02 and b > 1.0


def test_posterior_moments_rao_blackwell():
    n, r = 9, 6
    B = prior.KLEBasis(n, 0.1, 1.0, r)
    rng = np.random.default_rng(2)
    A = rng.standard_normal((r, r))
    S = A @ A.T / r
    mu = rng.standard_normal(r)
    tr = (mu + rng.standard_normal((5000, 4, r)) @ np.linalg.cholesky(S).T)
    mean, var, xbar, Shat = stats.posterior_moments(tr, B, burn_in_frac=0.0)
    np.testing.assert_allclose(mean, B.dec @ xbar, rtol=1e-12)
    C = prior.prior_covariance_dense(n, 0.1, 1.0)
    # field covariance = Dec S Dec^T + (C_pr - Dec Dec^T) (complement prior distributed)
    F = B.dec @ Shat @ B.dec.T + C - B.dec @ B.dec.T
    np.testing.assert_allclose(var, np.diag(F), rtol=1e-10, atol=1e-16)
