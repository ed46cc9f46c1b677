"""Chain diagnostics and posterior estimators (oracle; test infrastructure).

Paper basis: Sec. 6.2 (Markov chain diagnostics):
* eq. covariance_estimator: within-chain covariance W_s and the pooled V_s;
* Wasserstein MPSRF (Sec. 6.2.1): Tr(W + V - 2 (W^1/2 V W^1/2)^1/2);
* ESS% (Sec. 6.2.2, eq. ess), multichain, one value per degree of freedom.

Reading of the garbled eq. ess (the printed sum runs over "MAC", the definition
names "MACT", and AC is called an autocorrelation):
    rho_t = 1 - (w - (1/n_c) sum_k AC(t, k)) / v,
with AC(t, k) the biased (divide by n) autocovariance of chain k at lag t, w the
mean within-chain variance and v the 1-D pooled variance of eq. covariance_estimator;
    ESS% = 1 / (1 + 2 sum_{t=1}^{2n'+1} rho_t),
where n' is the largest index such that every pair sum rho_{2t'} + rho_{2t'+1},
t' = 0..n', is positive (rho_0 = 1).

Posterior moments (the Gaussian lemma of Sec. 5.3: the complement is prior distributed and independent
of the reduced part under the surrogate posterior): field mean Psi_r xbar and field
variance diag(Psi_r S Psi_r^T) + var_perp, with xbar, S the pooled sample mean and
covariance of the reduced coordinates.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def within_between(samples: np.ndarray):
    """1-D w and v of eq. covariance_estimator for samples (n_c, n)."""
    n_c, n = samples.shape
    means = samples.mean(axis=1)
    w = np.sum((samples - means[:, None]) ** 2) / (n_c * (n - 1))
    v = (n - 1) / n * w
    if n_c > 1:
        v += (n_c + 1) / (n_c * (n_c - 1)) * np.sum((means - means.mean()) ** 2)
    return w, v


def autocovariance(chain: np.ndarray, t: int) -> float:
    """Biased lag-t autocovariance (divide by n) of one chain."""
    n = len(chain)
    c = chain - chain.mean()
    return float(np.dot(c[: n - t], c[t:]) / n)


def ess_fraction(samples: np.ndarray) -> float:
    """ESS% / 100 of one degree of freedom from samples (n_c, n) (eq. ess reading)."""
    n_c, n = samples.shape
    w, v = within_between(samples)
    if v <= 0.0:
        return float("nan")

    def rho(t):
        ac = np.mean([autocovariance(samples[k], t) for k in range(n_c)])
        return 1.0 - (w - ac) / v

    total = 0.0
    tp = 0
    while 2 * tp + 1 < n:
        r_even = 1.0 if tp == 0 else rho(2 * tp)
        r_odd = rho(2 * tp + 1)
        if r_even + r_odd <= 0.0:
            break
        total += (r_even if tp > 0 else 0.0) + r_odd
        tp += 1
    return 1.0 / (1.0 + 2.0 * total)


def ess_per_coordinate(trace: np.ndarray) -> np.ndarray:
    """ESS fraction for each coordinate of a trace (n, n_c, dim)."""
    n, n_c, dim = trace.shape
    return np.array([ess_fraction(trace[:, :, j].T) for j in range(dim)])


def wasserstein_mpsrf(trace: np.ndarray) -> float:
    """Wasserstein MPSRF (Sec. 6.2.1) of a trace (n, n_c, dim) in its own coordinates."""
    n, n_c, dim = trace.shape
    X = np.transpose(trace, (1, 0, 2))  # (n_c, n, dim)
    means = X.mean(axis=1)
    Wm = np.zeros((dim, dim))
    for k in range(n_c):
        D = X[k] - means[k]
        Wm += D.T @ D
    Wm /= n_c * (n - 1)
    Dm = means - means.mean(axis=0)
    Vm = (n - 1) / n * Wm + (n_c + 1) / (n_c * (n_c - 1)) * (Dm.T @ Dm)
    Ws = sla.sqrtm(Wm)
    cross = sla.sqrtm(Ws @ Vm @ Ws)
    return float(np.real(np.trace(Wm + Vm - 2.0 * cross)))


def posterior_moments(trace: np.ndarray, basis, burn_in_frac: float = 0.2):
    """Rao-Blackwellised field mean and variance from a reduced trace (n, n_c, r)."""
    n = trace.shape[0]
    b = int(np.floor(burn_in_frac * n))
    X = trace[b:].reshape(-1, trace.shape[2])
    xbar = X.mean(axis=0)
    S = np.cov(X.T, bias=True)
    mean = basis.dec @ xbar
    var = np.einsum("pj,jk,pk->p", basis.dec, S, basis.dec) + basis.var_perp
    return mean, var, xbar, S
