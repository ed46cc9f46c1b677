"""Pins for oracle/da.py (the second stage of Alg. 1; Sec. 2.5 eq. da_second, Sec. 5.4
eq. da_dino_trr_2).

* The second-stage ratio equals the textbook MH ratio of the delayed-acceptance proposal
  Q_DA(m, dm+) = alpha1(m, m+) Q(m, dm+) with respect to the true posterior, built from
  explicit Gaussian densities (scipy) of the full proposal: the reduced mMALA part and
  the pCN complement part, and alpha1 from the surrogate posterior. A planted sign
  error fails it.
* A true model equal to the surrogate gives log rho^(2) == 0, and the DA chain is the
  first-stage chain, draw for draw.
* The DA chain's stationary law is the true posterior: 2-D quadrature for a nonlinear
  true model that reads the first complement coordinate, and the closed-form Gaussian
  posterior for a linear one. The first-stage chain alone misses the quadrature moments
  (so the pin has power).
"""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import da, mcmc, network, stats
from synth import draw_network, workload


def net(r, d_out, seed, width=6, scale=2.0, bias=0.2):
    w = workload("tiny", r=r, width=width, depth=2, d_out=d_out, d_y=d_out, arch="mlp")
    layers = draw_network(w, seed=seed, bias_scale=bias)
    return [(k, scale * W, b) for (k, W, b) in layers]


def restricted(layers, r):
    """The network with inputs beyond the first r fixed at zero (a network on R^r)."""
    k, W, b = layers[0]
    return [(k, W[:, :r].copy(), b)] + list(layers[1:])


def problem(surrogate, d_y, noise, dt, seed):
    y = np.random.default_rng(seed).standard_normal(d_y)
    return mcmc.Problem(surrogate, y, np.full(d_y, noise ** 2), dt, seed=seed, request_id=3)


def textbook_log_da_ratio(prob, tm, x, z, xp, zp):
    """log [pi(m+) alpha1(m+, m) q(m+ -> m)] - log [pi(m) alpha1(m, m+) q(m -> m+)], pi the
    true posterior and alpha1 the first-stage acceptance w.r.t. the surrogate posterior,
    all from explicit densities on R^r x R^(d_m - r) (prior N(0, I))."""
    s, beta = prob.s, prob.beta
    r = x.shape[0]

    def log_q(a, za, b, zb):
        c = mcmc.geometry(prob, a[None])
        K = np.linalg.inv(np.eye(r) + c.H[0])
        mean = K @ ((s * np.eye(r) + c.H[0]) @ a - (1 - s) * c.g[0])
        return (multivariate_normal.logpdf(b, mean, beta ** 2 * K)
                + multivariate_normal.logpdf(zb, s * za, beta ** 2 * np.eye(len(za))))

    def log_prior(a, za):
        return -0.5 * (a @ a) - 0.5 * (za @ za)

    def log_sur(a, za):
        return -mcmc.geometry(prob, a[None]).phi[0] + log_prior(a, za)

    def log_true(a, za):
        return -da.true_misfit(prob, tm, a[None], za[None])[0] + log_prior(a, za)

    q_fwd, q_rev = log_q(x, z, xp, zp), log_q(xp, zp, x, z)
    a_fwd = min(0.0, log_sur(xp, zp) + q_rev - log_sur(x, z) - q_fwd)
    a_rev = min(0.0, log_sur(x, z) + q_fwd - log_sur(xp, zp) - q_rev)
    return log_true(xp, zp) + a_rev + q_rev - log_true(x, z) - a_fwd - q_fwd


def test_second_stage_ratio_is_the_textbook_da_ratio():
    r, rT, dperp, dy = 3, 5, 4, 3
    prob = problem(net(r, dy, 3), dy, 0.4, 0.5, 4)
    tm = da.TrueModel(net(rT, dy, 8))
    rng = np.random.default_rng(5)
    for k in range(5):
        x, z = rng.standard_normal(r), rng.standard_normal(dperp)
        c = mcmc.geometry(prob, x[None])
        xp = mcmc.propose(prob, x[None], c, rng.standard_normal((1, r)))[0]
        zp = prob.s * z + prob.beta * rng.standard_normal(dperp)
        phi_x, phi_p = c.phi[0], mcmc.geometry(prob, xp[None]).phi[0]
        phit_x = da.true_misfit(prob, tm, x[None], z[None])[0]
        phit_p = da.true_misfit(prob, tm, xp[None], zp[None])[0]
        got = da.log_rho2(phi_x, phit_x, phi_p, phit_p)
        ref = textbook_log_da_ratio(prob, tm, x, z, xp, zp)
        scale = 1 + phi_x + phi_p + phit_x + phit_p
        assert abs(got - ref) < 1e-11 * scale, (k, got, ref)
        # planted mistake: the true misfits entered with the surrogate's sign
        planted = (phi_p - phi_x) - (phit_x - phit_p)
        assert abs(planted - ref) > 1e-3


def test_exact_surrogate_gives_the_first_stage_chain():
    r, dy, dperp = 4, 3, 5
    prob = problem(net(r, dy, 3), dy, 0.3, 0.6, 6)
    tm = da.TrueModel(prob.layers)            # the true model is the surrogate
    C, N = 6, 40
    rng = np.random.default_rng(7)
    x0, z0 = rng.standard_normal((C, r)), rng.standard_normal((C, dperp))
    ds = da.init_da_state(prob, tm, x0, z0)
    st = mcmc.init_state(prob, x0, z0)
    passes = 0
    for _ in range(N):
        rec = da.transition_da(prob, tm, ds)
        ref = mcmc.transition(prob, st)
        np.testing.assert_array_equal(rec.passed, ref.accept)
        np.testing.assert_array_equal(rec.accept, ref.accept)
        # zero up to the rounding of two evaluations of the same misfit
        assert np.all(np.abs(rec.log_rho2[rec.passed]) < 1e-12 * (1 + ds.phi_true[rec.passed]))
        passes += rec.passed.sum()
    np.testing.assert_array_equal(ds.chain.x, st.x)
    np.testing.assert_array_equal(ds.chain.z, st.z)
    np.testing.assert_array_equal(ds.passes, st.accepts)
    assert passes > 0.1 * C * N


def quadrature_true_posterior(prob, tm, lim=7.0, npts=401):
    g = np.linspace(-lim, lim, npts)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    phi = da.true_misfit(prob, tm, pts[:, :1], pts[:, 1:])
    logw = -phi - 0.5 * np.sum(pts * pts, axis=1)
    w = np.exp(logw - logw.max())
    w /= w.sum()
    mean = w @ pts
    cov = (pts - mean).T @ ((pts - mean) * w[:, None])
    return mean, cov


def test_da_chain_matches_true_posterior_quadrature():
    """r = 1 surrogate = the true model with the complement coordinate it reads fixed at 0;
    the true model reads (z_0, z_1) = (x, z_perp[0])."""
    dy = 2
    true_layers = net(2, dy, 15, scale=1.0)   # a unimodal true posterior (the chains mix)
    tm = da.TrueModel(true_layers)
    prob = problem(restricted(true_layers, 1), dy, 0.5, 1.0, 10)
    mean, cov = quadrature_true_posterior(prob, tm)
    C, N = 24, 2500
    rng = np.random.default_rng(12)
    x0 = rng.standard_normal((C, 1)) * np.sqrt(cov[0, 0]) + mean[0]
    z0 = np.concatenate([rng.standard_normal((C, 1)) * np.sqrt(cov[1, 1]) + mean[1],
                         rng.standard_normal((C, 1))], axis=1)
    ds = da.init_da_state(prob, tm, x0, z0)
    xs, zs, _ = da.run_da(prob, tm, ds, N)
    acc = ds.chain.accepts.sum() / (C * N)
    assert 0.1 < acc <= 1.0 and ds.passes.sum() >= ds.chain.accepts.sum()
    burn = N // 5
    tr = np.concatenate([xs[burn:], zs[burn:]], axis=2)          # (n, C, 2)
    e = stats.ess_per_coordinate(tr)
    n_eff = tr.shape[0] * C * e
    mcse = np.sqrt(np.diag(cov) / n_eff)
    X = tr.reshape(-1, 2)
    assert np.all(np.abs(X.mean(0) - mean) < 4.5 * mcse)
    var_tol = 5.0 * np.sqrt(2.0 / n_eff) * np.diag(cov) + 5 * mcse * np.abs(X.mean(0) - mean)
    assert np.all(np.abs(X.var(0) - np.diag(cov)) < var_tol)
    # power: the first-stage chain alone targets the surrogate posterior and misses
    st = mcmc.init_state(prob, x0, z0)
    xs1, _ = mcmc.run(prob, st, N)
    x1 = xs1[burn:].reshape(-1)
    assert abs(x1.mean() - mean[0]) > 8 * mcse[0]


def test_da_chain_matches_linear_gaussian_closed_form():
    """Linear surrogate on r = 2 and a different linear true model on r_T = 3 (it reads the
    first complement coordinate): the DA chain targets N(mu, Sigma) with
    Sigma = (I + A^T Gamma^-1 A)^-1, mu = Sigma A^T Gamma^-1 (y - b); the unread
    complement coordinate stays N(0, 1)."""
    rng = np.random.default_rng(13)
    dy = 4
    A_T = rng.standard_normal((dy, 3))
    b_T = rng.standard_normal(dy)
    A_s = A_T[:, :2] + 0.3 * rng.standard_normal((dy, 2))
    y = rng.standard_normal(dy)
    nv = np.full(dy, 0.7 ** 2)
    prob = mcmc.Problem([("linear", A_s, b_T)], y, nv, 0.8, seed=14, request_id=1)
    tm = da.TrueModel([("linear", A_T, b_T)])
    Gi = np.diag(1.0 / nv)
    Sigma = np.linalg.inv(np.eye(3) + A_T.T @ Gi @ A_T)
    mu = Sigma @ A_T.T @ Gi @ (y - b_T)
    C, N = 16, 3000
    x0 = rng.standard_normal((C, 2))
    z0 = rng.standard_normal((C, 2))
    ds = da.init_da_state(prob, tm, x0, z0)
    st = ds.chain
    X = np.empty((N, C, 4))
    for t in range(N):
        da.transition_da(prob, tm, ds)
        X[t, :, :2] = st.x
        X[t, :, 2:] = st.z
    burn = N // 5
    tr = X[burn:]
    e = stats.ess_per_coordinate(tr)
    n_eff = tr.shape[0] * C * e
    full_mu = np.concatenate([mu, [0.0]])
    full_var = np.concatenate([np.diag(Sigma), [1.0]])
    mcse = np.sqrt(full_var / n_eff)
    F = tr.reshape(-1, 4)
    assert np.all(np.abs(F.mean(0) - full_mu) < 4.5 * mcse)
    assert np.all(np.abs(F.var(0) - full_var) < 5.0 * np.sqrt(2.0 / n_eff) * full_var + 5 * mcse * np.abs(F.mean(0) - full_mu))
    S = np.cov(F[:, :3].T)
    off = np.abs(S - Sigma)[np.triu_indices(3, 1)]
    assert np.all(off < 6.0 * np.sqrt(np.outer(np.diag(Sigma), np.diag(Sigma)))[np.triu_indices(3, 1)] / np.sqrt(n_eff.min()))
