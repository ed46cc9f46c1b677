"""Pins for oracle/mcmc.py (Alg. 1 first stage, the splitting proposition of Sec. 5.3, Sec. 5.4 ratios).

* The paper-form first-stage ratio equals the textbook finite-dimensional MH ratio
  built from explicit Gaussian proposal densities (scipy), and rho_0 equals the
  mMALA / pCN density ratio.
* Linear surrogate: the proposal is the pCN proposal of the Gaussian posterior, so
  log rho == 0 for every dt, the chain is AR(1) with coefficient s, and its moments
  converge to the closed-form posterior.
* Zero likelihood (Gamma^-1 = 0): H = 0, g = 0 and the proposal is pCN, which is
  prior reversible (Sec. 2.5), so log rho == 0.
* Brute force on R^1 / R^2: quadrature of a nonlinear surrogate posterior.
* Planted mistakes: the printed ppg sign and the printed additive determinant term
  both fail these pins.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.stats import multivariate_normal

from oracle import mcmc, network, philox, stats
from synth import draw_network, workload


def nonlinear_problem(r=4, d_out=3, dt=0.4, noise=0.2, seed=3, arch="mlp"):
    w = workload("tiny", r=r, width=6, depth=2, d_out=d_out, d_y=d_out, arch=arch)
    layers = draw_network(w, seed=seed, bias_scale=0.2)
    layers = [(k, 2.0 * W, b) for (k, W, b) in layers]  # stronger nonlinearity
    y = np.random.default_rng(seed + 1).standard_normal(d_out)
    return mcmc.Problem(layers, y, np.full(d_out, noise ** 2), dt, seed=seed, request_id=2)


def linear_problem(r=3, d_y=4, dt=0.5, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((d_y, r))
    b = rng.standard_normal(d_y)
    y = rng.standard_normal(d_y)
    return mcmc.Problem([("linear", A, b)], y, rng.uniform(0.2, 1.0, d_y) ** 2, dt, seed=seed + 10), A, b


def textbook_log_ratio(prob, a, b):
    """log of pi(b) q(b->a) / (pi(a) q(a->b)) with q(u->.) = N(mean(u), beta^2 (I+H_u)^-1)."""
    s, beta = prob.s, prob.beta
    r = a.shape[0]

    def parts(u):
        c = mcmc.geometry(prob, u[None])
        H, g = c.H[0], c.g[0]
        K = np.linalg.inv(np.eye(r) + H)
        mean = K @ ((s * np.eye(r) + H) @ u - (1 - s) * g)
        return c.phi[0], mean, beta ** 2 * K

    phi_a, mean_a, cov_a = parts(a)
    phi_b, mean_b, cov_b = parts(b)
    log_pi = lambda phi, u: -phi - 0.5 * u @ u
    return (log_pi(phi_b, b) + multivariate_normal.logpdf(a, mean_b, cov_b)
            - log_pi(phi_a, a) - multivariate_normal.logpdf(b, mean_a, cov_a))


@pytest.mark.parametrize("arch", ["mlp", "resnet"])
def test_textbook_identity(arch):
    prob = nonlinear_problem(arch=arch)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 4))
    cx = mcmc.geometry(prob, x)
    xp = mcmc.propose(prob, x, cx, rng.standard_normal((4, 4)))
    cp = mcmc.geometry(prob, xp)
    lr = mcmc.log_rho1(prob, x, cx, xp, cp)
    for c in range(4):
        ref = textbook_log_ratio(prob, x[c], xp[c])
        # the ratio is a difference of terms of size ~ Phi and ~ eigenvalues of H
        scale = 1 + cx.phi[c] + cp.phi[c] + cx.d[c].sum() + cp.d[c].sum()
        assert abs(lr[c] - ref) < 1e-12 * scale


def test_rho0_is_mmala_over_pcn_density():
    prob = nonlinear_problem()
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4))
    x2 = rng.standard_normal((3, 4))
    cx = mcmc.geometry(prob, x)
    l0 = mcmc.log_rho0(prob, x, x2, cx)
    s, beta = prob.s, prob.beta
    for c in range(3):
        K = np.linalg.inv(np.eye(4) + cx.H[c])
        mean = K @ ((s * np.eye(4) + cx.H[c]) @ x[c] - (1 - s) * cx.g[c])
        ref = (multivariate_normal.logpdf(x2[c], mean, beta ** 2 * K)
               - multivariate_normal.logpdf(x2[c], s * x[c], beta ** 2 * np.eye(4)))
        scale = 1 + cx.phi[c] + cx.d[c].sum() * (1 + x2[c] @ x2[c] / beta ** 2)
        assert abs(l0[c] - ref) < 1e-12 * scale


def test_proposal_law_eigen_vs_cholesky():
    """eq. reduced_space_sampling mean, and the Cholesky noise map has the law
    N(0, (1 - s^2)(I + H)^-1) = P diag((1 - s^2)/(d + 1)) P^T."""
    prob = nonlinear_problem()
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4))
    c = mcmc.geometry(prob, x)
    s = prob.s
    m0 = mcmc.propose(prob, x, c, np.zeros((2, 4)))
    for k in range(2):
        ref = np.linalg.solve(np.eye(4) + c.H[k], (s * np.eye(4) + c.H[k]) @ x[k] - (1 - s) * c.g[k])
        np.testing.assert_allclose(m0[k], ref, rtol=1e-12, atol=1e-12)
        T = np.stack([mcmc.propose(prob, x[k:k + 1], _one(c, k), np.eye(4)[j][None])[0] - m0[k]
                      for j in range(4)], axis=1)
        cov = T @ T.T
        ref_cov = c.P[k] @ np.diag((1 - s * s) / (c.d[k] + 1)) @ c.P[k].T
        np.testing.assert_allclose(cov, ref_cov, rtol=1e-11, atol=1e-13)


def _one(cache, k):
    return mcmc.Cache(**{f: getattr(cache, f)[k:k + 1] for f in cache.__dataclass_fields__})


@pytest.mark.parametrize("dt", [1e-3, 0.1, 0.7, 2.0, 3.9])
def test_linear_surrogate_log_rho_is_zero(dt):
    prob, A, b = linear_problem(dt=dt)
    rng = np.random.default_rng(4)
    x = 3.0 * rng.standard_normal((6, 3))
    cx = mcmc.geometry(prob, x)
    xp = mcmc.propose(prob, x, cx, rng.standard_normal((6, 3)))
    lr = mcmc.log_rho1(prob, x, cx, xp, mcmc.geometry(prob, xp))
    assert np.max(np.abs(lr)) < 1e-10 * (1 + np.max(cx.phi))
    # the proposal is pCN about the Gaussian posterior mean
    Hm = A.T @ np.diag(1 / prob.noise_var) @ A
    mu = np.linalg.solve(np.eye(3) + Hm, A.T @ ((prob.y - b) / prob.noise_var))
    m0 = mcmc.propose(prob, x, cx, np.zeros_like(x))
    np.testing.assert_allclose(m0 - mu, prob.s * (x - mu), rtol=1e-10, atol=1e-10)


def test_zero_likelihood_is_pcn_and_reversible():
    prob = nonlinear_problem()
    prob.noise_var = np.full(prob.d_y, np.inf)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 4))
    c = mcmc.geometry(prob, x)
    assert np.all(c.phi == 0) and np.all(c.g == 0) and np.all(c.H == 0)
    np.testing.assert_array_equal(c.L, np.broadcast_to(np.eye(4), (4, 4, 4)))
    xi = rng.standard_normal((4, 4))
    xp = mcmc.propose(prob, x, c, xi)
    np.testing.assert_allclose(xp, prob.s * x + prob.beta * xi, rtol=1e-14, atol=1e-14)
    lr = mcmc.log_rho1(prob, x, c, xp, mcmc.geometry(prob, xp))
    assert np.max(np.abs(lr)) < 1e-13


# ---- planted mistakes: the printed forms fail the pins -------------------------------

def test_printed_ppg_sign_fails_linear_invariant():
    prob, A, b = linear_problem(dt=0.5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((5, 3))
    flip = lambda c: mcmc.Cache(**{**c.__dict__, "g": -c.g})
    cx = flip(mcmc.geometry(prob, x))
    xp = mcmc.propose(prob, x, cx, rng.standard_normal((5, 3)))
    lr = mcmc.log_rho1(prob, x, cx, xp, flip(mcmc.geometry(prob, xp)))
    assert np.max(np.abs(lr)) > 1e-2


def test_printed_additive_determinant_fails_textbook():
    prob = nonlinear_problem()
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, 4))
    cx = mcmc.geometry(prob, x)
    xp = mcmc.propose(prob, x, cx, rng.standard_normal((3, 4)))
    cp = mcmc.geometry(prob, xp)

    def printed_log_rho0(m1, m2, c1):
        full = mcmc.log_rho0(prob, m1, m2, c1)
        det = 0.5 * np.sum(np.log(c1.d + 1.0), axis=1)
        return np.log(np.exp(full - det) + np.exp(det))  # exp(...) + prod (d+1)^1/2

    lr_printed = cx.phi - cp.phi + printed_log_rho0(xp, x, cp) - printed_log_rho0(x, xp, cx)
    ref = np.array([textbook_log_ratio(prob, x[c], xp[c]) for c in range(3)])
    assert np.max(np.abs(lr_printed - ref)) > 1e-3


# ---- chains ------------------------------------------------------------------------------

def test_resume_is_bitwise():
    prob = nonlinear_problem()
    x0 = np.random.default_rng(8).standard_normal((3, 4))
    z0 = np.random.default_rng(9).standard_normal((3, 11))
    a = mcmc.init_state(prob, x0, z0)
    mcmc.run(prob, a, 40, trace=False)
    b = mcmc.init_state(prob, x0, z0)
    mcmc.run(prob, b, 25, trace=False)
    mcmc.run(prob, b, 15, trace=False)
    assert a.step == b.step == 40
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.z, b.z)
    np.testing.assert_array_equal(a.accepts, b.accepts)


def test_complement_moves_only_on_accept():
    prob = nonlinear_problem(dt=2.0, noise=0.02)
    x0 = np.random.default_rng(10).standard_normal((6, 4))
    st = mcmc.init_state(prob, x0, np.zeros((6, 5)))
    z_before = st.z.copy()
    rec = mcmc.transition(prob, st)
    moved = np.any(st.z != z_before, axis=1)
    np.testing.assert_array_equal(moved, rec.accept)
    zeta = philox.normals(prob.seed, prob.request_id, philox.STREAM_COMPLEMENT, 0, np.arange(6), 5)
    np.testing.assert_allclose(st.z[rec.accept], prob.beta * zeta[rec.accept], rtol=1e-15)


def test_linear_chain_matches_closed_form_posterior():
    prob, A, b = linear_problem(dt=0.5)
    C, N = 16, 3000
    x0 = np.random.default_rng(11).standard_normal((C, 3))
    st = mcmc.init_state(prob, x0, np.zeros((C, 4)))
    xs, _ = mcmc.run(prob, st, N)
    assert np.all(st.accepts == N)
    Gi = np.diag(1 / prob.noise_var)
    Sigma = np.linalg.inv(np.eye(3) + A.T @ Gi @ A)
    mu = Sigma @ A.T @ Gi @ (prob.y - b)
    burn = N // 5
    X = xs[burn:].reshape(-1, 3)
    ess_frac = (1 - prob.s) / (1 + prob.s)   # AR(1) with coefficient s
    assert abs(ess_frac - prob.dt / 4) < 1e-15
    n_eff = X.shape[0] * ess_frac
    mcse = np.sqrt(np.diag(Sigma) / n_eff)
    assert np.all(np.abs(X.mean(0) - mu) < 4.5 * mcse)
    S = np.cov(X.T)
    assert np.all(np.abs(np.diag(S) - np.diag(Sigma)) < 5 * np.sqrt(2 / n_eff) * np.diag(Sigma))
    # ESS estimator on the chain reproduces dt/4
    e = stats.ess_per_coordinate(xs[burn:])
    assert np.all(np.abs(e - prob.dt / 4) < 0.25 * prob.dt / 4)


def test_complement_stationary_law():
    prob = nonlinear_problem(dt=0.8)
    prob.noise_var = np.full(prob.d_y, np.inf)   # every move accepted
    C, N, dz = 8, 1500, 6
    st = mcmc.init_state(prob, np.zeros((C, 4)), np.zeros((C, dz)))
    zs = np.empty((N, C, dz))
    for t in range(N):
        mcmc.transition(prob, st)
        zs[t] = st.z
    Z = zs[300:]
    v = Z.var()
    n_eff = Z.size * (1 - prob.s) / (1 + prob.s)
    assert abs(v - 1.0) < 5 * np.sqrt(2 / n_eff)
    lag1 = np.mean(Z[1:] * Z[:-1]) / np.mean(Z * Z)
    assert abs(lag1 - prob.s) < 0.03


def quadrature_moments(prob, r, lim=7.0, npts=2001):
    g1 = np.linspace(-lim, lim, npts)
    if r == 1:
        pts = g1[:, None]
    else:
        g1 = np.linspace(-lim, lim, 401)
        X, Y = np.meshgrid(g1, g1, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    f, _ = network.forward(prob.layers, pts)
    phi = 0.5 * np.sum((prob.y - f[:, : prob.d_y]) ** 2 / prob.noise_var, axis=1)
    logw = -phi - 0.5 * np.sum(pts * pts, axis=1)
    w = np.exp(logw - logw.max())
    w /= w.sum()
    mean = w @ pts
    cov = (pts - mean).T @ ((pts - mean) * w[:, None])
    return mean, cov


@pytest.mark.parametrize("r", [1, 2])
def test_nonlinear_chain_matches_quadrature(r):
    prob = nonlinear_problem(r=r, d_out=2, dt=1.0, noise=0.5, seed=5)
    mean, cov = quadrature_moments(prob, r)
    C, N = 24, 2500
    x0 = np.random.default_rng(12).standard_normal((C, r)) * np.sqrt(np.diag(cov)) + mean
    st = mcmc.init_state(prob, x0)
    xs, _ = mcmc.run(prob, st, N)
    acc = st.accepts.sum() / (C * N)
    assert 0.2 < acc <= 1.0
    burn = N // 5
    tr = xs[burn:]
    e = stats.ess_per_coordinate(tr)
    n_eff = tr.shape[0] * C * e
    mcse = np.sqrt(np.diag(cov) / n_eff)
    X = tr.reshape(-1, r)
    assert np.all(np.abs(X.mean(0) - mean) < 4.5 * mcse)
    var_tol = 5.0 * np.sqrt(2.0 / n_eff) * np.diag(cov) + 5 * mcse * np.abs(X.mean(0) - mean)
    assert np.all(np.abs(X.var(0) - np.diag(cov)) < var_tol)


# ---- pCN baseline (Sec. 2.6, eq. pCN_proposal; the pCN row of the baselines of Sec. 6.1) ----

def test_pcn_misfit_is_the_geometry_misfit():
    prob = nonlinear_problem()
    x = np.random.default_rng(21).standard_normal((5, 4))
    f, phi = mcmc.misfit(prob, x)
    c = mcmc.geometry(prob, x)
    np.testing.assert_array_equal(phi, c.phi)
    np.testing.assert_array_equal(f, c.f)


def test_pcn_log_rho_is_the_textbook_mh_ratio():
    """log rho = log pi(x+) q(x+ -> x) - log pi(x) q(x -> x+), with pi = exp(-Phi) N(0, I)
    and the pCN law q(a -> .) = N(s a, (1 - s^2) I), evaluated by scipy's Gaussian density."""
    prob = nonlinear_problem(dt=0.6)
    prob.method = "pcn"
    rng = np.random.default_rng(22)
    x = rng.standard_normal((6, 4))
    st = mcmc.init_state(prob, x)
    xi = rng.standard_normal((6, 4))
    rec = mcmc.transition(prob, st, xi=xi, u=np.full(6, 0.5))
    np.testing.assert_allclose(rec.xp, prob.s * x + prob.beta * xi, rtol=1e-15, atol=1e-15)
    cov = (1.0 - prob.s ** 2) * np.eye(4)
    for c in range(6):
        a, b = x[c], rec.xp[c]
        phi_a = mcmc.geometry(prob, a[None]).phi[0]
        phi_b = mcmc.geometry(prob, b[None]).phi[0]
        ref = (-phi_b - 0.5 * b @ b + multivariate_normal.logpdf(a, prob.s * b, cov)
               + phi_a + 0.5 * a @ a - multivariate_normal.logpdf(b, prob.s * a, cov))
        assert abs(rec.log_rho[c] - ref) < 1e-10 * max(1.0, abs(ref))
    np.testing.assert_array_equal(rec.accept, np.log(0.5) <= rec.log_rho)


def test_pcn_without_likelihood_is_the_prior_ar1():
    """With Phi = 0 every pCN move is accepted and each coordinate is the AR(1) chain with
    coefficient s and stationary law N(0, 1)."""
    prob = nonlinear_problem(dt=0.8)
    prob.method = "pcn"
    prob.noise_var = np.full(prob.d_y, np.inf)
    C, N = 8, 1500
    st = mcmc.init_state(prob, np.zeros((C, 4)))
    xs, _ = mcmc.run(prob, st, N)
    assert np.all(st.accepts == N)
    X = xs[300:]
    n_eff = X.size * (1 - prob.s) / (1 + prob.s)
    assert abs(X.var() - 1.0) < 5 * np.sqrt(2 / n_eff)
    lag1 = np.mean(X[1:] * X[:-1]) / np.mean(X * X)
    assert abs(lag1 - prob.s) < 0.03


def test_pcn_chain_matches_quadrature():
    prob = nonlinear_problem(r=1, d_out=2, dt=1.0, noise=0.5, seed=5)
    prob.method = "pcn"
    mean, cov = quadrature_moments(prob, 1)
    C, N = 24, 3000
    x0 = np.random.default_rng(13).standard_normal((C, 1)) * np.sqrt(np.diag(cov)) + mean
    st = mcmc.init_state(prob, x0, np.zeros((C, 3)))
    xs, _ = mcmc.run(prob, st, N)
    acc = st.accepts.sum() / (C * N)
    assert 0.05 < acc < 1.0
    tr = xs[N // 5:]
    e = stats.ess_per_coordinate(tr)
    n_eff = tr.shape[0] * C * e
    mcse = np.sqrt(np.diag(cov) / n_eff)
    X = tr.reshape(-1, 1)
    assert np.all(np.abs(X.mean(0) - mean) < 4.5 * mcse)
    var_tol = 5.0 * np.sqrt(2.0 / n_eff) * np.diag(cov) + 5 * mcse * np.abs(X.mean(0) - mean)
    assert np.all(np.abs(X.var(0) - np.diag(cov)) < var_tol)


def test_pcn_planted_beta_squared_fails_the_prior_ar1():
    """A pCN proposal that scales the noise by 1 - s^2 instead of its square root leaves
    the prior: the stationary variance pin fails."""
    prob = nonlinear_problem(dt=0.8)
    prob.noise_var = np.full(prob.d_y, np.inf)
    C, N = 8, 1500
    rng = np.random.default_rng(23)
    x = np.zeros((C, 4))
    xs = np.empty((N, C, 4))
    for t in range(N):
        x = prob.s * x + (1.0 - prob.s ** 2) * rng.standard_normal((C, 4))
        xs[t] = x
    X = xs[300:]
    n_eff = X.size * (1 - prob.s) / (1 + prob.s)
    assert abs(X.var() - 1.0) > 5 * np.sqrt(2 / n_eff)


# ---- MALA baseline (gradient, no metric: the MALA row of the baselines of Sec. 6.1) ----

def mala_textbook_log_ratio(prob, a, b):
    """log pi(b) q(b -> a) - log pi(a) q(a -> b) with the Langevin law
    q(u -> .) = N(s u - (1 - s) g(u), (1 - s^2) I), g the ppg of the geometry."""
    r = a.shape[0]
    cov = (1.0 - prob.s ** 2) * np.eye(r)

    def parts(u):
        c = mcmc.geometry(prob, u[None])
        return c.phi[0], prob.s * u - (1.0 - prob.s) * c.g[0]

    phi_a, mean_a = parts(a)
    phi_b, mean_b = parts(b)
    return (-phi_b - 0.5 * b @ b + multivariate_normal.logpdf(a, mean_b, cov)
            + phi_a + 0.5 * a @ a - multivariate_normal.logpdf(b, mean_a, cov))


@pytest.mark.parametrize("arch", ["mlp", "resnet"])
def test_mala_log_rho_is_the_textbook_mh_ratio(arch):
    prob = nonlinear_problem(dt=0.3, arch=arch)
    prob.method = "mala"
    rng = np.random.default_rng(31)
    x = rng.standard_normal((5, 4))
    st = mcmc.init_state(prob, x)
    xi = rng.standard_normal((5, 4))
    rec = mcmc.transition(prob, st, xi=xi, u=np.full(5, 0.5))
    g = mcmc.geometry(prob, x).g
    np.testing.assert_allclose(rec.xp, prob.s * x - (1 - prob.s) * g + prob.beta * xi, rtol=1e-13, atol=1e-13)
    for c in range(5):
        ref = mala_textbook_log_ratio(prob, x[c], rec.xp[c])
        assert abs(rec.log_rho[c] - ref) < 1e-9 * max(1.0, abs(ref))


def test_mala_without_likelihood_is_pcn():
    prob = nonlinear_problem(dt=0.5)
    prob.noise_var = np.full(prob.d_y, np.inf)
    rng = np.random.default_rng(32)
    x = rng.standard_normal((4, 4))
    xi = rng.standard_normal((4, 4))
    out = {}
    for method in ("mala", "pcn"):
        prob.method = method
        st = mcmc.init_state(prob, x.copy())
        out[method] = mcmc.transition(prob, st, xi=xi, u=np.full(4, 0.999))
    np.testing.assert_allclose(out["mala"].xp, out["pcn"].xp, rtol=1e-15, atol=1e-15)
    assert np.max(np.abs(out["mala"].log_rho)) < 1e-13 and np.all(out["mala"].accept)


def test_mala_chain_matches_quadrature():
    prob = nonlinear_problem(r=1, d_out=2, dt=0.05, noise=0.5, seed=5)   # acceptance about 0.5
    prob.method = "mala"
    mean, cov = quadrature_moments(prob, 1)
    C, N = 24, 2500
    x0 = np.random.default_rng(14).standard_normal((C, 1)) * np.sqrt(np.diag(cov)) + mean
    st = mcmc.init_state(prob, x0)
    xs, _ = mcmc.run(prob, st, N)
    acc = st.accepts.sum() / (C * N)
    assert 0.05 < acc < 1.0
    tr = xs[N // 5:]
    e = stats.ess_per_coordinate(tr)
    n_eff = tr.shape[0] * C * e
    mcse = np.sqrt(np.diag(cov) / n_eff)
    X = tr.reshape(-1, 1)
    assert np.all(np.abs(X.mean(0) - mean) < 4.5 * mcse)
    var_tol = 5.0 * np.sqrt(2.0 / n_eff) * np.diag(cov) + 5 * mcse * np.abs(X.mean(0) - mean)
    assert np.all(np.abs(X.var(0) - np.diag(cov)) < var_tol)


def test_mala_planted_dropped_gradient_norm_fails_textbook():
    """Dropping the -(dt/8)||g||^2 terms of rho_0 breaks the MH ratio pin."""
    prob = nonlinear_problem(dt=0.3)
    prob.method = "mala"
    rng = np.random.default_rng(33)
    x = rng.standard_normal((3, 4))
    st = mcmc.init_state(prob, x)
    rec = mcmc.transition(prob, st, xi=rng.standard_normal((3, 4)), u=np.full(3, 0.5))
    gx = mcmc.geometry(prob, x).g
    gp = mcmc.geometry(prob, rec.xp).g
    planted = rec.log_rho + (prob.dt / 8.0) * (np.sum(gp * gp, axis=1) - np.sum(gx * gx, axis=1))
    ref = np.array([mala_textbook_log_ratio(prob, x[c], rec.xp[c]) for c in range(3)])
    assert np.max(np.abs(planted - ref)) > 1e-3


# ---- LA-pCN baseline (metric fixed at the MAP, no ppg; eq. MAP) ----------------------

def laplace_fixed(prob, r):
    """MAP by Gauss-Newton on the oracle's geometry, and the factor of I + H there."""
    x = np.zeros(r)
    for _ in range(200):
        c = mcmc.geometry(prob, x[None])
        step = np.linalg.solve(np.eye(r) + c.H[0], x + c.g[0])
        x = x - step
        if np.linalg.norm(step) < 1e-13:
            break
    c = mcmc.geometry(prob, x[None])
    return x, c.L[0]


def test_lapcn_log_rho_is_the_textbook_mh_ratio():
    prob = nonlinear_problem(dt=0.5)
    prob.method = "lapcn"
    x_map, L = laplace_fixed(prob, 4)
    prob.fixed = (x_map, L)
    cov = (1.0 - prob.s ** 2) * np.linalg.inv(L @ L.T)
    rng = np.random.default_rng(41)
    x = x_map + 0.5 * rng.standard_normal((5, 4))
    st = mcmc.init_state(prob, x)
    rec = mcmc.transition(prob, st, xi=rng.standard_normal((5, 4)), u=np.full(5, 0.5))
    for c in range(5):
        a, b = x[c], rec.xp[c]
        pa, pb = mcmc.geometry(prob, a[None]).phi[0], mcmc.geometry(prob, b[None]).phi[0]
        mean = lambda v: x_map + prob.s * (v - x_map)
        ref = (-pb - 0.5 * b @ b + multivariate_normal.logpdf(a, mean(b), cov)
               + pa + 0.5 * a @ a - multivariate_normal.logpdf(b, mean(a), cov))
        assert abs(rec.log_rho[c] - ref) < 1e-9 * max(1.0, abs(ref))


def test_lapcn_is_exact_on_a_linear_gaussian_posterior():
    """Linear network: the Laplace approximation at the MAP is the posterior, so every
    LA-pCN proposal has log rho = 0 and is accepted."""
    prob, A, b = linear_problem(dt=0.7)
    prob.method = "lapcn"
    x_map, L = laplace_fixed(prob, 3)
    Gi = np.diag(1 / prob.noise_var)
    Sigma = np.linalg.inv(np.eye(3) + A.T @ Gi @ A)
    np.testing.assert_allclose(x_map, Sigma @ A.T @ Gi @ (prob.y - b), rtol=1e-12, atol=1e-12)
    prob.fixed = (x_map, L)
    st = mcmc.init_state(prob, np.random.default_rng(42).standard_normal((6, 3)))
    for _ in range(5):
        rec = mcmc.transition(prob, st)
        assert np.max(np.abs(rec.log_rho)) < 1e-11 and np.all(rec.accept)


def test_lapcn_printed_mean_fails_the_textbook_ratio():
    """The printed mean m_MAP - s m with the Laplace-reversible ratio disagrees with the
    textbook MH ratio of that proposal: the printed form is not the method."""
    prob, A, b = linear_problem(dt=0.7)
    x_map, L = laplace_fixed(prob, 3)
    cov = (1.0 - prob.s ** 2) * np.linalg.inv(L @ L.T)
    rng = np.random.default_rng(43)
    a = rng.standard_normal(3)
    printed = lambda v: x_map - prob.s * v
    bpt = printed(a) + np.linalg.cholesky(cov) @ rng.standard_normal(3)
    phi = lambda v: mcmc.geometry(prob, v[None]).phi[0]
    textbook = (-phi(bpt) - 0.5 * bpt @ bpt + multivariate_normal.logpdf(a, printed(bpt), cov)
                + phi(a) + 0.5 * a @ a - multivariate_normal.logpdf(bpt, printed(a), cov))
    assert abs(textbook) > 1e-3   # the closed-form ratio is 0 on this posterior
