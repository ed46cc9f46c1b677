"""Pins for the dense reduced basis (oracle/prior.py DenseBasis; Sec. 4.2), DIS-mMALA
(oracle/mcmc.py, the DIS-mMALA row of the baselines of Sec. 6.1 with eq. dis_gnh) and
delayed acceptance on a dense basis (oracle/da.py, Alg. 1's assembly of the full proposal).

* Dense basis against dense-matrix definitions on a small grid: H_mu-orthonormality
  Psi^T C_pr^-1 Psi = I, the encoder of eq. projector <m, psi_j>_{C_pr^-1}, and the
  complement variance diag(C_pr) - diag(Psi Psi^T), with C_pr = A^-2 formed densely (no
  DCT); identity columns reproduce the closed-form KLE basis.
* DIS-mMALA: the ratio equals the textbook MH ratio of its Gaussian proposal (scipy);
  lam = 0 is the MALA transition draw for draw; a linear surrogate whose J^T Gamma^-1 J is
  diag(lam) makes DIS-mMALA exact mMALA (log rho == 0).
* DA on a dense basis: a linear true model reading the first r_T whitened coordinates of
  U x + (I - U U^T) w targets the closed-form Gaussian posterior of those coordinates.
"""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import da, mcmc, prior, stats
from synth import draw_network, workload


def random_dense_basis(n, r, support, seed):
    """Orthonormal U (d_m, r) supported on the first `support` whitened coordinates."""
    rng = np.random.default_rng(seed)
    U = np.zeros((n * n, r))
    U[:support], _ = np.linalg.qr(rng.standard_normal((support, r)))
    return U


def test_identity_columns_give_the_kle_basis():
    n, r = 9, 7
    K = prior.KLEBasis(n, 0.1, 1.0, r)
    D = prior.DenseBasis(n, 0.1, 1.0, np.eye(n * n)[:, :r])
    np.testing.assert_allclose(D.dec, K.dec, atol=1e-15)
    np.testing.assert_allclose(D.var_perp, K.var_perp, atol=1e-15)
    m = np.random.default_rng(0).standard_normal((3, n * n))
    np.testing.assert_allclose(D.encode(m), K.encode(m), rtol=1e-10, atol=1e-12)


def test_dense_basis_against_the_dense_prior():
    n, r = 6, 5
    U = random_dense_basis(n, r, 14, 1)
    D = prior.DenseBasis(n, 0.3, 1.0, U)
    Cpr = prior.prior_covariance_dense(n, 0.3, 1.0)
    Ci = np.linalg.inv(Cpr)
    np.testing.assert_allclose(D.dec.T @ Ci @ D.dec, np.eye(r), atol=1e-9)
    m = np.random.default_rng(2).standard_normal((4, n * n))
    np.testing.assert_allclose(D.encode(m), m @ Ci @ D.dec, rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(D.var_perp, np.diag(Cpr) - np.sum(D.dec ** 2, axis=1), rtol=1e-10, atol=1e-15)
    # field covariance of U x + (I - U U^T) w with x ~ N(0, S), w ~ N(0, I): its diagonal is the
    # Rao-Blackwell formula diag(Psi S Psi^T) + var_perp
    S = np.diag(np.linspace(0.2, 1.5, r))
    Pp = np.eye(n * n) - U @ U.T
    whiten_inv = D.kle.unwhiten_full(np.eye(n * n))      # rows: Q Lambda^1/2 e_k
    T = whiten_inv.T                                     # m = T z
    cov_m = T @ (U @ S @ U.T + Pp) @ T.T
    np.testing.assert_allclose(np.diag(cov_m), np.einsum("pj,jk,pk->p", D.dec, S, D.dec) + D.var_perp,
                               rtol=1e-10, atol=1e-15)


def dis_problem(r=4, d_out=3, dt=0.4, noise=0.3, seed=3, lam=None):
    w = workload("tiny", r=r, width=6, depth=2, d_out=d_out, d_y=d_out, arch="mlp")
    layers = [(k, 2.0 * W, b) for (k, W, b) in draw_network(w, seed=seed, bias_scale=0.2)]
    y = np.random.default_rng(seed + 1).standard_normal(d_out)
    lam = np.linspace(3.0, 0.2, r) if lam is None else lam
    return mcmc.Problem(layers, y, np.full(d_out, noise ** 2), dt, seed=seed, request_id=2, method="dis_mmala",
                        fixed=lam)


def test_dis_mmala_log_rho_is_the_textbook_mh_ratio():
    prob = dis_problem()
    lam = prob.fixed
    s, beta = prob.s, prob.beta
    K = np.diag(1.0 / (1.0 + lam))
    rng = np.random.default_rng(4)
    x = rng.standard_normal((5, 4))
    cx = mcmc.method_geometry(prob, x)
    xp = mcmc.propose(prob, x, cx, rng.standard_normal((5, 4)))
    cp = mcmc.method_geometry(prob, xp)
    lr = mcmc.log_rho1(prob, x, cx, xp, cp)
    for c in range(5):
        def log_q(a, ga, b):
            mean = K @ ((np.diag(lam) + s * np.eye(4)) @ a - (1 - s) * ga)
            return multivariate_normal.logpdf(b, mean, beta ** 2 * K)
        ref = (-cp.phi[c] - 0.5 * xp[c] @ xp[c] + log_q(xp[c], cp.g[c], x[c])
               + cx.phi[c] + 0.5 * x[c] @ x[c] - log_q(x[c], cx.g[c], xp[c]))
        assert abs(lr[c] - ref) < 1e-11 * (1 + cx.phi[c] + cp.phi[c] + lam.sum())


def test_dis_mmala_with_zero_eigenvalues_is_mala():
    p_dis = dis_problem(lam=np.zeros(4))
    p_mala = dis_problem()
    p_mala.method, p_mala.fixed = "mala", None
    rng = np.random.default_rng(5)
    x0 = rng.standard_normal((6, 4))
    s1, s2 = mcmc.init_state(p_dis, x0), mcmc.init_state(p_mala, x0)
    for _ in range(15):
        a = mcmc.transition(p_dis, s1)
        b = mcmc.transition(p_mala, s2)
        np.testing.assert_array_equal(a.accept, b.accept)
        np.testing.assert_allclose(a.log_rho, b.log_rho, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(s1.x, s2.x, rtol=1e-13, atol=1e-13)


def test_dis_mmala_is_exact_when_the_metric_is_the_constant_hessian():
    rng = np.random.default_rng(6)
    r, dy = 3, 5
    lam = np.array([4.0, 1.5, 0.3])
    V, _ = np.linalg.qr(rng.standard_normal((dy, r)))
    nv = rng.uniform(0.3, 1.0, dy) ** 2
    A = np.sqrt(nv)[:, None] * V * np.sqrt(lam)[None, :]        # A^T Gamma^-1 A = diag(lam)
    prob = mcmc.Problem([("linear", A, rng.standard_normal(dy))], rng.standard_normal(dy), nv, 0.7, seed=1,
                        method="dis_mmala", fixed=lam)
    x = rng.standard_normal((4, r))
    cx = mcmc.method_geometry(prob, x)
    np.testing.assert_allclose(mcmc.geometry(prob, x).H[0], np.diag(lam), atol=1e-12)
    xp = mcmc.propose(prob, x, cx, rng.standard_normal((4, r)))
    lr = mcmc.log_rho1(prob, x, cx, xp, mcmc.method_geometry(prob, xp))
    assert np.max(np.abs(lr)) < 1e-10


def test_da_on_a_dense_basis_matches_the_linear_gaussian_posterior():
    """Dense basis U (supported on the first 12 of 36 whitened coordinates, r = 3), linear
    surrogate on x = U^T z, linear true model on z[0:5] of the assembled full parameter."""
    n, r, rT, dy = 6, 3, 5, 4
    rng = np.random.default_rng(13)
    U = random_dense_basis(n, r, 12, 14)
    basis = prior.DenseBasis(n, 0.1, 1.0, U)
    A_T = rng.standard_normal((dy, rT))
    b_T = rng.standard_normal(dy)
    A_s = A_T @ U[:rT] + 0.3 * rng.standard_normal((dy, r))   # roughly the true model on span(U)
    y = rng.standard_normal(dy)
    nv = np.full(dy, 0.7 ** 2)
    prob = mcmc.Problem([("linear", A_s, b_T)], y, nv, 0.8, seed=15, request_id=1)
    tm = da.TrueModel([("linear", A_T, b_T)], basis=basis)
    Gi = np.diag(1.0 / nv)
    Sigma = np.linalg.inv(np.eye(rT) + A_T.T @ Gi @ A_T)
    mu = Sigma @ A_T.T @ Gi @ (y - b_T)
    C, N = 16, 3000
    ds = da.init_da_state(prob, tm, rng.standard_normal((C, r)), rng.standard_normal((C, n * n)))
    st = ds.chain
    Z = np.empty((N, C, rT))
    for t in range(N):
        da.transition_da(prob, tm, ds)
        Z[t] = basis.full(st.x, st.z)[:, :rT]
    tr = Z[N // 5:]
    e = stats.ess_per_coordinate(tr)
    n_eff = tr.shape[0] * C * e
    mcse = np.sqrt(np.diag(Sigma) / n_eff)
    F = tr.reshape(-1, rT)
    assert np.all(np.abs(F.mean(0) - mu) < 4.5 * mcse)
    assert np.all(np.abs(F.var(0) - np.diag(Sigma)) < 5.0 * np.sqrt(2.0 / n_eff) * np.diag(Sigma)
                  + 5 * mcse * np.abs(F.mean(0) - mu))
