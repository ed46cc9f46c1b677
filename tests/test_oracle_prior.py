"""Pins for oracle/prior.py: the closed-form KLE against dense eigensolves of the grid
operator, orthonormality, Psi_r^* Psi_r = I (eq. projector), white encoded prior
(eq. encoded_white_noise) and the complement variance against the dense covariance."""
import numpy as np
import pytest

from oracle import prior


@pytest.mark.parametrize("n", [5, 9, 16])
def test_1d_closed_form_matches_eigh(n):
    L1 = prior.laplacian_1d_neumann(n)
    w = np.linalg.eigvalsh(L1)
    np.testing.assert_allclose(np.sort(prior.mu_1d(n)), w, atol=1e-13)
    Q = prior.q_1d(n)
    np.testing.assert_allclose(L1 @ Q, Q * prior.mu_1d(n)[None, :], atol=1e-13)
    np.testing.assert_allclose(Q.T @ Q, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("n,gamma,delta", [(9, 0.1, 1.0), (12, 0.03, 3.33), (17, 0.1, 1.0)])
def test_kle_matches_dense_covariance(n, gamma, delta):
    C = prior.prior_covariance_dense(n, gamma, delta)
    k1, k2, lam = prior.kle_eigenvalues(n, gamma, delta)
    w = np.sort(np.linalg.eigvalsh(C))[::-1]
    np.testing.assert_allclose(lam, w, rtol=1e-10, atol=1e-15)
    eta = prior.kle_vectors(n, k1, k2)
    np.testing.assert_allclose(C @ eta, eta * lam[None, :], atol=1e-12 * lam[0])
    np.testing.assert_allclose(eta.T @ eta, np.eye(n * n), atol=1e-12)
    assert np.all(np.diff(lam) <= 0.0)


def test_tied_subspaces_by_projector():
    """Dense eigh returns an arbitrary rotation inside a tied pair; compare projectors."""
    n = 9
    C = prior.prior_covariance_dense(n, 0.1, 1.0)
    w, V = np.linalg.eigh(C)
    order = np.argsort(w)[::-1]
    w, V = w[order], V[:, order]
    k1, k2, lam = prior.kle_eigenvalues(n, 0.1, 1.0)
    eta = prior.kle_vectors(n, k1, k2)
    i = 0
    while i < 20:
        j = i + 1
        while j < len(lam) and abs(lam[j] - lam[i]) < 1e-12 * lam[i]:
            j += 1
        P1 = eta[:, i:j] @ eta[:, i:j].T
        P2 = V[:, i:j] @ V[:, i:j].T
        np.testing.assert_allclose(P1, P2, atol=1e-9)
        i = j


def test_tie_break_and_cut():
    """The canonical cuts split exact symmetric pairs; the tie-break fixes the order."""
    k1, k2, s = prior.kle_order(33)
    assert (k1[31], k2[31]) == (3, 5) and (k1[32], k2[32]) == (5, 3)
    assert s[31] == s[32]
    k1, k2, s = prior.kle_order(129)
    assert (k1[199], k2[199]) == (8, 13) and (k1[200], k2[200]) == (13, 8)
    # away from exact symmetric ties, consecutive sums are well separated
    for n, r in [(33, 32), (129, 200), (257, 400)]:
        k1, k2, s = prior.kle_order(n)
        head = s[: r + 2]
        gaps = np.diff(head)
        pos = gaps[gaps > 0]
        assert np.min(pos / head[1:][gaps > 0]) > 1e-9


@pytest.mark.parametrize("n,r", [(9, 12), (17, 30)])
def test_encoder_decoder(n, r):
    B = prior.KLEBasis(n, 0.1, 1.0, r)
    np.testing.assert_allclose(B.enc @ B.dec, np.eye(r), atol=1e-12)
    # psi_j are C_pr^-1-orthonormal: dec^T C^-1 dec = I
    C = prior.prior_covariance_dense(n, 0.1, 1.0)
    np.testing.assert_allclose(B.dec.T @ np.linalg.solve(C, B.dec), np.eye(r), atol=1e-8)
    # the encoder is <m, psi_j>_{C^-1}
    m = np.random.default_rng(1).standard_normal(n * n)
    np.testing.assert_allclose(B.encode(m), B.dec.T @ np.linalg.solve(C, m), rtol=1e-8, atol=1e-8)
    # complement variance = diag(C) - sum_j dec_pj^2
    np.testing.assert_allclose(B.var_perp, np.diag(C) - np.sum(B.dec ** 2, axis=1), atol=1e-14)
    z = B.whiten_full(m)
    np.testing.assert_allclose(z[:r], B.encode(m), atol=1e-10)
    np.testing.assert_allclose(B.unwhiten_full(z), m, atol=1e-12)


def test_encoded_prior_is_white():
    """Psi_r^* M ~ N(0, I_r) for M ~ N(0, C_pr), with M drawn by a dense Cholesky of C_pr."""
    n, r = 9, 10
    B = prior.KLEBasis(n, 0.1, 1.0, r)
    C = prior.prior_covariance_dense(n, 0.1, 1.0)
    Lc = np.linalg.cholesky(C + 1e-300 * np.eye(n * n))
    rng = np.random.default_rng(7)
    N = 40000
    M = rng.standard_normal((N, n * n)) @ Lc.T
    X = B.encode(M)
    S = X.T @ X / N
    assert np.max(np.abs(S - np.eye(r))) < 6.0 * np.sqrt(2.0 / N)
