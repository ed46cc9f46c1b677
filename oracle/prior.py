"""Grid Matern prior and its Karhunen-Loeve reduced basis (oracle; test infrastructure).

Paper basis:
* Gaussian prior N(0, C_pr) (Sec. 2.1, Assumption 2); the Matern-type covariance
  C_pr = (-gamma Lap + delta I)^-2 used in the experiments (Sec. 7.1 prior).
* KLE reduced basis (Sec. 4.2): eigenpairs (lambda_j, eta_j) of C_pr with
  M-orthonormal eta_j and decreasing lambda_j; H_mu-orthonormal basis
  psi_j = sqrt(lambda_j) eta_j.
* Encoder / decoder (Sec. 4, eq. projector): Psi_r^* m = sum_j <m, psi_j>_{C_pr^-1} e_j,
  Psi_r x = sum_j x_j psi_j, with Psi_r^* Psi_r = I_r.

Discretisation (a reading; the paper uses finite elements):
* n x n nodes on the unit square, h = 1/(n-1), flat index p = j*n + i with i the
  x-index (fastest).
* -Lap_h = (I (x) L1 + L1 (x) I) / h^2 where L1 is the 1-D zero-flux (Neumann)
  graph Laplacian: tridiagonal, -1 off the diagonal, 2 on the diagonal except 1
  at both ends. A = gamma(-Lap_h) + delta I, C_pr = A^-2 (l2 nodal inner product).
* Closed form: L1 q_k = mu_k q_k with mu_k = 4 sin^2(pi k / 2n) and the DCT-II
  vectors q_k(i) = sqrt((2 - [k=0]) / n) cos(pi k (i + 1/2) / n); the 2-D modes are
  q_k1 (x) q_k2 (x-index k1) with a = gamma (mu_k1 + mu_k2)/h^2 + delta, lambda = a^-2.
* KLE order: by decreasing lambda, i.e. increasing mu_k1 + mu_k2, with exact ties
  (the symmetric pairs (k1,k2)/(k2,k1)) broken by (k1, k2) ascending. The sum is
  formed as mu[min] + mu[max] so swapped pairs compare equal bit for bit.
* Whitened coordinates z = Lambda^-1/2 Q^T m: the prior becomes N(0, I); the
  reduced state is x = z[:r] and the complement z[r:].
"""
from __future__ import annotations

import numpy as np


def laplacian_1d_neumann(n: int) -> np.ndarray:
    """Dense L1: tridiagonal (-1, 2, -1) with the two end diagonal entries set to 1."""
    L = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    L[0, 0] = 1.0
    L[-1, -1] = 1.0
    return L


def matern_operator(n: int, gamma: float, delta: float) -> np.ndarray:
    """Dense A = gamma(-Lap_h) + delta I on the n x n grid (small n only)."""
    h = 1.0 / (n - 1)
    L1 = laplacian_1d_neumann(n)
    I = np.eye(n)
    lap = (np.kron(I, L1) + np.kron(L1, I)) / h ** 2
    return gamma * lap + delta * np.eye(n * n)


def prior_covariance_dense(n: int, gamma: float, delta: float) -> np.ndarray:
    """Dense C_pr = A^-2 (small n only)."""
    A = matern_operator(n, gamma, delta)
    Ainv = np.linalg.inv(A)
    return Ainv @ Ainv


def mu_1d(n: int) -> np.ndarray:
    """Eigenvalues of L1: mu_k = 4 sin^2(pi k / (2n)), k = 0..n-1."""
    k = np.arange(n)
    return 4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2


def q_1d(n: int) -> np.ndarray:
    """Columns q_k of the DCT-II basis: Q[i, k] = sqrt((2 - [k=0])/n) cos(pi k (i+1/2)/n)."""
    i = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    scale = np.where(k == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))
    return scale * np.cos(np.pi * k * (i + 0.5) / n)


def kle_order(n: int):
    """All n^2 modes in KLE order: arrays (k1, k2, musum) sorted by (musum, k1, k2)."""
    mu = mu_1d(n)
    k1, k2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    k1 = k1.ravel()
    k2 = k2.ravel()
    lo = np.minimum(k1, k2)
    hi = np.maximum(k1, k2)
    musum = mu[lo] + mu[hi]
    order = np.lexsort((k2, k1, musum))
    return k1[order], k2[order], musum[order]


def kle_eigenvalues(n: int, gamma: float, delta: float):
    """(k1, k2, lambda) for all modes in KLE order."""
    h = 1.0 / (n - 1)
    k1, k2, musum = kle_order(n)
    a = gamma * musum / h ** 2 + delta
    return k1, k2, 1.0 / a ** 2


def kle_vectors(n: int, k1: np.ndarray, k2: np.ndarray) -> np.ndarray:
    """l2-orthonormal eigenvectors eta for the listed modes, shape (n^2, len(k1))."""
    Q = q_1d(n)
    # eta[p = j*n + i, m] = q_k2(j) q_k1(i)
    return np.einsum("jm,im->jim", Q[:, k2], Q[:, k1]).reshape(n * n, len(k1))


class KLEBasis:
    """Rank-r KLE basis of the grid Matern prior (Sec. 4.2).

    Attributes: lam (r,), eta (d_m, r), dec = eta * sqrt(lam) (the decoder Psi_r),
    enc = (eta / sqrt(lam))^T (the encoder Psi_r^* in nodal coordinates),
    lam_all (d_m,) all eigenvalues in KLE order, var_perp (d_m,) the pointwise prior
    variance of the complement, sum_{k >= r} lambda_k eta_k(p)^2.
    """

    def __init__(self, n: int, gamma: float, delta: float, r: int):
        self.n, self.gamma, self.delta, self.r = n, gamma, delta, r
        self.d_m = n * n
        k1, k2, lam = kle_eigenvalues(n, gamma, delta)
        self.k1_all, self.k2_all, self.lam_all = k1, k2, lam
        self.k1, self.k2, self.lam = k1[:r], k2[:r], lam[:r]
        self.eta = kle_vectors(n, self.k1, self.k2)
        self.dec = self.eta * np.sqrt(self.lam)[None, :]
        self.enc = (self.eta / np.sqrt(self.lam)[None, :]).T
        self.var_perp = self._complement_variance()

    def _complement_variance(self) -> np.ndarray:
        """sum over modes k >= r of lambda_k eta_k(p)^2, via the separable structure."""
        n = self.n
        Q2 = q_1d(n) ** 2  # Q2[i, k] = q_k(i)^2
        lamgrid = np.zeros((n, n))  # lamgrid[k1, k2]
        lamgrid[self.k1_all[self.r:], self.k2_all[self.r:]] = self.lam_all[self.r:]
        # V[j, i] = sum_{k1,k2} q_k1(i)^2 lam[k1,k2] q_k2(j)^2
        V = Q2 @ lamgrid @ Q2.T  # V[i, j]
        return V.T.reshape(-1)

    # --- whitened <-> nodal maps -------------------------------------------------
    def encode(self, m: np.ndarray) -> np.ndarray:
        """Reduced coordinates x = Psi_r^* m for fields m (..., d_m)."""
        return m @ self.enc.T

    def decode(self, x: np.ndarray) -> np.ndarray:
        """Psi_r x for reduced coordinates x (..., r)."""
        return x @ self.dec.T

    def whiten_full(self, m: np.ndarray) -> np.ndarray:
        """All d_m whitened coordinates z = Lambda^-1/2 Q^T m in KLE order (..., d_m)."""
        n = self.n
        Q = q_1d(n)
        M = m.reshape(m.shape[:-1] + (n, n))  # M[..., j, i]
        Z = np.einsum("...ji,ik,jl->...kl", M, Q, Q)  # Z[k1, k2] = sum q_k1(i) q_k2(j) M[j,i]
        coef = Z[..., self.k1_all, self.k2_all]
        return coef / np.sqrt(self.lam_all)

    def unwhiten_full(self, z: np.ndarray) -> np.ndarray:
        """Nodal field m = Q Lambda^1/2 z from all d_m whitened coordinates."""
        n = self.n
        Q = q_1d(n)
        Z = np.zeros(z.shape[:-1] + (n, n))
        Z[..., self.k1_all, self.k2_all] = z * np.sqrt(self.lam_all)
        M = np.einsum("...kl,ik,jl->...ji", Z, Q, Q)
        return M.reshape(z.shape[:-1] + (n * n,))


def prior_pointwise_variance(n: int, gamma: float, delta: float) -> np.ndarray:
    """diag(C_pr) on the grid: sum over all modes of lambda_k eta_k(p)^2 (separable)."""
    k1, k2, lam = kle_eigenvalues(n, gamma, delta)
    Q2 = q_1d(n) ** 2
    lamgrid = np.zeros((n, n))
    lamgrid[k1, k2] = lam
    return (Q2 @ lamgrid @ Q2.T).T.reshape(-1)


class DenseBasis:
    """A dense reduced basis given in whitened KLE coordinates (Sec. 4.2): U (d_m, r) with
    orthonormal columns, psi_j = Q Lambda^1/2 u_j, which is H_mu-orthonormal (the Cameron-
    Martin inner product is Euclidean in whitened coordinates). A DIS basis (eq.
    jtj_eigenvalue) is of this form, with eigenvalues lam_dis (eq. dis_gnh) attached.

    Encoder x = U^T z for the whitened coordinates z of m; decoder Psi_r x = Q Lambda^1/2 U x
    (eq. projector); the complement of z is (I - U U^T) z. Attributes as KLEBasis: dec
    (d_m, r) = Psi_r in nodal coordinates and var_perp (d_m), the pointwise prior variance
    of the complement, diag(C_pr) - sum_j psi_j(p)^2."""

    def __init__(self, n: int, gamma: float, delta: float, U: np.ndarray, lam_dis=None):
        self.n, self.gamma, self.delta = n, gamma, delta
        self.d_m = n * n
        self.U = np.asarray(U, dtype=np.float64)
        assert self.U.shape[0] == self.d_m
        self.r = self.U.shape[1]
        self.lam_dis = None if lam_dis is None else np.asarray(lam_dis, dtype=np.float64)
        self.kle = KLEBasis(n, gamma, delta, 1)  # the full whitening transform (every mode)
        self.dec = self.kle.unwhiten_full(self.U.T).T
        self.var_perp = prior_pointwise_variance(n, gamma, delta) - np.sum(self.dec ** 2, axis=1)

    def encode(self, m: np.ndarray) -> np.ndarray:
        """Reduced coordinates x = U^T z(m) of fields m (..., d_m)."""
        return self.kle.whiten_full(m) @ self.U

    def decode(self, x: np.ndarray) -> np.ndarray:
        return x @ self.dec.T

    def project_complement(self, w: np.ndarray) -> np.ndarray:
        """(I - U U^T) w for whitened vectors w (..., d_m)."""
        return w - (w @ self.U) @ self.U.T

    def full(self, x: np.ndarray, w: np.ndarray) -> np.ndarray:
        """The whitened coordinates of the full parameter U x + (I - U U^T) w (Alg. 1's
        assembly Psi_r x + m_perp - Psi_r Psi_r^* m_perp, in whitened coordinates)."""
        return x @ self.U.T + self.project_complement(w)
