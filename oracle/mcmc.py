"""DINO-mMALA in reduced coordinates: Alg. 1 first stage + the splitting proposition of Sec. 5.3 (oracle; test infrastructure).

State of a chain: reduced whitened KLE coordinates x in R^r and the complement
coordinates z_perp in R^(d_m - r) (prior N(0, I) in both). Everything the MH
decision depends on lives in R^r (Sec. 5.4: the first stage runs entirely in the
reduced coefficient space); the complement follows the pCN move of the splitting proposition of Sec. 5.3.

Readings of the paper taken here (listed with reasons in the design notes):
* Observable basis: the network outputs physical observables and each problem has
  its own diagonal noise covariance Gamma = diag(noise_var); the whitened quantities
  are V^* y -> Gamma^-1/2 y and V^* G~ -> Gamma^-1/2 f (equivalent to V = Gamma^1/2).
  A problem observes the first d_y outputs of the network.
* Reduced ppg sign (Sec. 5.1, eq. surrogate_rppg): the ppg of the misfit is
  J^T Gamma^-1 (f - y), as in eq. ppg; the printed form has the opposite sign.
* The determinant factor of the reduced RN derivative (Sec. 5.4) multiplies the
  exponential, prod_j (d_j + 1)^(1/2), as in eq. mmala_trr; the printed form adds it.
* The complement move is the pCN move of the splitting proposition of Sec. 5.3 (item 1), z_perp <- s z_perp + beta zeta.
* The noise of the reduced proposal (eq. reduced_space_sampling) is mapped through the
  Cholesky factor L of I + H (L L^T = I + H) instead of P (d+1)^-1/2: the same law,
  N(0, (1 - s^2)(I + H)^-1), with a unique factor, so both sides draw the same point.
  With factor="dual" (observation-space form, for d_y < r) the same law is drawn as
  beta (I + H)^-1 (xi_1 + B^T xi_2), xi_1 in R^r, xi_2 in R^d_y, B = Gamma^-1/2 J: its
  covariance is (I + H)^-1 (I + B^T B) (I + H)^-1 = (I + H)^-1, and (I + H)^-1 can then
  be applied through the d_y x d_y matrix I + B B^T (Woodbury). xi_1 and xi_2 are the
  first r and the next d_y normals of the proposal stream.
* The acceptance uses the surrogate misfit (the first-stage ratio eq. da_dino_trr_1);
  accept iff log xi_1 <= log rho (Alg. 1 rejects iff alpha < xi_1, so ties accept).
* A proposal whose misfit is not finite or whose I + H is not positive definite is
  rejected and counted.
* The pCN baseline (method "pcn") uses the same s = (4 - dt)/(4 + dt): it is the
  mMALA proposal with H = 0 and g = 0, x+ = s x + beta xi (xi: the first r normals of
  the proposal stream), accepted with exp(Phi(x) - Phi(x+)).
* The LA-pCN baseline (method "lapcn", eq. MAP): the printed proposal mean m_MAP - s m
  is read as m_MAP + s (m - m_MAP), the pCN move about the MAP with the Laplace
  covariance, which is reversible with respect to the Laplace approximation
  N(m_MAP, C_post(m_MAP)); the printed mean is not. In whitened reduced coordinates:
  x+ = x_map + s (x - x_map) + beta L^-T xi with L L^T = I + H(x_map), and
  log rho = Phi(x) - Phi(x+) + (|x|^2 - |x+|^2)/2 + (|L^T(x+ - x_map)|^2 - |L^T(x - x_map)|^2)/2
  (target over Laplace density). The complement keeps its pCN move (the Laplace
  approximation equals the prior there).
* The DIS-mMALA baseline (method "dis_mmala", Sec. 6.1 with eq. dis_gnh) is the mMALA
  transition with the metric fixed at the DIS approximation of the expected ppGNH, which is
  diag(lam) in the coordinates of a DIS basis (lam its eigenvalues), and the ppg kept.
* The MALA baseline (method "mala") is the mMALA transition with the metric removed
  (H = 0, so d = 0, P = L = I and B = 0 in the noise mapping) and the ppg kept: x+ =
  s x - (1 - s) g + beta xi, and rho_0 keeps its ppg terms only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import network, philox


@dataclass
class Problem:
    """One inverse problem: network, data y (d_y,), noise variances (d_y,), step size."""
    layers: list
    y: np.ndarray
    noise_var: np.ndarray
    dt: float
    seed: int = 0
    request_id: int = 0
    factor: str = "primal"   # proposal noise mapping: "primal" (L^-T xi) or "dual"
    method: str = "mmala"    # "mmala"; baselines of Sec. 6.1: "pcn" (no metric, no ppg), "mala" (ppg only),
                             # "lapcn" (metric fixed at the MAP, no ppg), "dis_mmala" (fixed DIS metric, ppg)
    fixed: tuple = None      # "lapcn": (x_map (r,), lower Cholesky factor of I + H(x_map) (r, r));
                             # "dis_mmala": the DIS eigenvalues lam (r,) (the metric diag(lam))

    @property
    def d_y(self) -> int:
        return len(self.y)

    @property
    def s(self) -> float:
        """s = (4 - dt)/(4 + dt) (Sec. 2.7, eq. mmala)."""
        return (4.0 - self.dt) / (4.0 + self.dt)

    @property
    def beta(self) -> float:
        """sqrt(1 - s^2)."""
        return math.sqrt(1.0 - self.s ** 2)


@dataclass
class Cache:
    """What Alg. 1 keeps "known at m_j": misfit, reduced ppg, ppGNH and its factors."""
    f: np.ndarray        # (C, d_y) network output at x
    phi: np.ndarray      # (C,) surrogate reduced misfit
    g: np.ndarray        # (C, r) reduced ppg
    H: np.ndarray        # (C, r, r) reduced ppGNH
    d: np.ndarray        # (C, r) eigenvalues of H (eq. surrogate_eigendecomposition)
    P: np.ndarray        # (C, r, r) eigenvectors of H
    L: np.ndarray        # (C, r, r) lower Cholesky factor of I + H
    ok: np.ndarray       # (C,) finite misfit and positive definite I + H
    B: np.ndarray = None # (C, d_y, r) whitened reduced Jacobian Gamma^-1/2 J


def geometry(prob: Problem, x: np.ndarray) -> Cache:
    """Surrogate misfit, reduced ppg and reduced ppGNH at x (Sec. 5.1), plus the
    eigendecomposition of H (Sec. 5.2) and the Cholesky factor of I + H."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    C, r = x.shape
    f_full, _ = network.forward(prob.layers, x)
    J_full = network.jacobian_reverse(prob.layers, x)
    dy = prob.d_y
    f = f_full[:, :dy]
    J = J_full[:, :dy, :]
    w = 1.0 / np.sqrt(np.asarray(prob.noise_var, dtype=np.float64))
    Jw = J * w[None, :, None]                      # V^* J~_r : whitened reduced Jacobian
    return cache_from_jacobian(prob, f, Jw)


def cache_from_jacobian(prob: Problem, f: np.ndarray, Jw: np.ndarray) -> Cache:
    """The cache of Sec. 5.1-5.2 from the network output f (C, d_y) and a whitened reduced
    Jacobian Jw = Gamma^-1/2 J (C, d_y, r) given as data (geometry() passes the network's
    own; a caller may pass a rounded copy to evaluate the method on it)."""
    f = np.atleast_2d(np.asarray(f, dtype=np.float64))
    Jw = np.asarray(Jw, dtype=np.float64)
    C, r = Jw.shape[0], Jw.shape[2]
    w = 1.0 / np.sqrt(np.asarray(prob.noise_var, dtype=np.float64))
    res = (prob.y[None, :] - f) * w[None, :]       # V^* y - f_NN (whitened)
    phi = 0.5 * np.sum(res * res, axis=1)          # eq. (reduced data misfit)
    g = -np.einsum("cir,ci->cr", Jw, res)          # J^T Gamma^-1 (f - y)  (sign reading)
    H = np.einsum("cir,cis->crs", Jw, Jw)          # eq. surrogate_rppgnh
    d = np.zeros((C, r))
    P = np.zeros((C, r, r))
    L = np.zeros((C, r, r))
    ok = np.isfinite(phi) & np.all(np.isfinite(g), axis=1)
    for c in range(C):
        if not ok[c] or not np.all(np.isfinite(H[c])):
            ok[c] = False
            continue
        d[c], P[c] = np.linalg.eigh(H[c])
        try:
            L[c] = np.linalg.cholesky(np.eye(r) + H[c])
        except np.linalg.LinAlgError:
            ok[c] = False
    return Cache(f=f, phi=phi, g=g, H=H, d=d, P=P, L=L, ok=ok, B=Jw)


def misfit(prob: Problem, x: np.ndarray):
    """Network output f (C, d_y) and surrogate reduced misfit phi (C,) at x, without
    derivatives (Sec. 5.1): all that the pCN baseline evaluates per proposal."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    f_full, _ = network.forward(prob.layers, x)
    f = f_full[:, :prob.d_y]
    w = 1.0 / np.sqrt(np.asarray(prob.noise_var, dtype=np.float64))
    res = (prob.y[None, :] - f) * w[None, :]
    return f, 0.5 * np.sum(res * res, axis=1)


def without_metric(c: Cache) -> Cache:
    """The cache with the Gauss-Newton metric removed (H = 0: d = 0, P = L = I, B = 0)
    and the misfit and ppg kept: the geometry the MALA baseline proposes with (the MALA
    row of the baselines of Sec. 6.1: gradient, no Hessian)."""
    C, r = c.g.shape
    eye = np.broadcast_to(np.eye(r), (C, r, r)).copy()
    return Cache(f=c.f, phi=c.phi, g=c.g, H=np.zeros((C, r, r)), d=np.zeros((C, r)), P=eye, L=eye.copy(),
                 ok=np.isfinite(c.phi) & np.all(np.isfinite(c.g), axis=1),
                 B=None if c.B is None else np.zeros_like(c.B))


def with_diagonal_metric(c: Cache, lam: np.ndarray) -> Cache:
    """The cache with the Gauss-Newton metric replaced by the fixed diag(lam) and the misfit
    and ppg kept: the geometry DIS-mMALA proposes with (the DIS-mMALA row of the baselines
    of Sec. 6.1: the DIS approximation of the expected ppGNH, eq. dis_gnh, which is diagonal
    in the coordinates of a DIS basis, with its eigenvalues lam, and the gradient)."""
    C, r = c.g.shape
    lam = np.asarray(lam, dtype=np.float64)
    H = np.broadcast_to(np.diag(lam), (C, r, r)).copy()
    L = np.broadcast_to(np.diag(np.sqrt(1.0 + lam)), (C, r, r)).copy()
    return Cache(f=c.f, phi=c.phi, g=c.g, H=H, d=np.broadcast_to(lam, (C, r)).copy(),
                 P=np.broadcast_to(np.eye(r), (C, r, r)).copy(), L=L,
                 ok=np.isfinite(c.phi) & np.all(np.isfinite(c.g), axis=1),
                 B=None if c.B is None else np.zeros_like(c.B))


def method_geometry(prob: Problem, x: np.ndarray) -> Cache:
    """The geometry a transition of prob.method proposes and accepts with."""
    c = geometry(prob, x)
    if prob.method == "mala":
        return without_metric(c)
    if prob.method == "dis_mmala":
        return with_diagonal_metric(c, prob.fixed)
    return c


def propose(prob: Problem, x: np.ndarray, cache: Cache, xi: np.ndarray) -> np.ndarray:
    """Reduced proposal of the splitting proposition of Sec. 5.3, item 2 (eq. reduced_space_sampling):

        x+ = P diag((d+s)/(d+1)) P^T x - P diag((1-s)/(d+1)) P^T g + noise,

    noise = sqrt(1 - s^2) L^-T xi (Cholesky reading of P diag((1-s^2)/(d+1))^1/2 xi), or,
    with factor "dual", sqrt(1 - s^2) (I + H)^-1 (xi_1 + B^T xi_2) (xi of length r + d_y)."""
    s, beta = prob.s, prob.beta
    C, r = x.shape
    out = np.empty_like(x)
    for c in range(C):
        d, P = cache.d[c], cache.P[c]
        mean = P @ (((d + s) / (d + 1.0)) * (P.T @ x[c])) - P @ (((1.0 - s) / (d + 1.0)) * (P.T @ cache.g[c]))
        if prob.factor == "dual":
            w = xi[c, :r] + cache.B[c].T @ xi[c, r:]
            noise = beta * np.linalg.solve(np.eye(r) + cache.H[c], w)
        else:
            noise = beta * sla.solve_triangular(cache.L[c], xi[c], lower=True, trans="T")
        out[c] = mean + noise
    return out


def log_rho0(prob: Problem, m1: np.ndarray, m2: np.ndarray, cache1: Cache) -> np.ndarray:
    """log of the reduced RN derivative rho~_0,r(m1, m2) of the surrogate mMALA proposal
    with respect to pCN (Sec. 5.4), evaluated with the geometry cached at m1:

        -(dt/8) || D P^T m1 - P^T g ||^2_{(D+I)^-1} + (sqrt(dt)/2) mhat^T (H m1 - g)
        - (1/2) ||mhat||^2_H + (1/2) sum_j log(d_j + 1),   mhat = (m2 - s m1)/sqrt(1 - s^2)."""
    dt, s, beta = prob.dt, prob.s, prob.beta
    C = m1.shape[0]
    out = np.empty(C)
    for c in range(C):
        d, P, g, H = cache1.d[c], cache1.P[c], cache1.g[c], cache1.H[c]
        a = d * (P.T @ m1[c]) - P.T @ g
        t1 = -(dt / 8.0) * np.sum(a * a / (d + 1.0))
        mhat = (m2[c] - s * m1[c]) / beta
        t2 = (math.sqrt(dt) / 2.0) * (mhat @ (H @ m1[c] - g))
        t3 = -0.5 * (mhat @ (H @ mhat))
        t4 = 0.5 * np.sum(np.log(d + 1.0))
        out[c] = t1 + t2 + t3 + t4
    return out


def log_rho0_terms(prob: Problem, m1: np.ndarray, m2: np.ndarray, cache1: Cache) -> np.ndarray:
    """The four terms of log rho~_0,r(m1, m2) (Sec. 5.4) as columns (C, 4), in the order of
    log_rho0's docstring; their sum is log_rho0. A caller bounds rounding in the sum by
    the magnitudes of the terms that cancel in it."""
    dt, s, beta = prob.dt, prob.s, prob.beta
    C = m1.shape[0]
    out = np.empty((C, 4))
    for c in range(C):
        d, P, g, H = cache1.d[c], cache1.P[c], cache1.g[c], cache1.H[c]
        a = d * (P.T @ m1[c]) - P.T @ g
        mhat = (m2[c] - s * m1[c]) / beta
        out[c] = [-(dt / 8.0) * np.sum(a * a / (d + 1.0)), (math.sqrt(dt) / 2.0) * (mhat @ (H @ m1[c] - g)),
                  -0.5 * (mhat @ (H @ mhat)), 0.5 * np.sum(np.log(d + 1.0))]
    return out


def log_rho1(prob: Problem, x: np.ndarray, cache_x: Cache, xp: np.ndarray, cache_p: Cache) -> np.ndarray:
    """log of the first-stage transition-rate ratio rho^(1)_r(x, x+) (eq. da_dino_trr_1)."""
    return (cache_x.phi - cache_p.phi
            + log_rho0(prob, xp, x, cache_p) - log_rho0(prob, x, xp, cache_x))


@dataclass
class ChainState:
    x: np.ndarray                 # (C, r)
    z: np.ndarray | None          # (C, d_m - r) complement, or None when not tracked
    cache: Cache
    step: int = 0                 # global step counter of the stream layout
    accepts: np.ndarray = None
    failures: np.ndarray = None
    chains: np.ndarray = None     # chain indices used in the stream counter

    def __post_init__(self):
        C = self.x.shape[0]
        if self.accepts is None:
            self.accepts = np.zeros(C, dtype=np.int64)
        if self.failures is None:
            self.failures = np.zeros(C, dtype=np.int64)
        if self.chains is None:
            self.chains = np.arange(C)


def init_state(prob: Problem, x0: np.ndarray, z0: np.ndarray | None = None, chains=None) -> ChainState:
    x0 = np.array(x0, dtype=np.float64)
    return ChainState(x=x0, z=None if z0 is None else np.array(z0, dtype=np.float64),
                      cache=method_geometry(prob, x0), chains=None if chains is None else np.asarray(chains))


def _select(cache_a: Cache, cache_b: Cache, mask: np.ndarray) -> Cache:
    def pick(a, b):
        m = mask.reshape((-1,) + (1,) * (a.ndim - 1))
        return np.where(m, b, a)
    return Cache(**{k: pick(getattr(cache_a, k), getattr(cache_b, k)) for k in cache_a.__dataclass_fields__})


@dataclass
class StepRecord:
    xp: np.ndarray
    cache_p: Cache
    log_rho: np.ndarray
    log_u: np.ndarray
    accept: np.ndarray


def transition(prob: Problem, st: ChainState, xi=None, u=None, zeta=None) -> StepRecord:
    """One Markov transition for every chain (Alg. 1 first stage, the splitting proposition of Sec. 5.3).

    xi (C, r), u (C,) and zeta (C, d_m - r) default to the Philox streams at the
    current step; pass them to evaluate the transition at given draws."""
    if prob.method == "pcn":
        return transition_pcn(prob, st, xi, u, zeta)
    if prob.method == "lapcn":
        return transition_lapcn(prob, st, xi, u, zeta)
    C, r = st.x.shape
    if xi is None:
        count = r + prob.d_y if prob.factor == "dual" else r
        xi = philox.normals(prob.seed, prob.request_id, philox.STREAM_XI, st.step, st.chains, count)
    if u is None:
        u = philox.uniforms(prob.seed, prob.request_id, st.step, st.chains)
    # Alg. 1: reduced proposal sampling, surrogate evaluation at x+, first-stage ratio
    xp = propose(prob, st.x, st.cache, xi)
    cp = method_geometry(prob, xp)
    lr = log_rho1(prob, st.x, st.cache, xp, cp)
    lr = np.where(cp.ok & np.isfinite(lr), lr, -np.inf)
    log_u = np.log(u)
    acc = log_u <= lr
    st.failures += (~cp.ok).astype(np.int64)
    _move_complement(prob, st, acc, zeta)
    st.x = np.where(acc[:, None], xp, st.x)
    st.cache = _select(st.cache, cp, acc)
    st.accepts += acc.astype(np.int64)
    st.step += 1
    return StepRecord(xp=xp, cache_p=cp, log_rho=lr, log_u=log_u, accept=acc)


def _move_complement(prob: Problem, st: ChainState, acc: np.ndarray, zeta) -> None:
    """The pCN move of the complement (splitting proposition of Sec. 5.3, item 1), realised
    on accepted moves only."""
    if st.z is None or not np.any(acc):
        return
    idx = np.nonzero(acc)[0]
    if zeta is None:
        zeta_a = philox.normals(prob.seed, prob.request_id, philox.STREAM_COMPLEMENT, st.step,
                                st.chains[idx], st.z.shape[1])
    else:
        zeta_a = zeta[idx]
    st.z[idx] = prob.s * st.z[idx] + prob.beta * zeta_a


def transition_pcn(prob: Problem, st: ChainState, xi=None, u=None, zeta=None) -> StepRecord:
    """One transition of the pCN baseline for every chain (Sec. 2.6, eq. pCN_proposal and
    its transition rate ratio; the pCN row of the table of baselines in Sec. 6.1).

    In whitened coordinates the prior is N(0, I), so the proposal N(s m, (1 - s^2) C_pr)
    reads x+ = s x + beta xi in R^r and, for the complement, the same move as in the
    splitting proposition. The proposal is prior-reversible, so the ratio is
    exp(Phi(x) - Phi(x+)). s = (4 - dt)/(4 + dt) as for mMALA: it is the mMALA proposal
    with the geometry removed (H = 0, g = 0). xi (C, r): the first r normals of the
    proposal stream. The cache keeps f and phi current; its derivative fields are those
    of the initial states."""
    C, r = st.x.shape
    if xi is None:
        xi = philox.normals(prob.seed, prob.request_id, philox.STREAM_XI, st.step, st.chains, r)
    if u is None:
        u = philox.uniforms(prob.seed, prob.request_id, st.step, st.chains)
    xp = prob.s * st.x + prob.beta * xi[:, :r]
    fp, phip = misfit(prob, xp)
    lr = st.cache.phi - phip
    good = np.isfinite(lr)
    lr = np.where(good, lr, -np.inf)
    log_u = np.log(u)
    acc = log_u <= lr
    st.failures += (~good).astype(np.int64)
    _move_complement(prob, st, acc, zeta)
    st.x = np.where(acc[:, None], xp, st.x)
    st.cache.phi = np.where(acc, phip, st.cache.phi)
    st.cache.f = np.where(acc[:, None], fp, st.cache.f)
    st.accepts += acc.astype(np.int64)
    st.step += 1
    cp = Cache(f=fp, phi=phip, g=None, H=None, d=None, P=None, L=None, ok=good)
    return StepRecord(xp=xp, cache_p=cp, log_rho=lr, log_u=log_u, accept=acc)


def transition_lapcn(prob: Problem, st: ChainState, xi=None, u=None, zeta=None) -> StepRecord:
    """One transition of the LA-pCN baseline (eq. MAP and the LA-pCN proposal after it;
    the LA-pCN row of the baselines of Sec. 6.1), with the mean read as
    x_map + s (x - x_map). prob.fixed = (x_map, L_map)."""
    x_map, L_map = prob.fixed
    C, r = st.x.shape
    if xi is None:
        xi = philox.normals(prob.seed, prob.request_id, philox.STREAM_XI, st.step, st.chains, r)
    if u is None:
        u = philox.uniforms(prob.seed, prob.request_id, st.step, st.chains)
    noise = sla.solve_triangular(L_map, xi[:, :r].T, lower=True, trans="T").T
    xp = x_map + prob.s * (st.x - x_map) + prob.beta * noise
    fp, phip = misfit(prob, xp)

    def log_target_over_laplace(v, phi):
        q = (v - x_map) @ L_map          # rows: L^T (v - x_map)
        return -phi - 0.5 * np.sum(v * v, axis=1) + 0.5 * np.sum(q * q, axis=1)

    lr = log_target_over_laplace(xp, phip) - log_target_over_laplace(st.x, st.cache.phi)
    good = np.isfinite(lr)
    lr = np.where(good, lr, -np.inf)
    log_u = np.log(u)
    acc = log_u <= lr
    st.failures += (~good).astype(np.int64)
    _move_complement(prob, st, acc, zeta)
    st.x = np.where(acc[:, None], xp, st.x)
    st.cache.phi = np.where(acc, phip, st.cache.phi)
    st.cache.f = np.where(acc[:, None], fp, st.cache.f)
    st.accepts += acc.astype(np.int64)
    st.step += 1
    cp = Cache(f=fp, phi=phip, g=None, H=None, d=None, P=None, L=None, ok=good)
    return StepRecord(xp=xp, cache_p=cp, log_rho=lr, log_u=log_u, accept=acc)


def run(prob: Problem, st: ChainState, n_steps: int, trace: bool = True):
    """Advance every chain n_steps; returns the reduced trace (n_steps, C, r) and
    the misfit trace (n_steps, C) of the states after each step."""
    C, r = st.x.shape
    xs = np.empty((n_steps, C, r)) if trace else None
    phis = np.empty((n_steps, C)) if trace else None
    for t in range(n_steps):
        transition(prob, st)
        if trace:
            xs[t] = st.x
            phis[t] = st.cache.phi
    return xs, phis
