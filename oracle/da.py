"""Delayed acceptance: the second stage of Alg. 1 (oracle; test infrastructure).

The first stage is the surrogate mMALA transition of mcmc.transition (eq.
reduced_space_sampling, eq. da_dino_trr_1). A proposal that passes it is assembled into
a full parameter and judged by the true data misfit (Sec. 2.5, eq. da_second; Sec. 5.4,
eq. da_dino_trr_2):

    rho^(2)(m, m+) = exp(-Phi~(x) - Phi(m+)) / (exp(-Phi~(x+) - Phi(m))),

with Phi~ the surrogate misfit of the reduced coordinates and Phi the true misfit of
the full parameter. The chain keeps the true misfit of its state (Alg. 1, "known at
m_j" item (i)).

True model. The paper's true model is a PDE solve, which is out of scope; its stand-in
here is a second network ("true model") that reads the first r_T >= r whitened KLE
coordinates of the full parameter, z[0:r_T] = (x, z_perp[0:r_T - r]), so that it sees
the complement as well as the reduced part. A problem observes its first d_y outputs
with the problem's noise variances, as the surrogate does.

Readings (listed with reasons in the design notes):
* The full proposal's complement is the pCN move of the splitting proposition of
  Sec. 5.3 (item 1), z_perp+ = s z_perp + beta zeta, drawn only when the first stage
  passes, with the complement stream of the step; Alg. 1's "sample prior" line is read
  through that proposition, as for the first stage (reading 3).
* The second-stage uniform is word 0 of block 0 of stream 5 at (step, chain); accept iff
  log u2 <= log rho^(2) (ties accept, as in the first stage).
* A non-finite true misfit at the full proposal rejects it and is counted as a failure.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import mcmc, network, philox

STREAM_UNIFORM2 = 5


@dataclass
class TrueModel:
    """The true parameter-to-observable map's stand-in: a network on z[0:r_T]. basis: a
    prior.DenseBasis when the reduced basis is dense (else the KLE basis)."""
    layers: list
    basis: object = None

    @property
    def r_T(self) -> int:
        return self.layers[0][1].shape[1]


def true_misfit(prob: mcmc.Problem, tm: TrueModel, x: np.ndarray, z: np.ndarray | None, basis=None) -> np.ndarray:
    """Phi(m) = 1/2 |Gamma^-1/2 (y - G(m))|^2 (eq. data_model and the Gaussian likelihood of
    Sec. 2.1) of full parameters given by reduced coordinates x (C, r) and complement z.
    KLE basis (basis None): z (C, d_m - r) holds the whitened coordinates past r (None when
    r_T = r). Dense basis (prior.DenseBasis): z (C, d_m) is the unprojected complement draw
    w and the full parameter is U x + (I - U U^T) w (Alg. 1's assembly of m+)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    r = x.shape[1]
    extra = tm.r_T - r
    if basis is not None:
        zin = basis.full(x, np.asarray(z, dtype=np.float64))[:, :tm.r_T]
    else:
        zin = x if extra == 0 else np.concatenate([x, np.asarray(z, dtype=np.float64)[:, :extra]], axis=1)
    f, _ = network.forward(tm.layers, zin)
    w = 1.0 / np.sqrt(np.asarray(prob.noise_var, dtype=np.float64))
    res = (prob.y[None, :] - f[:, :prob.d_y]) * w[None, :]
    return 0.5 * np.sum(res * res, axis=1)


def log_rho2(phi_x, phi_true_x, phi_p, phi_true_p) -> np.ndarray:
    """log rho^(2) (eq. da_dino_trr_2): surrogate misfits phi at the state and the
    proposal, true misfits phi_true at the state and the full proposal."""
    return (np.asarray(phi_p) - np.asarray(phi_x)) + (np.asarray(phi_true_x) - np.asarray(phi_true_p))


def second_stage_uniforms(seed: int, request_id: int, step, chain) -> np.ndarray:
    step = np.asarray(step, dtype=np.uint64)
    chain = np.asarray(chain, dtype=np.uint64)
    step, chain = np.broadcast_arrays(step, chain)
    o = philox.philox4x64(np.zeros(step.shape, dtype=np.uint64),
                          np.full(step.shape, STREAM_UNIFORM2, dtype=np.uint64), step, chain, seed, request_id)
    return philox.to_uniform(o[0])


@dataclass
class DAState:
    chain: mcmc.ChainState
    phi_true: np.ndarray           # (C,) true misfit of the current states
    passes: np.ndarray = None      # (C,) first-stage passes (true-model evaluations)

    def __post_init__(self):
        if self.passes is None:
            self.passes = np.zeros(len(self.phi_true), dtype=np.int64)


@dataclass
class DARecord:
    xp: np.ndarray
    log_rho1: np.ndarray
    passed: np.ndarray
    phi_true_p: np.ndarray         # nan where the first stage rejected
    log_rho2: np.ndarray           # nan where the first stage rejected
    accept: np.ndarray


def init_da_state(prob: mcmc.Problem, tm: TrueModel, x0, z0=None, chains=None) -> DAState:
    st = mcmc.init_state(prob, x0, z0, chains=chains)
    return DAState(chain=st, phi_true=true_misfit(prob, tm, st.x, st.z, tm.basis))


def transition_da(prob: mcmc.Problem, tm: TrueModel, ds: DAState, xi=None, u=None, zeta=None, u2=None) -> DARecord:
    """One transition of Alg. 1 for every chain: the first stage (reduced proposal, surrogate
    geometry at x+, eq. da_dino_trr_1) and, for the chains it passes, the full proposal
    (x+, s z_perp + beta zeta), its true misfit and the second stage (eq. da_dino_trr_2).
    Draws default to the Philox streams at the current step."""
    if prob.method != "mmala":
        raise ValueError("delayed acceptance is defined here for the mMALA first stage")
    st = ds.chain
    C, r = st.x.shape
    if xi is None:
        count = r + prob.d_y if prob.factor == "dual" else r
        xi = philox.normals(prob.seed, prob.request_id, philox.STREAM_XI, st.step, st.chains, count)
    if u is None:
        u = philox.uniforms(prob.seed, prob.request_id, st.step, st.chains)
    if u2 is None:
        u2 = second_stage_uniforms(prob.seed, prob.request_id, st.step, st.chains)
    # first stage: reduced proposal, surrogate evaluation at x+, first-stage ratio
    xp = mcmc.propose(prob, st.x, st.cache, xi)
    cp = mcmc.geometry(prob, xp)
    lr1 = mcmc.log_rho1(prob, st.x, st.cache, xp, cp)
    lr1 = np.where(cp.ok & np.isfinite(lr1), lr1, -np.inf)
    passed = np.log(u) <= lr1
    # second stage, for the chains the first stage passed: full proposal, true misfit, ratio
    zp = None
    if st.z is not None:
        zp = st.z.copy()
        idx = np.nonzero(passed)[0]
        if len(idx):
            if zeta is None:
                zeta_a = philox.normals(prob.seed, prob.request_id, philox.STREAM_COMPLEMENT, st.step,
                                        st.chains[idx], st.z.shape[1])
            else:
                zeta_a = zeta[idx]
            zp[idx] = prob.s * st.z[idx] + prob.beta * zeta_a
    phi_tp = np.full(C, np.nan)
    lr2 = np.full(C, np.nan)
    if np.any(passed):
        idx = np.nonzero(passed)[0]
        phi_tp[idx] = true_misfit(prob, tm, xp[idx], None if zp is None else zp[idx], tm.basis)
        lr2[idx] = log_rho2(st.cache.phi[idx], ds.phi_true[idx], cp.phi[idx], phi_tp[idx])
    good2 = passed & np.isfinite(lr2)
    acc = good2 & (np.log(u2) <= np.where(good2, lr2, -np.inf))
    st.failures += (~cp.ok).astype(np.int64) + (passed & ~np.isfinite(lr2)).astype(np.int64)
    ds.passes += passed.astype(np.int64)
    if zp is not None:
        st.z = np.where(acc[:, None], zp, st.z)
    st.x = np.where(acc[:, None], xp, st.x)
    st.cache = mcmc._select(st.cache, cp, acc)
    ds.phi_true = np.where(acc, phi_tp, ds.phi_true)
    st.accepts += acc.astype(np.int64)
    st.step += 1
    return DARecord(xp=xp, log_rho1=lr1, passed=passed, phi_true_p=phi_tp, log_rho2=lr2, accept=acc)


def run_da(prob: mcmc.Problem, tm: TrueModel, ds: DAState, n_steps: int, trace: bool = True):
    """n_steps DA transitions; returns the reduced trace (n, C, r), the first r_T - r
    complement coordinates (n, C, r_T - r) and the true-misfit trace (n, C)."""
    st = ds.chain
    C, r = st.x.shape
    extra = tm.r_T - r
    xs = np.empty((n_steps, C, r)) if trace else None
    zs = np.empty((n_steps, C, extra)) if trace and extra and st.z is not None else None
    phis = np.empty((n_steps, C)) if trace else None
    for t in range(n_steps):
        transition_da(prob, tm, ds)
        if trace:
            xs[t] = st.x
            if zs is not None:
                zs[t] = st.z[:, :extra]
            phis[t] = ds.phi_true
    return xs, zs, phis
