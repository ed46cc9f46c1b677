"""Reduced Laplace approximation for chain initialisation (oracle; test infrastructure).

Paper basis: the appendix on tuning and initialisation starts chains from samples of
the Laplace approximation of the posterior; Sec. 5.1 gives the surrogate reduced
misfit, its gradient (ppg) and its Gauss-Newton Hessian (ppGNH) in whitened KLE
coordinates, where the prior is N(0, I_r).

Readings taken here (the paper does not say how its MAP point is found):
* The MAP of the reduced surrogate posterior minimises
      J(x) = Phi(x) + 1/2 ||x||^2,
  and is found by Gauss-Newton iterations with the ppGNH H:
      delta = -(I + H(x))^-1 (x + g(x)),
  accepting x + alpha delta for the largest alpha in {1, 1/2, 1/4, ...} (down to
  2^-30) with a finite J strictly below J(x); the iteration stops when
  ||delta|| <= tol (1 + ||x||) (converged), when no step length decreases J (the
  minimum is reached to rounding), or after `iters` iterations.
* The Laplace approximation is N(x_map, (I + H(x_map))^-1); a sample is
  x_map + L^-T xi with L L^T = I + H(x_map) and xi ~ N(0, I_r) given.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import mcmc


def objective(prob: mcmc.Problem, x: np.ndarray, cache: mcmc.Cache) -> np.ndarray:
    """J(x) = Phi(x) + 1/2 ||x||^2 per row (negative log posterior up to a constant)."""
    return cache.phi + 0.5 * np.sum(np.atleast_2d(x) ** 2, axis=1)


@dataclass
class MapResult:
    x: np.ndarray        # (r,) the last accepted iterate
    J: float             # objective there
    iters: int           # Gauss-Newton iterations taken (accepted steps)
    converged: bool      # stopped on the step-size test or because no step decreased J


def gauss_newton_map(prob: mcmc.Problem, x0: np.ndarray, iters: int = 300, tol: float = 1e-9) -> MapResult:
    """Damped Gauss-Newton minimisation of J from x0 (one point, shape (r,))."""
    x = np.array(x0, dtype=np.float64).reshape(1, -1)
    r = x.shape[1]
    cache = mcmc.geometry(prob, x)
    J = float(objective(prob, x, cache)[0])
    taken = 0
    for _ in range(iters):
        A = np.eye(r) + cache.H[0]
        delta = -np.linalg.solve(A, x[0] + cache.g[0])
        if np.linalg.norm(delta) <= tol * (1.0 + np.linalg.norm(x[0])):
            return MapResult(x=x[0], J=J, iters=taken, converged=True)
        alpha = 1.0
        while alpha >= 2.0 ** -30:
            xn = x + alpha * delta[None, :]
            cn = mcmc.geometry(prob, xn)
            Jn = float(objective(prob, xn, cn)[0])
            if np.isfinite(Jn) and bool(cn.ok[0]) and Jn < J:
                break
            alpha *= 0.5
        else:
            return MapResult(x=x[0], J=J, iters=taken, converged=True)
        x, cache, J = xn, cn, Jn
        taken += 1
    return MapResult(x=x[0], J=J, iters=taken, converged=False)


def laplace_samples(prob: mcmc.Problem, x_map: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """x_map + L^-T xi_c for each row of xi (C, r), L L^T = I + H(x_map)."""
    cache = mcmc.geometry(prob, np.asarray(x_map, dtype=np.float64).reshape(1, -1))
    L = cache.L[0]
    noise = sla.solve_triangular(L, np.asarray(xi, dtype=np.float64).T, lower=True, trans="T").T
    return x_map[None, :] + noise
