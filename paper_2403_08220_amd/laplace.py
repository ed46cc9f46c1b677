"""Chain initialisation from the reduced Laplace approximation (host orchestration).

The appendix on tuning and initialisation starts chains from samples of the Laplace
approximation. In whitened KLE coordinates the reduced surrogate posterior has
negative log density J(x) = Phi(x) + 1/2 ||x||^2 (Sec. 5.1), its Gauss-Newton
Hessian is I + H with H the ppGNH, and the Laplace approximation is
N(x_map, (I + H(x_map))^-1).

Every evaluation runs on the device through the library: the proposal entry point
at dt = 4 (s = 0, beta = 1) returns x - (I + H)^-1 (x + g) + L^-T xi, which is the
full Gauss-Newton step when xi = 0 and the step plus a Laplace draw otherwise. The
host only combines the returned vectors for the step-length search (halving from 1,
down to 2^-30, until J strictly decreases) and stops when the step is below
tol (1 + ||x||), when no step length decreases J, or after `iters` iterations.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .api import Context, Problem


@dataclass
class MapResult:
    x: np.ndarray
    J: float
    iters: int
    converged: bool


def _torch():
    import torch
    return torch


class _Evaluator:
    """One-chain evaluation problem at dt = 4 on the context's device."""

    def __init__(self, ctx: Context, y, noise_var, n: int, precision: str):
        self.p = Problem(ctx, n, y, noise_var, 4.0, precision=precision, track_complement=False)
        self.dev = f"cuda:{ctx.device}"
        self.r = ctx.r

    def geometry(self, x: np.ndarray):
        torch = _torch()
        xt = torch.tensor(np.atleast_2d(x), dtype=torch.float64, device=self.dev)
        return xt, self.p.eval_geometry(xt, want_H=False)

    def close(self):
        self.p.close()


def gauss_newton_map(ctx: Context, y, noise_var, x0=None, iters: int = 300, tol: float = 1e-9,
                     precision: str = "f64") -> MapResult:
    torch = _torch()
    ev = _Evaluator(ctx, y, noise_var, 1, precision)
    try:
        x = np.zeros(ctx.r) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
        xt, geo = ev.geometry(x)
        J = float(geo["phi"].cpu()[0]) + 0.5 * float(x @ x)
        zero = torch.zeros_like(xt)
        taken = 0
        for _ in range(iters):
            if int(geo["ok"].cpu()[0]) != 1:
                return MapResult(x=x, J=J, iters=taken, converged=False)
            full = ev.p.eval_propose(xt, geo["g"], geo["L"], zero).cpu().numpy()[0]
            delta = full - x
            if np.linalg.norm(delta) <= tol * (1.0 + np.linalg.norm(x)):
                return MapResult(x=x, J=J, iters=taken, converged=True)
            alpha = 1.0
            while alpha >= 2.0 ** -30:
                xn = x + alpha * delta
                xnt, gn = ev.geometry(xn)
                Jn = float(gn["phi"].cpu()[0]) + 0.5 * float(xn @ xn)
                if np.isfinite(Jn) and int(gn["ok"].cpu()[0]) == 1 and Jn < J:
                    break
                alpha *= 0.5
            else:
                return MapResult(x=x, J=J, iters=taken, converged=True)
            x, xt, geo, J = xn, xnt, gn, Jn
            taken += 1
        return MapResult(x=x, J=J, iters=taken, converged=False)
    finally:
        ev.close()


def laplace_samples(ctx: Context, y, noise_var, x_map, xi, precision: str = "f64") -> np.ndarray:
    """x_map + L^-T xi_c for each row of xi (C, r), L L^T = I + H(x_map)."""
    torch = _torch()
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    C = xi.shape[0]
    ev = _Evaluator(ctx, y, noise_var, 1, precision)
    batch = Problem(ctx, C, y, noise_var, 4.0, precision=precision, track_complement=False)
    try:
        xt, geo = ev.geometry(np.asarray(x_map, dtype=np.float64))
        X = xt.expand(C, -1).contiguous()
        G = geo["g"].expand(C, -1).contiguous()
        L = geo["L"].expand(C, -1, -1).contiguous()
        xit = torch.tensor(xi, dtype=torch.float64, device=xt.device)
        with_noise = batch.eval_propose(X, G, L, xit).cpu().numpy()
        without = batch.eval_propose(X, G, L, torch.zeros_like(xit)).cpu().numpy()
        return with_noise - without + np.asarray(x_map, dtype=np.float64)[None, :]
    finally:
        batch.close()
        ev.close()
