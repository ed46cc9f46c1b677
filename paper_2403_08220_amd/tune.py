"""Step-size tuning (host logic over the device path).

The appendix on tuning and initialisation chooses dt as follows: run a chain for each
candidate dt and measure the acceptance rate AR and the mean square jump
MSJ = (1/(n-1)) sum_j ||m_(j+1) - m_j||^2; keep the candidates up to the largest
dt_max over which AR decreases and MSJ increases monotonically with dt; among those
pick the one with the largest median ESS%.

Readings: the jumps are measured in the reduced whitened coordinates (the complement
moves by the same pCN rule at every dt and only adds a dt-monotone term); ESS% is the
multichain estimator of the library (the paper uses its single-chain version); the
monotone prefix starts at the smallest candidate, and a candidate that breaks either
monotonicity ends it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def select_step_size(dts, ar, msj, ess):
    """Index of the tuned candidate among dts (any order). Returns (index, kept indices)."""
    dts = np.asarray(dts, dtype=np.float64)
    order = np.argsort(dts)
    ar = np.asarray(ar, dtype=np.float64)[order]
    msj = np.asarray(msj, dtype=np.float64)[order]
    ess = np.asarray(ess, dtype=np.float64)[order]
    keep = [0]
    for k in range(1, len(order)):
        if ar[k] <= ar[k - 1] and msj[k] >= msj[k - 1]:
            keep.append(k)
        else:
            break
    scores = np.where(np.isfinite(ess[keep]), ess[keep], -np.inf)
    best = keep[int(np.argmax(scores))]
    return int(order[best]), [int(order[k]) for k in keep]


def mean_square_jump(trace: np.ndarray) -> float:
    """MSJ of a trace (n, C, r) averaged over chains."""
    t = np.asarray(trace, dtype=np.float64)
    return float(np.mean(np.sum(np.diff(t, axis=0) ** 2, axis=2)))


@dataclass
class TuneResult:
    dt: float
    table: list = field(default_factory=list)   # one dict per candidate


def tune_step_size(ctx, y, noise_var, x0, z0, candidates, burn: int, steps: int, seed: int = 0,
                   precision: str = "f64", stream=None, method: str = "mmala", fixed=None) -> TuneResult:
    """Run every candidate dt on the device from (x0, z0) and apply the selection rule
    (method: the transition kernel, "mmala" or a baseline; fixed: (x_map, L_map) of an
    "lapcn" problem)."""
    import torch

    from .api import Problem

    C = np.asarray(x0).shape[0]
    rows = []
    for dt in candidates:
        p = Problem(ctx, C, y, noise_var, float(dt), seed=seed, precision=precision,
                    track_complement=z0 is not None, trace_capacity=burn + steps, method=method)
        try:
            p.init(x0, z0, stream=stream)
            if fixed is not None:
                p.set_fixed_metric(*fixed)
            p.step(burn, stream=stream)
            a0, _, _ = p.diagnostics()
            p.step(steps, stream=stream)
            a1, f1, _ = p.diagnostics()
            xt, _ = p.trace()
            e = p.ess(burn)
        finally:
            p.close()
        per_chain = (a1 - a0) / steps
        rows.append(dict(dt=float(dt), AR=float(per_chain.mean()), AR_min=float(per_chain.min()),
                         AR_max=float(per_chain.max()), MSJ=mean_square_jump(xt[burn:]),
                         ess_frac=float(np.nanmedian(e)), failures=int(f1.sum())))
    idx, kept = select_step_size([r["dt"] for r in rows], [r["AR"] for r in rows], [r["MSJ"] for r in rows],
                                 [r["ess_frac"] for r in rows])
    for k, r in enumerate(rows):
        r["kept"] = k in kept
    return TuneResult(dt=rows[idx]["dt"], table=rows)
