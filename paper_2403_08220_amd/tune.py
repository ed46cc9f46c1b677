"""Step-size tuning (host logic over the device path).

The appendix on tuning and initialisation chooses dt as follows: run a chain for each
candidate dt and measure the acceptance rate AR and the mean square jump
MSJ = (1/(n-1)) sum_j ||m_(j+1) - m_j||^2; keep the candidates up to the largest
dt_max over which AR decreases and MSJ increases monotonically with dt; among those
pick the one with the largest median ESS%. For MALA and LA-pCN the appendix further
reduces the step until the acceptance rates of chains started at different positions
vary within +-5% of their average.

Readings: the jumps are measured in the reduced whitened coordinates (the complement
moves by the same pCN rule at every dt and only adds a dt-monotone term); ESS% is the
multichain estimator of the library (the paper uses its single-chain version); the
monotone prefix starts at the smallest candidate, and a candidate that breaks either
monotonicity ends it. The AR variation is the spread of the per-chain acceptance
rates in excess of their binomial sampling noise over the tuning run (a finite run
shows that noise even when every chain behaves alike), and "+-5%" is read as 5
percentage points. When every kept candidate's ESS% sits at the multichain
estimator's floor (chains that do not decorrelate within the tuning run), ESS%
cannot rank them; the rule then takes the kept candidate whose AR is closest to
AR_TARGET = 0.25 (inside the 20-40% band the design notes use for mMALA), and the
result records that fallback.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


AR_TARGET = 0.25
AR_SPREAD_TOL = 0.05


def ar_spread(per_chain_ar, steps: int) -> float:
    """Spread (standard deviation) of per-chain acceptance rates beyond the binomial noise
    of `steps` draws: sqrt(max(var(AR_c) - mean(AR_c (1 - AR_c)) / steps, 0))."""
    a = np.asarray(per_chain_ar, dtype=np.float64)
    excess = np.var(a) - np.mean(a * (1.0 - a)) / max(steps, 1)
    return float(np.sqrt(max(excess, 0.0)))


def select_step_size(dts, ar, msj, ess, spread=None, ess_floor_frac=None):
    """Index of the tuned candidate among dts (any order).

    spread: per-candidate AR spread (ar_spread) when the appendix's AR-variation
    reduction applies (MALA, LA-pCN), else None. ess_floor_frac: the ESS% of chains that
    do not decorrelate within the tuning run; when every kept candidate is at or below
    it, ESS% does not rank them and the AR closest to AR_TARGET decides.
    Returns (index, kept indices, rule) with rule "ess", "ar_target" or "ar_spread"."""
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
    cand = list(keep)
    if ess_floor_frac is not None and not np.any(np.nan_to_num(ess[cand], nan=-np.inf) > ess_floor_frac):
        best, rule = cand[int(np.argmin(np.abs(ar[cand] - AR_TARGET)))], "ar_target"
    else:
        scores = np.where(np.isfinite(ess[cand]), ess[cand], -np.inf)
        best, rule = cand[int(np.argmax(scores))], "ess"
    if spread is not None:
        sp = np.asarray(spread, dtype=np.float64)[order]
        if sp[best] > AR_SPREAD_TOL:
            # reduce the step: the largest smaller kept candidate whose chains agree
            ok = [k for k in cand if k < best and sp[k] <= AR_SPREAD_TOL]
            best = ok[-1] if ok else cand[0]
            rule = "ar_spread"
    return int(order[best]), [int(order[k]) for k in keep], rule


def mean_square_jump(trace: np.ndarray) -> float:
    """MSJ of a trace (n, C, r) averaged over chains."""
    t = np.asarray(trace, dtype=np.float64)
    return float(np.mean(np.sum(np.diff(t, axis=0) ** 2, axis=2)))


@dataclass
class TuneResult:
    dt: float
    table: list = field(default_factory=list)   # one dict per candidate
    rule: str = "ess"                            # what decided: "ess", "ar_target" or "ar_spread"


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
                         AR_max=float(per_chain.max()), AR_spread=ar_spread(per_chain, steps),
                         MSJ=mean_square_jump(xt[burn:]), ess_frac=float(np.nanmedian(e)),
                         failures=int(f1.sum())))
    # the multichain ESS% of chains that stay correlated over the n = steps samples after
    # burn-in is about (C / 2) / (C n); ESS% at or below 1.5 times that does not rank
    floor = 1.5 / (2.0 * steps)
    spread = [r["AR_spread"] for r in rows] if method in ("mala", "lapcn") else None
    idx, kept, rule = select_step_size([r["dt"] for r in rows], [r["AR"] for r in rows], [r["MSJ"] for r in rows],
                                       [r["ess_frac"] for r in rows], spread=spread, ess_floor_frac=floor)
    for k, r in enumerate(rows):
        r["kept"] = k in kept
    return TuneResult(dt=rows[idx]["dt"], table=rows, rule=rule)
