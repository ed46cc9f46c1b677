"""Benchmark of the DINO-mMALA hot path on one MI355X.

Workload (the one the headline throughput is quoted on): 129x129 grid Matern prior
(gamma 0.1, delta 1), r = 200 KLE basis, ResNet width 400 depth 4 with exact GELU,
d_y = 100 observations with sigma = 1% of max |f(x_true)|, 512 chains. One step is
one Markov transition of every chain through every stage of the hot path (proposal,
surrogate forward, reduced Jacobian, misfit/ppg, GN Hessian, Cholesky, acceptance,
complement, trace). Inputs are seeded and synthetic (no PDE data exists for this
surrogate); chain states stay resident in HBM for the whole timed region.

Prints ONE JSON line. --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "bf16_TFLOPs": 2500.0,
    "fp8_TFLOPs": 5000.0,
    "fp32_TFLOPs": 157.3,
    "fp64_TFLOPs": 78.6,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage_work(stage, w, C, r, dy, L_res, accepted_frac, d_perp, prec):
    """Algorithmic work of one launch group of a stage for one step of C chains.
    Returns (amount, unit, bound, peak)."""
    width = w
    if stage == "jacobian":
        flops = C * 2.0 * (L_res * dy * width * width + dy * width * r)
        if prec == "bf16":
            return flops, "TFLOP/s", "mfma", PEAKS["bf16_TFLOPs"]
        return flops, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if stage == "forward":
        flops = C * 2.0 * (r * width + L_res * width * width + width * dy)
        return flops, "TFLOP/s", "alu", PEAKS["fp32_TFLOPs"] if prec == "bf16" else PEAKS["fp64_TFLOPs"]
    if stage == "gn_hessian":
        flops = C * 2.0 * r * r * dy / 2.0  # symmetric product, lower half
        if prec == "bf16":
            return flops, "TFLOP/s", "mfma", PEAKS["bf16_TFLOPs"]
        return flops, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if stage == "cholesky":
        return C * r ** 3 / 3.0, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if stage in ("proposal", "accept"):
        # one read of the packed-equivalent lower triangle of the factor per chain
        return C * r * (r + 1) / 2.0 * 8.0, "GB/s", "hbm", PEAKS["hbm_GBps"]
    if stage == "complement":
        return C * accepted_frac * d_perp * 8.0, "GB/s", "hbm", PEAKS["hbm_GBps"]
    if stage == "misfit_ppg":
        return C * dy * r * 8.0, "GB/s", "hbm", PEAKS["hbm_GBps"]
    if stage == "trace":
        return C * r * (8.0 + 4.0), "GB/s", "hbm", PEAKS["hbm_GBps"]
    return 0.0, "GB/s", "hbm", PEAKS["hbm_GBps"]


def make_problem_inputs(w, layers, ctx_builder):
    """Data y = f(x_true) + sigma eps with f evaluated by the device path."""
    import torch
    from synth import draw_noise, draw_true_state

    x_true = draw_true_state(w)[: w.r]
    ctx = ctx_builder()
    from paper_2403_08220_amd import Problem
    tmp = Problem(ctx, 1, np.zeros(w.d_y), np.ones(w.d_y), 0.1, track_complement=False)
    geo = tmp.eval_geometry(torch.tensor(x_true[None], dtype=torch.float64, device="cuda:0"), want_H=False)
    f_true = geo["f"].cpu().numpy()[0]
    tmp.close()
    sigma = w.sigma * np.max(np.abs(f_true)) if w.sigma_rule == "rel_max" else w.sigma
    y = f_true + sigma * draw_noise(w)
    return ctx, y, np.full(w.d_y, sigma ** 2)


def cpu_baseline(w, layers, chains=32, budget_s=20.0, max_steps=6):
    """The FP64 oracle on a bounded sample of the same workload."""
    from threadpoolctl import threadpool_info

    from oracle import mcmc, network
    from synth import draw_initial_states, draw_noise, draw_true_state

    x_true = draw_true_state(w)[: w.r]
    f_true, _ = network.forward(layers, x_true[None])
    f_true = f_true[0, : w.d_y]
    sigma = w.sigma * np.max(np.abs(f_true)) if w.sigma_rule == "rel_max" else w.sigma
    y = f_true + sigma * draw_noise(w)
    prob = mcmc.Problem(layers, y, np.full(w.d_y, sigma ** 2), w.dt, seed=w.chain_seed)
    x0, z0 = draw_initial_states(w, chains=chains)
    st = mcmc.init_state(prob, x0, z0.astype(np.float64))
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and (time.perf_counter() - t0) < budget_s:
        mcmc.transition(prob, st)
        steps += 1
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": chains * steps / dt, "unit": "chain-steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{chains} chains x {steps} steps of the same workload (FP64 NumPy/SciPy oracle, "
                      f"{dt:.1f} s), the complement tracked", "seconds": dt}


def run_path(w, layers, ctx, y, nv, precision, steps, warmup, profile_steps, want_ess=True):
    import torch
    from paper_2403_08220_amd import Problem
    from synth import draw_initial_states

    C = w.chains
    cap = warmup + steps if want_ess else 0
    p = Problem(ctx, C, y, nv, w.dt, seed=w.chain_seed, precision=precision, track_complement=True,
                trace_capacity=cap)
    x0, z0 = draw_initial_states(w, chains=C)
    p.init(x0, z0)
    stream = torch.cuda.current_stream()
    p.step(warmup)
    torch.cuda.synchronize()
    a0, _, _ = p.diagnostics()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    p.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    acc, fail, nst = p.diagnostics()
    accept_frac = float((acc - a0).sum()) / (C * steps)
    out = dict(wall_s=wall, gpu_ms=gpu_ms, accept_rate=accept_frac, failures=int(fail.sum()))
    if want_ess:
        burn = warmup + int(0.2 * steps)
        e = p.ess(burn)
        n_post = warmup + steps - burn
        ess = e * C * n_post
        out["median_ess"] = float(np.nanmedian(ess))
        out["median_ess_frac"] = float(np.nanmedian(e))
    if profile_steps > 0:
        p.set_profiling(True)
        p.step(profile_steps)
        prof, nprof = p.profile()
        p.set_profiling(False)
        out["profile"] = {k: dict(ms_per_step=v["ms"] / max(nprof, 1), launches=v["launches"]) for k, v in prof.items()}
    p.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="f64", choices=["f64", "bf16"])
    ap.add_argument("--compare-f64", action="store_true", help="also time the plain FP64 path")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}). "
              "Chains are independent; sharding would place whole chain blocks or requests on separate GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_08220_amd import Context
    from synth import draw_network, workload

    w = workload("mid")
    layers = draw_network(w)
    L_res = sum(1 for k, _, _ in layers if k == "resid")

    def ctx_builder():
        c = Context(0)
        c.load_prior(w.n, w.gamma, w.delta, w.r)
        c.load_network(layers)
        return c

    log(f"bench: workload mid, {w.chains} chains, precision {args.precision}, steps {args.steps}")
    ctx, y, nv = make_problem_inputs(w, layers, ctx_builder)
    res = run_path(w, layers, ctx, y, nv, args.precision, args.steps, args.warmup, args.profile_steps)
    log(f"bench: {args.precision} path done: {res['wall_s']:.3f} s, accept {res['accept_rate']:.3f}")
    extra = {}
    if args.compare_f64 and args.precision != "f64":
        r64 = run_path(w, layers, ctx, y, nv, "f64", max(args.steps // 4, 10), args.warmup, 0)
        extra["fp64_plain"] = dict(value=w.chains * max(args.steps // 4, 10) / r64["wall_s"],
                                   unit="chain-steps/s", accept_rate=r64["accept_rate"],
                                   ess_per_s=r64["median_ess"] / r64["wall_s"])
    C, steps = w.chains, args.steps
    value = C * steps / res["wall_s"]
    ms_per_step = 1e3 * res["wall_s"] / steps

    # roofline of the dominant stage, from the live HIP-event profile
    prof = res.get("profile", {})
    stages = {}
    for name, v in prof.items():
        amt, unit, bound, peak = stage_work(name, w.width, C, w.r, w.d_y, L_res, res["accept_rate"],
                                            w.d_m - w.r, args.precision)
        t = v["ms_per_step"] * 1e-3
        ach = (amt / t / (1e12 if unit == "TFLOP/s" else 1e9)) if t > 0 else 0.0
        stages[name] = dict(ms=round(v["ms_per_step"], 4), launches=v["launches"], bound=bound,
                            achieved=round(ach, 3), peak=peak, unit=unit, frac=round(ach / peak, 4))
    dom = max(stages, key=lambda k: stages[k]["ms"]) if stages else None
    roof = None
    if dom:
        s = stages[dom]
        roof = dict(kernel=dom, bound=s["bound"], achieved=s["achieved"], peak=s["peak"], unit=s["unit"],
                    frac=s["frac"], traffic=None, launches_per_step=s["launches"])
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle) ...")
        cpu = cpu_baseline(w, layers)
    line = {
        "metric": "chain-steps/s",
        "value": round(value, 1),
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "bf16+f32+f64",
        "data": "synthetic (seeded Xavier-normal ResNet, KLE prior draws; no trained weights or PDE data)",
        "config": {"workload": "129x129 grid, r=200 KLE, ResNet 400x4 GELU, d_y=100, 512 chains",
                   "grid": w.n, "r": w.r, "width": w.width, "depth": w.depth, "d_y": w.d_y, "chains": C,
                   "dt": w.dt, "precision": args.precision},
        "ess_per_s": round(res["median_ess"] / res["wall_s"], 2),
        "median_ess_frac": res["median_ess_frac"],
        "accept_rate": round(res["accept_rate"], 4),
        "roofline": roof,
        "stages": stages,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
