"""Benchmark of the DINO-mMALA hot path on one MI355X.

Workload (the one the headline throughput is quoted on): 129x129 grid Matern prior
(gamma 0.1, delta 1), r = 200 KLE basis, ResNet width 400 depth 4 with exact GELU,
d_y = 100 observations with sigma = 1% of max |f(x_true)|, 512 chains, dt = 3e-4
(tuned by the appendix's rule and frozen). One step is one Markov transition of
every chain through every stage of the hot path (proposal, surrogate forward,
reduced Jacobian, misfit/ppg, GN Hessian, Cholesky, acceptance, complement, trace).
Inputs are seeded and synthetic (no PDE data or trained weights exist for this
surrogate); chains start from Laplace-approximation samples around the device
Gauss-Newton MAP, and their states stay resident in HBM for the whole timed region.

The primary path is the mixed-precision one (FP32 forward, BF16 MFMA Jacobian and
GN Hessian with FP32 accumulation, FP64 Cholesky, proposal and MH); the plain FP64
device path is timed beside it on the same workload, and the FP64 CPU oracle on a
bounded sample of it. Per-stage device times come from HIP events the library
records on its stream during the timed steps.

Prints ONE JSON line. --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "bf16_TFLOPs": 2500.0,
    "fp32_TFLOPs": 157.3,
    "fp64_TFLOPs": 78.6,
    "fp8_TFLOPs": 5000.0,
}

# device kernel of each stage on the mixed-precision path (rocprofv3 kernel names)
STAGE_KERNEL = {
    "proposal": "propose_kernel", "forward": "fwd_mfma_kernel", "jacobian": "jac_sweep_bf16_kernel",
    "misfit_ppg": "misfit_grad_kernel", "gn_hessian": "hess_bf16_kernel", "cholesky": "cholesky_reg_kernel",
    "accept": "accept_kernel", "complement": "complement_kernel", "trace": "accept_kernel",
}
# observation-space form (d_y < r): Gram matrix, d_y x d_y factor and Woodbury kernels
STAGE_KERNEL_DUAL = dict(STAGE_KERNEL, proposal="propose_dual_kernel", accept="accept_dual_kernel",
                         gn_hessian="gram_bf16_kernel")
# the dual form on the mixed path at d_y <= 104: Gram matrix and factor in one kernel (the
# metric stage; the factor stage has no kernel of its own)
FUSED_METRIC_KERNEL = "gram_chol_bf16_kernel"
# the width-416 sweep (layers of 401..416 units) has its own kernel
SWEEP416_KERNEL = "jac_sweep13_kernel"
KERNEL_SOURCES = {"cholesky_reg_kernel": ["kernels_chain.hip"],
                  "cholesky_wave_kernel": ["kernels_chain.hip", "chol_wave.hpp"],
                  "propose_kernel": ["kernels_chain.hip"],
                  "accept_kernel": ["kernels_chain.hip"], "complement_kernel": ["kernels_chain.hip"],
                  "propose_dual_kernel": ["kernels_chain.hip"],
                  "accept_dual_kernel": ["kernels_chain.hip"], "jac_sweep_bf16_kernel": ["kernels_mfma.hip"],
                  "jac_sweep13_kernel": ["kernels_mfma.hip", "sweep_asm.inc"],
                  "hess_bf16_kernel": ["kernels_mfma.hip"], "gram_bf16_kernel": ["kernels_mfma.hip"],
                  "gram_chol_bf16_kernel": ["kernels_mfma.hip", "chol_wave.hpp"],
                  "fwd_mfma_kernel": ["kernels_geometry.hip"],
                  "fwd_layer_kernel": ["kernels_geometry.hip"],
                  "jac_sweep_fp8_kernel": ["kernels_fp8.hip"], "hess_bf16_tiled_kernel": ["kernels_mfma.hip"],
                  "cholesky_kernel": ["kernels_chain.hip"], "cholesky_panel_kernel": ["kernels_chain.hip"]}
# the FP8 path at the large shape: FP8 sweep, tiled Gauss-Newton kernel, transposed-panel factor
STAGE_KERNEL_FP8_LARGE = dict(STAGE_KERNEL, jacobian="jac_sweep_fp8_kernel", gn_hessian="hess_bf16_tiled_kernel",
                              cholesky="cholesky_panel_kernel")


def source_sha256(kernel):
    """SHA-256 over the source files of `kernel` (None when one of them is missing)."""
    h = hashlib.sha256()
    names = KERNEL_SOURCES.get(kernel)
    if not names:
        return None
    for name in names:
        path = os.path.join(ROOT, "paper_2403_08220_amd", "csrc", name)
        if not os.path.isfile(path):
            return None
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stage_kernel(stage, dual, width, r, dy, fused=False):
    k = (STAGE_KERNEL_DUAL if dual else STAGE_KERNEL)[stage]
    if fused and stage == "gn_hessian":
        return FUSED_METRIC_KERNEL
    # the sweep instance covers the widest layer (the widths and r) in blocks of 32:
    # 8..13 blocks run the width-416 kernel
    if stage == "jacobian" and 224 < max(width, r) <= 416:
        k = SWEEP416_KERNEL
    # factors of order up to 104 run one wavefront per chain
    if stage == "cholesky" and (dy if dual else r) <= 104:
        k = "cholesky_wave_kernel"
    return k


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage_work(stage, w, C, r, dy, L_res, accepted_frac, d_perp, prec, dual=False, fused=False):
    """Algorithmic work of one step of a stage over C chains.
    Returns (amount, unit, bound, peak); the per-chain figures are in the design notes.
    dual: the observation-space form (Gram matrix I + B B^T, d_y x d_y factor); fused: the
    Gram matrix and its factor in one kernel (the metric stage), bound by the FP64 factor."""
    mixed = prec in ("bf16", "fp8")
    if dual and fused and stage == "gn_hessian":
        flops = C * (2.0 * (dy * (dy + 1) / 2.0 * r + dy * r) + dy ** 3 / 3.0)
        return flops, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if dual and stage == "gn_hessian":
        flops = C * 2.0 * (dy * (dy + 1) / 2.0 * r + dy * r)  # lower half of B B^T, and B^T e
        if mixed:
            return flops, "TFLOP/s", "mfma", PEAKS["bf16_TFLOPs"]
        return flops, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if dual and stage == "cholesky":
        return C * dy ** 3 / 3.0, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if dual and stage in ("proposal", "accept"):
        # one read of the chain's B (BF16 on the mixed path, FP64 otherwise) and of the lower
        # triangle of its FP64 d_y x d_y factor; on acceptance the proposal's B is copied
        bsz = 2.0 if mixed else 8.0
        per = dy * r * bsz + dy * (dy + 1) / 2.0 * 8.0
        if stage == "accept":
            per += accepted_frac * 2.0 * dy * r * bsz
        return C * per, "GB/s", "hbm", PEAKS["hbm_GBps"]
    if stage == "jacobian":
        flops = C * 2.0 * (L_res * dy * w * w + dy * w * r)
        if prec == "fp8":
            return flops, "TFLOP/s", "mfma", PEAKS["fp8_TFLOPs"]
        if mixed:
            return flops, "TFLOP/s", "mfma", PEAKS["bf16_TFLOPs"]
        return flops, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if stage == "forward":
        flops = C * 2.0 * (r * w + L_res * w * w + w * dy)
        return flops, "TFLOP/s", "alu", PEAKS["fp32_TFLOPs"] if mixed else PEAKS["fp64_TFLOPs"]
    if stage == "gn_hessian":
        flops = C * 2.0 * r * r * dy / 2.0  # symmetric product, lower half
        if mixed:
            return flops, "TFLOP/s", "mfma", PEAKS["bf16_TFLOPs"]
        return flops, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if stage == "cholesky":
        return C * r ** 3 / 3.0, "TFLOP/s", "alu", PEAKS["fp64_TFLOPs"]
    if stage in ("proposal", "accept"):
        # one read of the lower triangle of an FP64 factor per chain
        return C * r * (r + 1) / 2.0 * 8.0, "GB/s", "hbm", PEAKS["hbm_GBps"]
    if stage == "complement":
        # read + write of the FP32 complement of the accepted chains
        return C * accepted_frac * d_perp * 8.0, "GB/s", "hbm", PEAKS["hbm_GBps"]
    if stage == "misfit_ppg":
        # residual: read f and y, write e (FP32 path) / read B (FP64 path)
        if mixed:
            return C * dy * 12.0, "GB/s", "hbm", PEAKS["hbm_GBps"]
        return C * dy * r * 8.0, "GB/s", "hbm", PEAKS["hbm_GBps"]
    if stage == "trace":
        return C * r * (8.0 + 4.0), "GB/s", "hbm", PEAKS["hbm_GBps"]
    return 0.0, "GB/s", "hbm", PEAKS["hbm_GBps"]


def make_problem_inputs(w, ctx_builder):
    """Data y = f(x_true) + sigma eps with f evaluated by the device path."""
    ctx = ctx_builder()
    y, nv = device_data(w, ctx)
    return ctx, y, nv


def laplace_start(w, ctx, y, nv):
    from paper_2403_08220_amd import laplace
    from synth import draw_initial_states, draw_laplace_normals

    t0 = time.perf_counter()
    m = laplace.gauss_newton_map(ctx, y, nv)
    x0 = laplace.laplace_samples(ctx, y, nv, m.x, draw_laplace_normals(w))
    _, z0 = draw_initial_states(w)
    return x0, z0, dict(J_map=m.J, gn_iters=m.iters, seconds=round(time.perf_counter() - t0, 3)), m.x


def cpu_baseline(w, layers, x0, z0, chains=32, budget_s=20.0, max_steps=60, factor="primal", threads=None):
    """The FP64 oracle on a bounded sample of the same workload (same starting states and
    factorisation as the device path), about 10-20 s of host work, on all host cores or
    on `threads` BLAS threads."""
    from threadpoolctl import threadpool_info, threadpool_limits

    if threads is not None:
        with threadpool_limits(limits=threads):
            return cpu_baseline(w, layers, x0, z0, chains, budget_s, max_steps, factor, None)

    from oracle import mcmc, network
    from synth import draw_noise, draw_true_state

    x_true = draw_true_state(w)[: w.r]
    f_true, _ = network.forward(layers, x_true[None])
    f_true = f_true[0, : w.d_y]
    sigma = w.sigma * np.max(np.abs(f_true)) if w.sigma_rule == "rel_max" else w.sigma
    y = f_true + sigma * draw_noise(w)
    prob = mcmc.Problem(layers, y, np.full(w.d_y, sigma ** 2), w.dt, seed=w.chain_seed, factor=factor)
    st = mcmc.init_state(prob, x0[:chains], z0[:chains].astype(np.float64))
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and (time.perf_counter() - t0) < budget_s:
        mcmc.transition(prob, st)
        steps += 1
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": round(chains * steps / dt, 2), "unit": "chain-steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{chains} of the {w.chains} chains x {steps} steps of the same workload and starting states "
                      f"(FP64 NumPy/SciPy oracle, {factor} form, complement tracked, {dt:.1f} s)"}


def copy_calibration(nbytes=1 << 29):
    """A plain device copy of known size (read nbytes + write nbytes): the reference
    kernel that scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    return nbytes


def run_path(w, ctx, y, nv, x0, z0, precision, steps, warmup, profile=True, factorization="auto", method="mmala",
             dt=None, fixed=None, tune=True):
    import torch
    from paper_2403_08220_amd import Problem

    C = w.chains
    cap = warmup + steps
    p = Problem(ctx, C, y, nv, w.dt if dt is None else dt, seed=w.chain_seed, precision=precision,
                track_complement=True, trace_capacity=cap, factorization=factorization, method=method)
    p.init(x0, z0)
    if fixed is not None:
        p.set_fixed_metric(*fixed)
    if tune:
        p.autotune()  # implementation choices for this problem's shapes, before any timing
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
    out = dict(wall_s=wall, gpu_ms=gpu_ms, accept_rate=float((acc - a0).sum()) / (C * steps),
               failures=int(fail.sum()))
    if profile:
        # the same number of steps again with HIP events around every stage on the
        # library's stream (the events add a few microseconds per stage boundary, so
        # the headline value comes from the pass above)
        p.set_profiling(True)
        t1 = time.perf_counter()
        p.step(steps)
        torch.cuda.synchronize()
        out["profiled_ms_per_step"] = 1e3 * (time.perf_counter() - t1) / steps
        prof, nprof = p.profile()
        p.set_profiling(False)
        out["profile"] = {k: dict(ms_per_step=v["ms"] / max(nprof, 1), launches=v["launches"])
                          for k, v in prof.items()}
    # ESS over the timed window only (the warm-up steps are its burn-in), so that ESS and
    # wall time describe the same samples
    e = p.ess(warmup) if steps >= 2 else np.full(w.r, np.nan)
    out["median_ess"] = float(np.nanmedian(e * C * steps))
    out["median_ess_frac"] = float(np.nanmedian(e))
    p.close()
    return out


# step sizes the tuning rule chooses from, per baseline
BASELINE_DT_CANDIDATES = {"pcn": [1e-6, 3e-6, 1e-5, 3e-5, 1e-4, 3e-4, 1e-3, 3e-3, 1e-2],
                          "mala": [1e-5, 3e-5, 1e-4, 3e-4, 1e-3, 3e-3],
                          "lapcn": [1e-3, 3e-3, 1e-2, 3e-2, 1e-1, 3e-1, 1.0]}


def laplace_metric(w, ctx, y, nv, x_map):
    """(x_map, L_map) for LA-pCN: the factor of I + H(x_map), evaluated by the device's
    FP64 primal geometry."""
    import torch
    from paper_2403_08220_amd import Problem

    p = Problem(ctx, 1, y, nv, w.dt, precision="f64", track_complement=False, factorization="primal")
    try:
        x = torch.tensor(np.asarray(x_map, dtype=np.float64)[None], device="cuda:0")
        L = p.eval_geometry(x)["L"][0].cpu().numpy()
    finally:
        p.close()
    return np.asarray(x_map, dtype=np.float64), np.tril(L)
ESS_FLOOR_MARGIN = 1.5


def ess_floor(n_chains):
    """Multichain ESS of chains that do not decorrelate within the window (rho_t = 1 at
    every lag): n_chains * n / (2 n - 1), about n_chains / 2."""
    return n_chains / 2.0


def ess_rate(median_ess, wall_s, n_chains):
    """(ESS/s, note): median ESS over the timed window / its wall time, or None with the
    reason when the median ESS is within ESS_FLOOR_MARGIN of the multichain floor (chains
    that do not decorrelate within the window: the figure would measure the spread of
    the starting states and scale as 1 / steps, not mixing)."""
    fl = ESS_FLOOR_MARGIN * ess_floor(n_chains)
    if not np.isfinite(median_ess) or median_ess < fl or wall_s <= 0:
        return None, (f"median ESS {median_ess:.1f} is below {ESS_FLOOR_MARGIN} x the multichain floor "
                      f"({ess_floor(n_chains):.0f}): the chains do not decorrelate within the timed window")
    return round(median_ess / wall_s, 3), None


def baseline_leg(method, w, ctx, y, nv, x0, z0, precision, steps, warmup, mmala, fixed=None):
    """A baseline of Sec. 6.1 (pCN, MALA, or LA-pCN with `fixed` = (x_map, L_map)) on
    the same workload, chains and starting states: its step size chosen by the same
    tuning rule over BASELINE_DT_CANDIDATES, then timed like the main leg. The ratio of
    the two ESS rates is the effective sampling speedup (Sec. 6.3.1) of mMALA over the
    baseline on the surrogate posterior, at equal hardware. It is reported only when
    both median ESS values clear the multichain estimator's floor: chains that stay
    correlated over the whole window give rho_t near 1 at every lag and an ESS of about
    n_chains / 2 whatever the method, which measures the spread of the starting states,
    not mixing."""
    from paper_2403_08220_amd.tune import tune_step_size

    tr = tune_step_size(ctx, y, nv, x0, z0, BASELINE_DT_CANDIDATES[method], burn=20, steps=100,
                        seed=w.chain_seed, precision=precision, method=method, fixed=fixed)
    r = run_path(w, ctx, y, nv, x0, z0, precision, steps, warmup, profile=False, method=method, dt=tr.dt,
                 fixed=fixed)
    C = w.chains
    rate, note = ess_rate(r["median_ess"], r["wall_s"], C)
    mm_rate, _ = ess_rate(mmala["median_ess"], mmala["wall_s"], C)
    return dict(value=round(C * steps / r["wall_s"], 1), unit="chain-steps/s", steps=steps,
                ms_per_step=round(1e3 * r["wall_s"] / steps, 4), dt=tr.dt, accept_rate=round(r["accept_rate"], 4),
                step_cost_mmala_over_this=round(mmala["wall_s"] / r["wall_s"], 2),
                median_ess=round(r["median_ess"], 1), median_ess_frac=r["median_ess_frac"], ess_per_s=rate,
                ess_note=note, ess_speedup_mmala=round(mm_rate / rate, 2) if rate and mm_rate else None,
                tuning_rule=tr.rule,
                tuning=[dict(dt=t["dt"], AR=round(t["AR"], 4), AR_spread=round(t["AR_spread"], 4),
                             ess_frac=t["ess_frac"], kept=t["kept"]) for t in tr.table])


def device_data(w, ctx):
    """y = f(x_true) + sigma eps for workload w, f evaluated by the device path on ctx."""
    import torch
    from paper_2403_08220_amd import Problem
    from synth import draw_noise, draw_true_state

    x_true = draw_true_state(w)[: w.r]
    tmp = Problem(ctx, 1, np.zeros(w.d_y), np.ones(w.d_y), 0.1, track_complement=False)
    try:
        geo = tmp.eval_geometry(torch.tensor(x_true[None], dtype=torch.float64, device="cuda:0"), want_H=False)
        f_true = geo["f"].cpu().numpy()[0]
    finally:
        tmp.close()
    sigma = w.sigma * np.max(np.abs(f_true)) if w.sigma_rule == "rel_max" else w.sigma
    return f_true + sigma * draw_noise(w), np.full(w.d_y, sigma ** 2)


def ess_leg(ctx, steps, warmup):
    """ESS/s of the BF16 path against the plain FP64 path on the mix workload: the bench's
    shapes (129^2 grid, r = 200, ResNet 400 x 4, d_y = 100, 512 chains) with sigma = 30% of
    max |f(x_true)|, a posterior on which these chains decorrelate within the run (at the
    bench's sigma = 1% they do not, and ESS sits at the multichain floor). Both legs start
    from the same Laplace samples, take dt from the tuning rule (BF16 path, 200-step runs),
    and report ESS over their timed window of `steps` steps after `warmup` burn-in steps."""
    from paper_2403_08220_amd import laplace
    from paper_2403_08220_amd.tune import tune_step_size
    from synth import draw_initial_states, draw_laplace_normals, workload

    w = workload("mix")
    y, nv = device_data(w, ctx)
    m = laplace.gauss_newton_map(ctx, y, nv)
    x0 = laplace.laplace_samples(ctx, y, nv, m.x, draw_laplace_normals(w))
    _, z0 = draw_initial_states(w)
    tr = tune_step_size(ctx, y, nv, x0, z0, [0.01, 0.03, 0.1, 0.3], burn=50, steps=200, seed=w.chain_seed,
                        precision="bf16")
    out = dict(workload="mix: the bench shapes with sigma = 30% of max|f(x_true)|, 512 chains", dt=tr.dt,
               tuning_rule=tr.rule, steps=steps, burn_in=warmup)
    for prec in ("bf16", "f64"):
        r = run_path(w, ctx, y, nv, x0, z0, prec, steps, warmup, profile=False, factorization="auto", dt=tr.dt)
        rate, note = ess_rate(r["median_ess"], r["wall_s"], w.chains)
        out[prec] = dict(value=round(w.chains * steps / r["wall_s"], 1), unit="chain-steps/s",
                         ms_per_step=round(1e3 * r["wall_s"] / steps, 4), accept_rate=round(r["accept_rate"], 4),
                         median_ess=round(r["median_ess"], 1), ess_per_s=rate, ess_note=note)
    a, b = out["bf16"]["ess_per_s"], out["f64"]["ess_per_s"]
    out["ess_per_s_bf16_over_f64"] = round(a / b, 2) if a and b else None
    return out


def da_leg(ctx, w, layers, y, nv, x0, z0, precision, steps, warmup, mmala_wall):
    """DA-DINO-mMALA (Alg. 1 with its second stage) on the bench workload, the true model a
    stand-in network that reads 56 complement coordinates (r_T = 256; the surrogate's
    weights perturbed by 5%). Reports chain-steps/s, the first-stage pass rate (true-model
    evaluations per chain-step), the second-stage acceptance and the per-step cost
    relative to plain mMALA."""
    import torch
    from paper_2403_08220_amd import Problem
    from synth import draw_true_model

    ctx.load_true_model(draw_true_model(layers, 56))
    C = w.chains
    p = Problem(ctx, C, y, nv, w.dt, seed=w.chain_seed, precision=precision, track_complement=True,
                factorization="auto", method="da_mmala")
    try:
        p.init(x0, z0)
        p.step(warmup)
        torch.cuda.synchronize()
        a0, _, _ = p.diagnostics()
        _, q0 = p.delayed()
        t0 = time.perf_counter()
        p.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        a1, f1, _ = p.diagnostics()
        _, q1 = p.delayed()
    finally:
        p.close()
    passes, accepts = float((q1 - q0).sum()), float((a1 - a0).sum())
    return dict(value=round(C * steps / wall, 1), unit="chain-steps/s", steps=steps,
                ms_per_step=round(1e3 * wall / steps, 4), true_model="r_T = 256 (56 complement coordinates)",
                pass_rate=round(passes / (C * steps), 4), accept_rate=round(accepts / (C * steps), 4),
                second_stage_acceptance=round(accepts / passes, 4) if passes else None,
                failures=int(f1.sum()), step_cost_over_mmala=round(wall / mmala_wall, 3))


def run_logged(srv, total, what, slice_s=20.0):
    """srv.run() in slices of slice_s seconds of server clock, logging progress between them."""
    done = 0
    while done < total:
        done += srv.run(until=srv.clock() + slice_s)
        st = srv.stats()
        log(f"bench: serving {what}: {done} of {total} requests finished ({st['pending']} waiting, "
            f"{st['live']} admitted)")
        if st["pending"] == 0 and st["live"] == 0:
            break
    return done


def serving_leg(ctx, w, n_requests, load, slots=1024, max_requests=48, quantum=20, seed=11):
    """Poisson stream of inverse problems on the served workload (129x129 grid, r = 200,
    ResNet 400x4 with 100 outputs): per request d_y in {25, 50, 100}, chains in [8, 128],
    steps in [500, 5000], fresh seeded m_true and noise. The arrival rate is
    load * capacity / E[C N], with the capacity measured first by a saturating burst.
    Returns p50/p99 time-to-posterior-mean (arrival to mean field in host memory)."""
    import torch
    from paper_2403_08220_amd import Problem, Server
    from synth import draw_requests

    buckets = [(25, slots), (50, slots), (100, slots)]
    srv = Server(ctx, buckets, max_requests=max_requests, steps_per_quantum=quantum, dt=w.dt, precision="bf16")

    def data(reqs):
        """y = f(x_true)[:d_y] + sigma eps, sigma = 1% of max |f(x_true)[:d_y]| (f on the device)."""
        out = []
        chunk = 256
        ev = Problem(ctx, chunk, np.zeros(w.d_y), np.ones(w.d_y), 0.1, track_complement=False)
        for k0 in range(0, len(reqs), chunk):
            part = reqs[k0:k0 + chunk]
            xt = np.stack([np.random.default_rng(q.truth_seed).standard_normal(w.r) for q in part])
            f = ev.eval_geometry(torch.tensor(xt, dtype=torch.float64, device="cuda:0"), want_H=False)["f"]
            f = f.cpu().numpy()
            for q, fq in zip(part, f):
                fo = fq[: q.d_y]
                sigma = 0.01 * np.max(np.abs(fo))
                y = fo + sigma * np.random.default_rng(q.noise_seed).standard_normal(q.d_y)
                out.append((y, np.full(q.d_y, sigma ** 2)))
        ev.close()
        return out

    # capacity: a saturating burst (all requests at t = 0, 300 steps each)
    burst = draw_requests(24, 1.0, seed=seed + 1)
    for q, (y, nv) in zip(burst, data(burst)):
        srv.submit(seed=q.chain_seed, request_id=100000 + q.rid, y=y, noise_var=nv, n_chains=q.chains, n_steps=300)
    t0 = srv.clock()
    run_logged(srv, len(burst), "capacity burst")
    t1 = srv.clock()
    srv.poll(len(burst), with_means=False)
    kappa = sum(q.chains * 300 for q in burst) / (t1 - t0)

    mean_work = 68.0 * 2750.0
    rate = load * kappa / mean_work
    reqs = draw_requests(n_requests, rate, seed=seed)
    ys = data(reqs)
    start = srv.clock() + 0.05
    for q, (y, nv) in zip(reqs, ys):
        srv.submit(seed=q.chain_seed, request_id=q.rid + 1, y=y, noise_var=nv, n_chains=q.chains, n_steps=q.steps,
                   arrival=start + q.arrival)
    run_logged(srv, n_requests, "stream")
    res = srv.poll(n_requests, with_means=True)
    srv.close()
    lat = np.array([r["finished"] - r["arrival"] for r in res])
    wait = np.array([r["admitted"] - r["arrival"] for r in res])
    work = sum(r["n_chains"] * r["n_steps"] for r in res)
    span = max(r["finished"] for r in res) - start
    finite = all(np.all(np.isfinite(r["mean"])) for r in res)
    return {"requests": len(res), "load": load, "capacity_chain_steps_per_s": round(kappa, 1),
            "arrival_rate_per_s": round(rate, 4), "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4), "mean_s": round(float(lat.mean()), 4),
            "wait_p50_s": round(float(np.percentile(wait, 50)), 4),
            "wait_p99_s": round(float(np.percentile(wait, 99)), 4),
            "throughput_chain_steps_per_s": round(work / span, 1), "makespan_s": round(span, 3),
            "means_finite": bool(finite),
            "setup": f"buckets d_y 25/50/100 x {slots} slots, {max_requests} requests per bucket, "
                     f"{quantum} steps per quantum, BF16 path, dt {w.dt}"}


def traffic_record(kernel, workload_tag):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or
    None when that summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    sha = source_sha256(kernel)
    if sha is None or rec.get("source_sha256") != sha:
        return None
    return rec.get("bytes_per_launch")


def _csv_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


# The profiled bench commands of each workload's committed summaries (the kernel trace run,
# then one FETCH_SIZE and one WRITE_SIZE run of the counter command).
_PROFILE_ZERO = "--fp64-steps 0 --baseline-steps 0 --serve-requests 0 --ess-steps 0 --da-steps 0 --no-cpu-baseline"
PROFILE_RUNS = {
    "mid": dict(desc="BF16 path, 512 chains",
                trace=f"python3 bench.py --steps 100 {_PROFILE_ZERO} --large-steps 0",
                counters=f"python3 bench.py --steps 20 --warmup 5 {_PROFILE_ZERO} --large-steps 0"),
    "mid_f64": dict(desc="plain FP64 path, 512 chains",
                    trace=f"python3 bench.py --precision f64 --steps 100 {_PROFILE_ZERO} --large-steps 0",
                    counters=f"python3 bench.py --precision f64 --steps 20 --warmup 5 {_PROFILE_ZERO} "
                             "--large-steps 0"),
    "large": dict(desc="FP8 path at 257x257, r = 400, ResNet 800x6, d_y = 400, 4096 chains",
                  trace=f"python3 bench.py --steps 2 --warmup 1 {_PROFILE_ZERO} --large-steps 10 --large-fp64-steps 0",
                  counters=f"python3 bench.py --steps 2 --warmup 1 {_PROFILE_ZERO} --large-steps 3 "
                           "--large-fp64-steps 0"),
}


def summarize_profiles(trace_dir, fetch_dir, write_dir, command, workload_tag="mid", desc="BF16 path, 512 chains"):
    """Turns rocprofv3 output (one --kernel-trace --stats run, one --pmc FETCH_SIZE and
    one --pmc WRITE_SIZE run of the same bench command) into the committed summaries
    under profiles/: per-kernel statistics of the step kernels, and the HBM traffic per
    launch of every step kernel at its full-batch grid, each counter scaled by what it
    reads for the calibration copy (a 512 MiB device copy: 512 MiB read, 512 MiB written)."""
    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    trace = _csv_rows(os.path.join(trace_dir, "run_kernel_trace.csv"))
    groups = {}
    for r in trace:
        key = (r["Kernel_Name"].split("(")[0].replace("void ", ""),
               int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in groups.values())
    lines = [f"# rocprofv3 kernel statistics, {workload_tag} workload ({desc})", "",
             f"Command: `{command['trace']}`", "",
             "Grouped by kernel and grid size (work-items): the per-step launches cover all chains; "
             "launches at small grids belong to the Gauss-Newton start and the data setup.", "",
             "| Kernel | Grid | Calls | Average us | Min us | Max us | Share % |", "|---|---|---|---|---|---|---|"]
    for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:24]:
        lines.append(f"| `{k}` | {g} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} | "
                     f"{100.0 * sum(v) / total:.2f} |")
    with open(os.path.join(prof, f"step_kernels_{workload_tag}_kernel_stats.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    def per_kernel(rows):
        out = {}
        for r in rows:
            key = (r["Kernel_Name"].split("(")[0].replace("void ", ""), int(r["Grid_Size"]))
            out.setdefault(key, []).append(float(r["Counter_Value"]))
        return out

    fetch = per_kernel(_csv_rows(os.path.join(fetch_dir, "run_counter_collection.csv")))
    write = per_kernel(_csv_rows(os.path.join(write_dir, "run_counter_collection.csv")))
    cal_bytes = float(1 << 29)
    f_cal = max(v[0] for (k, g), v in fetch.items() if k == "__amd_rocclr_copyBuffer") * 1024.0
    w_cal = max(v[0] for (k, g), v in write.items() if k == "__amd_rocclr_copyBuffer") * 1024.0
    f_scale, w_scale = cal_bytes / f_cal, cal_bytes / w_cal
    lines = [f"# HBM traffic per launch, {workload_tag} workload ({desc})", "",
             f"FETCH_SIZE: `{command['fetch']}`", "", f"WRITE_SIZE: `{command['write']}`", "",
             f"Calibration: the 512 MiB device copy reads {f_cal / 2**20:.1f} MiB by FETCH_SIZE and writes "
             f"{w_cal / 2**20:.1f} MiB by WRITE_SIZE: scales {f_scale:.3f} (fetch) and {w_scale:.3f} (write).", "",
             "| Kernel | Grid | Launches | Read MB | Written MB | Total MB |", "|---|---|---|---|---|---|"]
    records = {}
    for (k, g), fv in sorted(fetch.items(), key=lambda kv: -max(kv[1]))[:24]:
        if not k.startswith("dino::") or (k, g) not in write:
            continue
        wv = write[(k, g)]
        rd = sum(fv) / len(fv) * 1024.0 * f_scale
        wr = sum(wv) / len(wv) * 1024.0 * w_scale
        lines.append(f"| `{k}` | {g} | {len(fv)} | {rd / 1e6:.2f} | {wr / 1e6:.2f} | {(rd + wr) / 1e6:.2f} |")
        base = k.split("::")[-1].split("<")[0]
        if base not in records or g > records[base]["grid"]:
            records[base] = dict(grid=g, read_bytes=rd, write_bytes=wr)
    with open(os.path.join(prof, f"step_kernels_{workload_tag}_traffic.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    for base, rec in records.items():
        sha = source_sha256(base)
        if sha is None:
            continue
        with open(os.path.join(prof, f"{base}_{workload_tag}_traffic.json"), "w") as fh:
            json.dump(dict(kernel=base, grid=rec["grid"], bytes_per_launch=round(rec["read_bytes"] + rec["write_bytes"]),
                           read_bytes=round(rec["read_bytes"]), write_bytes=round(rec["write_bytes"]),
                           fetch_scale=f_scale, write_scale=w_scale, source_sha256=sha,
                           commands=[command["fetch"], command["write"]]), fh, indent=1)
            fh.write("\n")


def fused_metric(prof, prec, dual):
    """The profile's factor stage has no kernel of its own: the metric kernel factorises."""
    return bool(dual and prec in ("bf16", "fp8") and prof.get("cholesky", {}).get("launches", 1) == 0)


def stage_table(prof, w, C, L_res, accept_rate, prec, dual):
    """Per-stage time, algorithmic work rate and roofline fraction from a stage profile."""
    stages = {}
    fused = fused_metric(prof, prec, dual)
    for name, v in prof.items():
        if v["launches"] == 0:  # a stage with no kernel of its own on this path
            continue
        amt, unit, bound, peak = stage_work(name, w.width, C, w.r, w.d_y, L_res, accept_rate, w.d_m - w.r, prec,
                                            dual=dual, fused=fused)
        t = v["ms_per_step"] * 1e-3
        ach = (amt / t / (1e12 if unit == "TFLOP/s" else 1e9)) if t > 0 else 0.0
        stages[name] = dict(ms=round(v["ms_per_step"], 4), launches=v["launches"], bound=bound,
                            achieved=round(ach, 3), peak=peak, unit=unit, frac=round(ach / peak, 4))
    return stages


def large_leg(steps, warmup, fp64_steps):
    """The largest shape: 257x257 grid, r = 400, ResNet 800x6, d_y = 400, 4096 chains, on the
    FP8 path (FP8 reverse sweep, BF16 Gauss-Newton tiles, FP64 factor and MH), beside the
    plain FP64 path on the same problem for a few steps."""
    from paper_2403_08220_amd import Context
    from synth import draw_network, workload

    w = workload("large")
    layers = draw_network(w)
    L_res = sum(1 for k, _, _ in layers if k == "resid")
    ctx = Context(0)
    try:
        ctx.load_prior(w.n, w.gamma, w.delta, w.r)
        ctx.load_network(layers)
        y, nv = device_data(w, ctx)
        x0, z0, init_info, _ = laplace_start(w, ctx, y, nv)
        log(f"bench: large leg, Laplace start ready {init_info}")
        res = run_path(w, ctx, y, nv, x0, z0, "fp8", steps, warmup, profile=True, factorization="primal")
        C = w.chains
        stages = stage_table(res.get("profile", {}), w, C, L_res, res["accept_rate"], "fp8", False)
        dom = max(stages, key=lambda k: stages[k]["ms"])
        jac = stages.get("jacobian")
        kern = STAGE_KERNEL_FP8_LARGE.get(dom, dom)
        out = dict(
            workload="257x257 grid, r=400 KLE, ResNet 800x6 GELU, d_y=400, 4096 chains, dt=3e-4",
            precision="fp8", value=round(C * steps / res["wall_s"], 1), unit="chain-steps/s", steps=steps,
            ms_per_step=round(1e3 * res["wall_s"] / steps, 4), accept_rate=round(res["accept_rate"], 4),
            failures=res["failures"], stages=stages,
            dominant=dict(stage=dom, kernel=kern, **{k: stages[dom][k] for k in ("bound", "achieved", "peak",
                                                                                 "unit", "frac")}),
            roofline_fp8_sweep=None if jac is None else dict(
                bound="mfma", achieved=jac["achieved"], peak=PEAKS["fp8_TFLOPs"], unit="TFLOP/s",
                frac=jac["frac"], kernel="jac_sweep_fp8_kernel", ms_per_launch=jac["ms"],
                traffic=traffic_record("jac_sweep_fp8_kernel", "large")),
            init=init_info)
        if fp64_steps > 0:
            r64 = run_path(w, ctx, y, nv, x0, z0, "f64", fp64_steps, 1, profile=False, factorization="primal")
            out["fp64_plain"] = dict(value=round(C * fp64_steps / r64["wall_s"], 1), unit="chain-steps/s",
                                     steps=fp64_steps, ms_per_step=round(1e3 * r64["wall_s"] / fp64_steps, 4),
                                     accept_rate=round(r64["accept_rate"], 4))
        return out
    finally:
        ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="bf16", choices=["f64", "bf16"])
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="steps of the plain FP64 leg (default: --steps, so both ESS windows match; 0: skip)")
    ap.add_argument("--no-profile", action="store_true", help="time without the per-stage events")
    ap.add_argument("--factorization", default="auto", choices=["auto", "primal", "dual"],
                    help="auto: the observation-space (d_y x d_y) factorisation when d_y < r")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--baseline-steps", type=int, default=400,
                    help="steps of each baseline leg, pCN, MALA and LA-pCN (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests of the serving leg (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="offered load as a fraction of capacity")
    ap.add_argument("--ess-steps", type=int, default=1000,
                    help="timed steps of the ESS/s leg on the mix workload (0: skip)")
    ap.add_argument("--da-steps", type=int, default=None,
                    help="timed steps of the delayed-acceptance leg (default: --steps; 0: skip)")
    ap.add_argument("--large-steps", type=int, default=40,
                    help="steps of the FP8 leg at the largest shape (4096 chains; 0: skip)")
    ap.add_argument("--large-fp64-steps", type=int, default=4, help="plain FP64 steps at the largest shape")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write the profiles/ summaries from rocprofv3 output (no GPU needed) and exit")
    ap.add_argument("--profile-workload", default="mid", choices=sorted(PROFILE_RUNS),
                    help="which workload's bench commands the rocprofv3 output came from")
    args = ap.parse_args()
    if args.summarize_profiles:
        run = PROFILE_RUNS[args.profile_workload]
        summarize_profiles(*args.summarize_profiles, command={
            "trace": f"rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- {run['trace']}",
            "fetch": f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- {run['counters']}",
            "write": f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o run -- {run['counters']}"},
            workload_tag=args.profile_workload, desc=run["desc"])
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}). "
              "Chains are independent; sharding would place whole chain blocks or requests on separate GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import torch  # noqa: F401
    from paper_2403_08220_amd import Context, tuning_table
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
    ctx, y, nv = make_problem_inputs(w, ctx_builder)
    x0, z0, init_info, x_map = laplace_start(w, ctx, y, nv)
    log(f"bench: Laplace start ready {init_info}")
    copy_calibration()
    res = run_path(w, ctx, y, nv, x0, z0, args.precision, args.steps, args.warmup, profile=not args.no_profile,
                   factorization=args.factorization)
    log(f"bench: {args.precision} path: {res['wall_s']:.3f} s, accept {res['accept_rate']:.3f}")
    C, steps = w.chains, args.steps
    value = C * steps / res["wall_s"]
    ms_per_step = 1e3 * res["wall_s"] / steps

    fp64 = None
    fp64_steps = steps if args.fp64_steps is None else args.fp64_steps
    if fp64_steps > 0 and args.precision != "f64":
        r64 = run_path(w, ctx, y, nv, x0, z0, "f64", fp64_steps, args.warmup, profile=False,
                       factorization=args.factorization)
        rate64, note64 = ess_rate(r64["median_ess"], r64["wall_s"], C)
        fp64 = dict(value=round(C * fp64_steps / r64["wall_s"], 1), unit="chain-steps/s",
                    steps=fp64_steps, ms_per_step=round(1e3 * r64["wall_s"] / fp64_steps, 4),
                    accept_rate=round(r64["accept_rate"], 4), median_ess=round(r64["median_ess"], 1),
                    ess_per_s=rate64, ess_note=note64)
        log(f"bench: f64 path: {r64['wall_s']:.3f} s, accept {r64['accept_rate']:.3f}")

    baselines = None
    if args.baseline_steps > 0:
        baselines = {}
        fixed = laplace_metric(w, ctx, y, nv, x_map)
        for method in ("pcn", "mala", "lapcn"):
            b = baseline_leg(method, w, ctx, y, nv, x0, z0, args.precision, args.baseline_steps, args.warmup, res,
                             fixed=fixed if method == "lapcn" else None)
            baselines[method] = b
            log(f"bench: {method} baseline: dt {b['dt']}, accept {b['accept_rate']}, {b['value']} chain-steps/s")

    ess = None
    if args.ess_steps > 0:
        log(f"bench: ESS/s leg (mix workload), {args.ess_steps} steps per path ...")
        ess = ess_leg(ctx, args.ess_steps, 200)
        log(f"bench: ESS/s bf16 {ess['bf16']['ess_per_s']} f64 {ess['f64']['ess_per_s']}")
    da_res = None
    da_steps = steps if args.da_steps is None else args.da_steps
    if da_steps > 0:
        da_res = da_leg(ctx, w, layers, y, nv, x0, z0, args.precision, da_steps, args.warmup,
                        res["wall_s"] * da_steps / steps)
        log(f"bench: DA leg {da_res['value']} chain-steps/s, pass rate {da_res['pass_rate']}")
    prof = res.get("profile", {})
    # the observation-space form is taken when asked for, or by "auto" when d_y < r
    dual = args.factorization == "dual" or (args.factorization == "auto" and w.d_y < w.r)
    stages = stage_table(prof, w, C, L_res, res["accept_rate"], args.precision, dual)
    roof = None
    if stages:
        dom = max(stages, key=lambda k: stages[k]["ms"])
        s = stages[dom]
        kern = (stage_kernel(dom, dual, w.width, w.r, w.d_y, fused=fused_metric(prof, args.precision, dual))
                if args.precision == "bf16" else dom)
        roof = dict(bound=s["bound"], achieved=s["achieved"], peak=s["peak"], unit=s["unit"], frac=s["frac"],
                    traffic=traffic_record(kern, "mid") if args.precision == "bf16" else None,
                    kernel=kern, stage=dom, ms_per_launch=round(s["ms"] / max(s["launches"], 1), 4),
                    profiled_ms_per_step=round(res.get("profiled_ms_per_step", 0.0), 4))
    large = None
    if args.large_steps > 0:
        log(f"bench: large leg (FP8), {args.large_steps} steps ...")
        large = large_leg(args.large_steps, max(2, args.warmup // 4), args.large_fp64_steps)
        log(f"bench: large FP8 {large['value']} chain-steps/s, {large['ms_per_step']} ms/step, "
            f"accept {large['accept_rate']}")
    serving = None
    if args.serve_requests > 0:
        log(f"bench: serving leg, {args.serve_requests} requests at load {args.serve_load} ...")
        serving = serving_leg(ctx, workload("serve"), args.serve_requests, args.serve_load)
        log(f"bench: serving p50 {serving['p50_s']} s, p99 {serving['p99_s']} s")
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle) ...")
        cpu = cpu_baseline(w, layers, x0, z0, factor="dual" if dual else "primal")
        one = cpu_baseline(w, layers, x0, z0, factor="dual" if dual else "primal", threads=1, budget_s=12.0)
        cpu["one_core"] = {k: one[k] for k in ("value", "unit", "cores", "sample")}
    main_rate, main_note = ess_rate(res["median_ess"], res["wall_s"], C)
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
        "dtype": "f64" if args.precision == "f64" else "bf16",
        "data": "synthetic: seeded Xavier-normal ResNet and KLE prior draws (no trained weights or PDE data); "
                "chains start from Laplace samples at the Gauss-Newton MAP",
        "config": {"workload": "129x129 grid, r=200 KLE, ResNet 400x4 GELU, d_y=100, 512 chains, dt=3e-4",
                   "grid": w.n, "r": w.r, "width": w.width, "depth": w.depth, "d_y": w.d_y, "chains": C,
                   "dt": w.dt, "precision": args.precision, "factorization": args.factorization},
        "ess_per_s": main_rate,
        "ess_note": main_note,
        "median_ess": round(res["median_ess"], 1),
        "ess_floor": ess_floor(C),
        "median_ess_frac": res["median_ess_frac"],
        "accept_rate": round(res["accept_rate"], 4),
        "roofline": roof,
        "stages": stages,
        "fp64_plain": fp64,
        "ess_leg": ess,
        "delayed_acceptance": da_res,
        "large_fp8": large,
        "baselines": baselines,
        "serving": serving,
        "cpu_baseline": cpu,
        "init": init_info,
        "launch": "graphs of 8 steps (dino_step default)",
        "autotune": [dict(kind=e["kind"], shape=list(e["shape"]), choice=e["choice"],
                          ms=[round(v, 4) for v in e["ms"]]) for e in tuning_table()],
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
