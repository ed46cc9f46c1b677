"""Posterior statistics of the mixed-precision path against FP64.

Target: the BF16 path (FP32 forward, BF16 Jacobian and GN Hessian, FP64 factor and
MH) matches the FP64 posterior mean and pointwise variance fields (Rao-Blackwellised:
Psi_r xbar and diag(Psi_r S Psi_r^T) + v_perp) to within 1% relative L2.

* Well-mixing case (ResNet r = 40, d_y = 20, sigma = 0.5, dt = 0.1, about 43% accepted;
  32768 chains x 1000 steps from prior draws, burn-in 20%): BF16 and FP64 run on coupled
  streams (same keys and initial states). An FP64 replicate with another seed gives the
  Monte Carlo scale of the comparison; the BF16 deviation must be within 1% and below
  that scale. The chain count keeps the Monte Carlo scale well under 1% (at 4096 chains
  and sigma = 0.2 the replicate itself differed by 1-2%, so 1% could not be resolved).
  The FP64 device path is the oracle's arithmetic (stage parity 1e-10, identical
  decisions on coupled streams, test_gpu_parity), so FP64 here stands for the oracle
  at a chain count the CPU oracle cannot run in a test.
* Configured case (33x33 grid, r = 32, MLP 64x2, d_y = 16, sigma = 0.01, tuned
  dt = 3e-3): FP64 device vs the CPU oracle itself over 4 chains x 2000 steps from prior
  draws (1e-6 relative, coupled; the device trace holds FP32 states), and BF16 vs the
  oracle, reported. This posterior is a thin curved manifold far from the prior: chains
  started at prior draws are still travelling after 8000 steps (the chain mean moves
  from about 0.8 to 2.3 in norm), and the BF16 and FP64 transients differ by more than
  their Monte Carlo scale, so moments of such runs compare transients, not posteriors.
  The stationarity check: 2048 chains are run 40000 FP64 steps from prior draws; from
  those states BF16 and FP64 run 8000 steps on coupled streams, and an FP64 replicate
  with another seed gives the Monte Carlo scale. An inexact BF16 transition would drift
  away from the FP64 stationary law; its deviation must stay within that scale.
"""
import numpy as np
import pytest

from oracle import mcmc, prior, stats
from tests.helpers import device_problem, make_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(case, precision, steps, seed=None):
    ctx, p = device_problem(case, precision=precision, trace_capacity=steps)
    if seed is not None:
        p.close()
        from paper_2403_08220_amd import Problem
        prob = case["prob"]
        p = Problem(ctx, case["C"], prob.y, prob.noise_var, prob.dt, seed=seed, precision=precision,
                    track_complement=False, trace_capacity=steps)
    p.init(case["x0"], None)
    p.step(steps)
    acc, fail, _ = p.diagnostics()
    mean, var, xbar, S = p.posterior(steps // 5)
    p.close()
    ctx.close()
    return dict(mean=mean, var=var, accept=acc.sum() / (case["C"] * steps), failures=int(fail.sum()))


def test_bf16_posterior_within_one_percent_of_fp64():
    case = make_case("tiny", chains=32768, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                     bias_scale=0.3, noise_scale=0.5, dt=0.1)
    steps = 1000
    print("statistics: bf16 vs fp64, 32768 chains x 1000 steps", flush=True)
    f64 = run(case, "f64", steps)
    b16 = run(case, "bf16", steps)
    rep = run(case, "f64", steps, seed=case["prob"].seed + 1000)
    dm, dv = rel_l2(b16["mean"], f64["mean"]), rel_l2(b16["var"], f64["var"])
    rm, rv = rel_l2(rep["mean"], f64["mean"]), rel_l2(rep["var"], f64["var"])
    print(f"accept fp64 {f64['accept']:.3f} bf16 {b16['accept']:.3f}; rel L2 bf16 vs fp64: mean {dm:.2e} "
          f"var {dv:.2e}; independent fp64 replicate: mean {rm:.2e} var {rv:.2e}", flush=True)
    print(f"failures: fp64 {f64['failures']}, bf16 {b16['failures']} of {case['C'] * steps} transitions", flush=True)
    # a failure (non-finite misfit or non-positive pivot) rejects its proposal; it must stay rare
    assert f64["failures"] <= 1e-5 * case["C"] * steps and b16["failures"] <= 1e-5 * case["C"] * steps
    assert dm < 0.01 and dv < 0.01
    assert dm < max(rm, 1e-3) and dv < max(rv, 1e-3)


def test_configured_case_against_oracle():
    case = make_case("tiny", chains=4, dt=3e-3)
    steps = 2000
    print("statistics: configured 33x33 case vs the oracle, 4 chains x 2000 steps", flush=True)
    st = mcmc.init_state(case["prob"], case["x0"])
    xs, _ = mcmc.run(case["prob"], st, steps)
    B = prior.KLEBasis(case["w"].n, case["w"].gamma, case["w"].delta, case["w"].r)
    o_mean, o_var = stats.posterior_moments(xs, B)[:2]
    f64 = run(case, "f64", steps)
    b16 = run(case, "bf16", steps)
    dm64, dv64 = rel_l2(f64["mean"], o_mean), rel_l2(f64["var"], o_var)
    dm16, dv16 = rel_l2(b16["mean"], o_mean), rel_l2(b16["var"], o_var)
    print(f"oracle accept {st.accepts.sum() / (4 * steps):.3f}, fp64 {f64['accept']:.3f}, bf16 {b16['accept']:.3f}; "
          f"rel L2 vs oracle: fp64 mean {dm64:.2e} var {dv64:.2e}; bf16 mean {dm16:.2e} var {dv16:.2e}", flush=True)
    # the device trace holds FP32 states: 1e-6 relative on the moments
    assert dm64 < 1e-6 and dv64 < 1e-6
    assert np.isfinite(dm16) and np.isfinite(dv16)

    # stationarity: 2048 chains warmed up by 40000 FP64 steps, then BF16 and FP64 on coupled
    # streams and an FP64 replicate (another seed) from the same states
    from paper_2403_08220_amd import Context, Problem

    wide = make_case("tiny", chains=2048, dt=3e-3)
    w, prob = wide["w"], wide["prob"]
    ctx = Context(0)
    try:
        ctx.load_prior(w.n, w.gamma, w.delta, w.r)
        ctx.load_network(wide["layers"])

        def chains(precision, seed, x0, n_steps, trace):
            p = Problem(ctx, wide["C"], prob.y, prob.noise_var, prob.dt, seed=seed, request_id=prob.request_id,
                        precision=precision, track_complement=False, trace_capacity=n_steps if trace else 0)
            try:
                p.init(x0, None)
                p.step(n_steps)
                acc, fail, _ = p.diagnostics()
                out = dict(accept=acc.sum() / (wide["C"] * n_steps), failures=int(fail.sum()))
                if trace:
                    out["mean"], out["var"] = p.posterior(0)[:2]
                else:
                    out["x"] = p.states()[0]
                return out
            finally:
                p.close()

        warm = chains("f64", prob.seed + 7, wide["x0"], 40000, False)
        f64 = chains("f64", prob.seed, warm["x"], 8000, True)
        b16 = chains("bf16", prob.seed, warm["x"], 8000, True)
        rep = chains("f64", prob.seed + 1000, warm["x"], 8000, True)
    finally:
        ctx.close()
    dm, dv = rel_l2(b16["mean"], f64["mean"]), rel_l2(b16["var"], f64["var"])
    rm, rv = rel_l2(rep["mean"], f64["mean"]), rel_l2(rep["var"], f64["var"])
    print(f"configured case from 40000-step FP64 states, 2048 chains x 8000: accept fp64 {f64['accept']:.4f} "
          f"bf16 {b16['accept']:.4f} (delta {b16['accept'] - f64['accept']:+.4f}); rel L2 bf16 vs fp64: mean {dm:.2e} "
          f"var {dv:.2e}; fp64 replicate: mean {rm:.2e} var {rv:.2e}; failures fp64 {f64['failures']} "
          f"bf16 {b16['failures']}", flush=True)
    assert f64["failures"] == 0 and b16["failures"] == 0
    assert dm < max(rm, 1e-3) and dv < max(rv, 1e-3)


def test_bf16_dual_posterior_at_the_bench_shape():
    """The bench's path (BF16, observation-space form) at its shapes: 129^2 grid, r = 200,
    ResNet 400 x 4, d_y = 100, on the mix workload (sigma = 30% of max |f(x_true)|, dt = 0.1,
    where these chains decorrelate within the run), 4096 chains x 600 steps from Laplace
    samples, burn-in 20%. BF16 and FP64 run on coupled streams (same keys and starts); an
    independent BF16 replicate (another seed) gives the Monte Carlo scale. Measured: coupled
    deviation 1.5% (mean field) and 0.7% (variance) against a Monte Carlo scale of 2.8% and
    1.4%. At 16384 chains the variance scale halves (0.63%, coupled 0.46%) but the mean
    field's stays at 2.9% (coupled 1.8%): this weakly informed mean field has a Monte Carlo
    component that more chains of this length do not reduce, so 1% is not resolvable here
    at a test's cost; the 1% target is asserted on the well-mixing case above. Here the
    BF16 deviation must lie below the Monte Carlo scale (no bias beyond sampling error) and
    below 2%."""
    from paper_2403_08220_amd import Context, Problem, laplace
    from synth import draw_laplace_normals, draw_network, draw_noise, draw_true_state, workload

    w = workload("mix")
    C, steps = 4096, 600
    ctx = Context(0)
    try:
        ctx.load_prior(w.n, w.gamma, w.delta, w.r)
        ctx.load_network(draw_network(w))
        x_true = draw_true_state(w)[: w.r]
        tmp = Problem(ctx, 1, np.zeros(w.d_y), np.ones(w.d_y), 0.1, track_complement=False)
        f_true = tmp.eval_geometry(torch.tensor(x_true[None], device="cuda:0"), want_H=False)["f"].cpu().numpy()[0]
        tmp.close()
        sigma = w.sigma * np.max(np.abs(f_true))
        y, nv = f_true + sigma * draw_noise(w), np.full(w.d_y, sigma ** 2)
        m = laplace.gauss_newton_map(ctx, y, nv)
        x0 = laplace.laplace_samples(ctx, y, nv, m.x, draw_laplace_normals(w, chains=C))
        out = {}
        for tag, prec, seed in (("f64", "f64", w.chain_seed), ("bf16", "bf16", w.chain_seed),
                                ("bf16_rep", "bf16", w.chain_seed + 1000)):
            print(f"statistics at the bench shape: {tag}", flush=True)
            p = Problem(ctx, C, y, nv, w.dt, seed=seed, precision=prec, track_complement=False,
                        trace_capacity=steps, factorization="auto")
            p.init(x0, None)
            p.step(steps)
            acc, fail, _ = p.diagnostics()
            mean, var, _, _ = p.posterior(steps // 5)
            out[tag] = dict(mean=mean, var=var, accept=acc.sum() / (C * steps), failures=int(fail.sum()))
            p.close()
    finally:
        ctx.close()
    f64, b16, rep = out["f64"], out["bf16"], out["bf16_rep"]
    dm, dv = rel_l2(b16["mean"], f64["mean"]), rel_l2(b16["var"], f64["var"])
    rm, rv = rel_l2(rep["mean"], b16["mean"]), rel_l2(rep["var"], b16["var"])
    print(f"bench shape: accept fp64 {f64['accept']:.3f} bf16 {b16['accept']:.3f}; rel L2 bf16 vs fp64 (coupled): "
          f"mean {dm:.2e} var {dv:.2e}; independent replicate: mean {rm:.2e} var {rv:.2e}", flush=True)
    assert f64["failures"] == 0 and b16["failures"] == 0
    assert abs(b16["accept"] - f64["accept"]) < 0.01
    assert dm < rm and dv < rv
    assert dm < 0.02 and dv < 0.02
