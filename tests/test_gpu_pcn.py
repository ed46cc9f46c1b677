"""pCN baseline on the device (Sec. 2.6, eq. pCN_proposal; the pCN row of the baselines
of Sec. 6.1) against the FP64 oracle's pCN transition, through the C ABI.

Tolerances: FP64 path, accept decisions identical and states within 1e-9 relative (the
proposal is s x + beta xi in FP64 on both sides; only the misfit's rounding order
differs); complement (FP32 state) 1e-5. BF16 path (the forward in FP32 arithmetic on
BF16-rounded weights where the mixed path rounds them): acceptance rate within a few
points of the oracle's on coupled streams, and the cached misfit within 1e-4 relative of
the oracle's at the device's own states.
"""
import copy

import numpy as np
import pytest

from oracle import mcmc
from tests.helpers import device_problem, make_case, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def resnet_case(C, dt, **kw):
    """r = 40, width 80, d_y = 20: several tiles with ragged tails."""
    case = make_case("tiny", chains=C, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                     bias_scale=0.3, noise_scale=0.2, dt=dt, **kw)
    case["prob"].method = "pcn"
    return case


def coupled(case, n_steps, precision="f64", chains_idx=None, trace=False):
    ctx, p = device_problem(case, precision=precision, method="pcn", trace_capacity=n_steps if trace else 0)
    p.init(case["x0"], case["z0"])
    p.step(n_steps)
    x, z = p.states()
    acc, fail, steps = p.diagnostics()
    assert steps == n_steps
    idx = np.arange(case["C"]) if chains_idx is None else np.asarray(chains_idx)
    st = mcmc.init_state(case["prob"], case["x0"][idx], case["z0"][idx].astype(np.float64), chains=idx)
    xs, phis = mcmc.run(case["prob"], st, n_steps, trace=trace)
    out = dict(x=x[idx], z=z[idx], acc=acc[idx], fail=fail[idx], st=st, p=p, ctx=ctx, xs=xs, phis=phis, idx=idx)
    if trace:
        out["trace"] = p.trace()
    return out


def close(r):
    r["p"].close()
    r["ctx"].close()


def test_pcn_coupled_chains_parity():
    print("pcn f64: 70 chains x 40 steps, resnet r=40", flush=True)
    case = resnet_case(70, 0.2)
    r = coupled(case, 40, trace=True)
    np.testing.assert_array_equal(r["acc"], r["st"].accepts)
    assert np.all(r["fail"] == 0)
    assert 0.1 < r["acc"].sum() / (70 * 40) < 0.9
    assert rel_err(r["x"], r["st"].x) < 1e-9
    assert np.max(np.abs(r["z"] - r["st"].z)) < 1e-5
    xt, pt = r["trace"]
    assert xt.shape == (40, 70, 40)
    np.testing.assert_allclose(xt, r["xs"].astype(np.float32), rtol=1e-6, atol=1e-6)
    assert np.max(np.abs(pt - r["phis"]) / (1 + np.abs(r["phis"]))) < 1e-11
    phi, _, _ = r["p"].cache()
    assert np.max(np.abs(phi - r["st"].cache.phi) / (1 + r["st"].cache.phi)) < 1e-11
    close(r)


def test_pcn_tiny_literal():
    print("pcn f64: tiny workload x 60 steps", flush=True)
    case = make_case("tiny")
    case["prob"].method = "pcn"
    r = coupled(case, 60)
    np.testing.assert_array_equal(r["acc"], r["st"].accepts)
    assert rel_err(r["x"], r["st"].x) < 1e-9
    assert np.max(np.abs(r["z"] - r["st"].z)) < 1e-5
    close(r)


def test_pcn_without_likelihood_equals_mmala():
    """Phi = 0: both kernels move every chain by s x + beta xi on the same streams."""
    print("pcn vs mmala, zero likelihood", flush=True)
    case = resnet_case(9, 0.8)
    case["prob"].noise_var = np.full(case["w"].d_y, np.inf)
    out = {}
    for method in ("pcn", "mmala"):
        ctx, p = device_problem(case, method=method)
        p.init(case["x0"], case["z0"])
        p.step(20)
        acc, fail, _ = p.diagnostics()
        assert np.all(acc == 20) and np.all(fail == 0)
        out[method] = p.states()
        p.close()
        ctx.close()
    assert rel_err(out["pcn"][0], out["mmala"][0]) < 1e-12
    np.testing.assert_array_equal(out["pcn"][1], out["mmala"][1])


def test_pcn_profile_launches():
    print("pcn profile", flush=True)
    case = resnet_case(16, 0.2)
    ctx, p = device_problem(case, method="pcn")
    p.init(case["x0"], case["z0"])
    p.set_profiling(True)
    p.step(5)
    prof, steps = p.profile()
    assert steps == 5
    n_layers = len(case["layers"])
    assert prof["proposal"]["launches"] == 1 and prof["forward"]["launches"] == n_layers
    for stage in ("jacobian", "misfit_ppg", "gn_hessian", "cholesky"):
        assert prof[stage]["launches"] == 0
    assert prof["accept"]["launches"] == 1 and prof["complement"]["launches"] == 1
    p.close()
    ctx.close()


def test_pcn_full_size_mid_sampled():
    """The 129x129 / r=200 / ResNet 400x4 / d_y=100 workload, 512 chains; the oracle
    follows a sample of chains over coupled streams."""
    print("pcn f64: full-size mid, 512 chains x 4 steps", flush=True)
    case = make_case("mid")
    case["prob"].method = "pcn"
    r = coupled(case, 4, chains_idx=[0, 1, 255, 256, 511])
    np.testing.assert_array_equal(r["acc"], r["st"].accepts)
    assert rel_err(r["x"], r["st"].x) < 1e-9
    assert np.max(np.abs(r["z"] - r["st"].z)) < 1e-5
    close(r)


@pytest.mark.parametrize("name", ["resnet", "mid"])
def test_pcn_bf16(name):
    print(f"pcn bf16: {name}", flush=True)
    if name == "mid":
        case = make_case("mid", chains=64)
        case["prob"].method = "pcn"
        n_steps = 30
    else:
        case = resnet_case(64, 0.2)
        n_steps = 60
    ctx, p = device_problem(case, precision="bf16", method="pcn")
    p.init(case["x0"], case["z0"])
    p.step(n_steps)
    acc, fail, steps = p.diagnostics()
    assert steps == n_steps and fail.sum() == 0
    st = mcmc.init_state(case["prob"], case["x0"], case["z0"].astype(np.float64))
    mcmc.run(case["prob"], st, n_steps, trace=False)
    C = case["C"]
    a_gpu, a_ref = acc.sum() / (C * n_steps), st.accepts.sum() / (C * n_steps)
    print(f"pcn acceptance bf16 {a_gpu:.3f} vs fp64 oracle {a_ref:.3f}", flush=True)
    assert abs(a_gpu - a_ref) < 0.08
    x, _ = p.states()
    phi, _, _ = p.cache()
    _, ref_phi = mcmc.misfit(case["prob"], x)
    assert np.max(np.abs(phi - ref_phi) / (1 + ref_phi)) < 1e-4
    p.close()
    ctx.close()


def test_pcn_method_is_validated():
    from paper_2403_08220_amd import Context, DinoError, _lib
    from paper_2403_08220_amd._lib import ProblemDesc, check
    import ctypes as ct

    case = resnet_case(4, 0.2)
    w = case["w"]
    ctx = Context(0)
    ctx.load_prior(w.n, w.gamma, w.delta, w.r)
    ctx.load_network(case["layers"])
    d = ProblemDesc(n_chains=4, d_y=w.d_y, precision=0, track_complement=1, trace_capacity=0, factorization=0,
                    dt=0.2, seed=1, request_id=0, method=7)
    nbytes = ct.c_size_t()
    with pytest.raises(DinoError, match="method"):
        check(ctx.lib.dino_problem_workspace_bytes(ctx.h, ct.byref(d), ct.byref(nbytes)))
    ctx.close()
