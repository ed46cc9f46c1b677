"""MALA baseline on the device (the MALA row of the baselines of Sec. 6.1: the ppg, no
metric) against the FP64 oracle's MALA transition, through the C ABI.

Tolerances: FP64 path, accept decisions identical, states and ppg within 1e-9 relative;
complement (FP32 state) 1e-5. BF16 path: acceptance within 0.08 of the oracle's on
coupled streams; the cached misfit within 1e-4 relative and the ppg within 3e-2
Frobenius relative of the oracle's at the device's own states (the mixed-path bars of
the geometry).
"""
import numpy as np
import pytest

from oracle import mcmc
from tests.helpers import device_problem, make_case, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def resnet_case(C, dt):
    case = make_case("tiny", chains=C, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                     bias_scale=0.3, noise_scale=0.2, dt=dt)
    case["prob"].method = "mala"
    return case


def coupled(case, n_steps, precision="f64", chains_idx=None, trace=False, factorization="primal"):
    ctx, p = device_problem(case, precision=precision, method="mala", trace_capacity=n_steps if trace else 0,
                            factorization=factorization)
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


def test_mala_coupled_chains_parity():
    print("mala f64: 70 chains x 40 steps, resnet r=40", flush=True)
    case = resnet_case(70, 0.01)
    r = coupled(case, 40, trace=True)
    np.testing.assert_array_equal(r["acc"], r["st"].accepts)
    assert np.all(r["fail"] == 0)
    assert 0.1 < r["acc"].sum() / (70 * 40) < 0.95
    assert rel_err(r["x"], r["st"].x) < 1e-9
    assert np.max(np.abs(r["z"] - r["st"].z)) < 1e-5
    _, pt = r["trace"]
    assert np.max(np.abs(pt - r["phis"]) / (1 + np.abs(r["phis"]))) < 1e-11
    phi, g, _ = r["p"].cache()
    assert np.max(np.abs(phi - r["st"].cache.phi) / (1 + r["st"].cache.phi)) < 1e-11
    assert rel_err(g, r["st"].cache.g) < 1e-9
    close(r)


def test_mala_dual_descriptor_is_the_same_chain():
    """MALA forms no factor, so the factorisation field changes nothing."""
    print("mala f64: dual descriptor", flush=True)
    case = resnet_case(37, 0.01)
    r = coupled(case, 20, factorization="dual")
    np.testing.assert_array_equal(r["acc"], r["st"].accepts)
    assert rel_err(r["x"], r["st"].x) < 1e-9
    close(r)


def test_mala_without_likelihood_equals_pcn():
    print("mala vs pcn, zero likelihood", flush=True)
    case = resnet_case(9, 0.8)
    case["prob"].noise_var = np.full(case["w"].d_y, np.inf)
    out = {}
    for method in ("mala", "pcn"):
        ctx, p = device_problem(case, method=method)
        p.init(case["x0"], case["z0"])
        p.step(20)
        acc, fail, _ = p.diagnostics()
        assert np.all(acc == 20) and np.all(fail == 0)
        out[method] = p.states()
        p.close()
        ctx.close()
    assert rel_err(out["mala"][0], out["pcn"][0]) < 1e-12
    np.testing.assert_array_equal(out["mala"][1], out["pcn"][1])


@pytest.mark.parametrize("precision", ["f64", "bf16"])
def test_mala_profile_launches(precision):
    print(f"mala profile {precision}", flush=True)
    case = resnet_case(16, 0.01)
    ctx, p = device_problem(case, precision=precision, method="mala")
    p.init(case["x0"], case["z0"])
    p.set_profiling(True)
    p.step(5)
    prof, steps = p.profile()
    assert steps == 5
    n_layers = len(case["layers"])
    assert prof["proposal"]["launches"] == 1 and prof["forward"]["launches"] == n_layers
    assert prof["cholesky"]["launches"] == 0 and prof["accept"]["launches"] == 1
    if precision == "f64":
        assert prof["jacobian"]["launches"] == n_layers and prof["misfit_ppg"]["launches"] == 1
        assert prof["gn_hessian"]["launches"] == 0
    else:
        assert prof["jacobian"]["launches"] == 1 and prof["gn_hessian"]["launches"] == 1
    p.close()
    ctx.close()


def test_mala_full_size_mid_sampled():
    print("mala f64: full-size mid, 512 chains x 3 steps", flush=True)
    case = make_case("mid")
    case["prob"].method = "mala"
    r = coupled(case, 3, chains_idx=[0, 1, 255, 256, 511])
    np.testing.assert_array_equal(r["acc"], r["st"].accepts)
    assert rel_err(r["x"], r["st"].x) < 1e-9
    assert np.max(np.abs(r["z"] - r["st"].z)) < 1e-5
    close(r)


def test_mala_bf16():
    print("mala bf16: resnet, 64 chains x 60 steps", flush=True)
    case = resnet_case(64, 0.01)
    ctx, p = device_problem(case, precision="bf16", method="mala")
    p.init(case["x0"], case["z0"])
    p.step(60)
    acc, fail, steps = p.diagnostics()
    assert steps == 60 and fail.sum() == 0
    st = mcmc.init_state(case["prob"], case["x0"], case["z0"].astype(np.float64))
    mcmc.run(case["prob"], st, 60, trace=False)
    a_gpu, a_ref = acc.sum() / (64 * 60), st.accepts.sum() / (64 * 60)
    print(f"mala acceptance bf16 {a_gpu:.3f} vs fp64 oracle {a_ref:.3f}", flush=True)
    assert abs(a_gpu - a_ref) < 0.08
    x, _ = p.states()
    phi, g, _ = p.cache()
    ref = mcmc.geometry(case["prob"], x)
    assert np.max(np.abs(phi - ref.phi) / (1 + ref.phi)) < 1e-4
    assert np.linalg.norm(g - ref.g) / np.linalg.norm(ref.g) < 3e-2
    p.close()
    ctx.close()
