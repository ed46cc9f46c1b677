"""Parity of the HIP path (through the C ABI) with the FP64 oracle, stage by stage
at identical inputs and for coupled multi-step runs.

Tolerances (FP64 path): 1e-10 relative on f, phi, g, H, L, x+; log rho within
1e-10 of the size of the terms that cancel in it; complement (FP32 state) 1e-5.
"""
import numpy as np
import pytest

from oracle import mcmc, philox, prior, stats
from tests.helpers import device_problem, make_case, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_dev(a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


def small_resnet_case(C=70, **kw):
    """Shapes spanning several tiles with ragged tails: r=40, width 80, d_y=20."""
    return make_case("tiny", chains=C, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                     bias_scale=0.3, noise_scale=0.2, **kw)


@pytest.mark.parametrize("n,r", [(33, 32), (129, 200), (10, 7)])
def test_basis_parity(n, r):
    from paper_2403_08220_amd import Context
    print(f"basis n={n} r={r}", flush=True)
    ctx = Context(0)
    ctx.load_prior(n, 0.1, 1.0, r)
    got = ctx.read_basis()
    B = prior.KLEBasis(n, 0.1, 1.0, r)
    np.testing.assert_array_equal(got["modes"][:, 0], B.k1)
    np.testing.assert_array_equal(got["modes"][:, 1], B.k2)
    np.testing.assert_allclose(got["lam"], B.lam, rtol=1e-14)
    assert np.max(np.abs(got["dec"] - B.dec)) < 1e-13 * np.max(np.abs(B.dec))
    np.testing.assert_allclose(got["var_perp"], B.var_perp, rtol=1e-11, atol=1e-17)
    ctx.close()


def test_normals_parity():
    case = make_case("tiny", chains=5)
    ctx, p = device_problem(case)
    for stream_id, step, count in [(0, 0, 32), (1, 17, 1057), (3, 0, 9)]:
        got = p.eval_normals(5, stream_id, step, count).cpu().numpy()
        ref = philox.normals(case["prob"].seed, 0, stream_id, step, np.arange(5), count)
        assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    p.close()
    ctx.close()


def geometry_case(kind):
    if kind == "mlp":
        return make_case("tiny", chains=70, bias_scale=0.3, noise_scale=0.2)
    if kind == "resnet":
        return small_resnet_case()
    # reduced dimensions that select the other factorisation kernels (r in 65..128 and r > 208),
    # and the largest reduced dimension the library takes (512)
    r = {"resnet-r100": 100, "resnet-r230": 230, "resnet-r512": 512}[kind]
    return make_case("tiny", chains=70 if r < 512 else 12, arch="resnet", r=r, width=96, depth=2, d_out=80,
                     d_y=70, bias_scale=0.3, noise_scale=0.2)


@pytest.mark.parametrize("kind", ["mlp", "resnet", "resnet-r100", "resnet-r230", "resnet-r512"])
def test_geometry_parity(kind):
    case = geometry_case(kind)
    print(f"geometry {kind}", flush=True)
    ctx, p = device_problem(case)
    x = np.random.default_rng(1).standard_normal((case["C"], case["w"].r))
    got = {k: v.cpu().numpy() for k, v in p.eval_geometry(to_dev(x)).items()}
    ref = mcmc.geometry(case["prob"], x)
    assert rel_err(got["f"], ref.f) < 1e-12
    assert np.max(np.abs(got["phi"] - ref.phi) / (1 + ref.phi)) < 1e-11
    assert rel_err(got["g"], ref.g) < 1e-10
    assert rel_err(got["H"], ref.H) < 1e-10
    assert rel_err(np.tril(got["L"]), ref.L) < 1e-10
    np.testing.assert_allclose(got["logdet"], np.sum(np.log(np.diagonal(ref.L, axis1=1, axis2=2)), axis=1),
                               rtol=1e-11)
    assert np.all(got["ok"] == 1)
    p.close()
    ctx.close()


@pytest.mark.parametrize("kind", ["resnet", "resnet-r230", "resnet-r512"])
def test_propose_and_log_rho_parity(kind):
    # r = 40: two solve blocks; r = 230: eight blocks with a 6-row tail, panels of up to
    # seven 32-column chunks (two load batches) and back-solve columns of 190+ rows;
    # r = 512: the largest reduced dimension (sixteen blocks, four load batches)
    if kind == "resnet":
        case = small_resnet_case(C=70, dt=0.7)
    else:
        r = 230 if kind == "resnet-r230" else 512
        case = make_case("tiny", chains=70 if r < 512 else 12, arch="resnet", r=r, width=96, depth=2, d_out=80,
                         d_y=70, bias_scale=0.3, noise_scale=0.2, dt=0.7)
    print(f"propose/log rho {kind}", flush=True)
    ctx, p = device_problem(case)
    prob = case["prob"]
    r, C = case["w"].r, case["C"]
    rng = np.random.default_rng(2)
    x = rng.standard_normal((C, r))
    xi = rng.standard_normal((C, r))
    cx = mcmc.geometry(prob, x)
    xp_ref = mcmc.propose(prob, x, cx, xi)
    xp = p.eval_propose(to_dev(x), to_dev(cx.g), to_dev(cx.L), to_dev(xi))
    assert rel_err(xp.cpu().numpy(), xp_ref) < 1e-10
    # log rho on the oracle's caches
    cp = mcmc.geometry(prob, xp_ref)
    lr_ref = mcmc.log_rho1(prob, x, cx, xp_ref, cp)
    dev = lambda c: dict(phi=to_dev(c.phi), g=to_dev(c.g), L=to_dev(c.L),
                         logdet=to_dev(np.sum(np.log(np.diagonal(c.L, axis1=1, axis2=2)), axis=1)))
    lr = p.eval_log_rho(to_dev(x), dev(cx), to_dev(xp_ref), dev(cp)).cpu().numpy()
    scale = 1 + cx.phi + cp.phi + cx.d.sum(1) + cp.d.sum(1)
    assert np.all(np.abs(lr - lr_ref) < 1e-10 * scale)
    p.close()
    ctx.close()


def run_coupled(case, n_steps, chains_idx=None, trace=False):
    """Run the oracle and the device for n_steps from the same initial state."""
    ctx, p = device_problem(case, trace_capacity=n_steps if trace else 0)
    C = case["C"]
    p.init(case["x0"], case["z0"])
    p.step(n_steps)
    x, z = p.states()
    acc, fail, steps = p.diagnostics()
    assert steps == n_steps
    idx = np.arange(C) if chains_idx is None else np.asarray(chains_idx)
    st = mcmc.init_state(case["prob"], case["x0"][idx], case["z0"][idx].astype(np.float64), chains=idx)
    xs, _ = mcmc.run(case["prob"], st, n_steps, trace=trace)
    out = dict(x=x[idx], z=z[idx], acc=acc[idx], fail=fail[idx], ox=st.x, oz=st.z, oacc=st.accepts, p=p, ctx=ctx,
               st=st, otrace=xs)
    if trace:
        out["trace"] = p.trace()
    return out


def test_coupled_chains_tiny_literal():
    """The literal tiny workload (stiff: dt = 0.1, sigma = 0.01), coupled streams."""
    case = make_case("tiny")
    r = run_coupled(case, 60)
    np.testing.assert_array_equal(r["acc"], r["oacc"])
    assert rel_err(r["x"], r["ox"]) < 1e-9
    assert np.max(np.abs(r["z"] - r["oz"])) < 1e-5
    r["p"].close()
    r["ctx"].close()


def test_coupled_chains_mixing():
    """A well-mixing variant (sigma = 0.2, several tiles of chains, ragged sizes)."""
    case = small_resnet_case(C=70, dt=0.5)
    r = run_coupled(case, 40)
    flips = np.sum(r["acc"] != r["oacc"])
    assert flips == 0
    assert r["acc"].sum() > 70 * 40 * 0.05   # decisions are not trivially all-reject
    assert rel_err(r["x"], r["ox"]) < 1e-9
    assert np.max(np.abs(r["z"] - r["oz"])) < 1e-5
    r["p"].close()
    r["ctx"].close()


def test_zero_likelihood_is_pcn_on_device():
    case = small_resnet_case(C=8, dt=0.8)
    case["prob"].noise_var = np.full(case["w"].d_y, np.inf)
    ctx, p = device_problem(case)
    p.init(case["x0"], case["z0"])
    p.step(25)
    acc, fail, _ = p.diagnostics()
    assert np.all(acc == 25) and np.all(fail == 0)
    x, _ = p.states()
    st = mcmc.init_state(case["prob"], case["x0"], case["z0"].astype(np.float64))
    mcmc.run(case["prob"], st, 25, trace=False)
    assert rel_err(x, st.x) < 1e-12
    p.close()
    ctx.close()


def test_full_size_mid_sampled():
    """The 129x129 / r=200 / ResNet 400x4 / d_y=100 workload with 512 chains, in the
    launch configuration the bench times; the oracle follows a sample of chains."""
    case = make_case("mid")
    idx = [0, 1, 255, 256, 511]
    print("full-size mid: 3 coupled steps", flush=True)
    r = run_coupled(case, 3, chains_idx=idx)
    np.testing.assert_array_equal(r["acc"], r["oacc"])
    assert rel_err(r["x"], r["ox"]) < 1e-9
    assert np.max(np.abs(r["z"] - r["oz"])) < 1e-5
    # geometry of the sampled chains at their current states
    x, _ = r["p"].states()
    phi, g, L = r["p"].cache()
    c = mcmc.geometry(case["prob"], x[idx])
    assert np.max(np.abs(phi[idx] - c.phi) / (1 + c.phi)) < 1e-11
    assert rel_err(g[idx], c.g) < 1e-9
    assert rel_err(L[idx], c.L) < 1e-9
    r["p"].close()
    r["ctx"].close()


def test_posterior_and_ess_parity():
    case = small_resnet_case(C=16, dt=0.5)
    r = run_coupled(case, 120, trace=True)
    p = r["p"]
    xt, pt = r["trace"]
    assert xt.shape == (120, 16, 40)
    assert np.max(np.abs(xt - r["otrace"])) < 1e-5
    mean, var, xbar, S = p.posterior(24)
    B = prior.KLEBasis(case["w"].n, 0.1, 1.0, 40)
    om, ov, oxbar, oS = stats.posterior_moments(xt.astype(np.float64), B, burn_in_frac=24 / 120)
    assert rel_err(xbar, oxbar) < 1e-10
    assert rel_err(S, oS) < 1e-9
    assert rel_err(mean, om) < 1e-9
    assert rel_err(var, ov) < 1e-9
    e = p.ess(24)
    oe = stats.ess_per_coordinate(xt[24:].astype(np.float64))
    assert rel_err(e, oe) < 1e-8
    p.close()
    r["ctx"].close()


def test_single_chain_and_minimal_output():
    case = make_case("tiny", chains=1, d_y=1, noise_scale=0.3)
    r = run_coupled(case, 30)
    np.testing.assert_array_equal(r["acc"], r["oacc"])
    assert rel_err(r["x"], r["ox"]) < 1e-9
    r["p"].close()
    r["ctx"].close()


def test_abi_errors_on_device():
    from paper_2403_08220_amd import Context, DinoError, Problem
    case = make_case("tiny", chains=2)
    ctx = Context(0)
    with pytest.raises(DinoError):
        Problem(ctx, 2, case["y"], case["noise_var"], 0.1)   # no prior / network yet
    ctx.load_prior(33, 0.1, 1.0, 32)
    ctx.load_network(case["layers"])
    with pytest.raises(DinoError):
        Problem(ctx, 2, case["y"], case["noise_var"], -0.1)  # dt <= 0
    with pytest.raises(DinoError):
        Problem(ctx, 2, case["y"], -case["noise_var"], 0.1)  # negative variance
    p = Problem(ctx, 2, case["y"], case["noise_var"], 0.1)
    with pytest.raises(DinoError):
        p.step(1)                                           # step before init
    p.init(case["x0"], case["z0"])
    p.step(0)
    assert p.diagnostics()[2] == 0
    p.close()
    ctx.close()
