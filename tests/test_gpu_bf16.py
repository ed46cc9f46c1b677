"""Mixed-precision path (FP32 forward, BF16 MFMA Jacobian / GN Hessian with FP32
accumulation, FP64 factorisation and MH) against the FP64 oracle.

Tolerances derived from the arithmetic: the forward is FP32 (unit roundoff 6e-8, a
few hundred accumulations: 1e-5 relative is generous); the Jacobian is a chain of
BF16-operand products (unit roundoff 2^-8 = 3.9e-3 per rounded operand, random
signs, a handful of layers), so B, g and H carry O(1e-2) relative error in
Frobenius norm; 3e-2 is the bound used here and the measured values are printed.
A wrong operand layout or permutation in the sweep gives O(1) errors.
"""
import numpy as np
import pytest

from oracle import mcmc
from tests.helpers import device_problem, make_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fro_rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


CASES = {
    "tiny-mlp": dict(name="tiny", chains=70, bias_scale=0.3, noise_scale=0.2),
    "resnet-ragged": dict(name="tiny", chains=37, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                          bias_scale=0.3, noise_scale=0.2),
    "mid": dict(name="mid", chains=64),
}


@pytest.mark.parametrize("key", list(CASES))
def test_bf16_geometry_against_oracle(key):
    kw = dict(CASES[key])
    case = make_case(kw.pop("name"), **kw)
    print(f"bf16 geometry {key}", flush=True)
    ctx, p = device_problem(case, precision="bf16")
    C, r = case["C"], case["w"].r
    x = np.random.default_rng(3).standard_normal((C, r))
    got = {k: v.cpu().numpy() for k, v in p.eval_geometry(to_dev(x)).items()}
    ref = mcmc.geometry(case["prob"], x)
    errs = dict(f=fro_rel(got["f"], ref.f), phi=float(np.max(np.abs(got["phi"] - ref.phi) / (1 + ref.phi))),
                g=fro_rel(got["g"], ref.g), H=fro_rel(got["H"], ref.H),
                L=fro_rel(np.tril(got["L"]), ref.L))
    print(f"bf16 errors vs FP64 oracle ({key}): " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert errs["f"] < 1e-5 and errs["phi"] < 1e-4
    assert errs["g"] < 3e-2 and errs["H"] < 3e-2 and errs["L"] < 3e-2
    assert np.all(got["ok"] == 1)
    p.close()
    ctx.close()


def test_bf16_chains_step_and_agree_on_decisions_mostly():
    """Coupled streams: the BF16 chains see the same draws as the FP64 oracle; the
    proposals differ at the BF16 level, so only the statistics of decisions are
    compared here (acceptance rates within a few points)."""
    case = make_case("tiny", chains=64, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                     bias_scale=0.3, noise_scale=0.2, dt=0.5)
    ctx, p = device_problem(case, precision="bf16")
    p.init(case["x0"], case["z0"])
    p.step(60)
    acc, fail, steps = p.diagnostics()
    assert steps == 60 and fail.sum() == 0
    st = mcmc.init_state(case["prob"], case["x0"], case["z0"].astype(np.float64))
    mcmc.run(case["prob"], st, 60, trace=False)
    a_gpu = acc.sum() / (64 * 60)
    a_ref = st.accepts.sum() / (64 * 60)
    print(f"acceptance bf16 {a_gpu:.3f} vs fp64 oracle {a_ref:.3f}", flush=True)
    assert abs(a_gpu - a_ref) < 0.08
    p.close()
    ctx.close()


@pytest.mark.gpu
def test_bf16_primal_refuses_shapes_beyond_its_lds():
    """The BF16 Gauss-Newton Hessian stages B^T (r x d_y) in LDS: a shape that does not fit
    is refused when the problem is described (the FP64 path takes it)."""
    from paper_2403_08220_amd import Context, DinoError, Problem

    rng = np.random.default_rng(4)
    r, dy = 200, 400
    ctx = Context(0)
    try:
        ctx.load_prior(33, 0.1, 1.0, r)
        layers = [("act", rng.standard_normal((32, r)) / np.sqrt(r), None),
                  ("linear", rng.standard_normal((dy, 32)) / np.sqrt(32), None)]
        ctx.load_network(layers)
        y, nv = np.zeros(dy), np.ones(dy)
        with pytest.raises(DinoError, match="too large for the BF16 Gauss-Newton Hessian"):
            Problem(ctx, 4, y, nv, 1e-3, precision="bf16", factorization="primal")
        p = Problem(ctx, 4, y, nv, 1e-3, precision="f64", factorization="primal")
        p.close()
    finally:
        ctx.close()


@pytest.mark.gpu
def test_bf16_refuses_networks_wider_than_the_sweep():
    """The BF16 reverse sweep holds at most 512 rows (16 blocks of 32): a wider hidden
    layer is refused when the problem is described instead of being cut short (the FP64
    path takes it)."""
    from paper_2403_08220_amd import Context, DinoError, Problem

    rng = np.random.default_rng(5)
    r, width, dy = 64, 544, 20
    ctx = Context(0)
    try:
        ctx.load_prior(33, 0.1, 1.0, r)
        layers = [("act", rng.standard_normal((width, r)) / np.sqrt(r), None),
                  ("linear", rng.standard_normal((dy, width)) / np.sqrt(width), None)]
        ctx.load_network(layers)
        y, nv = np.zeros(dy), np.ones(dy)
        with pytest.raises(DinoError, match="at most 512 units"):
            Problem(ctx, 4, y, nv, 1e-3, precision="bf16")
        p = Problem(ctx, 4, y, nv, 1e-3, precision="f64")
        p.close()
    finally:
        ctx.close()
