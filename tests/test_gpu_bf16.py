"""Mixed-precision path (FP32 forward, BF16 MFMA Jacobian / GN Hessian with FP32
accumulation, FP64 factorisation and MH) against the FP64 oracle, per chain.

Bars derived from the arithmetic. The forward is FP32 (unit roundoff 6e-8, a few hundred
accumulations: 1e-5 relative is generous). The Jacobian is a chain of about L + 2
products whose operands are rounded to bfloat16 (unit roundoff u = 2^-8 = 3.9e-3): with
randomly signed rounding errors each product adds ~0.8 u relative rms error to an output
element, so a row of B, and g and H of a chain, carry ~sqrt(L + 2) * 0.8 u ~ 8e-3 rms at
L = 4. Every row of B and every chain's g, H and factor is held to 3e-2 (about 4x that
estimate): errors are compared per row or per chain, never through a norm over all
chains, so an error confined to one wave's 32 Jacobian columns (one or two chains) shows
at its own size. A wrong operand layout or permutation gives O(1) errors.
"""
import numpy as np
import pytest

from oracle import mcmc
from tests.helpers import device_problem, make_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def per_chain_rel(a, b):
    """max over chains of |a_c - b_c| / |b_c| (Frobenius norms over each chain's entries)."""
    a = np.asarray(a, dtype=np.float64).reshape(len(b), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


CASES = {
    "configured": dict(name="tiny", chains=64),
    "tiny-mlp": dict(name="tiny", chains=70, bias_scale=0.3, noise_scale=0.2),
    "resnet-ragged": dict(name="tiny", chains=37, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                          bias_scale=0.3, noise_scale=0.2),
    "mid": dict(name="mid", chains=64),
    "mid-dual": dict(name="mid", chains=96, factorization="dual"),
}

BAR = 3e-2


@pytest.mark.parametrize("key", list(CASES))
def test_bf16_geometry_against_oracle(key):
    kw = dict(CASES[key])
    fact = kw.pop("factorization", "primal")
    case = make_case(kw.pop("name"), **kw)
    if fact == "dual":
        case["prob"].factor = "dual"
    print(f"bf16 geometry {key}", flush=True)
    ctx, p = device_problem(case, precision="bf16", factorization=fact)
    C, r, dy = case["C"], case["w"].r, case["prob"].d_y
    x = np.random.default_rng(3).standard_normal((C, r))
    got = {k: v.cpu().numpy() for k, v in p.eval_geometry(to_dev(x)).items()}
    ref = mcmc.geometry(case["prob"], x)
    if fact == "dual":
        K = got["L"].reshape(C, -1)[:, : dy * dy].reshape(C, dy, dy)
        Kref = np.linalg.cholesky(np.eye(dy)[None] + np.einsum("cir,ckr->cik", ref.B, ref.B))
        e_fac = per_chain_rel(np.tril(K), Kref)
    else:
        e_fac = per_chain_rel(np.tril(got["L"]), ref.L)
    B = p.eval_jacobian(to_dev(x)).cpu().numpy()
    e_rows = np.linalg.norm(B - ref.B, axis=2) / np.linalg.norm(ref.B, axis=2)   # (C, d_y)
    errs = dict(f=per_chain_rel(got["f"], ref.f), phi=float(np.max(np.abs(got["phi"] - ref.phi) / (1 + ref.phi))),
                B_row=float(e_rows.max()), g=per_chain_rel(got["g"], ref.g), H=per_chain_rel(got["H"], ref.H),
                factor=e_fac)
    print(f"bf16 per-chain max errors vs FP64 oracle ({key}): " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f"; B row error rms {np.sqrt(np.mean(e_rows ** 2)):.2e}", flush=True)
    assert errs["f"] < 1e-5 and errs["phi"] < 1e-4
    assert errs["B_row"] < BAR and errs["g"] < BAR and errs["H"] < BAR and errs["factor"] < BAR
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
def test_bf16_primal_beyond_the_staged_lds_takes_the_tiled_kernel():
    """B^T (r x d_y) of a chain too large for one block's LDS (r = 200, d_y = 400): the
    Gauss-Newton kernel streams B in 64 x 64 output tiles instead. H and g equal FP64 sums
    over the device's own B and FP32 residual to FP32 accumulation accuracy, and the
    oracle's within the BF16 bar."""
    from paper_2403_08220_amd import Context, Problem

    rng = np.random.default_rng(4)
    r, dy, C = 200, 400, 6
    ctx = Context(0)
    try:
        ctx.load_prior(33, 0.1, 1.0, r)
        layers = [("act", rng.standard_normal((32, r)) / np.sqrt(r), np.zeros(32)),
                  ("linear", rng.standard_normal((dy, 32)) / np.sqrt(32), np.zeros(dy))]
        ctx.load_network(layers)
        y, nv = 0.1 * rng.standard_normal(dy), np.full(dy, 0.05)
        p = Problem(ctx, C, y, nv, 1e-3, precision="bf16", factorization="primal")
        try:
            x = 0.5 * rng.standard_normal((C, r))
            B = p.eval_jacobian(to_dev(x)).cpu().numpy()
            got = {k: v.cpu().numpy() for k, v in p.eval_geometry(to_dev(x)).items()}
        finally:
            p.close()
        e = ((got["f"] - y[None, :]) / np.sqrt(nv)[None, :]).astype(np.float32).astype(np.float64)
        for c in range(C):
            H = B[c].T @ B[c]
            assert np.max(np.abs(got["H"][c] - H)) < 1e-5 * np.max(np.abs(H))
            assert np.max(np.abs(got["g"][c] - B[c].T @ e[c])) < 1e-9 * np.max(np.abs(B[c].T @ e[c]))
        prob = mcmc.Problem(layers, y, nv, 1e-3)
        ref = mcmc.geometry(prob, x)
        assert per_chain_rel(got["H"], ref.H) < BAR and per_chain_rel(got["g"], ref.g) < BAR
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
