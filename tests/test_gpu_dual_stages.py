"""Element-wise parity of the observation-space (dual) stages that dino_step runs for a
dual problem, in both precisions, against the oracle evaluated on the same inputs.

The device's dual proposal kernel (with its forward transition term) and the code of the
acceptance kernel's reverse term are called through stage entry points with given
states, caches and normals (Sec. 5.3 eq. reduced_space_sampling; Sec. 5.4 eq.
da_dino_trr_1). The Jacobian handed to both sides is the oracle's; for a BF16 problem it
is first rounded to bfloat16 on the host, which gives exactly the values the BF16 path
stores and stages in LDS. Both sides therefore evaluate the method on identical numbers
and differ only by FP64 rounding order, so the bars are FP64 bars:

* x+ per chain within 1e-10 relative (max over the chain's coordinates / max |x+|): the
  device applies (I + H)^-1 by Woodbury through the d_y x d_y factor, the oracle by a
  dense r x r solve; both are backward stable, so the difference is ~ eps * cond(I + H)
  with cond <= 1 + |B|^2 ~ 1e4 here, i.e. ~1e-12;
* log rho_0 and log rho^(1) per chain within 1e-10 of the sum of the magnitudes of the
  terms that cancel in them (the oracle's term breakdown), the FP64 bar of the primal
  stage tests.

Cases span the bench's full shape (129^2 grid, r = 200, ResNet 400 x 4, d_y = 100, all
512 chains), a ragged r (230 = 7 x 32 + 6, ragged LDS chunks and solve blocks), a ragged
small shape (r = 40, d_y = 20, 37 chains) and the degenerate d_y = 1.
"""
import numpy as np
import pytest

from oracle import mcmc
from tests.helpers import device_problem, make_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def bf16_round(a):
    """Round float64 values to bfloat16 (through float32, round to nearest even); the
    result is returned as float64 and is exactly representable in bfloat16."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


CASES = {
    "mid-bf16": dict(kw=dict(name="mid"), precision="bf16"),
    "mid-f64-64": dict(kw=dict(name="mid", chains=64), precision="f64"),
    "ragged-r230-bf16": dict(kw=dict(name="tiny", chains=70, r=230, width=96, d_out=100, d_y=100, bias_scale=0.3,
                                     noise_scale=0.2), precision="bf16"),
    "ragged-small-bf16": dict(kw=dict(name="tiny", chains=37, arch="resnet", r=40, width=80, depth=2, d_out=24,
                                      d_y=20, bias_scale=0.3, noise_scale=0.2), precision="bf16"),
    "dy1-bf16": dict(kw=dict(name="tiny", chains=9, r=40, width=64, d_out=4, d_y=1, bias_scale=0.3,
                             noise_scale=0.2), precision="bf16"),
}


def stage_cache(prob, x, precision):
    """The oracle's cache at x, evaluated on the Jacobian the device path stores."""
    c = mcmc.geometry(prob, x)
    if precision == "bf16":
        c = mcmc.cache_from_jacobian(prob, c.f, bf16_round(c.B))
    return c


def device_cache(p, c):
    dev = dict(device="cuda:0", dtype=torch.float64)
    dy = c.B.shape[1]
    K = np.linalg.cholesky(np.eye(dy)[None] + np.einsum("cir,ckr->cik", c.B, c.B))
    logdet = np.sum(np.log(np.diagonal(K, axis1=1, axis2=2)), axis=1)
    return dict(phi=torch.tensor(c.phi, **dev), g=torch.tensor(c.g, **dev),
                B=p.jacobian_storage(torch.tensor(c.B, **dev)), K=torch.tensor(np.ascontiguousarray(K), **dev),
                logdet=torch.tensor(logdet, **dev))


@pytest.mark.parametrize("key", list(CASES))
def test_dual_stages_elementwise(key):
    spec = CASES[key]
    kw = dict(spec["kw"])
    case = make_case(kw.pop("name"), **kw)
    prob = case["prob"]
    prob.factor = "dual"
    C, r, dy = case["C"], case["w"].r, prob.d_y
    print(f"dual stages {key}: C={C} r={r} d_y={dy} {spec['precision']}", flush=True)
    ctx, p = device_problem(case, precision=spec["precision"], factorization="dual")
    try:
        rng = np.random.default_rng(11)
        x = 0.5 * rng.standard_normal((C, r))
        xi = rng.standard_normal((C, r + dy))
        cx = stage_cache(prob, x, spec["precision"])
        xp_ref = mcmc.propose(prob, x, cx, xi)
        t_fwd = mcmc.log_rho0_terms(prob, x, xp_ref, cx)

        dev = dict(device="cuda:0", dtype=torch.float64)
        dcx = device_cache(p, cx)
        xp_dev, lfwd_dev = p.eval_propose_dual(torch.tensor(x, **dev), dcx["g"], dcx["B"], dcx["K"], dcx["logdet"],
                                               torch.tensor(xi, **dev))
        xp_dev, lfwd_dev = xp_dev.cpu().numpy(), lfwd_dev.cpu().numpy()
        e_xp = np.max(np.abs(xp_dev - xp_ref), axis=1) / np.max(np.abs(xp_ref), axis=1)
        e_fwd = np.abs(lfwd_dev - t_fwd.sum(axis=1)) / np.abs(t_fwd).sum(axis=1)
        print(f"  x+ per-chain max rel {e_xp.max():.2e} (chain {e_xp.argmax()}), "
              f"log rho_0 fwd {e_fwd.max():.2e}", flush=True)
        assert e_xp.max() < 1e-10
        assert e_fwd.max() < 1e-10

        cp = stage_cache(prob, xp_ref, spec["precision"])
        t_rev = mcmc.log_rho0_terms(prob, xp_ref, x, cp)
        lr_ref = mcmc.log_rho1(prob, x, cx, xp_ref, cp)
        dcp = device_cache(p, cp)
        lr_dev = p.eval_log_rho_dual(torch.tensor(x, **dev), dcx, torch.tensor(xp_ref, **dev), dcp).cpu().numpy()
        scale = np.abs(cx.phi) + np.abs(cp.phi) + np.abs(t_fwd).sum(axis=1) + np.abs(t_rev).sum(axis=1)
        e_lr = np.abs(lr_dev - lr_ref) / scale
        print(f"  log rho per-chain {e_lr.max():.2e} of the cancelling terms (chain {e_lr.argmax()})", flush=True)
        assert np.all(np.isfinite(lr_dev))
        assert e_lr.max() < 1e-10
    finally:
        p.close()
        ctx.close()


def test_dual_stage_entry_argument_errors():
    from paper_2403_08220_amd import DinoError

    case = make_case("tiny", chains=4, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20, noise_scale=0.2)
    ctx, p = device_problem(case, precision="bf16", factorization="primal")
    try:
        z = torch.zeros((4, 40), dtype=torch.float64, device="cuda:0")
        with pytest.raises(DinoError, match="serves the dual form"):
            p.eval_propose_dual(z, z, z, z, z[:, 0].contiguous(), z)
    finally:
        p.close()
        ctx.close()
