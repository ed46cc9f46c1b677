"""FP8 reverse sweep of the reduced Jacobian (the display after eq. rb_dino; e4m3 products
with FP32 accumulation) and the tiled Gauss-Newton kernel (eq. surrogate_rppgnh,
surrogate_rppg) against the oracle.

* Layout, scales and the residual branch, exactly: a network whose FP8 and BF16
  operands are all representable (signed-permutation weights with power-of-two entries
  and per-column power-of-two scales, evaluated at x = 0, where every gelu' is 1/2
  exactly) gives B with every entry equal to the oracle's J Gamma^-1/2 rounded to
  bfloat16. The test checks its own precondition (every A block and every stored
  Lambda exactly representable) before comparing, so a case that would not be exact
  fails as a construction error, not as a parity failure.
* Both left-operand forms: one e4m3 term (fp8_single) and the two-term expansion (fp8),
  whose remainder term is zero on the representable network.
* Tolerance on Xavier networks. e4m3 keeps 3 mantissa bits: round to nearest leaves a
  relative error uniform in +-2^-4 of the leading binade, ~0.026 rms over a binade.
  Each term of a product rounds both operands (~0.037 rms) and, with randomly signed
  errors, a row of a layer's product carries the same relative rms error. On a residual
  layer only the product branch (Lambda d) W carries it, and with Xavier weights that
  branch is ~0.6 of the row's norm: ~0.02 per layer; six layers in quadrature plus the
  lift layer (all product) give ~0.06 per row of B at L = 6 (~0.045 with the two-term
  left operand, where only the weights' rounding remains at that size). Bars: every row of B, and
  every chain's H and g, within 0.15 relative Frobenius error (about 2.5x the estimate;
  a wrong operand layout, scale or residual term gives O(1) errors). Errors are compared
  per row or per chain, never through a norm over all chains.
* The tiled Gauss-Newton kernel equals the LDS-staged one bit for bit where both apply
  (the same products in the same order), and at the large shape (r = d_y = 400, where
  only the tiled kernel applies) it matches I + B^T B and B^T e formed in FP64 from the
  device's own B and residual to FP32 accumulation accuracy (1e-5 relative).
"""
import numpy as np
import pytest

from oracle import mcmc, network
from tests.helpers import device_problem, make_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def bf16_round(a):
    """float64 -> float32 (round to nearest even) -> bfloat16 (round to nearest even) -> float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3_exact(v):
    """Whether every entry of v is exactly an OCP e4m3 value (|v| <= 448)."""
    v = np.abs(np.asarray(v, dtype=np.float64))
    nz = v[v > 0]
    if np.any(nz > 448):
        return False
    e = np.maximum(np.floor(np.log2(nz)), -6.0)   # subnormals share the exponent 2^-6
    q = nz / 2.0 ** (e - 3)                        # 3 mantissa bits: integer multiples of 2^(e-3)
    return bool(np.all(q == np.round(q)))


def mx_blocks_exact(A):
    """A (rows, K): every 32-block of a row scaled by 2^-(ilogb(max) - 7) is e4m3-exact."""
    rows, K = A.shape
    Kp = (K + 31) // 32 * 32
    P = np.zeros((rows, Kp))
    P[:, :K] = A
    for blk in P.reshape(rows, Kp // 32, 32).reshape(-1, 32):
        m = np.max(np.abs(blk))
        if m == 0:
            continue
        e = int(np.floor(np.log2(m))) - 7
        if not e4m3_exact(blk * 2.0 ** -e):
            return False
    return True


def permutation_network(r, width, depth, d_out, seed):
    """ResNet [lift, resid x depth, output] with one nonzero per column (resid layers, a
    derangement so that a row's terms never add), one per row (lift and output layers),
    entries +-1 times per-column powers of two."""
    rng = np.random.default_rng(seed)
    layers = []
    W0 = np.zeros((width, r))
    W0[np.arange(width), rng.integers(0, r, width)] = rng.choice([-1.0, 1.0], width) * 2.0 ** rng.integers(-2, 3, width)
    layers.append(("linear", W0, np.zeros(width)))
    for _ in range(depth):
        sigma = (np.arange(width) + rng.integers(1, width)) % width
        W = np.zeros((width, width))
        W[sigma, np.arange(width)] = rng.choice([-1.0, 1.0], width) * 2.0 ** rng.integers(-1, 1, width)
        layers.append(("resid", W, np.zeros(width)))
    Wout = np.zeros((d_out, width))
    Wout[np.arange(d_out), rng.integers(0, width, d_out)] = rng.choice([-1.0, 1.0], d_out)
    layers.append(("linear", Wout, np.zeros(d_out)))
    return layers


def sweep_preconditions(layers, d_y):
    """The reverse sweep at x = 0 (gelu' = 1/2 on every resid layer): every A = Lambda d of
    a layer is exactly representable in MX e4m3 blocks, every stored Lambda in bfloat16."""
    lam = layers[-1][1][:d_y].copy()
    ok = np.array_equal(bf16_round(lam), lam)
    for kind, W, _ in reversed(layers[:-1]):
        d = 0.5 if kind == "resid" else 1.0
        A = lam * d
        ok = ok and mx_blocks_exact(A)
        lam = (lam if kind == "resid" else 0.0) + A @ W
        if kind == "resid":
            ok = ok and np.array_equal(bf16_round(lam), lam)
    return ok, lam


@pytest.mark.parametrize("precision", ["fp8", "fp8_single"])
@pytest.mark.parametrize("r,width,depth,d_y,chains", [(40, 96, 3, 20, 37), (400, 800, 6, 400, 3)])
def test_fp8_sweep_exact_on_a_representable_network(r, width, depth, d_y, chains, precision):
    layers = None
    for seed in range(20):
        cand = permutation_network(r, width, depth, d_y + 4, seed)
        ok, lam0 = sweep_preconditions(cand, d_y)
        if ok:
            layers = cand
            break
    assert layers is not None, "no seed gave an exactly representable sweep"
    case = make_case("tiny", chains=chains, arch="resnet", r=r, width=width, depth=depth, d_out=d_y + 4, d_y=d_y,
                     noise_scale=0.3)
    case["layers"] = layers
    nv = np.random.default_rng(5).uniform(0.5, 2.0, d_y) ** 2
    case["prob"].noise_var = nv
    case["prob"].layers = layers
    print(f"{precision} exact r={r} width={width} depth={depth}", flush=True)
    ctx, p = device_problem(case, precision=precision)
    try:
        B = p.eval_jacobian(to_dev(np.zeros((chains, r)))).cpu().numpy()
        ref = bf16_round(lam0 / np.sqrt(nv)[:, None])
        J = network.jacobian_reverse(layers, np.zeros((1, r)))[0][:d_y]
        assert np.array_equal(J, lam0)   # the precondition's sweep is the oracle's Jacobian
        for c in range(chains):
            np.testing.assert_array_equal(B[c], ref)
    finally:
        p.close()
        ctx.close()


CASES = {
    "resnet-ragged": dict(name="tiny", chains=37, arch="resnet", r=40, width=96, depth=2, d_out=24, d_y=20,
                          bias_scale=0.3, noise_scale=0.2),
    "mid": dict(name="mid", chains=40),
    "large": dict(name="large", chains=6),
}
BAR = 0.15


@pytest.mark.parametrize("precision", ["fp8", "fp8_single"])
@pytest.mark.parametrize("key", list(CASES))
def test_fp8_geometry_against_oracle(key, precision):
    kw = dict(CASES[key])
    case = make_case(kw.pop("name"), **kw)
    print(f"{precision} geometry {key}", flush=True)
    ctx, p = device_problem(case, precision=precision)
    C, r, dy = case["C"], case["w"].r, case["prob"].d_y
    try:
        x = 0.5 * np.random.default_rng(3).standard_normal((C, r))
        B = p.eval_jacobian(to_dev(x)).cpu().numpy()
        got = {k: v.cpu().numpy() for k, v in p.eval_geometry(to_dev(x)).items()}
        ref = mcmc.geometry(case["prob"], x)
        Bref = ref.B if hasattr(ref, "B") else None
        if Bref is None:
            Bref = network.jacobian_reverse(case["layers"], x)[:, :dy] / np.sqrt(case["prob"].noise_var)[None, :, None]
        row_err = np.linalg.norm(B - Bref, axis=2) / np.linalg.norm(Bref, axis=2)
        h_err = np.linalg.norm((got["H"] - ref.H).reshape(C, -1), axis=1) / np.linalg.norm(ref.H.reshape(C, -1), axis=1)
        g_err = np.linalg.norm(got["g"] - ref.g, axis=1) / np.linalg.norm(ref.g, axis=1)
        print(f"  B rows: median {np.median(row_err):.3e} max {row_err.max():.3e}; "
              f"H max {h_err.max():.3e}; g max {g_err.max():.3e}", flush=True)
        assert row_err.max() < BAR and h_err.max() < BAR and g_err.max() < BAR
        assert np.max(np.abs(got["phi"] - ref.phi) / (1 + ref.phi)) < 1e-4     # FP32 forward
        assert np.all(got["ok"] == 1)
    finally:
        p.close()
        ctx.close()


@pytest.mark.parametrize("name,kw", [("ragged", dict(name="tiny", chains=37, arch="resnet", r=40, width=80, depth=2,
                                                     d_out=24, d_y=20, bias_scale=0.3, noise_scale=0.2)),
                                      ("mid", dict(name="mid", chains=33))])
def test_tiled_hessian_matches_the_lds_kernel_bitwise(name, kw):
    from paper_2403_08220_amd import tune_set
    kw = dict(kw)
    case = make_case(kw.pop("name"), **kw)
    print(f"tiled hessian bitwise {name}", flush=True)
    ctx, p = device_problem(case, precision="bf16")
    C, r, dy = case["C"], case["w"].r, case["prob"].d_y
    try:
        x = to_dev(0.5 * np.random.default_rng(4).standard_normal((C, r)))
        tune_set("hess", (r, dy, 0), 0)
        a = {k: v.cpu().numpy() for k, v in p.eval_geometry(x).items()}
        tune_set("hess", (r, dy, 0), 1)
        b = {k: v.cpu().numpy() for k, v in p.eval_geometry(x).items()}
        for k in ("f", "phi", "g", "H", "L", "logdet", "ok"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    finally:
        tune_set("hess", (r, dy, 0), -1)
        p.close()
        ctx.close()


def test_tiled_hessian_at_the_large_shape():
    """r = d_y = 400: B^T (333 KB) exceeds LDS, so the tiled kernel is the only one; H, g and
    phi against FP64 sums over the device's own B and FP32 output."""
    case = make_case("large", chains=5)
    print("tiled hessian large", flush=True)
    ctx, p = device_problem(case, precision="fp8")
    C, r = case["C"], case["w"].r
    prob = case["prob"]
    try:
        x = to_dev(0.5 * np.random.default_rng(6).standard_normal((C, r)))
        B = p.eval_jacobian(x).cpu().numpy()
        got = {k: v.cpu().numpy() for k, v in p.eval_geometry(x).items()}
        winv = 1.0 / np.sqrt(prob.noise_var)
        e = ((got["f"] - prob.y[None, :]) * winv[None, :]).astype(np.float32).astype(np.float64)
        H = np.einsum("cir,cis->crs", B, B)
        g = np.einsum("cir,ci->cr", B, e)
        for c in range(C):
            assert np.max(np.abs(got["H"][c] - H[c])) < 1e-5 * np.max(np.abs(H[c]))
            assert np.max(np.abs(got["g"][c] - g[c])) < 1e-9 * np.max(np.abs(g[c]))
        phi = 0.5 * np.sum(((got["f"] - prob.y[None, :]) * winv[None, :]) ** 2, axis=1)
        assert np.max(np.abs(got["phi"] - phi) / phi) < 1e-12
    finally:
        p.close()
        ctx.close()


def test_fp8_problem_argument_errors():
    from paper_2403_08220_amd import Context, DinoError, Problem

    case = make_case("tiny", chains=4, arch="resnet", r=40, width=1024, depth=1, d_out=24, d_y=20)
    w = case["w"]
    ctx = Context(0)
    try:
        ctx.load_prior(w.n, w.gamma, w.delta, w.r)
        ctx.load_network(case["layers"])
        prob = case["prob"]
        for prec in ("fp8", "fp8_single"):
            with pytest.raises(DinoError, match="FP8 reverse sweep"):
                Problem(ctx, 4, prob.y, prob.noise_var, 0.1, precision=prec)
        with pytest.raises(DinoError, match="BF16 reverse sweep"):
            Problem(ctx, 4, prob.y, prob.noise_var, 0.1, precision="bf16")
    finally:
        ctx.close()
