"""The autotuner (dino_autotune) and its tuning table.

Every implementation the tuner may pick must compute the method's quantities: each
factor-kernel variant is forced through the table at orders it holds (20, 40, 100,
150; ragged against its register blocks) and its factor and log det compared with the
oracle's (1e-10 relative, the FP64 stage bar). A tuned FP64 problem then reproduces
the oracle's coupled chains (identical decisions, x 1e-9), and the table holds the
timed choice of every shape the problem launches. The table is process-wide: each test
clears what it set.
"""
import numpy as np
import pytest

from oracle import mcmc
from tests.helpers import device_problem, make_case, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAX_ORDER = [32, 56, 104, 128, 208, 512, 512]


@pytest.mark.parametrize("r", [20, 40, 100, 150, 300])
def test_every_factor_variant_matches_the_oracle(r):
    from paper_2403_08220_amd import clear_tuning, tune_set

    case = make_case("tiny", chains=13, arch="resnet", r=r, width=64, depth=1, d_out=r + 8, d_y=r + 8,
                     bias_scale=0.3, noise_scale=0.3)
    ctx, p = device_problem(case, precision="f64", factorization="primal")
    x = 0.3 * np.random.default_rng(r).standard_normal((13, r))
    ref = mcmc.geometry(case["prob"], x)
    ref_logdet = np.sum(np.log(np.diagonal(ref.L, axis1=1, axis2=2)), axis=1)
    try:
        for v, mx in enumerate(MAX_ORDER):
            if mx < r:
                continue
            print(f"factor variant {v} at order {r}", flush=True)
            tune_set("chol", (13, r, 0), v)
            got = {k: t.cpu().numpy() for k, t in p.eval_geometry(torch.tensor(x, device="cuda:0")).items()}
            assert rel_err(np.tril(got["L"]), ref.L) < 1e-10, v
            np.testing.assert_allclose(got["logdet"], ref_logdet, rtol=1e-10)
            assert np.all(got["ok"] == 1)
    finally:
        clear_tuning()
        p.close()
        ctx.close()


def test_tuned_problem_reproduces_the_oracle_chains():
    from paper_2403_08220_amd import clear_tuning, tuning_table

    case = make_case("tiny", chains=64, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20, bias_scale=0.3,
                     noise_scale=0.2, dt=0.5)
    ctx, p = device_problem(case, precision="f64", factorization="dual")
    try:
        p.init(case["x0"], case["z0"])
        n = p.autotune()
        table = tuning_table()
        print(f"tuned {n} entries: {table}", flush=True)
        chol = [e for e in table if e["kind"] == "chol" and e["shape"] == (64, 20, 0)]
        assert len(chol) == 1 and n >= 2
        ms = np.array(chol[0]["ms"])
        valid = ms > 0
        assert chol[0]["choice"] == int(np.argmin(np.where(valid, ms, np.inf)))
        assert valid[:3].all()                           # orders up to 32 / 56 / 104 hold d_y = 20
        assert any(e["kind"] == "fwd64" for e in table)
        p.step(30)
        x, _ = p.states()
        acc, _, _ = p.diagnostics()
        case["prob"].factor = "dual"
        st = mcmc.init_state(case["prob"], case["x0"], case["z0"].astype(np.float64))
        mcmc.run(case["prob"], st, 30, trace=False)
        np.testing.assert_array_equal(acc, st.accepts)
        assert rel_err(x, st.x) < 1e-9
    finally:
        clear_tuning()
        p.close()
        ctx.close()


def test_bf16_autotune_keeps_the_chains_identical_to_the_untuned_run():
    """The mixed path's tunable choices (FP32 forward block order, factor kernel) change no
    value here but the factor's rounding order: a tuned and an untuned run of the same
    chains take the same decisions."""
    from paper_2403_08220_amd import clear_tuning

    case = make_case("tiny", chains=256, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20, bias_scale=0.3,
                     noise_scale=0.2, dt=0.5)
    runs = []
    for tuned in (False, True):
        ctx, p = device_problem(case, precision="bf16", factorization="dual")
        try:
            p.init(case["x0"], case["z0"])
            if tuned:
                p.autotune()
            p.step(20)
            acc, _, _ = p.diagnostics()
            x, _ = p.states()
            runs.append((acc, x))
        finally:
            p.close()
            ctx.close()
    clear_tuning()
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    assert rel_err(runs[1][1], runs[0][1]) < 1e-9


def test_tune_set_rejects_a_variant_that_cannot_hold_the_order():
    from paper_2403_08220_amd import DinoError, tune_set

    with pytest.raises(DinoError, match="does not hold this order"):
        tune_set("chol", (8, 100, 0), 0)
    with pytest.raises(DinoError, match="out of range"):
        tune_set("fwd32", (64, 40, 80), 2)


@pytest.mark.parametrize("key", ["mid-512", "resnet-ragged"])
def test_one_launch_forward_is_bit_identical_to_per_layer_launches(key):
    """The mixed path's forward in one launch (row blocks handing layers on through device
    counters) runs the same tile arithmetic as one launch per layer: f, g, the metric and B
    agree bit for bit, on two evaluations in a row (the counters clear themselves), the
    second with fewer chains."""
    from paper_2403_08220_amd import clear_tuning, tune_set

    if key == "mid-512":
        case = make_case("mid", chains=512)
        fact = "dual"
    else:
        case = make_case("tiny", chains=37, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                         bias_scale=0.3, noise_scale=0.2)
        fact = "primal"
    ctx, p = device_problem(case, precision="bf16", factorization=fact)
    C, r = case["C"], case["w"].r
    L = len(case["layers"])
    wmax = max(W.shape[0] for _, W, _ in case["layers"][:-1])
    x = 0.5 * np.random.default_rng(11).standard_normal((C, r))
    try:
        for n in (C, C - 13):
            xd = torch.tensor(x[:n], dtype=torch.float64, device="cuda:0")
            outs = []
            for choice in (0, 1, 1):
                tune_set("fwdchain", (n, L, wmax), choice)
                got = {k: t.cpu().numpy() for k, t in p.eval_geometry(xd).items()}
                got["B"] = p.eval_jacobian(xd).cpu().numpy()
                outs.append(got)
            print(f"one-launch forward {key}: n {n}, layers {L}, width {wmax}", flush=True)
            for got in outs[1:]:
                for k in ("f", "phi", "g", "H", "L", "B"):
                    np.testing.assert_array_equal(got[k], outs[0][k], err_msg=k)
            assert np.all(np.isfinite(outs[1]["f"]))
    finally:
        clear_tuning()
        p.close()
        ctx.close()
