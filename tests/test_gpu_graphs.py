"""Launch graphs: dino_step replays a captured graph of the step loop (DINO_LAUNCH_GRAPH,
the default). A graph runs the same kernels with the same arguments as the eager loop,
so every replay must give bit-identical chains: each case replays several graphs (a
full one and the remainder), with eager device work, stream synchronisations and host
reads between the replays, and compares states, complement, decisions, caches and trace
with an eager twin problem after every call."""
import numpy as np
import pytest

from synth import draw_true_model
from tests.helpers import device_problem, make_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "bf16-dual": dict(precision="bf16", factorization="dual", method="mmala"),
    "bf16-primal": dict(precision="bf16", factorization="primal", method="mmala"),
    "f64-dual": dict(precision="f64", factorization="dual", method="mmala"),
    "f64-pcn": dict(precision="f64", factorization="primal", method="pcn"),
    "bf16-mala": dict(precision="bf16", factorization="primal", method="mala", dt=0.005),
    "bf16-da": dict(precision="bf16", factorization="dual", method="da_mmala"),
}


def twin(case, spec, mode):
    ctx, p = device_problem(case, precision=spec["precision"], factorization=spec["factorization"],
                            method="mmala" if spec["method"] == "da_mmala" else spec["method"], trace_capacity=40,
                            chains=1)
    p.close()
    if spec["method"] == "da_mmala":
        ctx.load_true_model(draw_true_model(case["layers"], 8))
    from paper_2403_08220_amd import Problem
    prob = case["prob"]
    p = Problem(ctx, case["C"], prob.y, prob.noise_var, prob.dt, seed=prob.seed, request_id=prob.request_id,
                precision=spec["precision"], track_complement=True, trace_capacity=40,
                factorization=spec["factorization"], method=spec["method"])
    p.set_launch_mode(mode, steps_per_graph=4)
    p.init(case["x0"], case["z0"])
    return ctx, p


def snapshot(p):
    x, z = p.states()
    acc, fail, steps = p.diagnostics()
    phi, g, _ = p.cache()
    xt, pt = p.trace()
    return dict(x=x, z=z, acc=acc, fail=fail, steps=steps, phi=phi, g=g, xt=xt, pt=pt)


@pytest.mark.parametrize("key", list(CASES))
def test_graph_replays_equal_eager(key):
    spec = CASES[key]
    case = make_case("tiny", chains=70, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20, bias_scale=0.3,
                     noise_scale=0.2, dt=spec.get("dt", 0.5))
    print(f"graphs {key}", flush=True)
    ctx_e, pe = twin(case, spec, "eager")
    ctx_g, pg = twin(case, spec, "graph")
    try:
        scratch = torch.randn(512, 512, device="cuda:0")
        for n in (6, 1, 9, 4):                   # full graphs of 4 and remainders of 2, 1, 1, 0
            pe.step(n)
            pg.step(n)
            scratch = scratch @ scratch.T / 512.0  # eager device work between replays
            torch.cuda.synchronize()
            a, b = snapshot(pe), snapshot(pg)
            for k in a:
                np.testing.assert_array_equal(a[k], b[k], err_msg=f"{key}: {k} after {n} more steps")
        assert a["steps"] == 20 and a["acc"].sum() > 0
    finally:
        pe.close()
        pg.close()
        ctx_e.close()
        ctx_g.close()


def test_launch_mode_arguments():
    from paper_2403_08220_amd import DinoError

    case = make_case("tiny", chains=4)
    ctx, p = device_problem(case)
    try:
        with pytest.raises(DinoError, match="steps_per_graph"):
            p.set_launch_mode("graph", steps_per_graph=0)
        with pytest.raises(KeyError):
            p.set_launch_mode("persistent")
    finally:
        p.close()
        ctx.close()
