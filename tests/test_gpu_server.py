"""Serving path (continuous batching) through the C ABI.

* Parity: every request's posterior mean field equals the oracle's run of the same
  request (key (seed, request id), prior initial states of streams 3 and 4, n_steps
  transitions, burn-in 20%, Rao-Blackwellised mean Psi_r xbar, the observation-space
  form since every bucket has d_y < r), on the FP64 path, to 1e-9 relative; the
  acceptance counts are identical. Requests whose d_y is below
  their bucket's observe the first d_y outputs (the oracle problem has d_y outputs).
* Isolation: a request's result is the same alone and in a mix of requests that
  arrive while it runs and occupy other slots of its pool; the chains of different
  requests never mix, so the results agree to rounding (1e-12 relative).
* Admission: more requests than slots or rows wait and are admitted as others finish.
"""
import numpy as np
import pytest

from oracle import mcmc, network, philox, prior
from synth import draw_network, workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

W = workload("tiny", arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=24)
LAYERS = draw_network(W, bias_scale=0.3)


def request_data(rid, d_y, noise=0.2):
    rng = np.random.default_rng(1000 + rid)
    x_true = rng.standard_normal(W.r)
    f, _ = network.forward(LAYERS, x_true[None])
    y = f[0, :d_y] + noise * rng.standard_normal(d_y)
    return y, np.full(d_y, noise ** 2)


def make_ctx():
    from paper_2403_08220_amd import Context
    ctx = Context(0)
    ctx.load_prior(W.n, W.gamma, W.delta, W.r)
    ctx.load_network(LAYERS)
    return ctx


def oracle_mean(seed, rid, y, nv, C, N, dt, dec):
    # the pools take the observation-space form when d_y < r (every bucket here)
    prob = mcmc.Problem(LAYERS, y, nv, dt, seed=seed, request_id=rid, factor="dual" if len(y) < W.r else "primal")
    x0 = philox.normals(seed, rid, philox.STREAM_INIT_X, 0, np.arange(C), W.r)
    st = mcmc.init_state(prob, x0)
    xs, _ = mcmc.run(prob, st, N)
    burn = N // 5
    xbar = xs[burn:].reshape(-1, W.r).mean(axis=0)
    return dec @ xbar, int(st.accepts.sum()), int(st.failures.sum())


REQS = [  # (request id, d_y, chains, steps)
    (1, 10, 3, 30),
    (2, 20, 5, 25),
    (3, 24, 4, 40),
    (4, 7, 6, 20),
]


def test_server_matches_oracle_fp64():
    from paper_2403_08220_amd import Server
    print("server parity fp64", flush=True)
    ctx = make_ctx()
    dt = 0.5
    srv = Server(ctx, [(10, 12), (24, 12)], max_requests=3, steps_per_quantum=7, dt=dt, precision="f64")
    for rid, dy, C, N in REQS:
        y, nv = request_data(rid, dy)
        srv.submit(seed=9, request_id=rid, y=y, noise_var=nv, n_chains=C, n_steps=N)
    srv.run()
    res = {r["request_id"]: r for r in srv.poll()}
    assert sorted(res) == [1, 2, 3, 4]
    dec = prior.KLEBasis(W.n, W.gamma, W.delta, W.r).dec
    for rid, dy, C, N in REQS:
        y, nv = request_data(rid, dy)
        ref, acc, fail = oracle_mean(9, rid, y, nv, C, N, dt, dec)
        got = res[rid]
        err = np.max(np.abs(got["mean"] - ref)) / np.max(np.abs(ref))
        print(f"request {rid}: d_y {dy}, {C} chains x {N}: rel err {err:.2e}, accepts {got['accepts']} "
              f"(oracle {acc})", flush=True)
        assert err < 1e-9
        assert got["accepts"] == acc and got["failures"] == fail
        assert got["arrival"] <= got["admitted"] <= got["finished"]
    srv.close()
    ctx.close()


def test_request_alone_equals_request_in_mix():
    from paper_2403_08220_amd import Server
    print("server isolation bf16", flush=True)
    ctx = make_ctx()
    dt = 0.5
    yA, nvA = request_data(7, 20)

    srv = Server(ctx, [(10, 32), (24, 32)], max_requests=4, steps_per_quantum=5, dt=dt, precision="bf16")
    srv.submit(seed=3, request_id=7, y=yA, noise_var=nvA, n_chains=6, n_steps=40)
    srv.run()
    alone = srv.poll()[0]
    srv.close()

    srv = Server(ctx, [(10, 32), (24, 32)], max_requests=4, steps_per_quantum=5, dt=dt, precision="bf16")
    for rid, dy, C, N in [(11, 24, 10, 60), (12, 10, 8, 30), (13, 20, 7, 50)]:
        y, nv = request_data(rid, dy)
        srv.submit(seed=3, request_id=rid, y=y, noise_var=nv, n_chains=C, n_steps=N)
    t = srv.clock()
    srv.submit(seed=3, request_id=7, y=yA, noise_var=nvA, n_chains=6, n_steps=40, arrival=t + 0.02)
    y, nv = request_data(14, 24)
    srv.submit(seed=3, request_id=14, y=y, noise_var=nv, n_chains=9, n_steps=45, arrival=t + 0.03)
    srv.run()
    mix = {r["request_id"]: r for r in srv.poll()}
    srv.close()
    assert sorted(mix) == [7, 11, 12, 13, 14]
    a, m = alone["mean"], mix[7]["mean"]
    diff = np.max(np.abs(a - m)) / np.max(np.abs(a))
    print(f"alone vs mix: max rel diff {diff:.2e} (bitwise equal: {np.array_equal(a, m)}), "
          f"admitted at {mix[7]['admitted']:.4f} s while {sum(1 for k in mix if k != 7)} others ran", flush=True)
    assert diff <= 1e-12
    assert alone["accepts"] == mix[7]["accepts"]
    ctx.close()


def test_admission_waits_for_slots_and_rows():
    from paper_2403_08220_amd import Server
    print("server admission", flush=True)
    ctx = make_ctx()
    srv = Server(ctx, [(24, 8)], max_requests=2, steps_per_quantum=4, dt=0.5, precision="bf16")
    plan = [(21, 5, 12), (22, 4, 16), (23, 8, 8), (24, 3, 20), (25, 4, 10)]
    for rid, C, N in plan:
        y, nv = request_data(rid, 24)
        srv.submit(seed=5, request_id=rid, y=y, noise_var=nv, n_chains=C, n_steps=N)
    srv.run()
    res = {r["request_id"]: r for r in srv.poll()}
    assert sorted(res) == [21, 22, 23, 24, 25]
    # never more than 8 slots or 2 requests at once
    events = sorted([(r["admitted"], +1, r["n_chains"]) for r in res.values()]
                    + [(r["finished"], -1, -r["n_chains"]) for r in res.values()])
    live = slots = 0
    for _, d, c in events:
        live += d
        slots += c
        assert live <= 2 and slots <= 8
    for r in res.values():
        assert r["arrival"] <= r["admitted"] <= r["finished"]
        assert np.all(np.isfinite(r["mean"]))
    srv.close()
    ctx.close()


def test_server_argument_errors():
    from paper_2403_08220_amd import DinoError, Server
    ctx = make_ctx()
    with pytest.raises(DinoError):
        Server(ctx, [(24, 8), (10, 8)], max_requests=2, steps_per_quantum=4, dt=0.5)   # buckets must ascend
    with pytest.raises(DinoError):
        Server(ctx, [(24, 8)], max_requests=2, steps_per_quantum=4, dt=0.5, hbm_budget_bytes=1e3)
    srv = Server(ctx, [(10, 8)], max_requests=2, steps_per_quantum=4, dt=0.5)
    y, nv = request_data(1, 20)
    with pytest.raises(DinoError):
        srv.submit(seed=1, request_id=1, y=y, noise_var=nv, n_chains=4, n_steps=10)     # d_y above every bucket
    y, nv = request_data(1, 10)
    with pytest.raises(DinoError):
        srv.submit(seed=1, request_id=1, y=y, noise_var=nv, n_chains=9, n_steps=10)     # more chains than slots
    srv.close()
    ctx.close()
