"""Shared test fixtures: seeded problems built from synth/ and the oracle's data model."""
from __future__ import annotations

import numpy as np

from oracle import mcmc, network, prior
from synth import draw_initial_states, draw_network, draw_noise, draw_true_state, workload


def make_case(name="tiny", chains=None, bias_scale=0.0, noise_scale=None, dt=None, **overrides):
    """Workload + network + data y = f(x_true) + sigma eps (the data model, eq. data_model)."""
    w = workload(name, **overrides)
    layers = draw_network(w, bias_scale=bias_scale)
    x_true = draw_true_state(w)[: w.r]
    f_true, _ = network.forward(layers, x_true[None])
    f_obs = f_true[0, : w.d_y]
    if w.sigma_rule == "abs":
        sigma = w.sigma
    else:
        sigma = w.sigma * np.max(np.abs(f_obs))
    if noise_scale is not None:
        sigma = noise_scale
    y = f_obs + sigma * draw_noise(w)
    nv = np.full(w.d_y, sigma ** 2)
    C = w.chains if chains is None else chains
    prob = mcmc.Problem(layers, y, nv, w.dt if dt is None else dt, seed=w.chain_seed, request_id=0)
    x0, z0 = draw_initial_states(w, chains=C)
    return dict(w=w, layers=layers, y=y, noise_var=nv, prob=prob, x0=x0, z0=z0, C=C)


def device_problem(case, precision="f64", trace_capacity=0, track_complement=True, chains=None,
                   factorization="primal", method="mmala"):
    """Context + problem on cuda:0 holding the case's prior, network and data."""
    from paper_2403_08220_amd import Context, Problem

    w = case["w"]
    ctx = Context(0)
    ctx.load_prior(w.n, w.gamma, w.delta, w.r)
    ctx.load_network(case["layers"])
    prob = case["prob"]
    p = Problem(ctx, case["C"] if chains is None else chains, prob.y, prob.noise_var, prob.dt, seed=prob.seed,
                request_id=prob.request_id, precision=precision, track_complement=track_complement,
                trace_capacity=trace_capacity, factorization=factorization, method=method)
    return ctx, p


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)
