"""Seeded synthetic inputs shared by the oracle tests and the device path.

This package holds no arithmetic of the method: it only draws random numbers
(network weights, true reduced states, noise, initial states, request streams) and
states the workload sizes. Everything that evaluates the prior, the network, the
geometry or the sampler lives in ``oracle/`` (CPU reference) or in the HIP library,
and the two never import each other.
"""
from .workloads import (  # noqa: F401
    CONFIGS,
    TUNED_DT,
    Workload,
    draw_initial_states,
    draw_laplace_normals,
    draw_network,
    draw_noise,
    draw_requests,
    draw_true_model,
    draw_true_state,
    workload,
)
