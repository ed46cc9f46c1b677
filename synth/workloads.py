"""Workload sizes and seeded draws (no method arithmetic here).

Workloads mirror the shapes of the paper's experiments (reduced dimension r = 200
and width-400 GELU networks in Sec. 7.4/8.5, tens to hundreds of observables in
Sec. 7.2/8.3) on a synthetic grid Matern prior, since the paper's PDE data, trained
weights and meshes are not available:

    tiny  : 33x33 grid, r=32,  MLP 32->64->64->16 GELU, d_y=16, 4 chains x 2000 steps, dt=0.1,
            sigma = 0.01 absolute (FP64 path; also the BF16 precision study)
    mid   : 129x129 grid, r=200, ResNet width 400 depth 4, d_y=100, 512 chains x 1000 steps,
            sigma = 1% of max |f(x_true)|, dt = 3e-4
    serve : 129x129 grid, r=200, ResNet 400x4 (100 outputs); requests with d_y in {25,50,100},
            chains uniform in [8,128], steps uniform in [500,5000], Poisson arrivals
    large : 257x257 grid, r=400, ResNet width 800 depth 6, d_y=400, 4096 chains x 2000 steps
    mix   : the mid shapes with sigma = 30% of max |f(x_true)|: a weakly informed posterior
            on which the mid-shaped chains decorrelate within ~1000 steps (the ESS/s leg)

Step sizes: tiny keeps the literal dt = 0.1 of its definition; mid and serve use the
value chosen once by the appendix's tuning rule (AR decreasing and MSJ increasing up
to dt_max, then the largest median ESS%) on the FP64 device path from Laplace
samples, over the candidates 3e-5, 1e-4, 3e-4, 1e-3, 3e-3: 3e-4 (AR 0.27), and
frozen here. TUNED_DT records the tuned value of every workload that has one (tiny:
3e-3 over 1e-4 .. 3e-2, AR 0.13). large is not tuned.

Prior: (-gamma Lap + delta I)^-2 with gamma = 0.1, delta = 1 on every grid.
Weights: Xavier/Glorot normal, std sqrt(2/(fan_in + fan_out)), drawn with
numpy.random.default_rng(seed) in layer order as standard_normal((fan_out, fan_in));
biases zero unless ``bias_scale`` > 0 (tests use nonzero biases).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # grid points per side
    gamma: float
    delta: float
    r: int                 # reduced dimension
    arch: str              # "mlp" or "resnet"
    width: int
    depth: int             # hidden layers (mlp) or residual blocks (resnet)
    d_out: int             # network outputs
    d_y: int               # observed outputs
    chains: int
    steps: int
    dt: float
    sigma_rule: str        # "abs" or "rel_max"
    sigma: float           # absolute sigma, or the fraction of max |f_true|
    weight_seed: int = 1
    truth_seed: int = 2
    noise_seed: int = 3
    chain_seed: int = 4
    init_seed: int = 5
    laplace_seed: int = 6

    @property
    def d_m(self) -> int:
        return self.n * self.n


CONFIGS = {
    "tiny": Workload("tiny", 33, 0.1, 1.0, 32, "mlp", 64, 2, 16, 16, 4, 2000, 0.1, "abs", 0.01),
    "mid": Workload("mid", 129, 0.1, 1.0, 200, "resnet", 400, 4, 100, 100, 512, 1000, 3e-4, "rel_max", 0.01),
    "serve": Workload("serve", 129, 0.1, 1.0, 200, "resnet", 400, 4, 100, 100, 68, 2750, 3e-4, "rel_max", 0.01),
    "large": Workload("large", 257, 0.1, 1.0, 400, "resnet", 800, 6, 400, 400, 4096, 2000, 3e-4, "rel_max", 0.01),
    "mix": Workload("mix", 129, 0.1, 1.0, 200, "resnet", 400, 4, 100, 100, 512, 1200, 0.1, "rel_max", 0.3),
}

TUNED_DT = {"tiny": 3e-3, "mid": 3e-4, "serve": 3e-4}


def workload(name: str, **overrides) -> Workload:
    w = CONFIGS[name]
    if overrides:
        d = dict(w.__dict__)
        d.update(overrides)
        w = Workload(**d)
    return w


def layer_shapes(arch: str, r: int, width: int, depth: int, d_out: int):
    """(kind, fan_out, fan_in) of every layer."""
    if arch == "mlp":
        dims = [r] + [width] * depth
        shapes = [("act", dims[i + 1], dims[i]) for i in range(depth)]
        shapes.append(("linear", d_out, dims[-1]))
    elif arch == "resnet":
        shapes = [("linear", width, r)]
        shapes += [("resid", width, width)] * depth
        shapes.append(("linear", d_out, width))
    else:
        raise ValueError(arch)
    return shapes


def draw_network(w: Workload, seed: int | None = None, bias_scale: float = 0.0):
    """Xavier-normal weights as a list of (kind, W, b) in float64."""
    rng = np.random.default_rng(w.weight_seed if seed is None else seed)
    layers = []
    shapes = layer_shapes(w.arch, w.r, w.width, w.depth, w.d_out)
    for kind, fo, fi in shapes:
        std = np.sqrt(2.0 / (fi + fo))
        W = std * rng.standard_normal((fo, fi))
        layers.append([kind, W, None])
    for layer in layers:
        fo = layer[1].shape[0]
        layer[2] = bias_scale * rng.standard_normal(fo) if bias_scale > 0 else np.zeros(fo)
    return [tuple(l) for l in layers]


def draw_true_state(w: Workload, seed: int | None = None) -> np.ndarray:
    """Whitened KLE coordinates of m_true, a prior draw: N(0, I_dm); x_true = first r."""
    rng = np.random.default_rng(w.truth_seed if seed is None else seed)
    return rng.standard_normal(w.d_m)


def draw_noise(w: Workload, d_y: int | None = None, seed: int | None = None) -> np.ndarray:
    """Standard normal noise eps (d_y,); the data are y = f(x_true) + sigma eps."""
    rng = np.random.default_rng(w.noise_seed if seed is None else seed)
    return rng.standard_normal(w.d_y if d_y is None else d_y)


def draw_initial_states(w: Workload, chains: int | None = None, seed: int | None = None,
                        complement: bool = True):
    """Independent prior draws: x0 (C, r) and, if asked, z0 (C, d_m - r) as float32."""
    C = w.chains if chains is None else chains
    rng = np.random.default_rng(w.init_seed if seed is None else seed)
    x0 = rng.standard_normal((C, w.r))
    z0 = rng.standard_normal((C, w.d_m - w.r)).astype(np.float32) if complement else None
    return x0, z0


def draw_laplace_normals(w: Workload, chains: int | None = None, seed: int | None = None) -> np.ndarray:
    """Standard normals xi (C, r) that map to Laplace-approximation samples x_map + L^-T xi."""
    C = w.chains if chains is None else chains
    rng = np.random.default_rng(w.laplace_seed if seed is None else seed)
    return rng.standard_normal((C, w.r))


@dataclass
class Request:
    rid: int
    arrival: float         # seconds after the stream starts
    d_y: int
    chains: int
    steps: int
    truth_seed: int
    noise_seed: int
    chain_seed: int


def draw_requests(count: int, rate: float, seed: int = 11):
    """Poisson stream: exponential inter-arrival times with mean 1/rate; d_y uniform in
    {25, 50, 100}, chains uniform in [8, 128], steps uniform in [500, 5000]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    dys = rng.choice([25, 50, 100], size=count)
    cs = rng.integers(8, 129, size=count)
    ns = rng.integers(500, 5001, size=count)
    base = rng.integers(1, 2 ** 31, size=(count, 3))
    return [Request(i, float(t[i]), int(dys[i]), int(cs[i]), int(ns[i]),
                    int(base[i, 0]), int(base[i, 1]), int(base[i, 2])) for i in range(count)]


def draw_true_model(layers, extra: int, eps: float = 0.05, seed: int = 17):
    """Layers of a true-model stand-in for delayed acceptance: the surrogate's weights with
    relative N(0, eps^2) perturbations and `extra` more input columns on the first layer
    (N(0, (std(W_1)/2)^2) entries), so that it also reads the first `extra` complement
    coordinates."""
    rng = np.random.default_rng(seed)
    out = []
    for l, (kind, W, b) in enumerate(layers):
        W2 = W * (1.0 + eps * rng.standard_normal(W.shape))
        if l == 0 and extra:
            cols = rng.standard_normal((W.shape[0], extra)) * (np.std(W) * 0.5)
            W2 = np.concatenate([W2, cols], axis=1)
        out.append((kind, W2, None if b is None else b.copy()))
    return out
