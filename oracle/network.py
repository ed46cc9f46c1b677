"""Reduced-basis neural operator f_NN and its reduced Jacobian (oracle; test infrastructure).

Paper basis: the surrogate G~(m) = V f_NN(Psi_r^* m) (Sec. 4, eq. rb_dino) and its
reduced Jacobian J~_r = d f_NN / d m_r (Sec. 4, the display after eq. rb_dino). The
paper's experiments use a dense GELU network (Sec. 7.2, Sec. 8.2).

Architectures (a network is a list of layers (kind, W, b), W of shape (fan_out, fan_in)):
    "linear": h <- W h + b
    "act":    z = W h + b, h <- sigma(z)            (dense layer with activation)
    "resid":  z = W h + b, h <- h + sigma(z)        (residual block, W square)
The MLP reading is [act, act, ..., linear]; the ResNet reading is
[linear (lift), resid x L, linear (output)].

sigma is the exact GELU, sigma(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2, with
sigma'(z) = Phi(z) + z phi(z) (phi the standard normal density).

All arrays carry a leading chain axis: x has shape (C, r), f (C, d_y), J (C, d_y, r).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def forward(layers, x):
    """f_NN(x) for a batch x (C, r). Returns (f, zs) with zs the pre-activations of
    every "act"/"resid" layer, in layer order (needed by the Jacobian)."""
    h = np.asarray(x, dtype=np.float64)
    zs = []
    for kind, W, b in layers:
        z = h @ W.T + b
        if kind == "linear":
            h = z
        elif kind == "act":
            zs.append(z)
            h = gelu(z)
        elif kind == "resid":
            zs.append(z)
            h = h + gelu(z)
        else:
            raise ValueError(kind)
    return h, zs


def jacobian_reverse(layers, x):
    """Reduced Jacobian by reverse-mode accumulation, shape (C, d_y, r).

    Lambda starts as the output layer's weights and is pulled back through the layers:
    linear: Lambda <- Lambda W; act: Lambda <- (Lambda D) W; resid: Lambda <- Lambda + (Lambda D) W,
    with D = diag sigma'(z) of that layer at x.
    """
    _, zs = forward(layers, x)
    C = np.asarray(x).shape[0]
    lam = None
    zi = len(zs)
    for kind, W, b in reversed(layers):
        if lam is None:
            if kind != "linear":
                raise ValueError("the last layer must be linear")
            lam = np.broadcast_to(W, (C,) + W.shape).copy()
            continue
        if kind == "linear":
            lam = lam @ W
        else:
            zi -= 1
            D = gelu_prime(zs[zi])  # (C, fan_out)
            upd = (lam * D[:, None, :]) @ W
            lam = upd if kind == "act" else lam + upd
    return lam


def jacobian_forward(layers, x):
    """Reduced Jacobian by forward-mode (tangent) propagation, shape (C, d_y, r)."""
    x = np.asarray(x, dtype=np.float64)
    C, r = x.shape
    h = x
    T = np.broadcast_to(np.eye(r), (C, r, r)).copy()  # dh/dx, (C, width, r)
    for kind, W, b in layers:
        z = h @ W.T + b
        Tz = W @ T  # (C, fan_out, r)
        if kind == "linear":
            h, T = z, Tz
        elif kind == "act":
            h, T = gelu(z), gelu_prime(z)[:, :, None] * Tz
        else:
            h, T = h + gelu(z), T + gelu_prime(z)[:, :, None] * Tz
    return T
