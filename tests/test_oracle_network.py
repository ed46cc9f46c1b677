"""Pins for oracle/network.py and the geometry of oracle/mcmc.py: central finite
differences of the network and of the misfit, forward == reverse mode, linear
networks (J = product of weights), the GELU definition, and H = J^T Gamma^-1 J."""
import math

import numpy as np
import pytest

from oracle import mcmc, network
from synth import draw_network, workload


def small_net(arch, r=5, width=7, depth=3, d_out=4, seed=3, bias=0.3):
    w = workload("tiny", r=r, width=width, depth=depth, d_out=d_out, d_y=d_out, arch=arch)
    return draw_network(w, seed=seed, bias_scale=bias)


def test_gelu_definition():
    assert network.gelu(0.0) == 0.0
    assert network.gelu_prime(0.0) == 0.5
    z = np.array([-3.0, -0.7, 0.2, 1.5, 4.0])
    Phi = np.array([0.5 * math.erfc(-v / math.sqrt(2.0)) for v in z])
    np.testing.assert_allclose(network.gelu(z), z * Phi, rtol=1e-14, atol=1e-16)
    h = 1e-6
    fd = (network.gelu(z + h) - network.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(network.gelu_prime(z), fd, rtol=1e-8, atol=1e-10)
    # exact GELU, not the tanh approximation (they differ by ~1e-3 near |z| ~ 2)
    tanh_approx = 0.5 * z * (1 + np.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))
    assert np.max(np.abs(network.gelu(z) - tanh_approx)) > 1e-5


@pytest.mark.parametrize("arch", ["mlp", "resnet"])
def test_jacobian_fd_and_modes(arch):
    layers = small_net(arch)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5))
    Jr = network.jacobian_reverse(layers, x)
    Jf = network.jacobian_forward(layers, x)
    np.testing.assert_allclose(Jr, Jf, rtol=1e-12, atol=1e-13)
    h = 1e-6
    for j in range(5):
        e = np.zeros(5)
        e[j] = h
        fp, _ = network.forward(layers, x + e)
        fm, _ = network.forward(layers, x - e)
        fd = (fp - fm) / (2 * h)
        np.testing.assert_allclose(Jr[:, :, j], fd, rtol=1e-6, atol=1e-8)


def test_linear_network_jacobian_is_weight_product():
    rng = np.random.default_rng(4)
    Ws = [rng.standard_normal((6, 3)), rng.standard_normal((5, 6)), rng.standard_normal((2, 5))]
    layers = [("linear", W, rng.standard_normal(W.shape[0])) for W in Ws]
    x = rng.standard_normal((2, 3))
    J = network.jacobian_reverse(layers, x)
    np.testing.assert_allclose(J[0], Ws[2] @ Ws[1] @ Ws[0], rtol=1e-13)
    f, _ = network.forward(layers, x)
    ref = ((x @ Ws[0].T + layers[0][2]) @ Ws[1].T + layers[1][2]) @ Ws[2].T + layers[2][2]
    np.testing.assert_allclose(f, ref, rtol=1e-13)


def test_resnet_structure():
    """h_l = h_{l-1} + gelu(W_l h_{l-1} + b_l) between a linear lift and a linear output."""
    layers = small_net("resnet", depth=2)
    x = np.random.default_rng(1).standard_normal((1, 5))
    (k0, W0, b0), (k1, W1, b1), (k2, W2, b2), (k3, W3, b3) = layers
    assert (k0, k1, k2, k3) == ("linear", "resid", "resid", "linear")
    h = x @ W0.T + b0
    h = h + network.gelu(h @ W1.T + b1)
    h = h + network.gelu(h @ W2.T + b2)
    f = h @ W3.T + b3
    np.testing.assert_allclose(network.forward(layers, x)[0], f, rtol=1e-14)


def make_problem(arch="mlp", d_out=4, noise=(0.05, 0.1, 0.2, 0.3), dt=0.3):
    layers = small_net(arch, d_out=d_out)
    y = np.random.default_rng(2).standard_normal(d_out) * 0.5
    return mcmc.Problem(layers, y, np.asarray(noise[:d_out]) ** 2, dt)


@pytest.mark.parametrize("arch", ["mlp", "resnet"])
def test_gradient_is_misfit_derivative(arch):
    """g = J^T Gamma^-1 (f - y) is the gradient of Phi (fixes the printed sign)."""
    prob = make_problem(arch)
    x = np.random.default_rng(5).standard_normal((2, 5))
    c = mcmc.geometry(prob, x)
    h = 1e-6
    for j in range(5):
        e = np.zeros(5)
        e[j] = h
        fd = (mcmc.geometry(prob, x + e).phi - mcmc.geometry(prob, x - e).phi) / (2 * h)
        np.testing.assert_allclose(c.g[:, j], fd, rtol=1e-6, atol=1e-7)


def test_hessian_gauss_newton_and_exact_for_linear():
    prob = make_problem("mlp")
    x = np.random.default_rng(6).standard_normal((2, 5))
    c = mcmc.geometry(prob, x)
    J = network.jacobian_reverse(prob.layers, x)
    ref = np.einsum("cir,i,cis->crs", J, 1.0 / prob.noise_var, J)
    np.testing.assert_allclose(c.H, ref, rtol=1e-13)
    np.testing.assert_allclose(c.H, np.transpose(c.H, (0, 2, 1)), atol=1e-14)
    assert np.all(np.linalg.eigvalsh(c.H) > -1e-12)
    # for an affine network the Gauss-Newton Hessian is the exact Hessian of Phi
    rng = np.random.default_rng(8)
    A = rng.standard_normal((4, 5))
    lin = mcmc.Problem([("linear", A, rng.standard_normal(4))], prob.y, prob.noise_var, 0.3)
    cl = mcmc.geometry(lin, x)
    h = 1e-5
    for j in range(5):
        e = np.zeros(5)
        e[j] = h
        fd = (mcmc.geometry(lin, x + e).g - mcmc.geometry(lin, x - e).g) / (2 * h)
        np.testing.assert_allclose(cl.H[:, :, j], fd, rtol=1e-7, atol=1e-7)
    # Cholesky factor and eigendecomposition describe the same I + H
    np.testing.assert_allclose(c.L @ np.transpose(c.L, (0, 2, 1)), np.eye(5) + c.H, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(np.einsum("crk,ck,csk->crs", c.P, c.d, c.P), c.H, rtol=1e-10, atol=1e-10)


def test_partial_observation_is_prefix():
    """A problem observing d_y < d_out outputs sees the first d_y outputs."""
    layers = small_net("mlp", d_out=4)
    x = np.random.default_rng(9).standard_normal((1, 5))
    f, _ = network.forward(layers, x)
    p2 = mcmc.Problem(layers, f[0, :2] + 0.1, np.full(2, 0.01), 0.2)
    c = mcmc.geometry(p2, x)
    np.testing.assert_allclose(c.f, f[:, :2])
    np.testing.assert_allclose(c.phi, 0.5 * 2 * (0.1 ** 2) / 0.01, rtol=1e-12)
