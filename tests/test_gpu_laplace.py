"""Device Gauss-Newton MAP and Laplace samples (proposal entry point at dt = 4)
against the oracle's plain-solve iteration.

Near the minimum J is flat to rounding within about sqrt(eps) |x|, so the two
iterations may stop one step apart: the MAP points are compared to 1e-6 relative and
the objective to 1e-10 relative. The samples at a given MAP and given xi are a
triangular solve of the FP64 factor: 1e-9 relative.
"""
import numpy as np
import pytest

from oracle import laplace as olap
from tests.helpers import device_problem, make_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "tiny": dict(name="tiny", chains=8),
    "resnet-ragged": dict(name="tiny", chains=8, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                          bias_scale=0.3, noise_scale=0.05),
}


@pytest.mark.parametrize("key", list(CASES))
def test_gauss_newton_map_and_laplace_samples(key):
    from paper_2403_08220_amd import laplace

    kw = dict(CASES[key])
    case = make_case(kw.pop("name"), **kw)
    print(f"laplace {key}", flush=True)
    ctx, p = device_problem(case)
    p.close()
    prob = case["prob"]
    r = case["w"].r
    ref = olap.gauss_newton_map(prob, np.zeros(r))
    got = laplace.gauss_newton_map(ctx, prob.y, prob.noise_var, np.zeros(r))
    print(f"MAP {key}: oracle J {ref.J:.12g} ({ref.iters} it), device J {got.J:.12g} ({got.iters} it)", flush=True)
    assert ref.converged and got.converged
    assert abs(got.J - ref.J) <= 1e-10 * (1 + abs(ref.J))
    assert np.max(np.abs(got.x - ref.x)) <= 1e-6 * (1 + np.max(np.abs(ref.x)))
    xi = np.random.default_rng(5).standard_normal((case["C"], r))
    s_ref = olap.laplace_samples(prob, ref.x, xi)
    s_got = laplace.laplace_samples(ctx, prob.y, prob.noise_var, ref.x, xi)
    assert np.max(np.abs(s_got - s_ref)) <= 1e-9 * (1 + np.max(np.abs(s_ref)))
    ctx.close()
