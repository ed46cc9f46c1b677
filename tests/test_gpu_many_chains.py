"""More chains than the grid's y extent (65535): the kernels that put chains (or fields)
on grid y or z loop over them, so every chain is stepped, its complement moved and its
statistics formed."""
import numpy as np
import pytest

from tests.helpers import device_problem, make_case

C = 70000


@pytest.mark.gpu
@pytest.mark.parametrize("precision,factorization", [("bf16", "dual"), ("f64", "primal")])
def test_more_chains_than_grid_y(precision, factorization):
    case = make_case("tiny", chains=C, noise_scale=0.1)
    print(f"many chains {precision} {factorization}", flush=True)
    ctx, p = device_problem(case, precision=precision, trace_capacity=3, factorization=factorization)
    try:
        z0 = case["z0"].astype(np.float32)
        p.init(case["x0"], z0)
        p.step(3)
        x, z = p.states()
        acc, fail, steps = p.diagnostics()
        assert steps == 3
        assert np.all(np.isfinite(x))
        hi = np.arange(C) >= 65535
        moved = np.any(z != z0, axis=1)
        # a chain's complement moves exactly when one of its steps was accepted
        np.testing.assert_array_equal(moved, acc > 0)
        assert np.sum(acc[hi] > 0) > 100
        ess = p.ess(0)
        assert ess.shape == (case["w"].r,)
    finally:
        p.close()
        ctx.close()
