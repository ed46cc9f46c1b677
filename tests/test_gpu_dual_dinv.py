"""Inverted diagonal blocks of the dual factor (mixed path).

The fused Gram + factor kernel stores D_b = L_bb^-1 for every diagonal block of 32 rows
in the factor's unused upper triangle (D_b[k][m], m < k, at row b0 + m, column b0 + k),
and the dual proposal and acceptance then solve block by block through D_b instead of a
serial substitution. The stored blocks are checked against numpy's inverse of the
factor's own diagonal blocks (FP64, 1e-12 relative per block, full and ragged blocks, d_y
from 20 to 104),
and chains stepped with these solves against the same chains stepped with the
substitution (tuning kind dualsolve = 0): identical decisions and states to 1e-10, the
solves differing only in FP64 rounding.
"""
import numpy as np
import pytest

from tests.helpers import device_problem, make_case, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "mid-96": dict(name="mid", chains=96, dt=1e-5),
    "resnet-37": dict(name="tiny", chains=37, arch="resnet", r=40, width=80, depth=2, d_out=24, d_y=20,
                      bias_scale=0.3, noise_scale=0.2, dt=0.5),
}
# d_y at the edges of the inversion's split: three full blocks and no short one (96), a
# short block of 8 rows (72, 104), one full block and a short one of 9 rows (41)
EDGES = {f"resnet-dy{dy}": dict(name="tiny", chains=19, arch="resnet", r=128, width=80, depth=2, d_out=dy, d_y=dy,
                                bias_scale=0.3, noise_scale=0.2, dt=0.05) for dy in (41, 72, 96, 104)}


def stepped(case, n_steps, choice=None):
    from paper_2403_08220_amd import clear_tuning, tune_set
    from paper_2403_08220_amd._lib import check, dptr

    dy = case["prob"].d_y
    if choice is not None:
        tune_set("dualsolve", (dy, 0, 0), choice)
    try:
        ctx, p = device_problem(case, precision="bf16", factorization="dual")
        p.init(case["x0"], None)
        p.step(n_steps)
        x, _ = p.states()
        acc, fail, _ = p.diagnostics()
        # the factors as stored (Problem.cache clears the upper triangle of the r x r view)
        L = np.empty((case["C"], case["w"].r, case["w"].r))
        check(p.lib.dino_read_cache(p.h, None, None, dptr(L)))
        p.close()
        ctx.close()
    finally:
        clear_tuning()
    return x, acc, fail, L


@pytest.mark.parametrize("key", list(CASES) + list(EDGES))
def test_factor_carries_its_inverted_diagonal_blocks(key):
    kw = dict({**CASES, **EDGES}[key])
    case = make_case(kw.pop("name"), **kw)
    C, r, dy = case["C"], case["w"].r, case["prob"].d_y
    print(f"inverted diagonal blocks {key}: {C} chains, d_y {dy}", flush=True)
    _, _, fail, L = stepped(case, 3)
    assert np.all(fail == 0)
    K = L.reshape(C, -1)[:, : dy * dy].reshape(C, dy, dy)
    worst = 0.0
    for b0 in range(0, dy, 32):
        nb = min(32, dy - b0)
        blk = K[:, b0 : b0 + nb, b0 : b0 + nb]
        Dref = np.linalg.inv(np.tril(blk))
        Dstored = np.transpose(np.triu(blk, 1), (0, 2, 1))    # strictly lower part of D_b
        for c in range(C):
            e = np.linalg.norm(Dstored[c] - np.tril(Dref[c], -1)) / np.linalg.norm(Dref[c])
            worst = max(worst, e)
    print(f"  worst block relative error {worst:.2e}", flush=True)
    assert worst < 1e-12


@pytest.mark.parametrize("key", list(CASES))
def test_block_inverse_solves_match_substitution(key):
    kw = dict(CASES[key])
    case = make_case(kw.pop("name"), **kw)
    print(f"dual solves {key}: substitution vs inverted blocks", flush=True)
    x0, acc0, fail0, _ = stepped(case, 6, choice=0)
    x1, acc1, fail1, _ = stepped(case, 6, choice=1)
    print(f"  accepts {acc0.sum()} / {acc1.sum()}, state difference {rel_err(x1, x0):.2e}", flush=True)
    np.testing.assert_array_equal(acc1, acc0)
    np.testing.assert_array_equal(fail1, fail0)
    assert acc0.sum() > 0
    assert rel_err(x1, x0) < 1e-10
