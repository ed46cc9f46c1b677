"""Host logic of the step-size rule (appendix on tuning): monotone down-selection of
candidates by AR and MSJ, then the largest median ESS% among those kept."""
import numpy as np

from paper_2403_08220_amd.tune import AR_TARGET, ar_spread, mean_square_jump, select_step_size


def test_selects_max_ess_within_monotone_prefix():
    dts = [0.01, 0.03, 0.1, 0.3, 1.0]
    ar = [0.9, 0.8, 0.6, 0.3, 0.35]       # AR rises again at 1.0: prefix ends at 0.3
    msj = [0.1, 0.2, 0.5, 0.7, 0.2]
    ess = [0.01, 0.02, 0.05, 0.04, 0.5]   # the large ESS at 1.0 lies outside the prefix
    idx, kept, _ = select_step_size(dts, ar, msj, ess)
    assert kept == [0, 1, 2, 3] and dts[idx] == 0.1


def test_msj_break_ends_prefix_and_order_is_irrelevant():
    dts = [0.3, 0.01, 0.1, 0.03]
    ar = [0.3, 0.9, 0.6, 0.8]
    msj = [0.4, 0.1, 0.5, 0.2]            # MSJ falls from 0.1 to 0.3
    ess = [0.9, 0.01, 0.05, 0.02]
    idx, kept, _ = select_step_size(dts, ar, msj, ess)
    assert sorted(dts[k] for k in kept) == [0.01, 0.03, 0.1] and dts[idx] == 0.1


def test_nan_ess_never_selected():
    idx, kept, _ = select_step_size([1, 2], [0.5, 0.4], [1, 2], [0.1, float("nan")])
    assert idx == 0 and kept == [0, 1]


def test_mean_square_jump():
    t = np.zeros((3, 2, 2))
    t[1, 0] = [1, 0]
    t[2, 0] = [1, 2]
    # chain 0 jumps 1 then 4; chain 1 never moves
    assert mean_square_jump(t) == (1 + 4 + 0 + 0) / 4


def test_ess_at_floor_falls_back_to_ar_target():
    dts = [1e-4, 3e-4, 1e-3, 3e-3]
    ar = [0.8, 0.5, 0.27, 0.1]
    msj = [1, 2, 3, 4]
    ess = [0.004, 0.0051, 0.0049, 0.005]   # all at the floor of 1.5 / (2 * 100)
    idx, kept, rule = select_step_size(dts, ar, msj, ess, ess_floor_frac=0.0075)
    assert rule == "ar_target" and dts[idx] == 1e-3 and abs(ar[idx] - AR_TARGET) < 0.05
    # one candidate above the floor: ESS decides again
    ess[1] = 0.02
    idx, _, rule = select_step_size(dts, ar, msj, ess, ess_floor_frac=0.0075)
    assert rule == "ess" and dts[idx] == 3e-4


def test_ar_spread_reduces_the_step():
    dts = [0.01, 0.03, 0.1, 0.3]
    ar = [0.9, 0.7, 0.5, 0.3]
    msj = [1, 2, 3, 4]
    ess = [0.1, 0.2, 0.3, 0.4]
    spread = [0.01, 0.02, 0.08, 0.2]       # chains disagree from dt = 0.1 on
    idx, _, rule = select_step_size(dts, ar, msj, ess, spread=spread)
    assert rule == "ar_spread" and dts[idx] == 0.03


def test_ar_spread_excludes_binomial_noise():
    rng = np.random.default_rng(0)
    steps = 100
    same = rng.binomial(steps, 0.3, size=4000) / steps          # every chain alike: only sampling noise
    assert ar_spread(same, steps) < 0.01
    mixed = np.concatenate([rng.binomial(steps, 0.1, size=2000), rng.binomial(steps, 0.5, size=2000)]) / steps
    assert abs(ar_spread(mixed, steps) - 0.2) < 0.01             # two groups 0.4 apart: sd 0.2
