"""Host logic of the step-size rule (appendix on tuning): monotone down-selection of
candidates by AR and MSJ, then the largest median ESS% among those kept."""
import numpy as np

from paper_2403_08220_amd.tune import mean_square_jump, select_step_size


def test_selects_max_ess_within_monotone_prefix():
    dts = [0.01, 0.03, 0.1, 0.3, 1.0]
    ar = [0.9, 0.8, 0.6, 0.3, 0.35]       # AR rises again at 1.0: prefix ends at 0.3
    msj = [0.1, 0.2, 0.5, 0.7, 0.2]
    ess = [0.01, 0.02, 0.05, 0.04, 0.5]   # the large ESS at 1.0 lies outside the prefix
    idx, kept = select_step_size(dts, ar, msj, ess)
    assert kept == [0, 1, 2, 3] and dts[idx] == 0.1


def test_msj_break_ends_prefix_and_order_is_irrelevant():
    dts = [0.3, 0.01, 0.1, 0.03]
    ar = [0.3, 0.9, 0.6, 0.8]
    msj = [0.4, 0.1, 0.5, 0.2]            # MSJ falls from 0.1 to 0.3
    ess = [0.9, 0.01, 0.05, 0.02]
    idx, kept = select_step_size(dts, ar, msj, ess)
    assert sorted(dts[k] for k in kept) == [0.01, 0.03, 0.1] and dts[idx] == 0.1


def test_nan_ess_never_selected():
    idx, kept = select_step_size([1, 2], [0.5, 0.4], [1, 2], [0.1, float("nan")])
    assert idx == 0 and kept == [0, 1]


def test_mean_square_jump():
    t = np.zeros((3, 2, 2))
    t[1, 0] = [1, 0]
    t[2, 0] = [1, 2]
    # chain 0 jumps 1 then 4; chain 1 never moves
    assert mean_square_jump(t) == (1 + 4 + 0 + 0) / 4
