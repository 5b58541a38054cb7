"""Host logic of the learned correction's training script (no GPU): the
choice of the fallback's trust bound from validation errors."""
import math

import pytest

from paper_2303_11767_amd.train_learned import pick_kappa


def test_pick_kappa_prefers_the_tightest_near_best_bound():
    # the validation errors measured for the stored model (metres)
    errs = {1.0: 0.246, 2.0: 0.0477, 4.0: 0.0327, 8.0: 0.0311, 16.0: 0.0310, 1e30: 0.0310}
    assert pick_kappa(errs) == 8.0
    assert pick_kappa(errs, tol=0.10) == 4.0
    assert pick_kappa(errs, tol=0.0) == 16.0


def test_pick_kappa_ignores_nonfinite_and_rejects_all_nonfinite():
    assert pick_kappa({1.0: math.nan, 2.0: 0.5, 4.0: math.inf}) == 2.0
    with pytest.raises(ValueError):
        pick_kappa({1.0: math.nan, 2.0: math.inf})
