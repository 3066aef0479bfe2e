"""The simulated-sensitivity experiment of Section 4.1.1 on a small scale:
planted duplications with error at most delta (split into substitutions and
gaps, each below min(0.15, delta)) are found by the seed filter and the
extension, one region covering more than 95% of both copies, and by the
final SDs of Section 3.3, one alignment covering more than 95% of both."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("delta", [0.02, 0.15, 0.30])
def test_sensitivity_small(delta):
    sys.path.insert(0, ROOT)
    import bench
    res = bench.sensitivity_trial_set(delta, 40, seed=7)
    print(res)
    assert res["found"] >= 36, res  # 40, 39 and 38 of 40 when last measured
    assert res["found_final_sd"] >= 36, res
