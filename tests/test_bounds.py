"""Bounds the GPU chaining relies on to skip work without changing results
(Section 3.3 readings; CPU only).

Tier 2 skips a block of earlier chains when its best score does not exceed
the least cost of a link from the block's last end: min(d, 10 + ceil(d/10))
for a distance d from that end to the start of the chain being scored.  The
cost of a link with gaps dx, dy after a cut o is min(dx, dy) + (10 +
ceil(|dx - dy| / 10) when dx != dy) + o, and its dx is at least d.  Checked
here by enumeration: the bound grows with d and never exceeds a cost."""
import numpy as np


def least_cost(d):
    return np.minimum(d, 10 + (d + 9) // 10)


def link_cost(dx, dy, o):
    g = np.abs(dx - dy)
    return np.minimum(dx, dy) + np.where(g > 0, 10 + (g + 9) // 10, 0) + o


def test_least_cost_grows_with_distance():
    d = np.arange(0, 20001)
    lc = least_cost(d)
    assert np.all(np.diff(lc) >= 0)
    assert lc[0] == 0 and lc[11] == 11 and lc[12] == 12 and lc[20] == 12 and lc[10000] == 1010


def test_least_cost_bounds_every_link():
    dx, dy = np.meshgrid(np.arange(0, 601), np.arange(0, 601), indexing="ij")
    for o in range(0, 4):
        cost = link_cost(dx, dy, o)
        # any distance d <= dx: the bound at d is at most the bound at dx
        assert np.all(least_cost(dx) <= cost)
        # and it is reached (o = 0): by dy = dx, or by dy = 0
        if o == 0:
            assert np.array_equal(least_cost(dx[:, 0]), cost.min(axis=1))
