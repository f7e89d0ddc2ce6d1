"""Pins of the oracle's training-time ray cap (oracle/tiles.py, lidar_training_dropped; App. A:
a tile holding more than 256 lidar rays renders a random 256 of them during training): a worked
example, the kept count per tile, priorities on either side of the cut, ties by ray index, and
rays outside every tile."""
import numpy as np

from oracle import tiles as ot


def test_worked_example():
    # tiles (az, el) of 7 rays on a 2 x 1 grid; cap 2
    az = np.array([0, 0, 0, 1, 0, 1, 1])
    el = np.zeros(7, int)
    pr = np.array([5, 1, 3, 9, 3, 0, 0])
    d = ot.lidar_training_dropped(az, el, np.ones(7, bool), pr, 2, cap=2)
    # tile 0 holds rays 0, 1, 2, 4 with priorities 5, 1, 3, 3: keeps 1 and 2 (3 ties with 4, 2 < 4)
    # tile 1 holds rays 3, 5, 6 with priorities 9, 0, 0: keeps 5 and 6
    np.testing.assert_array_equal(d, [True, False, False, True, True, False, False])


def test_counts_and_cut():
    rng = np.random.default_rng(1)
    R, n_az = 20000, 16
    az, el = rng.integers(0, n_az, R), rng.integers(0, 3, R)
    valid = rng.uniform(size=R) > 0.02
    pr = rng.integers(0, 1 << 16, R).astype(np.uint16)
    d = ot.lidar_training_dropped(az, el, valid, pr, n_az)
    assert not d[~valid].any()
    tile = el * n_az + az
    for t in np.unique(tile[valid]):
        m = valid & (tile == t)
        kept = m & ~d
        assert kept.sum() == min(m.sum(), 256)
        if d[m].any():
            assert pr[kept].max() <= pr[m & d].min()


def test_small_tiles_keep_everything_and_ties_go_by_index():
    az = np.repeat(np.arange(4), 300)[:1000]
    el = np.zeros(1000, int)
    pr = np.zeros(1000, np.uint16)
    d = ot.lidar_training_dropped(az, el, np.ones(1000, bool), pr, 4)
    for t in range(4):
        idx = np.nonzero(az == t)[0]
        kept = idx[~d[idx]]
        np.testing.assert_array_equal(kept, idx[:256])   # equal priorities: the first 256 by index
    assert not d[az == 3].any()                          # 100 rays: all kept
