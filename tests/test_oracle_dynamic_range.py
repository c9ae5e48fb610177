"""The oracle's local dynamic range (the T of Sec. 3 measured on an image)
pinned to brute force, to scipy's maximum/minimum filters, and to closed
forms."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


@pytest.mark.parametrize("W", [1, 2, 3])
def test_matches_brute_force(W):
    rng = np.random.default_rng(W)
    for shape in [(5, 7), (8, 4), (6, 6)]:
        f = rng.integers(0, 50, size=shape).astype(np.float64)
        assert oracle.local_dynamic_range(f, W) == oracle.brute_local_dynamic_range(f.tolist(), W)


@pytest.mark.parametrize("W", [0, 1, 4, 9])
def test_equals_clipped_max_and_min_filters(W):
    """A folded neighbour is a pixel at most as far away as its offset, so T is
    the largest rise to the window maximum (or fall to the minimum) with the
    window clipped at the borders -- scipy's 'nearest' mode."""
    rng = np.random.default_rng(100 + W)
    f = rng.normal(100, 30, size=(23, 31))
    t = oracle.local_dynamic_range(f, W)
    up = (ndimage.maximum_filter(f, size=2 * W + 1, mode="nearest") - f).max()
    down = (f - ndimage.minimum_filter(f, size=2 * W + 1, mode="nearest")).max()
    assert abs(t - up) < 1e-12 and abs(t - down) < 1e-12


def test_closed_forms():
    H, Wd = 20, 30
    assert oracle.local_dynamic_range(np.full((H, Wd), 7.0), 3) == 0.0
    # a vertical step edge of height h
    f = np.zeros((H, Wd))
    f[:, 15:] = 37.0
    assert oracle.local_dynamic_range(f, 1) == 37.0
    assert oracle.local_dynamic_range(f, 5) == 37.0
    # a ramp of slope a along x: the range is a W (and is reached in the interior)
    x = np.arange(Wd, dtype=np.float64)
    f = np.tile(2.5 * x, (H, 1))
    for W in (1, 3, 7):
        assert oracle.local_dynamic_range(f, W) == pytest.approx(2.5 * W)
    # a diagonal ramp: the window corner gives a (W + W)
    y = np.arange(H, dtype=np.float64)[:, None]
    f = 1.5 * (y + x[None, :])
    assert oracle.local_dynamic_range(f, 4) == pytest.approx(1.5 * 8)
    # W = 0: no neighbours but the pixel itself
    assert oracle.local_dynamic_range(np.random.default_rng(0).normal(size=(5, 5)), 0) == 0.0


def test_border_fold_adds_nothing():
    """A bright pixel in a corner, W larger than its distance to the edge:
    only real neighbours contribute."""
    f = np.zeros((9, 9))
    f[0, 0] = 10.0
    f[8, 8] = 3.0
    assert oracle.local_dynamic_range(f, 2) == 10.0
    g = np.zeros((9, 9))
    g[4, 4] = 5.0
    assert oracle.local_dynamic_range(g, 1) == 5.0
