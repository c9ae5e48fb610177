"""Local dynamic range of an image (test infrastructure; see oracle/__init__).

The dynamic range T of Sec. 3 bounds the argument of the range kernel in
eq. (1): T = max over pixels i and offsets j in [-W, W]^2 of
|f(i - j) - f(i)|, where f(i - j) is taken with the half-sample symmetric
border that the filter uses.  Written here straight from that definition,
in FP64.
"""
from __future__ import annotations

import numpy as np


def fold(i: np.ndarray, n: int) -> np.ndarray:
    """Half-sample symmetric index: -1 -> 0, -2 -> 1, n -> n - 1, ..."""
    i = np.asarray(i)
    i = np.where(i < 0, -1 - i, i)
    return np.where(i >= n, 2 * n - 1 - i, i)


def local_dynamic_range(f, W: int) -> float:
    """max_i max_{j in [-W, W]^2} |f(fold(i - j)) - f(i)| in FP64."""
    f = np.asarray(f, dtype=np.float64)
    H, Wd = f.shape
    if W >= H or W >= Wd:
        raise ValueError("W must be smaller than both image sides (symmetric border)")
    ys = np.arange(H)
    xs = np.arange(Wd)
    best = 0.0
    for dy in range(-W, W + 1):
        rows = fold(ys - dy, H)
        for dx in range(-W, W + 1):
            cols = fold(xs - dx, Wd)
            best = max(best, float(np.abs(f[np.ix_(rows, cols)] - f).max()))
    return best


def brute_local_dynamic_range(f, W: int) -> float:
    """The same in pure Python loops, for tiny images."""
    H, Wd = len(f), len(f[0])

    def fo(i, n):
        if i < 0:
            i = -1 - i
        if i >= n:
            i = 2 * n - 1 - i
        return i

    best = 0.0
    for y in range(H):
        for x in range(Wd):
            for dy in range(-W, W + 1):
                for dx in range(-W, W + 1):
                    d = abs(float(f[fo(y - dy, H)][fo(x - dx, Wd)]) - float(f[y][x]))
                    best = max(best, d)
    return best
