"""Pins of the FP64 filters: eq. (1) against a pure-Python brute force and
textbook special cases, eq. (9) against Algorithm 1 in complex form, the
exact full-order case and the bound of eq. (12)."""
import math
import zlib

import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import polygon_image


def _rand_int_image(h, w, seed, hi=255):
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi + 1, size=(h, w)).astype(np.float32)


def _phi(kind, s, table=None):
    if kind == "gaussian":
        return lambda t: math.exp(-t * t / (2 * s * s))
    if kind == "exponential":
        return lambda t: math.exp(-abs(t) / s)
    return lambda t: table[min(int(round(abs(t))), len(table) - 1)]


@pytest.mark.parametrize("shape,W", [((5, 7), 1), ((5, 7), 4), ((8, 6), 2), ((9, 9), 3)])
@pytest.mark.parametrize("spatial", ["gaussian", "box"])
@pytest.mark.parametrize("rk", ["gaussian", "exponential", "table"])
def test_direct_matches_brute_force(shape, W, spatial, rk):
    f = _rand_int_image(*shape, seed=zlib.crc32(repr((shape, W, spatial, rk)).encode()) % 1000, hi=40)
    T = 40
    table = np.exp(-np.arange(T + 1) / 9.0) * (1 + 0.1 * np.cos(np.arange(T + 1)))
    sr = 12.0
    got = oracle.direct(f, spatial, 1.3, W, rk, sr, T=T, table=table)
    ref = oracle.brute_direct(f, spatial, 1.3, W, _phi(rk, sr, table))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_constant_image_unchanged():
    f = np.full((20, 23), 77.0, dtype=np.float32)
    r = oracle.fit_kernel("gaussian", 20.0, 255, 1e-3)
    for spatial in ("gaussian", "box"):
        np.testing.assert_allclose(oracle.direct(f, spatial, 2.0, 6, "gaussian", 20.0), 77.0, atol=1e-12)
        np.testing.assert_allclose(oracle.fourier(f, spatial, 2.0, 6, r.d, 255), 77.0, atol=1e-10)


def test_wide_range_kernel_is_plain_spatial_filter():
    """sigma_r -> infinity: phi == 1 and eq. (1) is the (unit-sum) spatial
    filter with symmetric borders, i.e. scipy's gaussian / uniform filters
    in 'reflect' mode."""
    f = polygon_image(40, 53, 7)
    for sigma_s, W in ((2.0, 6), (1.5, 4)):
        got = oracle.direct(f, "gaussian", sigma_s, W, "gaussian", 1e12)
        ref = ndimage.gaussian_filter(f.astype(np.float64), sigma_s, mode="reflect", truncate=W / sigma_s)
        np.testing.assert_allclose(got, ref, atol=1e-9)
    got = oracle.direct(f, "box", 0.0, 5, "gaussian", 1e12)
    ref = ndimage.uniform_filter(f.astype(np.float64), size=11, mode="reflect")
    np.testing.assert_allclose(got, ref, atol=1e-9)


def test_narrow_range_kernel_is_identity():
    """sigma_r -> 0 on integer images: only the centre pixel's own value
    (and equal neighbours) get weight, so the output is the input."""
    f = polygon_image(31, 29, 3)
    np.testing.assert_allclose(oracle.direct(f, "gaussian", 3.0, 9, "gaussian", 1e-3), f, rtol=0, atol=1e-9)


def test_output_is_convex_combination():
    """Each output lies between the min and max of its window (Appendix)."""
    f = polygon_image(37, 41, 11)
    W = 4
    out = oracle.direct(f, "gaussian", 1.5, W, "exponential", 15.0)
    fp = np.pad(f.astype(np.float64), W, mode="symmetric")
    win = np.lib.stride_tricks.sliding_window_view(fp, (2 * W + 1, 2 * W + 1))
    assert np.all(out >= win.min(axis=(2, 3)) - 1e-9)
    assert np.all(out <= win.max(axis=(2, 3)) + 1e-9)


def test_equivariances():
    """Transpose, flips and adding a constant commute with eq. (1)."""
    f = polygon_image(24, 30, 5)
    args = ("gaussian", 2.0, 5, "gaussian", 25.0)
    out = oracle.direct(f, *args)
    np.testing.assert_allclose(oracle.direct(f.T.copy(), *args), out.T, atol=1e-10)
    np.testing.assert_allclose(oracle.direct(f[::-1].copy(), *args), out[::-1], atol=1e-10)
    np.testing.assert_allclose(oracle.direct(f[:, ::-1].copy(), *args), out[:, ::-1], atol=1e-10)
    np.testing.assert_allclose(oracle.direct(f + 13.0, *args), out + 13.0, atol=1e-9)


@pytest.mark.parametrize("spatial,sigma_s,W", [("gaussian", 3.0, 9), ("box", 0.0, 4), ("gaussian", 1.2, 3)])
@pytest.mark.parametrize("rk,sr,eps", [("gaussian", 30.0, 1e-2), ("exponential", 20.0, 1e-1),
                                       ("gaussian", 10.0, 1e-4)])
def test_fourier_equals_algorithm1(spatial, sigma_s, W, rk, sr, eps):
    """Sec. 2 decomposition: eq. (9) summed directly (table of phi_K) equals
    Algorithm 1 (modulate / convolve / demodulate over n = -K..K)."""
    f = polygon_image(26, 33, 17)
    r = oracle.fit_kernel(rk, sr, 255, eps, K_max=40)
    a, Pa, Qa = oracle.fourier(f, spatial, sigma_s, W, r.d, 255, with_pq=True)
    b, Pb, Qb = oracle.shiftable_alg1(f, spatial, sigma_s, W, r.d, 255, with_pq=True)
    np.testing.assert_allclose(a, b, atol=1e-8)
    np.testing.assert_allclose(Pa, Pb.real, atol=1e-9 * np.abs(Pa).max())
    np.testing.assert_allclose(Qa, Qb.real, atol=1e-11)
    assert np.abs(Qb.imag).max() < 1e-12


def test_fourier_non_integer_image():
    """Non-integer gray levels take the summed-series branch of eq. (9)."""
    rng = np.random.default_rng(4)
    f = (rng.uniform(0, 255, size=(15, 17))).astype(np.float32)
    r = oracle.fit_kernel("gaussian", 25.0, 255, 1e-3)
    np.testing.assert_allclose(oracle.fourier(f, "gaussian", 2.0, 4, r.d, 255),
                               oracle.shiftable_alg1(f, "gaussian", 2.0, 4, r.d, 255), atol=1e-8)


def test_full_order_equals_direct():
    """K = T: the fit is exact on Lambda_T, so eq. (9) equals eq. (1) on
    integer images."""
    f = polygon_image(20, 22, 9)
    for rk, sr in (("gaussian", 10.0), ("exponential", 20.0)):
        r = oracle.fit_kernel(rk, sr, 255, 0.0, K_max=255)
        np.testing.assert_allclose(oracle.fourier(f, "gaussian", 2.0, 6, r.d, 255),
                                   oracle.direct(f, "gaussian", 2.0, 6, rk, sr), atol=1e-9)


@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-5])
def test_accuracy_bound_and_appendix_inequalities(eps):
    """Eq. (12) with eps the pointwise kernel error of eq. (10), and the
    Appendix steps Q_1 >= w(0), |Q_2| >= w(0) - eps, |P_1 - P_2| <= T eps."""
    T = 255
    f = polygon_image(48, 40, 21)
    sigma_s, W = 3.0, 9
    r = oracle.fit_kernel("gaussian", 30.0, T, eps)
    e_pt = np.abs(oracle.series(r.d, T, np.arange(T + 1)) - r.b).max()
    assert e_pt <= eps
    w0 = oracle.center_weight("gaussian", sigma_s, W)
    o1, P1, Q1 = oracle.direct(f, "gaussian", sigma_s, W, "gaussian", 30.0, with_pq=True)
    o2, P2, Q2 = oracle.fourier(f, "gaussian", sigma_s, W, r.d, T, with_pq=True)
    assert Q1.min() >= w0 - 1e-15
    assert np.abs(Q2).min() >= w0 - e_pt - 1e-15
    assert np.abs(Q1 - Q2).max() <= e_pt + 1e-15
    assert np.abs(P1 - P2).max() <= T * e_pt + 1e-12
    assert np.abs(o1 - o2).max() <= oracle.accuracy_bound(T, e_pt, w0)


def test_pixel_subset_matches_full():
    f = polygon_image(30, 35, 2)
    r = oracle.fit_kernel("gaussian", 20.0, 255, 1e-3)
    full = oracle.fourier(f, "box", 0.0, 5, r.d, 255)
    idx = np.array([0, 1, 34, 35, 500, 30 * 35 - 1])
    np.testing.assert_array_equal(oracle.fourier(f, "box", 0.0, 5, r.d, 255, pixels=idx), full.ravel()[idx])


def test_rejects_window_not_smaller_than_image():
    f = np.zeros((8, 10), dtype=np.float32)
    with pytest.raises(ValueError):
        oracle.direct(f, "gaussian", 3.0, 8, "gaussian", 10.0)
