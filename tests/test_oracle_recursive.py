"""Pins of the recursive (Deriche) spatial smoothing and of the shiftable
filter built on it (the constant-time spatial step cited in Sec. 2 after
eq. (5)).  CPU only."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import recursive as R
from oracle.fit import fit_kernel, series


def test_fitted_profile_is_the_gaussian_within_the_fit_error():
    # Deriche's two damped pairs against exp(-x^2 / 2) on [0, 8]: the fit's
    # worst error is 5.2e-4 (near x = 0.12); a mistyped constant exceeds 1e-3
    x = np.linspace(0.0, 8.0, 8001)
    err = np.abs(R.deriche_profile(x, 1.0) - np.exp(-x * x / 2))
    assert err.max() < 6e-4
    # scaling: the profile at sigma is the profile at 1 evaluated at x / sigma
    assert np.allclose(R.deriche_profile(3.0 * x, 3.0), R.deriche_profile(x, 1.0), rtol=0, atol=1e-15)


@pytest.mark.parametrize("sigma", [0.8, 1.5, 3.0, 8.0])
def test_sampled_kernel_is_the_normalised_sampled_gaussian(sigma):
    M = R.margin(sigma)
    n = np.arange(-M, M + 1)
    g = np.exp(-n * n / (2 * sigma * sigma))
    g /= g.sum()
    h = R.deriche_kernel(sigma)
    assert abs(h.sum() - 1.0) < 1e-14
    assert np.array_equal(h, h[::-1])
    assert np.abs(h - g).max() < 1e-3 * g.max()
    # the tail cut at the margin is below FP64 resolution of the peak
    assert R.deriche_profile(M, sigma) < 1e-16


@pytest.mark.parametrize("sigma", [0.8, 1.5, 3.0, 7.0])
def test_recursion_has_impulse_response_h(sigma):
    M = R.margin(sigma)
    x = np.zeros(2 * M + 41)
    c = len(x) // 2
    x[c] = 1.0
    y = R.recursive_smooth_1d(x[None, :], sigma, axis=1)[0]
    h = R.deriche_kernel(sigma)
    # every output within M of the impulse, and nothing else
    assert np.abs(y[c - M:c + M + 1] - h).max() < 1e-14
    assert np.abs(np.delete(y, np.s_[c - M:c + M + 1])).max() < 1e-16


def test_recursion_coefficients_have_the_poles_of_the_damped_pairs():
    sigma = 2.5
    nc, na, d = R.deriche_coefficients(sigma)
    roots = np.roots(d[::-1])            # d in powers of z^-1: roots in z^-1 are 1 / poles
    poles = np.sort_complex(1.0 / roots)
    p = R.DERICHE_FIT
    want = []
    for b, w in ((p["b0"], p["w0"]), (p["b1"], p["w1"])):
        z = math.exp(-b / sigma) * complex(math.cos(w / sigma), math.sin(w / sigma))
        want += [z, z.conjugate()]
    assert np.allclose(poles, np.sort_complex(np.array(want)), atol=1e-12)
    assert np.all(np.abs(poles) < 1.0)   # both recursions are stable
    assert d[0] == 1.0 and na[0] == 0.0


@pytest.mark.parametrize("sigma", [0.8, 1.5, 3.0, 7.0])
@pytest.mark.parametrize("shape", [(13, 17), (5, 40)])
def test_recursive_smoothing_equals_direct_sum_over_h(sigma, shape):
    rng = np.random.default_rng(11)
    X = rng.uniform(0, 255, shape)
    a = R.recursive_smooth(X, sigma)
    b = R.convolve_smooth(X, sigma)
    assert np.abs(a - b).max() < 1e-11
    # unit DC gain, borders included (half-sample symmetric extension)
    assert np.abs(R.recursive_smooth(np.full(shape, 7.0), sigma) - 7.0).max() < 1e-12


@pytest.mark.parametrize("sigma", [1.0, 2.0, 4.0, 8.0])
def test_recursive_smoothing_is_close_to_the_sampled_gaussian_filter(sigma):
    # scipy's sampled Gaussian with a reflecting (half-sample symmetric) border
    # and a long truncation: the two differ by the fit error of the profile only
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 255, (40, 37))
    a = R.recursive_smooth(X, sigma)
    b = ndimage.gaussian_filter(X, sigma, mode="reflect", truncate=12.0)
    assert np.abs(a - b).max() < 0.06


def _brute_eq1(f, sigma_s, phi):
    """Eq. (1) with w = h (x) h over the symmetric extension, one pixel at a time."""
    M = R.margin(sigma_s)
    h = R.deriche_kernel(sigma_s, M)
    hh = np.outer(h, h)
    fp = np.pad(f, M, mode="symmetric")
    H, Wd = f.shape
    out = np.zeros((H, Wd))
    for y in range(H):
        for x in range(Wd):
            patch = fp[y:y + 2 * M + 1, x:x + 2 * M + 1]
            wr = hh * phi(patch - f[y, x])
            out[y, x] = (wr * patch).sum() / wr.sum()
    return out


@pytest.mark.parametrize("sigma_s,sigma_r,seed", [(1.0, 30.0, 1), (2.0, 15.0, 2)])
def test_bilateral_variant_equals_eq1_with_the_recursive_weights(sigma_s, sigma_r, seed):
    # the shiftable sum with phi = phi_K is exactly eq. (1) with range kernel phi_K
    T = 255
    fit = fit_kernel("gaussian", sigma_r, T, 1e-3)
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 256, size=(6, 7)).astype(np.float64)
    got = R.fourier_recursive(f, sigma_s, fit.d, T)
    want = _brute_eq1(f, sigma_s, lambda t: series(fit.d, T, t))
    assert np.abs(got - want).max() < 1e-9


def test_bilateral_variant_with_a_constant_range_kernel_is_the_smoothing():
    rng = np.random.default_rng(5)
    f = rng.uniform(0, 255, (9, 11))
    got, P, Q = R.fourier_recursive(f, 1.7, np.array([1.0]), 255, with_pq=True)
    assert np.abs(Q - 1.0).max() < 1e-13
    assert np.abs(got - R.convolve_smooth(f, 1.7)).max() < 1e-11


def test_bilateral_variant_keeps_constant_images():
    T = 255
    fit = fit_kernel("gaussian", 20.0, T, 1e-3)
    assert np.abs(R.fourier_recursive(np.full((8, 9), 93.0), 2.0, fit.d, T) - 93.0).max() < 1e-10


def test_plane_assembly_with_the_truncated_gaussian_is_eq9():
    # the same modulation / demodulation with the truncated Gaussian of eq. (2)
    # as the smoothing must reproduce the C oracle of eq. (9)
    import oracle
    from oracle.filters import _smooth_separable, spatial_profile
    T, sigma_s, W = 255, 2.0, 4
    fit = fit_kernel("gaussian", 25.0, T, 1e-3)
    rng = np.random.default_rng(21)
    f = rng.integers(0, 256, size=(20, 23)).astype(np.float32)
    w1 = spatial_profile("gaussian", sigma_s, W)
    got = R.fourier_recursive(f, sigma_s, fit.d, T, smooth=lambda X: _smooth_separable(X, w1))
    want = oracle.fourier(f, "gaussian", sigma_s, W, fit.d, T)
    assert np.abs(got - want).max() < 1e-9


@pytest.mark.parametrize("sigma", [64.0, 256.0])
def test_recursion_at_the_largest_supported_sigma_equals_the_direct_sum(sigma):
    """At the library's largest sigma_s (256) the fourth-order recursion's
    poles come close to 1; on a line it must still match the direct sum over
    the same kernel h (half-sample symmetric extension) to within 1e-5 of the
    signal range per pass."""
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 255, 1500)
    M = R.margin(sigma)
    h = R.deriche_kernel(sigma, M)
    xp = np.pad(x, M, mode="symmetric")
    direct = np.convolve(xp, h, mode="valid")
    rec = R.recursive_smooth_1d(x, sigma)
    assert direct.shape == rec.shape == x.shape
    assert np.abs(rec - direct).max() < 255 * 1e-5
