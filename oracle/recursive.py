"""Recursive (Deriche) Gaussian smoothing and the shiftable filter built on
it -- TEST INFRASTRUCTURE ONLY, FP64, numpy.

Sec. 2 (after eq. (5)) notes that each Gaussian convolution of the shiftable
decomposition can run in time independent of sigma_s by separability and
recursion, citing Deriche (1993).  This module is the reference for that
variant of the spatial step:

* ``deriche_profile``: Deriche's fit of exp(-x^2 / 2) by two damped
  cosine/sine pairs, scaled to sigma (his published constants).
* ``deriche_kernel``: the two-sided sampled kernel h(n) = g(|n|) / sum_m g(|m|),
  its definition written out (the target of the recursion below).
* ``deriche_coefficients``: the causal and anti-causal recursions whose sum
  has impulse response h: the four poles of the damped pairs give the
  denominator, the partial fractions the numerator (derived here from the
  z-transform of the causal half, not copied from a table).
* ``recursive_smooth_1d`` / ``recursive_smooth``: the recursions run over a
  half-sample symmetric extension (the border the other oracles use), long
  enough that the truncated tail is below 1e-16 of the kernel's mass.
* ``convolve_smooth``: the same smoothing as a direct sum over h, for pins.
* ``fourier_recursive``: eq. (9)'s numerator and denominator with every
  spatial convolution replaced by the recursive smoothing (real cos/sin form,
  c_0 = d_0, c_{+-n} = d_n / 2 as after eq. (6)); the result therefore
  differs from the truncated-Gaussian parity path by the fit and truncation
  difference of the spatial kernels, not by the range approximation.

Pinned by tests/test_oracle_recursive.py: the fitted profile against
exp(-x^2 / 2) (the fit's own accuracy), the recursion against the direct sum
over h, unit DC gain, symmetry, the bilateral variant against eq. (1) by
brute force with the weights h (x) h, and its K = 0 limit.
"""
from __future__ import annotations

import math

import numpy as np

# Deriche's fit of exp(-x^2 / 2) for x >= 0 (sigma = 1):
#   g(x) = (a0 cos(w0 x) + a1 sin(w0 x)) e^{-b0 x} + (c0 cos(w1 x) + c1 sin(w1 x)) e^{-b1 x}
DERICHE_FIT = {"a0": 1.680, "a1": 3.735, "b0": 1.783, "w0": 0.6318,
               "c0": -0.6803, "c1": -0.2598, "b1": 1.723, "w1": 1.997}


def deriche_profile(x, sigma: float) -> np.ndarray:
    """Deriche's approximation of exp(-x^2 / (2 sigma^2)) for x >= 0."""
    p = DERICHE_FIT
    t = np.asarray(x, dtype=np.float64) / sigma
    return ((p["a0"] * np.cos(p["w0"] * t) + p["a1"] * np.sin(p["w0"] * t)) * np.exp(-p["b0"] * t)
            + (p["c0"] * np.cos(p["w1"] * t) + p["c1"] * np.sin(p["w1"] * t)) * np.exp(-p["b1"] * t))


def margin(sigma: float) -> int:
    """Samples beyond which the kernel's tail is below 1e-16 of its peak:
    the slowest decay is e^{-b1 n / sigma}."""
    return int(math.ceil(sigma * 16.0 * math.log(10.0) / DERICHE_FIT["b1"])) + 8


def deriche_kernel(sigma: float, M: int | None = None) -> np.ndarray:
    """h(n) for n = -M..M: the profile at |n|, normalised to unit sum over all
    integers (the sum over |n| > M is below the FP64 resolution)."""
    if M is None:
        M = margin(sigma)
    n = np.arange(-M, M + 1, dtype=np.float64)
    g = deriche_profile(np.abs(n), sigma)
    return g / g.sum()


def deriche_coefficients(sigma: float):
    """(n_causal[0..3], n_anti[1..4], d[1..4]) of the recursions

        y+(i) = sum_{k=0..3} n_causal[k] x(i - k) - sum_{k=1..4} d[k] y+(i - k)
        y-(i) = sum_{k=1..4} n_anti[k]  x(i + k) - sum_{k=1..4} d[k] y-(i + k)

    with y = y+ + y- having impulse response h of ``deriche_kernel``.

    The causal half g(n), n >= 0, is sum over the two pairs of
    Re[alpha p^n] with p = e^{(-b + i w) / sigma} and alpha = a - i a', so its
    z-transform is a sum of four one-pole terms; over the common denominator
    D(z^-1) = prod (1 - p z^-1) the numerator has degree 3.  The anti-causal
    half g(n), n >= 1, run backwards, has numerator N(z) - g(0) D(z).
    Both are scaled by one over the kernel's total sum, (N(1) + N(1) - g(0) D(1)) / D(1).
    """
    p = DERICHE_FIT
    pairs = [(p["a0"], p["a1"], p["b0"], p["w0"]), (p["c0"], p["c1"], p["b1"], p["w1"])]
    poles, residues = [], []
    for a_cos, a_sin, b, w in pairs:
        z = complex(math.exp(-b / sigma) * math.cos(w / sigma), math.exp(-b / sigma) * math.sin(w / sigma))
        alpha = complex(a_cos, -a_sin)
        poles += [z, z.conjugate()]
        residues += [alpha / 2, alpha.conjugate() / 2]
    # polynomials in z^-1, lowest power first
    D = np.array([1.0 + 0j])
    for z in poles:
        D = np.convolve(D, [1.0, -z])
    N = np.zeros(4, dtype=np.complex128)
    for j, (z, r) in enumerate(zip(poles, residues)):
        rest = np.array([1.0 + 0j])
        for m, z2 in enumerate(poles):
            if m != j:
                rest = np.convolve(rest, [1.0, -z2])
        N += r * rest
    D, N = D.real.copy(), N.real.copy()
    g0 = N[0]                      # g(0) = n_causal[0]
    anti = np.zeros(5)
    anti[1:4] = N[1:4] - g0 * D[1:4]
    anti[4] = -g0 * D[4]
    total = (N.sum() + anti.sum()) / D.sum()
    return N / total, anti / total, D


def recursive_smooth_1d(x: np.ndarray, sigma: float, axis: int = -1) -> np.ndarray:
    """The causal plus anti-causal recursions along ``axis`` over a half-sample
    symmetric extension of ``margin(sigma)`` samples each side, from zero
    state; the extension is then cut away.  Each recursion is one call of
    ``scipy.signal.lfilter`` (numerator over the denominator 1 + d1 z^-1 + ...
    + d4 z^-4); the anti-causal one runs on the reversed line."""
    from scipy.signal import lfilter
    nc, na, d = deriche_coefficients(sigma)
    M = margin(sigma)
    X = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    pad = [(0, 0)] * (X.ndim - 1) + [(M, M)]
    Xp = np.pad(X, pad, mode="symmetric")
    L = Xp.shape[-1]
    yp = lfilter(nc, d, Xp, axis=-1)
    ym = lfilter(na, d, Xp[..., ::-1], axis=-1)[..., ::-1]
    y = (yp + ym)[..., M:L - M]
    return np.moveaxis(y, -1, axis)


def recursive_smooth(X: np.ndarray, sigma: float) -> np.ndarray:
    """Separable 2-D recursive smoothing: along rows, then along columns."""
    return recursive_smooth_1d(recursive_smooth_1d(X, sigma, axis=1), sigma, axis=0)


def convolve_smooth(X: np.ndarray, sigma: float) -> np.ndarray:
    """The same 2-D smoothing as direct sums over h(n) h(m) with the same
    half-sample symmetric extension: the definition the recursion must meet."""
    M = margin(sigma)
    h = deriche_kernel(sigma, M)
    X = np.asarray(X, dtype=np.float64)
    H, Wd = X.shape
    Xp = np.pad(X, M, mode="symmetric")
    R = np.zeros((H + 2 * M, Wd))
    for t in range(-M, M + 1):
        R += h[t + M] * Xp[:, M - t:M - t + Wd]
    Y = np.zeros((H, Wd))
    for t in range(-M, M + 1):
        Y += h[t + M] * R[M - t:M - t + H, :]
    return Y


def fourier_recursive(f, sigma_s: float, d, T: int, smooth=None, with_pq: bool = False):
    """Eq. (9) in real form with recursive spatial smoothing:

        P = d_0 S(f) + sum_k d_k [cos(k w f) S(f cos(k w f)) + sin(k w f) S(f sin(k w f))]
        Q = d_0 S(1) + sum_k d_k [cos(k w f) S(cos(k w f))   + sin(k w f) S(sin(k w f))]

    with w = pi / T, S the 2-D smoothing (``recursive_smooth`` by default) and
    the output P / Q."""
    if smooth is None:
        def smooth(X):
            return recursive_smooth(X, sigma_s)
    f = np.asarray(f, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    omega = math.pi / T
    P = d[0] * smooth(f)
    Q = d[0] * smooth(np.ones_like(f))
    for k in range(1, len(d)):
        c, s = np.cos(k * omega * f), np.sin(k * omega * f)
        P += d[k] * (c * smooth(f * c) + s * smooth(f * s))
        Q += d[k] * (c * smooth(c) + s * smooth(s))
    out = P / Q
    return (out, P, Q) if with_pq else out
