"""Progressive Fourier approximation of a range kernel (Sec. 3, Algorithm 2), FP64.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU baseline; the GPU library has its own, independent fit.

The kernel phi is sampled on Lambda_T = {0, 1, ..., T}; the basis columns are
cos(n w t), w = pi / T (eq. (6)); the coefficients d minimise
||b - A d||_2^2 (eq. (7)/(8)).  Columns are added one at a time and the thin
QR factorisation A = Q R is grown by one modified Gram-Schmidt step per new
column; d is obtained from R d = Q^T b by back-substitution, and the loop
stops as soon as E = ||b - A d||_2 <= eps.

Reading taken where the printed algorithm is off by one: with N columns the
harmonics are 0..N-1, i.e. the column added when the column count becomes N
is cos((N-1) w t).  (Taken literally the first added column would be
cos(2 w t) and cos(w t) would never enter.)  With this reading the column
counts printed in Tables 3 and 4 are reproduced; the highest harmonic is
K = N - 1, which is what the rest of this code base calls K.

An optional cap K_max stops the loop after the column of harmonic K_max even
if E > eps; eps == 0 therefore asks for exactly K_max harmonics.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def sample_kernel(kind: str, sigma: float, T: int, table=None) -> np.ndarray:
    """b = [phi(t)] for t in Lambda_T (Algorithm 2, the sampling step).

    gaussian: eq. (3), exp(-t^2 / (2 sigma^2)); exponential: exp(-|t| / sigma);
    table: the given samples phi(0..T)."""
    t = np.arange(T + 1, dtype=np.float64)
    if kind == "gaussian":
        return np.exp(-t * t / (2.0 * sigma * sigma))
    if kind == "exponential":
        return np.exp(-t / sigma)
    if kind == "table":
        b = np.asarray(table, dtype=np.float64)
        if b.shape != (T + 1,):
            raise ValueError("table must hold phi(0..T)")
        return b.copy()
    raise ValueError(kind)


@dataclass
class FitResult:
    K: int               # highest harmonic (number of columns minus one)
    d: np.ndarray        # d_0..d_K
    E: float             # ||b - A d||_2 at exit
    converged: bool      # E <= eps
    E_history: list      # E after each column count 1..K+1
    Q: np.ndarray        # (T+1) x (K+1), orthonormal columns
    R: np.ndarray        # (K+1) x (K+1), upper triangular
    A: np.ndarray        # (T+1) x (K+1), the basis matrix
    b: np.ndarray        # samples of phi


def back_substitute(R: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Solve R d = p for upper-triangular R, last unknown first."""
    n = R.shape[0]
    d = np.zeros(n)
    for i in range(n - 1, -1, -1):
        d[i] = (p[i] - R[i, i + 1:] @ d[i + 1:]) / R[i, i]
    return d


def progressive_fit(b: np.ndarray, T: int, eps: float, K_max: int | None = None) -> FitResult:
    """Algorithm 2 on the samples b = phi(0..T)."""
    if K_max is None:
        K_max = T
    if T < 1 or eps < 0 or K_max < 0 or K_max > T:
        raise ValueError("need T >= 1, eps >= 0, 0 <= K_max <= T")
    omega = math.pi / T
    t = np.arange(T + 1, dtype=np.float64)
    # initialisation: one column, the all-ones vector
    N = 1
    a = np.ones(T + 1)
    A = a[:, None].copy()
    R = np.array([[np.linalg.norm(a)]])
    Q = (a / R[0, 0])[:, None]
    p = Q.T @ b
    d = p / R[0, 0]
    E = float(np.linalg.norm(b - Q @ p))
    hist = [E]
    while E > eps and N - 1 < K_max:
        r = np.zeros(N)
        N += 1
        a = np.cos((N - 1) * omega * t)     # harmonic N-1 (see module docstring)
        A = np.hstack([A, a[:, None]])
        for k in range(N - 1):              # modified Gram-Schmidt against q_1..q_{N-1}
            q_k = Q[:, k]
            r[k] = a @ q_k
            a = a - r[k] * q_k
        r_N = np.linalg.norm(a)
        a = a / r_N
        Q = np.hstack([Q, a[:, None]])
        p = np.append(p, a @ b)
        R = np.vstack([R, np.zeros((1, N - 1))])              # add a row of zeros
        R = np.hstack([R, np.append(r, r_N)[:, None]])      # append the new column
        d = back_substitute(R, p)
        E = float(np.linalg.norm(b - A @ d))
        hist.append(E)
    return FitResult(K=N - 1, d=d, E=E, converged=E <= eps, E_history=hist, Q=Q, R=R, A=A, b=b)


def fit_kernel(kind: str, sigma: float, T: int, eps: float, K_max: int | None = None,
               table=None) -> FitResult:
    return progressive_fit(sample_kernel(kind, sigma, T, table), T, eps, K_max)


def series(d: np.ndarray, T: int, t) -> np.ndarray:
    """phi_K(t) = d_0 + sum_k d_k cos(k w t), eq. (6)."""
    t = np.asarray(t, dtype=np.float64)
    k = np.arange(len(d), dtype=np.float64)
    return np.cos(np.multiply.outer(t, k) * (math.pi / T)) @ d


def accuracy_bound(T: int, eps: float, w0: float) -> float:
    """Right-hand side of eq. (12): 2 T eps / (w(0) - eps)."""
    return 2.0 * T * eps / (w0 - eps)
