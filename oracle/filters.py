"""FP64 reference filters -- TEST INFRASTRUCTURE ONLY.

* ``direct``  / ``fourier``: ctypes front ends of bf_oracle.c (eq. (1) and
  eq. (9), one output pixel at a time, OpenMP over pixels).
* ``shiftable_alg1``: Algorithm 1 written with numpy in complex FP64, term by
  term for n = -K..K with c_0 = d_0 and c_{+-n} = d_n / 2 (the relation stated
  after eq. (6)); each term modulates, convolves (separable, half-sample
  symmetric border), demodulates with the conjugate and accumulates P and Q.
  By the decomposition of Sec. 2 it must agree with ``fourier``.
* ``brute_direct``: eq. (1) in pure Python loops over a symmetrically padded
  array, for tiny images only.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bf_oracle.c")
_LIB = os.path.join(_HERE, "_bf_oracle.so")
_lock = threading.Lock()
_lib = None

SPATIAL = {"gaussian": 0, "box": 1}
RANGE = {"gaussian": 0, "exponential": 1, "table": 2}


def build(force: bool = False) -> str:
    """Compile bf_oracle.c (gcc, -O2, OpenMP, strict IEEE double)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            dp = ctypes.POINTER(ctypes.c_double)
            fp = ctypes.POINTER(ctypes.c_float)
            lp = ctypes.POINTER(ctypes.c_long)
            L, I, D = ctypes.c_long, ctypes.c_int, ctypes.c_double
            lib.oracle_direct.argtypes = [fp, L, L, L, I, D, I, I, D, dp, I, lp, L, dp, dp, dp]
            lib.oracle_direct.restype = I
            lib.oracle_fourier.argtypes = [fp, L, L, L, I, D, I, dp, I, I, lp, L, dp, dp, dp]
            lib.oracle_fourier.restype = I
            lib.oracle_center_weight.argtypes = [I, D, I]
            lib.oracle_center_weight.restype = D
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = I
            lib.oracle_set_threads.argtypes = [I]
            lib.oracle_set_threads.restype = I
            _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> int:
    """Threads of later oracle calls (n >= 1); returns the previous count."""
    return int(_load().oracle_set_threads(int(n)))


def center_weight(spatial: str, sigma_s: float, W: int) -> float:
    """w(0) of the unit-sum spatial kernel on [-W, W]^2."""
    return float(_load().oracle_center_weight(SPATIAL[spatial], float(sigma_s), int(W)))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def _prep(f, pixels):
    f = np.ascontiguousarray(f, dtype=np.float32)
    if f.ndim != 2:
        raise ValueError("2-D image expected")
    H, Wd = f.shape
    if pixels is None:
        pix, n = None, H * Wd
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64).ravel()
        if pix.size and (pix.min() < 0 or pix.max() >= H * Wd):
            raise ValueError("pixel index out of range")
        n = pix.size
    return f, H, Wd, pix, n


def _finish(out, P, Q, H, Wd, pixels, with_pq):
    if pixels is None:
        out = out.reshape(H, Wd)
        if with_pq:
            P, Q = P.reshape(H, Wd), Q.reshape(H, Wd)
    return (out, P, Q) if with_pq else out


def direct(f, spatial: str, sigma_s: float, W: int, range_kind: str, sigma_r: float = 1.0,
           T: int = 255, table=None, pixels=None, with_pq: bool = False):
    """Eq. (1) in FP64 at every pixel (or at the linear indices ``pixels``)."""
    f, H, Wd, pix, n = _prep(f, pixels)
    tab = None if table is None else np.ascontiguousarray(table, dtype=np.float64)
    out = np.empty(n)
    P = np.empty(n) if with_pq else None
    Q = np.empty(n) if with_pq else None
    rc = _load().oracle_direct(_ptr(f, ctypes.c_float), H, Wd, Wd, SPATIAL[spatial], float(sigma_s),
                               int(W), RANGE[range_kind], float(sigma_r), _ptr(tab, ctypes.c_double),
                               int(T), _ptr(pix, ctypes.c_long), n, _ptr(out, ctypes.c_double),
                               _ptr(P, ctypes.c_double), _ptr(Q, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_direct rejected its arguments")
    return _finish(out, P, Q, H, Wd, pixels, with_pq)


def fourier(f, spatial: str, sigma_s: float, W: int, d, T: int, pixels=None, with_pq: bool = False):
    """Eq. (9) in FP64 with phi_K from the coefficients d_0..d_K."""
    f, H, Wd, pix, n = _prep(f, pixels)
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty(n)
    P = np.empty(n) if with_pq else None
    Q = np.empty(n) if with_pq else None
    rc = _load().oracle_fourier(_ptr(f, ctypes.c_float), H, Wd, Wd, SPATIAL[spatial], float(sigma_s),
                                int(W), _ptr(d, ctypes.c_double), len(d) - 1, int(T),
                                _ptr(pix, ctypes.c_long), n, _ptr(out, ctypes.c_double),
                                _ptr(P, ctypes.c_double), _ptr(Q, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_fourier rejected its arguments")
    return _finish(out, P, Q, H, Wd, pixels, with_pq)


# ---------------------------------------------------------------------------
# numpy forms


def spatial_profile(spatial: str, sigma_s: float, W: int) -> np.ndarray:
    """1-D profile on [-W, W] with unit sum; the 2-D kernel is its outer product."""
    x = np.arange(-W, W + 1, dtype=np.float64)
    w = np.ones_like(x) if spatial == "box" else np.exp(-x * x / (2.0 * sigma_s * sigma_s))
    return w / w.sum()


def _smooth_separable(X: np.ndarray, w1: np.ndarray) -> np.ndarray:
    """sum_j w(j) X(i - j) with w = w1 (x) w1 and half-sample symmetric borders."""
    W = (len(w1) - 1) // 2
    H, Wd = X.shape
    Xp = np.pad(X, ((0, 0), (W, W)), mode="symmetric")
    Y = np.zeros_like(X)
    for j in range(-W, W + 1):
        Y += w1[j + W] * Xp[:, W - j: W - j + Wd]
    Yp = np.pad(Y, ((W, W), (0, 0)), mode="symmetric")
    Z = np.zeros_like(X)
    for j in range(-W, W + 1):
        Z += w1[j + W] * Yp[W - j: W - j + H, :]
    return Z


def shiftable_alg1(f, spatial: str, sigma_s: float, W: int, d, T: int, with_pq: bool = False):
    """Algorithm 1 (complex form) in FP64, n = -K..K."""
    f = np.asarray(f, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    K = len(d) - 1
    omega = math.pi / T
    w1 = spatial_profile(spatial, sigma_s, W)
    P = np.zeros(f.shape, dtype=np.complex128)
    Q = np.zeros(f.shape, dtype=np.complex128)
    for n in range(-K, K + 1):
        c_n = d[0] if n == 0 else 0.5 * d[abs(n)]
        G = np.exp(1j * n * omega * f)
        F = G * f
        Hn = c_n * np.conj(G)
        Fbar = _smooth_separable(F, w1)
        Gbar = _smooth_separable(G, w1)
        P += Hn * Fbar
        Q += Hn * Gbar
    out = (P / Q).real
    return (out, P, Q) if with_pq else out


def brute_direct(f, spatial: str, sigma_s: float, W: int, phi) -> np.ndarray:
    """Eq. (1) with explicit loops; ``phi`` is a Python callable. Tiny inputs only."""
    f = np.asarray(f, dtype=np.float64)
    H, Wd = f.shape
    fp = np.pad(f, W, mode="symmetric")
    out = np.zeros((H, Wd))
    for r in range(H):
        for c in range(Wd):
            num = den = 0.0
            for jy in range(-W, W + 1):
                for jx in range(-W, W + 1):
                    if spatial == "box":
                        w = 1.0
                    else:
                        w = math.exp(-(jx * jx + jy * jy) / (2.0 * sigma_s * sigma_s))
                    v = fp[r - jy + W, c - jx + W]
                    k = w * phi(v - f[r, c])
                    num += k * v
                    den += k
            out[r, c] = num / den
    return out
