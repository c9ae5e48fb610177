"""ctypes binding of libbf.so (include/bf.h), names as in the C ABI.

This layer only marshals arguments: torch tensors provide device memory and
streams, every step of the filter runs in the library's HIP kernels.  If the
library is missing the import fails; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbf.so")

BF_OK = 0
BF_FIT_NOT_CONVERGED = 1
BF_E_INVALID = -1
BF_E_DEVICE = -2
BF_E_WORKSPACE = -4
BF_E_UNSUPPORTED = -5
BF_MAX_T = 1024
BF_MAX_K = 255
BF_MAX_W = 64
BF_NOALLOC_SCRATCH_BYTES = 4 << 20

RANGE = {"gaussian": 0, "exponential": 1, "table": 2}
SPATIAL = {"gaussian": 0, "box": 1}
PLANES = {"fp32": 0, "fp16": 1, "bf16": 2}
BF_FLAG_INTEGER_INPUT = 1
BF_FLAG_OFFSETS16 = 2


class BfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libbf error %d: %s" % (code, msg))
        self.code = code


class bf_job(ctypes.Structure):
    _fields_ = [
        ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
        ("height", ctypes.c_int), ("width", ctypes.c_int),
        ("src_pitch", ctypes.c_int), ("dst_pitch", ctypes.c_int),
        ("spatial", ctypes.c_int), ("sigma_s", ctypes.c_double), ("W", ctypes.c_int),
        ("range", ctypes.c_int), ("sigma_r", ctypes.c_double),
        ("phi_table", ctypes.POINTER(ctypes.c_double)),
        ("T", ctypes.c_int), ("eps", ctypes.c_double), ("K_max", ctypes.c_int),
        ("d", ctypes.POINTER(ctypes.c_double)), ("K", ctypes.c_int),
        ("flags", ctypes.c_int), ("f_max", ctypes.c_int),
    ]


def _hip_runtimes():
    """Distinct HIP / HSA runtime files mapped into this process."""
    try:
        with open("/proc/self/maps") as fh:
            paths = {ln.split()[-1] for ln in fh if "libamdhip64" in ln or "libhsa-runtime64" in ln}
    except OSError:
        return set()
    return paths


def _load():
    # torch's wheel ships its own HIP runtime (same soname as /opt/rocm's).
    # Importing torch first makes libbf bind to that copy, so the process
    # holds one HIP runtime and torch's streams and pointers are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbf.so is not built (run `python -m paper_1603_08081_amd.build`); "
                          "there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    D, I, Z, P = ctypes.c_double, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    jp = ctypes.POINTER(bf_job)
    lib.bf_fit_coeffs.argtypes = [I, D, dp, I, D, I, dp, ip, dp, dp]
    lib.bf_fit_coeffs.restype = I
    lib.bf_workspace_bytes.argtypes = [jp, I, I]
    lib.bf_workspace_bytes.restype = Z
    lib.bf_filter.argtypes = [jp, I, P, Z, P]
    lib.bf_filter.restype = I
    lib.bf_filter_batched.argtypes = [jp, I, I, P, Z, P]
    lib.bf_filter_batched.restype = I
    lib.bf_filter_batched_noalloc.argtypes = [jp, I, I, P]
    lib.bf_filter_batched_noalloc.restype = I
    lib.bf_plan_create.argtypes = [jp, I, I, ctypes.POINTER(P)]
    lib.bf_plan_create.restype = I
    lib.bf_plan_workspace_bytes.argtypes = [P]
    lib.bf_plan_workspace_bytes.restype = Z
    lib.bf_plan_upload.argtypes = [P, P, Z, P]
    lib.bf_plan_upload.restype = I
    lib.bf_plan_launch.argtypes = [P, P, I]
    lib.bf_plan_launch.restype = I
    lib.bf_plan_tune.argtypes = [P, P, I]
    lib.bf_plan_tune.restype = I
    lib.bf_plan_describe.argtypes = [P, ctypes.c_char_p, Z]
    lib.bf_plan_describe.restype = I
    lib.bf_tune_save.argtypes = [ctypes.c_char_p]
    lib.bf_tune_save.restype = I
    lib.bf_tune_load.argtypes = [ctypes.c_char_p]
    lib.bf_tune_load.restype = I
    lib.bf_tune_clear.argtypes = []
    lib.bf_tune_clear.restype = None
    lib.bf_plan_destroy.argtypes = [P]
    lib.bf_plan_destroy.restype = None
    lib.bf_dynamic_range_workspace_bytes.argtypes = [I, I]
    lib.bf_dynamic_range_workspace_bytes.restype = Z
    lib.bf_dynamic_range.argtypes = [P, I, I, I, I, P, P, Z, P]
    lib.bf_dynamic_range.restype = I
    lib.bf_recursive_workspace_bytes.argtypes = [jp]
    lib.bf_recursive_workspace_bytes.restype = Z
    lib.bf_filter_recursive.argtypes = [jp, P, Z, P]
    lib.bf_filter_recursive.restype = I
    lib.bf_last_error.argtypes = []
    lib.bf_last_error.restype = ctypes.c_char_p
    hip = sorted(p for p in _hip_runtimes() if "libamdhip64" in p)
    if len(hip) > 1:
        raise ImportError("two HIP runtimes are loaded (%s); import torch before anything that "
                          "loads /opt/rocm's libamdhip64" % ", ".join(hip))
    return lib


lib = _load()


def bf_last_error() -> str:
    return lib.bf_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise BfError(rc, bf_last_error())
    return rc


def bf_fit_coeffs(kind: str, sigma_r: float, T: int, eps: float, K_max: int, phi_table=None):
    """Algorithm 2 on the host.  Returns (status, d[0..K], err_l2, err_max)."""
    tab = None
    if phi_table is not None:
        tab = np.ascontiguousarray(phi_table, dtype=np.float64)
    d = np.zeros(max(K_max, 0) + 1, dtype=np.float64)
    K = ctypes.c_int(-1)
    e2 = ctypes.c_double(0.0)
    em = ctypes.c_double(0.0)
    rc = lib.bf_fit_coeffs(RANGE[kind], float(sigma_r),
                           tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if tab is not None else None,
                           int(T), float(eps), int(K_max), d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           ctypes.byref(K), ctypes.byref(e2), ctypes.byref(em))
    _check(rc)
    return rc, d[:K.value + 1].copy(), e2.value, em.value


class Job:
    """Python-side holder of one bf_job (keeps host arrays alive)."""

    def __init__(self, src, dst, *, spatial="gaussian", sigma_s=1.0, W=-1, range_kind="gaussian",
                 sigma_r=30.0, T=255, eps=1e-2, K_max=None, d=None, phi_table=None,
                 integer_input=False, f_max=0, height=None, width=None, src_pitch=None, dst_pitch=None,
                 offsets16=False):
        self._keep = []
        s = bf_job()
        s.src = _ptr(src)
        s.dst = _ptr(dst)
        h, w = _hw(src) if height is None else (height, width)
        s.height, s.width = int(h), int(w)
        s.src_pitch = int(src_pitch if src_pitch is not None else _pitch(src, w))
        s.dst_pitch = int(dst_pitch if dst_pitch is not None else _pitch(dst, w))
        s.spatial = SPATIAL[spatial]
        s.sigma_s = float(sigma_s)
        s.W = int(W)
        s.range = RANGE[range_kind]
        s.sigma_r = float(sigma_r)
        if phi_table is not None:
            tab = np.ascontiguousarray(phi_table, dtype=np.float64)
            self._keep.append(tab)
            s.phi_table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.T = int(T)
        s.eps = float(eps)
        s.K_max = int(T if K_max is None else K_max)
        if d is not None:
            dd = np.ascontiguousarray(d, dtype=np.float64)
            self._keep.append(dd)
            s.d = dd.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            s.K = len(dd) - 1
        s.flags = (BF_FLAG_INTEGER_INPUT if integer_input else 0) | (BF_FLAG_OFFSETS16 if offsets16 else 0)
        s.f_max = int(f_max)
        self.struct = s


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _hw(t):
    return int(t.shape[-2]), int(t.shape[-1])


def _pitch(t, w):
    if t is None or isinstance(t, int):
        return w
    return int(t.stride(-2))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def bf_workspace_bytes(jobs: Sequence[Job], prec: str = "fp32") -> int:
    arr = (bf_job * len(jobs))(*[j.struct for j in jobs])
    n = lib.bf_workspace_bytes(arr, len(jobs), PLANES[prec])
    if n == ctypes.c_size_t(-1).value:
        raise BfError(BF_E_INVALID, bf_last_error())
    return int(n)


def bf_filter(job: Job, prec: str = "fp32", workspace=None, ws_bytes: int = 0, stream=None) -> int:
    return _check(lib.bf_filter(ctypes.byref(job.struct), PLANES[prec], _ptr(workspace), int(ws_bytes),
                                _stream_handle(stream)))


def bf_filter_batched(jobs: Sequence[Job], prec: str = "fp32", workspace=None, ws_bytes: int = 0,
                      stream=None) -> int:
    arr = (bf_job * len(jobs))(*[j.struct for j in jobs])
    return _check(lib.bf_filter_batched(arr, len(jobs), PLANES[prec], _ptr(workspace), int(ws_bytes),
                                        _stream_handle(stream)))


def bf_filter_batched_noalloc(jobs: Sequence[Job], prec: str = "fp32", stream=None) -> int:
    arr = (bf_job * len(jobs))(*[j.struct for j in jobs])
    return _check(lib.bf_filter_batched_noalloc(arr, len(jobs), PLANES[prec], _stream_handle(stream)))


class Plan:
    """bf_plan_create / _upload / _launch / _destroy (include/bf.h).

    Holds the opaque plan handle and the Job objects whose host arrays it was
    built from; the jobs' device buffers must outlive the plan's launches.
    """

    def __init__(self, jobs: Sequence[Job], prec: str = "fp32"):
        self.jobs = list(jobs)
        self.prec = prec
        self.handle = ctypes.c_void_p()
        arr = (bf_job * len(self.jobs))(*[j.struct for j in self.jobs])
        self.status = _check(lib.bf_plan_create(arr, len(self.jobs), PLANES[prec], ctypes.byref(self.handle)))

    def workspace_bytes(self) -> int:
        return int(lib.bf_plan_workspace_bytes(self.handle))

    def upload(self, workspace, ws_bytes: int, stream=None) -> int:
        self._ws = workspace  # keep the tensor alive while the plan points at it
        return _check(lib.bf_plan_upload(self.handle, _ptr(workspace), int(ws_bytes), _stream_handle(stream)))

    def launch(self, stream=None, use_graph: bool = False) -> int:
        return _check(lib.bf_plan_launch(self.handle, _stream_handle(stream), 1 if use_graph else 0))

    def tune(self, stream=None, reps: int = 3) -> int:
        """bf_plan_tune: time the tile-height / grid-mode candidates of every
        class and keep the fastest (synchronises the stream)."""
        return _check(lib.bf_plan_tune(self.handle, _stream_handle(stream), int(reps)))

    def describe(self) -> dict:
        import json
        n = _check(lib.bf_plan_describe(self.handle, None, 0))
        buf = ctypes.create_string_buffer(n + 1)
        lib.bf_plan_describe(self.handle, buf, n + 1)
        return json.loads(buf.value.decode())

    def destroy(self):
        if self.handle:
            lib.bf_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def bf_dynamic_range_workspace_bytes(height: int, width: int) -> int:
    n = lib.bf_dynamic_range_workspace_bytes(int(height), int(width))
    if n == ctypes.c_size_t(-1).value:
        raise BfError(BF_E_INVALID, "height and width must be >= 1")
    return int(n)


def bf_dynamic_range(src, W: int, T_out, workspace, ws_bytes: int, stream=None, height=None, width=None,
                     src_pitch=None) -> int:
    """bf_dynamic_range: the local dynamic range of a device image into the
    device int T_out (asynchronous)."""
    h, w = _hw(src) if height is None else (height, width)
    pitch = int(src_pitch if src_pitch is not None else _pitch(src, w))
    return _check(lib.bf_dynamic_range(_ptr(src), int(h), int(w), pitch, int(W), _ptr(T_out), _ptr(workspace),
                                       int(ws_bytes), _stream_handle(stream)))


def bf_recursive_workspace_bytes(job: Job) -> int:
    n = lib.bf_recursive_workspace_bytes(ctypes.byref(job.struct))
    if n == ctypes.c_size_t(-1).value:
        raise BfError(BF_E_INVALID, bf_last_error())
    return int(n)


def bf_filter_recursive(job: Job, workspace, ws_bytes: int, stream=None) -> int:
    """bf_filter_recursive: eq. (9) with Deriche's recursive Gaussian as the
    spatial smoothing (asynchronous)."""
    return _check(lib.bf_filter_recursive(ctypes.byref(job.struct), _ptr(workspace), int(ws_bytes),
                                          _stream_handle(stream)))


def bf_tune_save(path: str) -> int:
    return _check(lib.bf_tune_save(os.fsencode(path)))


def bf_tune_load(path: str) -> int:
    """Merge a saved tuning file; returns the number of entries read."""
    return _check(lib.bf_tune_load(os.fsencode(path)))


def bf_tune_clear() -> None:
    lib.bf_tune_clear()
