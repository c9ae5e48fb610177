"""Every-pixel GPU parity at the full sizes of the named workloads.

Each oracle image (eq. (9) in FP64, Sec. 4, through the Fourier coefficients
of Algorithm 2) is computed once per module and compared with every plane
format the kernels offer:

- gauss_8192 (8192 x 8192, Gaussian sigma_s = 10, W = 30, Gaussian range
  sigma_r = 10, K = 40): float32 planes <= 1e-3, float16 planes < 0.5,
  bfloat16 planes < 0.5 (bfloat16 planes with a float16 intermediate);
- frame 0 of frames32_2160x3840 (2160 x 3840 with gradients, sigma_s = 8,
  W = 24, sigma_r = 15, K = 32), through a one-frame plan at the 144-row tile
  height the benchmark's tuned plan runs: float32 <= 1e-3, float16 and
  bfloat16 < 0.5;
- exp_2048 and exp_2048_box (2048 x 2048, exponential range sigma = 20,
  K = 24, Gaussian sigma_s = 5 or box, W = 15): float32 <= 1e-3.

The oracle runs on all host threads: about a minute for 8192 x 8192.
"""
import numpy as np
import pytest

import oracle
from synth import WORKLOADS, workload_images
from tests.gpu_util import gpu_filter

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL_FP32 = 1e-3
TOL_16 = 0.5


def _report(name, err):
    print("%s: max err over every pixel %.4g" % (name, err), flush=True)


def _q_report(name, Q):
    """Share of pixels whose eq. (9) denominator (unit-sum weights) falls
    below the thresholds under which the kernels re-evaluate a pixel
    directly (float32 planes 0.005, float16 0.02, bfloat16 0.05)."""
    print("%s: min Q %.4g; share below 0.005 / 0.02 / 0.05: %.3g / %.3g / %.3g"
          % (name, Q.min(), (Q < 0.005).mean(), (Q < 0.02).mean(), (Q < 0.05).mean()), flush=True)


def _fit(wl):
    return oracle.fit_kernel(wl["range_kind"], wl["sigma_r"], wl["T"], wl["eps"], wl["K_max"])


@pytest.fixture(scope="module")
def gauss_8192():
    wl = WORKLOADS["gauss_8192"]
    f = workload_images("gauss_8192")[0]
    r = _fit(wl)
    assert r.K == 40
    print("gauss_8192: oracle over %d px on %d threads" % (f.size, oracle.num_threads()), flush=True)
    ref, _, Q = oracle.fourier(f, "gaussian", wl["sigma_s"], wl["W"], r.d, wl["T"], with_pq=True)
    _q_report("gauss_8192", Q)
    return wl, f, r, ref


@pytest.mark.parametrize("prec,tol", [("fp32", TOL_FP32), ("fp16", TOL_16), ("bf16", TOL_16)])
def test_gauss_8192_every_pixel(gauss_8192, prec, tol):
    wl, f, r, ref = gauss_8192
    out, _ = gpu_filter(f, prec, spatial="gaussian", sigma_s=wl["sigma_s"], W=wl["W"], T=wl["T"], d=r.d,
                        integer_input=True)
    err = float(np.abs(out - ref).max())
    _report("gauss_8192 %s" % prec, err)
    assert np.isfinite(out).all()
    assert (err <= tol) if prec == "fp32" else (err < tol)


@pytest.fixture(scope="module")
def frame0():
    wl = WORKLOADS["frames32_2160x3840"]
    f = workload_images("frames32_2160x3840", limit=1)[0]
    r = _fit(wl)
    assert r.K == 32
    ref, _, Q = oracle.fourier(f, "gaussian", wl["sigma_s"], wl["W"], r.d, wl["T"], with_pq=True)
    _q_report("frames32 frame 0", Q)
    return wl, f, r, ref


@pytest.mark.parametrize("prec,tol", [("fp32", TOL_FP32), ("fp16", TOL_16), ("bf16", TOL_16)])
def test_frames32_frame0_every_pixel(frame0, prec, tol, monkeypatch):
    import torch

    from paper_1603_08081_amd import native
    wl, f, r, ref = frame0
    if prec != "fp32":
        monkeypatch.setenv("BF_TILE_ROWS", "144")
    x = torch.from_numpy(f).cuda()
    y = torch.full_like(x, -1.0)
    job = native.Job(x, y, spatial="gaussian", sigma_s=wl["sigma_s"], W=wl["W"], T=wl["T"], d=r.d,
                     integer_input=True)
    plan = native.Plan([job], prec)
    try:
        classes = plan.describe()["classes"]
        n = plan.workspace_bytes()
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream()
        plan.upload(ws, n, stream)
        plan.launch(stream, use_graph=True)
        torch.cuda.synchronize()
    finally:
        plan.destroy()
    if prec != "fp32":
        assert classes[0]["tile_rows"] == 144 and classes[0]["family"] == 1
    out = y.cpu().numpy()
    err = float(np.abs(out - ref).max())
    _report("frames32 frame 0 %s (plan %s)" % (prec, classes), err)
    assert np.isfinite(out).all()
    assert (err <= tol) if prec == "fp32" else (err < tol)


@pytest.mark.parametrize("name", ["exp_2048", "exp_2048_box"])
def test_exp_2048_every_pixel(name):
    wl = WORKLOADS[name]
    f = workload_images(name)[0]
    r = _fit(wl)
    assert r.K == 24
    sig = wl["sigma_s"] or 1.0
    out, st = gpu_filter(f, "fp32", spatial=wl["spatial"], sigma_s=sig, W=wl["W"], T=wl["T"], d=r.d,
                         integer_input=True)
    ref = oracle.fourier(f, wl["spatial"], sig, wl["W"], r.d, wl["T"])
    err = float(np.abs(out - ref).max())
    _report("%s fp32" % name, err)
    assert np.isfinite(out).all() and err <= TOL_FP32
