"""GPU: the local dynamic range kernel (bf_dynamic_range) and filtering with
the measured T (smaller than the largest gray level) through f_max."""
import math

import numpy as np
import pytest

import oracle
from synth import polygon_image
from tests.gpu_util import gpu_filter

pytestmark = pytest.mark.gpu


def _gpu_range(f, W):
    import torch

    import paper_1603_08081_amd as bfm
    x = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
    return bfm.dynamic_range(x, W)


@pytest.mark.parametrize("shape", [(1, 1), (3, 700), (700, 3), (65, 257), (300, 130), (1031, 517)])
@pytest.mark.parametrize("W", [0, 1, 5, 24, 64])
def test_integer_images_exact(shape, W):
    H, Wd = shape
    f = polygon_image(max(H, 2), max(Wd, 2), seed=H * 7 + Wd)[:H, :Wd]
    if W >= min(H, Wd):
        # the oracle's definition folds borders, which needs W < min(H, W);
        # the clipped-window form gives the same value and has no such limit
        from scipy import ndimage
        ref = float((ndimage.maximum_filter(f.astype(np.float64), size=2 * W + 1, mode="nearest") - f).max())
    else:
        ref = oracle.local_dynamic_range(f, W)
    got = _gpu_range(f, W)
    print("range %s W=%d: gpu %d oracle %g" % (shape, W, got, ref), flush=True)
    assert got == int(math.ceil(ref))


def test_non_integer_and_pitched():
    import torch

    import paper_1603_08081_amd as bfm
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 255, size=(97, 131)).astype(np.float32)
    ref = oracle.local_dynamic_range(f, 4)
    assert abs(_gpu_range(f, 4) - math.ceil(ref)) <= 1
    # a pitched view (rows of 160 floats, 131 used)
    big = torch.zeros(97, 160, device="cuda")
    big[:, :131] = torch.from_numpy(f).cuda()
    assert abs(bfm.dynamic_range(big[:, :131], 4) - math.ceil(ref)) <= 1


def _smooth_image(H, Wd, seed):
    """Large-scale gradient over the full gray range plus small local detail:
    the local dynamic range is far below 255."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:Wd].astype(np.float64)
    f = 255.0 * (0.5 * x / Wd + 0.5 * y / H) + 6.0 * np.sin(x / 3.0) + rng.normal(0, 2.0, (H, Wd))
    return np.rint(np.clip(f, 0, 255)).astype(np.float32)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-3), ("fp16", 0.5)])
def test_filter_with_local_range(prec, tol):
    f = _smooth_image(200, 260, 9)
    W, sigma_s, sigma_r = 9, 3.0, 6.0
    T_loc = _gpu_range(f, W)
    assert T_loc == int(math.ceil(oracle.local_dynamic_range(f, W)))
    assert 0 < T_loc < 100 and f.max() > 200
    r_loc = oracle.fit_kernel("gaussian", sigma_r, T_loc, 1e-5, T_loc)
    r_full = oracle.fit_kernel("gaussian", sigma_r, 255, 1e-5, 255)
    print("T_loc %d: K %d (T = 255: K %d)" % (T_loc, r_loc.K, r_full.K), flush=True)
    assert r_loc.K < r_full.K
    out, st = gpu_filter(f, prec, spatial="gaussian", sigma_s=sigma_s, W=W, T=T_loc, d=r_loc.d,
                         f_max=255, integer_input=True)
    ref = oracle.fourier(f, "gaussian", sigma_s, W, r_loc.d, T_loc)
    err = np.abs(out - ref).max()
    print("local-range filter %s: max err %.3e" % (prec, err), flush=True)
    assert err <= tol
    dire = oracle.direct(f, "gaussian", sigma_s, W, "gaussian", sigma_r, T=255)
    assert np.abs(out - dire).max() < 0.5


def test_filter_with_local_range_batched_and_general_path():
    import torch

    from paper_1603_08081_amd import native
    f = _smooth_image(150, 170, 4)
    W = 6
    T_loc = _gpu_range(f, W)
    r = oracle.fit_kernel("gaussian", 5.0, T_loc, 1e-5, T_loc)
    ref = oracle.fourier(f, "gaussian", 2.0, W, r.d, T_loc)
    x = torch.from_numpy(f).cuda()
    outs = [torch.full_like(x, -1.0) for _ in range(3)]
    jobs = [native.Job(x, outs[0], sigma_s=2.0, W=W, T=T_loc, d=r.d, f_max=255, integer_input=True),
            native.Job(x, outs[1], sigma_s=2.0, W=W, T=T_loc, d=r.d, f_max=255, integer_input=False),
            native.Job(x, outs[2], sigma_s=2.0, W=W, T=T_loc, d=r.d, f_max=255, integer_input=True)]
    for prec in ("fp32", "fp16"):
        n = native.bf_workspace_bytes(jobs, prec)
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        native.bf_filter_batched(jobs, prec, ws, n, torch.cuda.current_stream())
        torch.cuda.synchronize()
        tol = 1e-3 if prec == "fp32" else 0.5
        for o in outs:
            assert np.abs(o.cpu().numpy() - ref).max() <= tol
