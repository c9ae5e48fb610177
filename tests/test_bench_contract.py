"""Host-side checks of bench.py: the multi-GPU refusal, the flop and byte
counts its rooflines use, and the lookup of committed HBM counter summaries.
No GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "one GPU" in r.stdout
    assert "{" not in r.stdout   # no JSON line


def test_algorithmic_flops_gaussian_and_box():
    # K = 32, W = 24: 129 planes, two passes of 49 MACs, plus 16 flops per
    # harmonic of modulation and demodulation
    assert bench.alg_flops_per_px(32, 24) == 129 * 2 * 49 * 2 + 16 * 32 == 25796
    # a box filter's passes are running sums: one add and one subtract each
    assert bench.alg_flops_per_px(24, 15, "box") == 97 * 2 * 2 + 16 * 24
    assert bench.alg_flops_per_px(24, 15, "box") < bench.alg_flops_per_px(24, 15)


@pytest.mark.parametrize("K,W,th", [(32, 24, 128), (32, 24, 32), (9, 9, 32), (40, 30, 64)])
def test_issued_mfma_flops_cover_the_algorithmic_count(K, W, th):
    issued = bench.issued_flops_per_px(K, W, th)
    assert issued >= bench.alg_flops_per_px(K, W)
    # taller tiles recompute fewer halo rows
    assert bench.issued_flops_per_px(K, W, 128) <= bench.issued_flops_per_px(K, W, 32)


def test_issued_flops_closed_form_at_the_benchmarked_shape():
    # NT = 4, KS = 2, NJ = 8: (11/8 * 2 + 2) products of 16x16x32 per 16x16 block
    per_plane = (11 / 8 * 2 + 2) * 2 * 16 * 16 * 32 / 256
    assert bench.issued_flops_per_px(32, 24, 128) == pytest.approx(per_plane * 129)


def test_traffic_comes_from_the_committed_summary_only_when_it_matches():
    path = os.path.join(ROOT, "profiles", "wave_batched_kernel_frames32_2160x3840_fp16.md")
    txt = open(path).read()
    if bench.kernel_sources_digest() not in txt:
        pytest.skip("kernel sources changed since the counters were taken")
    # the tile height the tuner keeps on this workload
    v = bench.measured_traffic("frames32_2160x3840", "fp16", 32, 144)
    assert v is not None and v > 8 * 32 * 2160 * 3840   # at least the algorithmic bytes
    # another frame count, a tile height without counters, or no summary: null
    assert bench.measured_traffic("frames32_2160x3840", "fp16", 8, 144) is None
    assert bench.measured_traffic("frames32_2160x3840", "fp16", 32, 48) is None
    assert bench.measured_traffic("gauss_8192", "fp16", 1, 128) is None


@pytest.mark.parametrize("K", [0, 3, 4, 32, 40])
def test_recursive_traffic_model_uses_the_library_harmonic_groups(K):
    """bench.py prices the recursive path per harmonic and per group of
    harmonics; the group count it assumes is the one the library's workspace
    is laid out for (float32 planes 16 (K + 1) B/px, float64 group shares
    16 B/px per group)."""
    import numpy as np

    from paper_1603_08081_amd import native
    job = native.Job(0x10000000, 0x20000000, spatial="gaussian", sigma_s=24.0, W=0, T=255,
                     d=np.ones(K + 1), height=64, width=64, integer_input=True)
    per_px = native.bf_recursive_workspace_bytes(job) // (64 * 64)
    groups = (per_px - 16 * (K + 1)) // 16
    assert 16 * (K + 1) + 16 * groups == per_px and groups >= 1
    assert bench.recursive_bytes_per_px(K) == (K + 1) * (56 + 48) + groups * (48 + 16) + 4
    if K == 32:
        assert bench.recursive_bytes_per_px(K) == 4012
