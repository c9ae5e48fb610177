"""C-ABI checks that need no GPU: the library loads, exports what
include/bf.h declares, its host fit agrees with the FP64 oracle, and every
argument error is reported before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1603_08081_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE_SRC = 0x10000000   # never dereferenced: validation fails before any device call
FAKE_DST = 0x20000000


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*\*?\s*\b(bf_[a-z_0-9]+)\s*\(", txt, re.M):
            names.add(m.group(1))
    return names


def test_exports_every_declared_symbol():
    names = _declared_functions()
    assert {"bf_fit_coeffs", "bf_filter", "bf_filter_batched", "bf_workspace_bytes", "bf_last_error"} <= names
    lib = ctypes.CDLL(native.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("kind,sigma,T,eps,kmax", [
    ("gaussian", 30.0, 217, 1e-3, 217), ("gaussian", 30.0, 255, 1e-2, 255),
    ("exponential", 20.0, 255, 1e-2, 24), ("gaussian", 10.0, 255, 0.0, 40),
    ("gaussian", 15.0, 255, 0.0, 32), ("gaussian", 80.0, 255, 1e-5, 255)])
def test_host_fit_matches_oracle(kind, sigma, T, eps, kmax):
    st, d, e2, em = native.bf_fit_coeffs(kind, sigma, T, eps, kmax)
    r = oracle.fit_kernel(kind, sigma, T, eps, kmax)
    assert len(d) == r.K + 1
    np.testing.assert_allclose(d, r.d, rtol=0, atol=1e-10)
    assert abs(e2 - r.E) < 1e-10
    em_ref = np.abs(oracle.series(r.d, T, np.arange(T + 1)) - r.b).max()
    assert abs(em - em_ref) < 1e-10
    assert st == (native.BF_OK if r.converged else native.BF_FIT_NOT_CONVERGED)


def test_host_fit_table_kernel():
    T = 100
    t = np.arange(T + 1)
    phi = 0.25 + 0.5 * np.cos(3 * np.pi * t / T) + 0.25 * np.cos(7 * np.pi * t / T)
    st, d, e2, _ = native.bf_fit_coeffs("table", 0.0, T, 1e-12, T, phi_table=phi)
    assert st == native.BF_OK and len(d) == 8 and e2 < 1e-12
    np.testing.assert_allclose(d[[0, 3, 7]], [0.25, 0.5, 0.25], atol=1e-12)


def test_tables_3_and_4_through_the_abi(golden_dir):
    for line in open(os.path.join(golden_dir, "paper_table3_table4.txt")):
        if line.strip() and not line.startswith("#"):
            eps, n, _ = line.split()
            st, d, _, _ = native.bf_fit_coeffs("gaussian", 30.0, 217, float(eps), 217)
            assert st == native.BF_OK and len(d) == int(n)


@pytest.mark.parametrize("args", [
    ("gaussian", 30.0, 0, 1e-3, 0), ("gaussian", 30.0, 2000, 1e-3, 10),
    ("gaussian", 30.0, 255, -1.0, 10), ("gaussian", 30.0, 255, 1e-3, 256),
    ("gaussian", 0.0, 255, 1e-3, 10), ("exponential", -1.0, 255, 1e-3, 10),
    ("table", 0.0, 255, 1e-3, 10)])
def test_fit_rejects_bad_arguments(args):
    with pytest.raises(native.BfError) as ei:
        native.bf_fit_coeffs(*args)
    assert ei.value.code == native.BF_E_INVALID
    assert native.bf_last_error()


def test_fit_cap_warns():
    st, d, e2, _ = native.bf_fit_coeffs("exponential", 20.0, 255, 1e-2, 24)
    assert st == native.BF_FIT_NOT_CONVERGED and len(d) == 25 and e2 > 1e-2


def _job(**kw):
    base = dict(spatial="gaussian", sigma_s=3.0, W=9, range_kind="gaussian", sigma_r=30.0, T=255,
                eps=1e-2, K_max=40, height=64, width=64)
    base.update(kw)
    src = base.pop("src", FAKE_SRC)
    dst = base.pop("dst", FAKE_DST)
    return native.Job(src, dst, **base)


@pytest.mark.parametrize("kw,code", [
    (dict(src=None), native.BF_E_INVALID),
    (dict(dst=None), native.BF_E_INVALID),
    (dict(height=0), native.BF_E_INVALID),
    (dict(width=-3), native.BF_E_INVALID),
    (dict(src_pitch=10), native.BF_E_INVALID),
    (dict(W=64, height=64), native.BF_E_INVALID),
    (dict(W=9, width=9), native.BF_E_INVALID),
    (dict(W=65, height=200, width=200), native.BF_E_UNSUPPORTED),
    (dict(sigma_s=0.0), native.BF_E_INVALID),
    (dict(spatial="box", W=-1), native.BF_E_INVALID),
    (dict(W=-1, sigma_s=30.0, height=500, width=500), native.BF_E_UNSUPPORTED),
    (dict(T=0), native.BF_E_INVALID),
    (dict(T=4096), native.BF_E_INVALID),
    (dict(K_max=300), native.BF_E_INVALID),
    (dict(T=1000, K_max=300), native.BF_E_UNSUPPORTED),
    (dict(sigma_r=-1.0), native.BF_E_INVALID),
    (dict(range_kind="table"), native.BF_E_INVALID),
    (dict(d=np.ones(300)), native.BF_E_UNSUPPORTED),
    (dict(d=np.array([1.0, np.nan])), native.BF_E_INVALID),
    (dict(dst=FAKE_SRC + 4 * 100), native.BF_E_INVALID),   # overlaps src
    (dict(flags=0x100), native.BF_E_INVALID),               # unknown flag bits
])
def test_filter_rejects_bad_jobs_before_device_work(kw, code):
    flags = kw.pop("flags", None)
    j = _job(**kw)
    if flags is not None:
        j.struct.flags = flags
    with pytest.raises(native.BfError) as ei:
        native.bf_filter(j, "fp32", stream=0)
    assert ei.value.code == code
    assert native.bf_last_error()
    with pytest.raises(native.BfError):
        native.bf_workspace_bytes([j])
    with pytest.raises(native.BfError) as ei:
        native.bf_filter_batched([_job(), j], "fp32", stream=0)
    assert ei.value.code == code


def test_unknown_precision_rejected():
    rc = native.lib.bf_filter(ctypes.byref(_job().struct), 7, None, 0, None)
    assert rc == native.BF_E_INVALID


def test_workspace_query_for_valid_jobs():
    assert native.bf_workspace_bytes([_job()], "fp32") >= 0
    assert native.bf_workspace_bytes([_job(), _job(W=-1, sigma_s=2.0, dst=FAKE_DST + (1 << 20))], "fp16") >= 0


def test_batched_workspace_grows_with_jobs_and_tiles():
    one = native.bf_workspace_bytes([_job()], "fp16")
    two = native.bf_workspace_bytes([_job(), _job(dst=FAKE_DST + (1 << 20))], "fp16")
    assert 0 < one < two
    big = native.bf_workspace_bytes([_job(height=2000, width=3000, src_pitch=3000, dst_pitch=3000,
                                          dst=FAKE_DST + (1 << 26))], "fp16")
    assert big > one
    # the table holds one 16-byte work item per output tile
    assert (big - one) % 16 == 0


def test_plan_host_side_without_device_work():
    pl = native.Plan([_job(), _job(W=-1, sigma_s=2.0, dst=FAKE_DST + (1 << 20))], "fp16")
    assert pl.status == native.BF_OK
    assert pl.workspace_bytes() == native.bf_workspace_bytes(pl.jobs, "fp16")
    # launch before upload, and uploads into a missing or small workspace, fail before any HIP call
    with pytest.raises(native.BfError) as ei:
        pl.launch(stream=0)
    assert ei.value.code == native.BF_E_INVALID
    with pytest.raises(native.BfError) as ei:
        pl.upload(None, 0, stream=0)
    assert ei.value.code == native.BF_E_WORKSPACE
    with pytest.raises(native.BfError) as ei:
        pl.upload(0x30000000, pl.workspace_bytes() - 1, stream=0)
    assert ei.value.code == native.BF_E_WORKSPACE
    with pytest.raises(native.BfError) as ei:
        pl.upload(0x30000008, pl.workspace_bytes(), stream=0)   # misaligned
    assert ei.value.code == native.BF_E_WORKSPACE
    pl.destroy()
    native.lib.bf_plan_destroy(None)


def test_plan_reports_unconverged_fit_and_rejects_bad_jobs():
    pl = native.Plan([_job(d=None, range_kind="exponential", sigma_r=20.0, eps=1e-2, K_max=24)], "fp32")
    assert pl.status == native.BF_FIT_NOT_CONVERGED
    pl.destroy()
    with pytest.raises(native.BfError) as ei:
        native.Plan([_job(), _job(T=0)], "fp32")
    assert ei.value.code == native.BF_E_INVALID
    assert "job 1" in native.bf_last_error()
    out = ctypes.c_void_p(1)
    assert native.lib.bf_plan_create(None, 0, 0, ctypes.byref(out)) == native.BF_E_INVALID
    assert out.value is None
    assert native.lib.bf_plan_workspace_bytes(None) == ctypes.c_size_t(-1).value


def test_plan_describe_lists_classes():
    jobs = [_job(), _job(W=30, sigma_s=10.0, height=200, width=300, src_pitch=300, dst_pitch=300,
                         dst=FAKE_DST + (1 << 24)),
            _job(integer_input=True, dst=FAKE_DST + (1 << 25))]
    pl = native.Plan(jobs, "fp16")
    info = pl.describe()
    assert info["jobs"] == 3 and info["planes"] == native.PLANES["fp16"]
    assert info["workspace_bytes"] == pl.workspace_bytes()
    # W = 9 non-integer, W = 30 non-integer, W = 9 integer: three kernel classes
    assert len(info["classes"]) == 3
    assert sum(c["jobs"] for c in info["classes"]) == 3
    for c in info["classes"]:
        assert c["tile_rows"] in (32, 64, 128) and c["items"] >= 1 and not c["tuned"]
    fam = sorted(c["family"] for c in info["classes"])
    assert fam == [0, 0, 1]   # general path for non-integer images, wave kernel for integer fp16
    with pytest.raises(native.BfError):
        pl.tune(stream=0)     # not uploaded yet
    pl.destroy()


def test_dynamic_range_rejects_bad_arguments_before_device_work():
    ws = native.bf_dynamic_range_workspace_bytes(64, 80)
    assert ws >= 4 * 64 * 80
    cases = [
        (dict(src=None), native.BF_E_INVALID),
        (dict(W=-1), native.BF_E_INVALID),
        (dict(W=65), native.BF_E_INVALID),
        (dict(height=0), native.BF_E_INVALID),
        (dict(src_pitch=10), native.BF_E_INVALID),
        (dict(T_out=None), native.BF_E_INVALID),
        (dict(workspace=None), native.BF_E_WORKSPACE),
        (dict(ws_bytes=ws - 1), native.BF_E_WORKSPACE),
        (dict(workspace=0x30000004), native.BF_E_WORKSPACE),
    ]
    for kw, code in cases:
        a = dict(src=FAKE_SRC, height=64, width=80, src_pitch=80, W=5, T_out=FAKE_DST, workspace=0x30000000,
                 ws_bytes=ws)
        a.update(kw)
        rc = native.lib.bf_dynamic_range(a["src"], a["height"], a["width"], a["src_pitch"], a["W"], a["T_out"],
                                         a["workspace"], a["ws_bytes"], None)
        assert rc == code, (kw, rc)
    with pytest.raises(native.BfError):
        native.bf_dynamic_range_workspace_bytes(0, 5)


def test_f_max_validated():
    with pytest.raises(native.BfError) as ei:
        native.bf_filter(_job(f_max=2000), "fp32", stream=0)
    assert ei.value.code == native.BF_E_INVALID


def test_tune_cache_round_trip(tmp_path):
    native.bf_tune_clear()
    p = tmp_path / "tune.txt"
    # fp16, window class 2 (W = 3), wave kernel, 64 x 64 = 2^12 pixels
    p.write_text("bf-tune 1\n1 2 1 12 32 -1\n")
    assert native.bf_tune_load(str(p)) == 1
    pl = native.Plan([_job(W=3, sigma_s=1.0, integer_input=True)], "fp16")
    c = pl.describe()["classes"][0]
    assert (c["nt"], c["family"], c["tile_rows"], c["grid"], c["tuned"]) == (2, 1, 32, -1, True)
    pl.destroy()
    q = tmp_path / "saved.txt"
    native.bf_tune_save(str(q))
    assert q.read_text() == "bf-tune 1\n1 2 1 12 32 -1\n"
    native.bf_tune_clear()
    pl = native.Plan([_job(W=3, sigma_s=1.0, integer_input=True)], "fp16")
    assert not pl.describe()["classes"][0]["tuned"]
    pl.destroy()
    for bad in ("nonsense\n", "bf-tune 1\n1 2 1 12 48 0\n", "bf-tune 1\n1 2 1 12 32\n", "bf-tune 1\n7 2 1 12 32 0\n"):
        p.write_text(bad)
        with pytest.raises(native.BfError):
            native.bf_tune_load(str(p))
    with pytest.raises(native.BfError):
        native.bf_tune_load(str(tmp_path / "missing.txt"))


def test_batched_rejects_outputs_that_overlap_other_jobs():
    a = dict(height=64, width=64)
    # two jobs reading the same image into different outputs: allowed
    ok = [_job(**a), _job(dst=FAKE_DST + (1 << 20), **a)]
    assert native.bf_workspace_bytes(ok, "fp16") > 0
    # two jobs writing the same output
    bad = [_job(**a), _job(src=FAKE_SRC + (1 << 20), **a)]
    with pytest.raises(native.BfError) as ei:
        native.bf_workspace_bytes(bad, "fp16")
    assert ei.value.code == native.BF_E_INVALID and "overlaps another job" in native.bf_last_error()
    # job 1 writes into job 0's input
    bad = [_job(**a), _job(src=FAKE_SRC + (1 << 21), dst=FAKE_SRC + 4 * 100, **a)]
    with pytest.raises(native.BfError):
        native.Plan(bad, "fp32")
    # job 0's output runs into job 1's input further up in memory
    bad = [_job(dst=FAKE_DST, **a), _job(src=FAKE_DST + 4 * 64 * 63, dst=FAKE_DST + (1 << 22), **a)]
    with pytest.raises(native.BfError):
        native.bf_filter_batched(bad, "fp32", stream=0)


@pytest.mark.parametrize("kw,code", [
    (dict(src=None), native.BF_E_INVALID),
    (dict(height=0), native.BF_E_INVALID),
    (dict(src_pitch=10), native.BF_E_INVALID),
    (dict(spatial="box", W=3), native.BF_E_INVALID),
    (dict(sigma_s=0.0), native.BF_E_INVALID),
    (dict(sigma_s=2000.0), native.BF_E_UNSUPPORTED),
    (dict(sigma_s=300.0), native.BF_E_UNSUPPORTED),
    (dict(T=0), native.BF_E_INVALID),
    (dict(sigma_r=-1.0), native.BF_E_INVALID),
    (dict(d=np.ones(300)), native.BF_E_UNSUPPORTED),
    (dict(dst=FAKE_SRC + 4 * 100), native.BF_E_INVALID),
    # 2^28 elements: beyond the 32-bit byte offsets of the recursive kernels
    (dict(height=16384, width=16384), native.BF_E_UNSUPPORTED),
    (dict(height=8192, width=16384, src_pitch=32768), native.BF_E_UNSUPPORTED),
])
def test_recursive_filter_rejects_bad_jobs_before_device_work(kw, code):
    j = _job(**kw)
    with pytest.raises(native.BfError) as ei:
        native.bf_filter_recursive(j, 0x30000000, 1 << 40, stream=0)
    assert ei.value.code == code
    assert native.bf_last_error()
    with pytest.raises(native.BfError):
        native.bf_recursive_workspace_bytes(j)


def test_recursive_filter_workspace_checks():
    # 16 (K + 1) + 16 ceil((K + 1) / 4) bytes per pixel (row-smoothed
    # float32 planes, float64 numerator and denominator shares of each group
    # of four harmonics), each of the three regions 256-byte aligned; one row
    # short of 2^28 elements is still taken
    assert native.bf_recursive_workspace_bytes(_job(W=0, d=np.array([1.0]), height=16383, width=16384,
                                                    dst=FAKE_SRC + (1 << 32))) > 0
    j = _job(W=0, d=np.array([1.0, 0.5, 0.25]))
    assert native.bf_recursive_workspace_bytes(j) == (16 * 3 + 16 * 1) * 64 * 64
    assert native.bf_recursive_workspace_bytes(_job(W=0, d=np.ones(6))) == (16 * 6 + 16 * 2) * 64 * 64
    assert native.bf_recursive_workspace_bytes(_job(W=0, d=np.array([1.0]), height=3, width=5)) == 3 * 256
    ws = native.bf_recursive_workspace_bytes(j)
    for ptr, n in ((None, ws), (0x30000000, ws - 1), (0x30000004, ws)):
        with pytest.raises(native.BfError) as ei:
            native.bf_filter_recursive(j, ptr, n, stream=0)
        assert ei.value.code == native.BF_E_WORKSPACE


def test_noalloc_batched_refuses_oversized_tables_before_device_work():
    # 1700 descriptors exceed the library's fixed table array; the refusal
    # comes from the host-side plan, before any HIP call
    jobs = [_job(height=32, width=32, dst=FAKE_DST + i * 4096) for i in range(1700)]
    assert native.bf_workspace_bytes(jobs, "fp16") > native.BF_NOALLOC_SCRATCH_BYTES
    with pytest.raises(native.BfError) as ei:
        native.bf_filter_batched_noalloc(jobs, "fp16", stream=0)
    assert ei.value.code == native.BF_E_UNSUPPORTED
    assert "BF_NOALLOC_SCRATCH_BYTES" in native.bf_last_error()
    # argument errors are reported as by bf_filter_batched
    with pytest.raises(native.BfError) as ei:
        native.bf_filter_batched_noalloc([_job(), _job(height=0)], "fp16", stream=0)
    assert ei.value.code == native.BF_E_INVALID
