"""GPU test of bf_filter_batched_noalloc (the batched filter with its job
table in the library's fixed device array instead of a caller workspace),
through the C ABI: its outputs equal bf_filter_batched's bit for bit on two
calls in a row, the second with fewer and smaller images, and a batch whose
table exceeds the array is refused without touching any output."""
import numpy as np
import pytest

from synth import polygon_image

pytestmark = pytest.mark.gpu


def _jobs(native, specs, srcs, dsts):
    return [native.Job(x, y, spatial=s["spatial"], sigma_s=s["sigma_s"], W=s["W"], range_kind=s["rk"],
                       sigma_r=s["sr"], T=255, eps=s["eps"], K_max=s.get("K_max", 40), integer_input=s["integer"])
            for s, x, y in zip(specs, srcs, dsts)]


SPECS_A = [
    dict(h=300, w=257, spatial="gaussian", sigma_s=8.0, W=24, rk="gaussian", sr=15.0, eps=0.0, K_max=32,
         integer=True),
    dict(h=130, w=200, spatial="gaussian", sigma_s=3.0, W=9, rk="exponential", sr=20.0, eps=1e-2, integer=True),
    dict(h=97, w=131, spatial="box", sigma_s=1.0, W=15, rk="gaussian", sr=30.0, eps=1e-3, integer=True),
    dict(h=111, w=99, spatial="gaussian", sigma_s=5.0, W=15, rk="gaussian", sr=25.0, eps=1e-3, integer=False),
    dict(h=150, w=141, spatial="gaussian", sigma_s=16.0, W=48, rk="exponential", sr=60.0, eps=1e-2,
         integer=True),
]
# the second call: fewer and smaller images
SPECS_B = [
    dict(h=70, w=90, spatial="gaussian", sigma_s=2.0, W=6, rk="gaussian", sr=10.0, eps=1e-4, integer=True),
    dict(h=64, w=80, spatial="gaussian", sigma_s=3.0, W=9, rk="gaussian", sr=30.0, eps=1e-3, integer=True),
]


def _inputs(torch, specs, seed):
    imgs = []
    for i, s in enumerate(specs):
        f = polygon_image(s["h"], s["w"], seed=seed + i)
        if not s["integer"]:
            f = np.clip(f + np.random.default_rng(i).uniform(-0.4, 0.4, f.shape), 0, 255).astype(np.float32)
        imgs.append(torch.from_numpy(f).cuda())
    return imgs


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_noalloc_equals_batched_on_two_calls(prec):
    import torch

    from paper_1603_08081_amd import native
    stream = torch.cuda.current_stream()
    for specs, seed in ((SPECS_A, 8100), (SPECS_B, 8200)):
        srcs = _inputs(torch, specs, seed)
        ref = [torch.full_like(x, -1.0) for x in srcs]
        out = [torch.full_like(x, -2.0) for x in srcs]
        jobs = _jobs(native, specs, srcs, ref)
        n = native.bf_workspace_bytes(jobs, prec)
        assert n <= native.BF_NOALLOC_SCRATCH_BYTES
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        native.bf_filter_batched(jobs, prec, ws, n, stream)
        st = native.bf_filter_batched_noalloc(_jobs(native, specs, srcs, out), prec, stream)
        torch.cuda.synchronize()
        assert st in (native.BF_OK, native.BF_FIT_NOT_CONVERGED)
        for i, (a, b) in enumerate(zip(ref, out)):
            print("%s %d x %d: max |noalloc - batched| = %.3g" % (prec, specs[i]["h"], specs[i]["w"],
                                                                  float((a - b).abs().max())), flush=True)
            assert torch.isfinite(b).all()
            assert torch.equal(a, b), "job %d" % i


def test_noalloc_refuses_a_table_beyond_its_array():
    import torch

    from paper_1603_08081_amd import native
    n = 1700   # 1700 job descriptors alone exceed the array
    x = torch.zeros(32, 32, device="cuda")
    Y = torch.full((n, 32, 32), -5.0, device="cuda")
    jobs = [native.Job(x, Y[i], spatial="gaussian", sigma_s=3.0, W=9, T=255, d=np.array([1.0, 0.5]),
                       integer_input=True) for i in range(n)]
    assert native.bf_workspace_bytes(jobs, "fp16") > native.BF_NOALLOC_SCRATCH_BYTES
    with pytest.raises(native.BfError) as ei:
        native.bf_filter_batched_noalloc(jobs, "fp16", torch.cuda.current_stream())
    assert ei.value.code == native.BF_E_UNSUPPORTED
    assert "BF_NOALLOC_SCRATCH_BYTES" in native.bf_last_error()
    torch.cuda.synchronize()
    assert bool((Y == -5.0).all())
