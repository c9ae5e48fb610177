"""GPU: the library's launches inside a caller's stream capture (torch CUDA
graphs).  bf_filter and bf_plan_launch enqueue kernels only; bf_filter_batched
also enqueues the copy of its job table from pinned memory, whose staging
buffer is then kept for the captured graph.  Every replay, with other device
work between replays, must equal the eager result."""
import numpy as np
import pytest

from synth import polygon_image

pytestmark = pytest.mark.gpu


def _setup(torch, native, n=3):
    imgs = [polygon_image(120 + 17 * i, 150 + 9 * i, seed=900 + i) for i in range(n)]
    srcs = [torch.from_numpy(f).cuda() for f in imgs]
    return imgs, srcs


def _jobs(native, srcs, outs):
    return [native.Job(x, y, sigma_s=2.0 + i, W=-1, range_kind="gaussian", sigma_r=20.0 + 5 * i, T=255,
                       eps=1e-3, K_max=40, integer_input=True) for i, (x, y) in enumerate(zip(srcs, outs))]


@pytest.mark.parametrize("entry", ["filter", "plan", "batched"])
def test_replays_of_captured_launches_match_eager(entry):
    import torch

    from paper_1603_08081_amd import native
    imgs, srcs = _setup(torch, native)
    ref = [torch.full_like(x, -1.0) for x in srcs]
    out = [torch.full_like(x, -1.0) for x in srcs]
    s = torch.cuda.Stream()
    # eager reference
    jobs_ref = _jobs(native, srcs, ref)
    n = native.bf_workspace_bytes(jobs_ref, "fp16")
    ws_ref = torch.empty(n, dtype=torch.uint8, device="cuda")
    native.bf_filter_batched(jobs_ref, "fp16", ws_ref, n, torch.cuda.current_stream())
    torch.cuda.synchronize()

    jobs = _jobs(native, srcs, out)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    plan = None
    if entry == "plan":
        plan = native.Plan(jobs, "fp16")
        plan.upload(ws, n, torch.cuda.current_stream())
        torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cap = torch.cuda.current_stream()
        if entry == "filter":
            for j in jobs:
                native.bf_filter(j, "fp16", stream=cap)
        elif entry == "plan":
            plan.launch(cap, use_graph=False)
        else:
            native.bf_filter_batched(jobs, "fp16", ws, n, cap)
    for rep in range(3):
        for o in out:
            o.fill_(-5.0)                      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(ref, out)):
            assert torch.equal(a, b), "%s replay %d image %d" % (entry, rep, i)
    if plan is not None:
        plan.destroy()
