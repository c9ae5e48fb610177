#!/usr/bin/env python3
"""Throughput of the Fourier-kernel bilateral filter on one MI355X.

One step = eq. (9) through Algorithm 1 (modulate, row and column smoothing,
demodulate, accumulate, divide) over one batch of synthetic input that is
already resident in HBM.  The default workload is 32 frames of 2160 x 3840
(integer gray levels with smooth gradients), Gaussian spatial kernel
sigma_s = 8 (W = 24), Gaussian range kernel sigma_r = 15, T = 255, K = 32,
filtered in one batched call with float16 planes and float32 accumulation
(float16 keeps the error below half a gray level here; bfloat16 planes are
timed and checked alongside, and so are float32 planes).

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp16|bf16|fp32]
    python bench.py --sweep     # Tables 1-3 analogues, one JSON line per setting
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s, FP32 vs BF16-plane batched, at max err <0.5 gray level; % HBM peak"
PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}   # dense MFMA, MI355X published
PEAK_HBM_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def alg_flops_per_px(K, W):
    """Separable smoothing of the 4K+1 planes: two passes of 2W+1 MACs each."""
    return (4 * K + 1) * 2 * (2 * W + 1) * 2


def kernel_sources_digest():
    """sha256 over the library's kernel and host sources (byte counters taken
    on other sources no longer describe the kernel)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1603_08081_amd", "csrc")
    h = hashlib.sha256()
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".h", ".hip", ".cpp")):
            h.update(fn.encode())
            with open(os.path.join(csrc, fn), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, prec, frames):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a copy of known size);
    None when there is none for this workload or the sources have changed
    since the counters were taken."""
    name = "%s_%s_%s.md" % ("wave_batched_kernel" if prec != "fp32" else "fused_batched_kernel", workload, prec)
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ":" in ln and ln.lstrip("- ").split(":")[0].strip() in (
                    "traffic_bytes_per_launch", "sources_sha256", "frames"):
                k, v = ln.lstrip("- ").split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("sources_sha256") != kernel_sources_digest() or int(vals.get("frames", -1)) != frames:
        return None
    return float(vals["traffic_bytes_per_launch"])


# Run-times the paper reports for one 512 x 512 image (Sec. 5, Matlab on a
# 1.3 GHz laptop CPU; the image had T = 217): Table 1 over sigma_s at
# sigma_r = 30, Table 2 over sigma_r at sigma_s = 3, Table 3 over eps at
# sigma_s = 3, sigma_r = 30 (eps = 1e-3 where not varied).
PAPER_MS = {
    "table1": {1: 630, 2: 635, 5: 638, 8: 640, 10: 645, 12: 650},
    "table2": {10: 2100, 15: 1500, 20: 840, 30: 634, 50: 450, 100: 200},
    "table3": {1e-5: 910, 1e-4: 850, 1e-3: 780, 1e-2: 715, 1e-1: 670},
}


def run_sweep(args):
    """Tables 1-3 analogues on the GPU: per setting, the fitted K, the latency
    of one 512 x 512 image, the throughput of a batch of 64 such images, and
    the error against the FP64 oracles.  One JSON line per setting."""
    import torch

    import oracle
    from paper_1603_08081_amd import native
    from synth import polygon_image

    T = 255
    n_img = 64
    imgs = [polygon_image(512, 512, seed=70000 + i) for i in range(n_img)]
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(np.stack(imgs)).to(dev)
    stream = torch.cuda.current_stream()
    cells = [("table1", dict(sigma_s=float(v), sigma_r=30.0, eps=1e-3)) for v in PAPER_MS["table1"]]
    cells += [("table2", dict(sigma_s=3.0, sigma_r=float(v), eps=1e-3)) for v in PAPER_MS["table2"]]
    cells += [("table3", dict(sigma_s=3.0, sigma_r=30.0, eps=float(v))) for v in PAPER_MS["table3"]]

    def events_ms(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for table, c in cells:
        st, d, e2, em = native.bf_fit_coeffs("gaussian", c["sigma_r"], T, c["eps"], T)
        K = len(d) - 1
        W = int(math.ceil(3.0 * c["sigma_s"]))
        line = {"sweep": table, "sigma_s": c["sigma_s"], "sigma_r": c["sigma_r"], "eps": c["eps"], "T": T,
                "K": K, "W": W}
        for prec in ("fp32", "fp16"):
            out = torch.empty_like(src)
            jobs = [native.Job(src[i], out[i], spatial="gaussian", sigma_s=c["sigma_s"], W=W, T=T, d=d,
                               integer_input=True) for i in range(n_img)]
            line[prec + "_ms_1img"] = round(events_ms(lambda: native.bf_filter(jobs[0], prec, stream=stream),
                                                      20), 4)
            plan = native.Plan(jobs, prec)
            ws = torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device=dev)
            plan.upload(ws, ws.numel(), stream)
            plan.tune(stream, reps=2)
            ms = events_ms(lambda: plan.launch(stream, use_graph=True), 10)
            line[prec + "_mpix_s_batch64"] = round(n_img * 512 * 512 / (ms * 1e-3) / 1e6, 1)
            torch.cuda.synchronize()
            o0 = out[0].cpu().numpy()
            ref = oracle.fourier(imgs[0], "gaussian", c["sigma_s"], W, d, T)
            line[prec + "_err_vs_fourier"] = float("%.3g" % np.abs(o0 - ref).max())
            if prec == "fp32":
                dire = oracle.direct(imgs[0], "gaussian", c["sigma_s"], W, "gaussian", c["sigma_r"], T=T)
                line["fp32_err_vs_direct"] = float("%.3g" % np.abs(o0 - dire).max())
            plan.destroy()
        key = {"table1": c["sigma_s"], "table2": c["sigma_r"], "table3": c["eps"]}[table]
        line["paper_ms_1img"] = PAPER_MS[table][int(key) if table != "table3" else key]
        print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp16", choices=["bf16", "fp16", "fp32"],
                    help="plane format of the headline number (fp16 meets the 0.5 gray-level bar "
                         "on this workload; bf16 is timed and checked alongside)")
    ap.add_argument("--workload", default="frames32_2160x3840")
    ap.add_argument("--frames", type=int, default=None, help="use only the first N frames")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32-plane comparison")
    ap.add_argument("--no-bf16", action="store_true", help="skip the bfloat16-plane comparison")
    ap.add_argument("--no-check", action="store_true", help="skip the error check against the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the plan autotuner (bf_plan_tune)")
    ap.add_argument("--eager", action="store_true",
                    help="launch the plan eagerly instead of replaying its HIP graph")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one plain elementwise copy (negation) of this many MiB of "
                         "float32, the known-size reference for HBM byte counters")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline line: the Tables 1-3 analogues (one JSON line per setting)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the path shards by whole images or by "
              "row stripes with W-row halos; no multi-GPU run is implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.sweep:
        run_sweep(args)
        return

    import torch

    import paper_1603_08081_amd as bfm  # noqa: F401
    from paper_1603_08081_amd import native
    from synth import WORKLOADS, workload_images

    wl = WORKLOADS[args.workload]
    if "height" not in wl:
        raise SystemExit("bench.py times the single-kernel-setting workloads only")
    t0 = time.time()
    imgs = workload_images(args.workload, limit=args.frames)
    n = len(imgs)
    H, Wd = imgs[0].shape
    log("generated %d x %dx%d in %.1fs" % (n, H, Wd, time.time() - t0))
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(np.stack(imgs)).to(dev)
    dst = torch.empty_like(src)
    st, d, e2, em = native.bf_fit_coeffs(wl["range_kind"], wl["sigma_r"], wl["T"], wl["eps"], wl["K_max"])
    K = len(d) - 1
    W = wl["W"]

    def make_jobs(prec_dst):
        return [native.Job(src[i], prec_dst[i], spatial=wl["spatial"], sigma_s=wl["sigma_s"] or 1.0, W=W,
                           range_kind=wl["range_kind"], sigma_r=wl["sigma_r"], T=wl["T"], d=d,
                           integer_input=True) for i in range(n)]

    stream = torch.cuda.current_stream()

    plans = {}

    def timed(prec, out, steps, warmup, use_graph=True):
        """Device time per step of one plan launch (graph replay by default)
        over all frames; the plan (fits, job table upload, autotuning) is made
        once, outside the timed region."""
        plan = native.Plan(make_jobs(out), prec)
        nbytes = plan.workspace_bytes()
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        plan.upload(ws, nbytes, stream)
        if not args.no_tune:
            t0 = time.time()
            plan.tune(stream, reps=2)
            log("%s: tuned in %.2fs: %s" % (prec, time.time() - t0, plan.describe()["classes"]))
        plans[prec] = plan.describe()
        for _ in range(warmup):
            plan.launch(stream, use_graph)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            plan.launch(stream, use_graph)
        e1.record(stream)
        torch.cuda.synchronize()
        plan.destroy()
        return e0.elapsed_time(e1) / steps

    def timed_call(prec, out, steps):
        """Device time per step of bf_filter_batched (job table copy included)."""
        jobs = make_jobs(out)
        nbytes = native.bf_workspace_bytes(jobs, prec)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        native.bf_filter_batched(jobs, prec, ws, nbytes, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            native.bf_filter_batched(jobs, prec, ws, nbytes, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms = timed(args.precision, dst, args.steps, args.warmup, use_graph=not args.eager)
    px = n * H * Wd
    value = px / (ms * 1e-3) / 1e6
    log("%s planes: %.3f ms/step, %.1f Mpix/s (plan, graph replay)" % (args.precision, ms, value))

    extra = {}
    ms_call = timed_call(args.precision, dst, max(2, args.steps // 2))
    log("%s planes: %.3f ms/step through bf_filter_batched" % (args.precision, ms_call))
    extra["batched_call_ms_per_step"] = round(ms_call, 3)
    dstb = None
    if not args.no_bf16 and args.precision != "bf16":
        dstb = torch.empty_like(src)
        msb = timed("bf16", dstb, args.steps, 1)
        vb = px / (msb * 1e-3) / 1e6
        log("bf16 planes: %.3f ms/step, %.1f Mpix/s" % (msb, vb))
        extra["bf16_value"] = round(vb, 1)
        extra["bf16_ms_per_step"] = round(msb, 3)
    if not args.no_fp32 and args.precision != "fp32":
        dst32 = torch.empty_like(src)
        ms32 = timed("fp32", dst32, max(2, args.steps // 4), 1)
        v32 = px / (ms32 * 1e-3) / 1e6
        log("fp32 planes: %.3f ms/step, %.1f Mpix/s" % (ms32, v32))
        extra["fp32_value"] = round(v32, 1)
        extra["fp32_ms_per_step"] = round(ms32, 3)
        extra["speedup_vs_fp32"] = round(value / v32, 3)
    else:
        dst32 = dst if args.precision == "fp32" else None

    if args.calib_copy_mib > 0:
        a = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))
        del a, b

    # ---- roofline of the dominant kernel: every frame has the same window and
    # K, so the plan is one launch per step
    launches = len(plans[args.precision]["classes"])
    avg_launch_s = ms * 1e-3 / launches
    flops = alg_flops_per_px(K, W) * px / launches   # algorithmic flops of one launch
    achieved = flops / avg_launch_s / 1e12
    peak = PEAK_TFLOPS[args.precision]
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(args.workload, args.precision, n),
            "kernel": ("wave_batched_kernel" if args.precision != "fp32" else "fused_batched_kernel") +
                      " (modulate + row/column MFMA Toeplitz + demodulate + divide)",
            "alg_flops_per_px": alg_flops_per_px(K, W), "launches_per_step": launches,
            "plan": plans[args.precision]["classes"]}

    # ---- error against the FP64 oracle (sampled rows of frame 0 and the last frame)
    if not args.no_check:
        import oracle
        out16 = dst.cpu().numpy()
        out32 = dst32.cpu().numpy() if dst32 is not None else None
        rows = np.unique(np.array([0, 1, W - 1, W, H // 2, H - W - 1, H - 2, H - 1] +
                                  list(np.random.default_rng(1).integers(0, H, 4))))
        pix = (rows[:, None] * Wd + np.arange(Wd)[None, :]).ravel()
        outb = dstb.cpu().numpy() if dstb is not None else None
        errs16, errs32, errsd, errsb = [], [], [], []
        for fi in sorted({0, n - 1}):
            ref = oracle.fourier(imgs[fi], wl["spatial"], wl["sigma_s"] or 1.0, W, d, wl["T"], pixels=pix)
            dire = oracle.direct(imgs[fi], wl["spatial"], wl["sigma_s"] or 1.0, W, wl["range_kind"],
                                 wl["sigma_r"], T=wl["T"], pixels=pix)
            errs16.append(np.abs(out16[fi].ravel()[pix] - ref).max())
            errsd.append(np.abs(out16[fi].ravel()[pix] - dire).max())
            if out32 is not None:
                errs32.append(np.abs(out32[fi].ravel()[pix] - ref).max())
            if outb is not None:
                errsb.append(np.abs(outb[fi].ravel()[pix] - ref).max())
        extra["max_err_vs_fourier_fp64"] = float("%.4g" % max(errs16))
        extra["max_err_vs_direct_fp64"] = float("%.4g" % max(errsd))
        if errs32:
            extra["fp32_max_err_vs_fourier_fp64"] = float("%.4g" % max(errs32))
        if errsb:
            extra["bf16_max_err_vs_fourier_fp64"] = float("%.4g" % max(errsb))
            extra["bf16_meets_0p5"] = bool(max(errsb) < 0.5)
        extra["err_sample"] = "all pixels of %d rows of frames %s" % (len(rows), sorted({0, n - 1}))
        extra["meets_0p5"] = bool(max(errs16) < 0.5)

    # ---- CPU baseline: the FP64 oracle of eq. (9) on a bounded sample of frame 0
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        f0 = imgs[0]
        oracle.fourier(f0, wl["spatial"], wl["sigma_s"] or 1.0, W, d, wl["T"],
                       pixels=np.arange(Wd))  # warm (threads, page-in)
        t1 = time.time()
        oracle.fourier(f0, wl["spatial"], wl["sigma_s"] or 1.0, W, d, wl["T"], pixels=np.arange(2 * Wd))
        per_row = (time.time() - t1) / 2
        nrows = int(max(1, min(H, args.cpu_seconds / max(per_row, 1e-6))))
        r0 = (H - nrows) // 2
        pix = np.arange(r0 * Wd, (r0 + nrows) * Wd)
        t1 = time.time()
        oracle.fourier(f0, wl["spatial"], wl["sigma_s"] or 1.0, W, d, wl["T"], pixels=pix)
        dt = time.time() - t1
        cpu = {"value": round(pix.size / dt / 1e6, 4), "unit": "Mpix/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "eq. (9) in FP64 on %d full rows (%d px) of frame 0, %.1f s" % (nrows, pix.size, dt)}

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": args.workload, "frames": n, "height": H, "width": Wd,
                   "spatial": wl["spatial"], "sigma_s": wl["sigma_s"], "W": W,
                   "range": wl["range_kind"], "sigma_r": wl["sigma_r"], "T": wl["T"], "K": K,
                   "planes": args.precision, "accumulation": "fp32"},
        "roofline": roof, "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
