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
PEAK_FP32_VECTOR_TFLOPS = 157.3   # 256 CUs x 2.4 GHz x 256 flop per clock (packed FMA)
PEAK_FP64_VECTOR_TFLOPS = 78.6    # 256 CUs x 2.4 GHz x 128 flop per clock


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def alg_flops_per_px(K, W, spatial="gaussian"):
    """Algorithmic flops per output pixel: the separable smoothing of the
    4K+1 planes (two passes of 2W+1 multiply-adds each for the Gaussian; for
    the box, whose passes are running sums, one add and one subtract per
    plane and pass) plus 16 per harmonic for the modulation ((f - c0) cos and
    (f - c0) sin, d_k cos and d_k sin) and the demodulation (two
    multiply-adds each into the numerator and the denominator)."""
    mod_demod = 16 * K
    if spatial == "box":
        return (4 * K + 1) * 2 * 2 + mod_demod
    return (4 * K + 1) * 2 * (2 * W + 1) * 2 + mod_demod


def issued_flops_per_px(K, W, tile_rows):
    """MFMA flops the 16-bit wave kernel issues per output pixel: each
    16 x 16 output block needs (NJ + NT - 1) / NJ row-pass steps of KS
    16x16x32 products per plane and KS column-pass products per plane,
    NT = max(2, ceil((16 + 2W) / 16)), KS = ceil(NT / 2), NJ = tile_rows / 16;
    4 planes per harmonic k >= 1, one plane for k = 0."""
    nt = max(2, (16 + 2 * W + 15) // 16)
    ks = (nt + 1) // 2
    nj = tile_rows // 16
    per_plane = ((nj + nt - 1) / nj * ks + ks) * 2 * 16 * 16 * 32 / 256.0
    return per_plane * (4 * K + 1)


# standalone HIP units that share no code with the filter kernels measured here
_OTHER_UNITS = ("bf_box.hip", "bf_noalloc.hip", "bf_range.hip", "bf_recursive.hip")


def kernel_sources_digest():
    """sha256 over the sources the filter kernels are compiled from (their HIP
    file and the headers it includes; byte counters taken on other sources no
    longer describe the kernel).  Host-only .cpp files and the standalone
    units of other operations are not part of it."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1603_08081_amd", "csrc")
    h = hashlib.sha256()
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".h", ".hip")) and fn not in _OTHER_UNITS:
            h.update(fn.encode())
            with open(os.path.join(csrc, fn), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, prec, frames, tile_rows):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a copy of known size),
    for the tile height the plan runs with; None when there is none for this
    workload, or the sources have changed since the counters were taken."""
    name = "%s_%s_%s.md" % ("wave_batched_kernel" if prec != "fp32" else "fused_batched_kernel", workload, prec)
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            ln = ln.strip().lstrip("- ")
            if ":" not in ln:
                continue
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    key = "traffic_bytes_per_launch[%d]" % tile_rows
    if vals.get("sources_sha256") != kernel_sources_digest() or vals.get("frames") != str(frames) or key not in vals:
        return None
    return float(vals[key])


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


def recursive_flops_per_px(K):
    """Recursions of the recursive-Gaussian path: per harmonic, four planes,
    two axes, a causal and an anti-causal fourth-order recursion of 8
    multiply-adds each (float64)."""
    return (K + 1) * 4 * 2 * 2 * 8 * 2


def recursive_bytes_per_px(K):
    """Bytes per pixel the recursive-Gaussian path moves to and from memory
    (before caches): per harmonic, the row pass reads f in both directions and
    writes, re-reads and rewrites four float32 planes (56), the column pass
    reads them in both directions, and f in both directions for each of the
    numerator and denominator shares (48); per group of four harmonics, the
    column pass writes the group's two float64 shares on the way down and
    reads and rewrites them on the way up (48), and the final sum reads them
    (16).  Plus the output."""
    groups = (K + 4) // 4
    return (K + 1) * (56 + 48) + groups * (48 + 16) + 4


def run_recursive(args):
    import torch

    import paper_1603_08081_amd as bfm  # noqa: F401
    from paper_1603_08081_amd import native
    from synth import WORKLOADS, workload_images
    wl = dict(WORKLOADS[args.workload])
    if args.sigma_s:
        wl["sigma_s"] = args.sigma_s
    img = workload_images(args.workload, limit=1)[0]
    H, Wd = img.shape
    src = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    out = torch.empty_like(src)
    job = native.Job(src, out, spatial="gaussian", sigma_s=wl["sigma_s"], W=0, range_kind=wl["range_kind"],
                     sigma_r=wl["sigma_r"], T=wl["T"], eps=wl["eps"], K_max=wl["K_max"], integer_input=True)
    K = len(native.bf_fit_coeffs(wl["range_kind"], wl["sigma_r"], wl["T"], wl["eps"], wl["K_max"])[1]) - 1
    n = native.bf_recursive_workspace_bytes(job)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        native.bf_filter_recursive(job, ws, n, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(args.steps):
        e0.record(stream)
        native.bf_filter_recursive(job, ws, n, stream=stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    px = H * Wd
    fl = recursive_flops_per_px(K) * px / (ms * 1e-3) / 1e12
    gbs = recursive_bytes_per_px(K) * px / (ms * 1e-3) / 1e9
    line = {"metric": "recursive_filter_throughput", "value": round(px / (ms * 1e-3) / 1e6, 1),
            "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "%s, first frame (%d x %d), recursive Gaussian sigma_s = %g, %s range "
                                   "sigma_r = %g, K = %d" % (args.workload, H, Wd, wl["sigma_s"],
                                                             wl["range_kind"], wl["sigma_r"], K)},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None,
                         "kernel": "rec_rows_kernel + rec_cols_kernel + rec_sum_kernel, 3 launches per step",
                         "bytes_per_px": recursive_bytes_per_px(K),
                         "fp64_tflops": round(fl, 2), "fp64_frac": round(fl / PEAK_FP64_VECTOR_TFLOPS, 4)}}
    if not args.no_check:
        import oracle.recursive as orec
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        d = native.bf_fit_coeffs(wl["range_kind"], wl["sigma_r"], wl["T"], wl["eps"], wl["K_max"])[1]
        ref = orec.fourier_recursive(img.astype(np.float64), wl["sigma_s"], d, wl["T"])
        line["max_err_vs_oracle_recursive_fp64"] = float("%.4g" % np.abs(got - ref).max())
        line["err_sample"] = "every pixel"
    print(json.dumps(line))


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
    ap.add_argument("--no-fp16-alongside", action="store_true",
                    help="mixed batches: skip the float16-plane comparison when timing another format")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the plan autotuner (bf_plan_tune)")
    ap.add_argument("--tune-cache", default=None,
                    help="file of remembered tuner choices: loaded before planning if it exists, "
                         "written after tuning")
    ap.add_argument("--eager", action="store_true",
                    help="launch the plan eagerly instead of replaying its HIP graph")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one plain elementwise copy (negation) of this many MiB of "
                         "float32, the known-size reference for HBM byte counters")
    ap.add_argument("--recursive", action="store_true",
                    help="instead of the headline line: bf_filter_recursive (Deriche's recursive "
                         "Gaussian as the spatial smoothing) on one frame of the workload")
    ap.add_argument("--sigma-s", type=float, default=None,
                    help="--recursive: spatial sigma instead of the workload's (above 21.3 the truncated "
                         "window W = ceil(3 sigma) exceeds the largest window of bf_filter, 64)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline line: the Tables 1-3 analogues (one JSON line per setting)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only (the path shards by whole images or by "
              "row stripes with W-row halos; no multi-GPU run is implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.sweep:
        run_sweep(args)
        return
    if args.recursive:
        run_recursive(args)
        return

    import torch

    import paper_1603_08081_amd as bfm  # noqa: F401
    from paper_1603_08081_amd import native
    from synth import WORKLOADS, batch_specs, range_table, workload_images

    wl = WORKLOADS[args.workload]
    t0 = time.time()
    imgs = workload_images(args.workload, limit=args.frames)
    n = len(imgs)
    uniform = "height" in wl
    log("generated %d images (%.1f Mpx) in %.1fs" % (n, sum(f.size for f in imgs) / 1e6, time.time() - t0))
    # per-image filter settings; coefficients from the library's own fit
    if uniform:
        params = [dict(spatial=wl["spatial"], sigma_s=wl["sigma_s"] or 1.0, W=wl["W"],
                       range_kind=wl["range_kind"], sigma_r=wl["sigma_r"]) for _ in range(n)]
    else:
        params = [dict(spatial=wl["spatial"], sigma_s=sp["sigma_s"], W=sp["W"], range_kind=sp["range_kind"],
                       sigma_r=sp["sigma_r"]) for sp in batch_specs(wl["n"], wl["seed"])[:n]]
    fits = {}
    t_fit = time.time()
    phi_table = range_table(wl["table"], wl["T"]) if "table" in wl else None
    for p in params:
        key = (p["range_kind"], p["sigma_r"])
        if key not in fits:
            fits[key] = native.bf_fit_coeffs(key[0], key[1], wl["T"], wl["eps"], wl["K_max"], phi_table=phi_table)[1]
        p["d"] = fits[key]
        p["K"] = len(p["d"]) - 1
    fit_ms = (time.time() - t_fit) * 1e3 / len(fits)
    dev = torch.device("cuda", 0)
    srcs = [torch.from_numpy(f).to(dev) for f in imgs]
    dst = [torch.empty_like(x) for x in srcs]
    px = sum(f.size for f in imgs)
    alg_flops = sum(alg_flops_per_px(p["K"], p["W"], p["spatial"]) * f.size for p, f in zip(params, imgs))
    all_box = all(p["spatial"] == "box" for p in params)

    def make_jobs(outs):
        return [native.Job(srcs[i], outs[i], spatial=p["spatial"], sigma_s=p["sigma_s"], W=p["W"],
                           range_kind=p["range_kind"], sigma_r=p["sigma_r"], T=wl["T"], d=p["d"],
                           integer_input=True) for i, p in enumerate(params)]

    stream = torch.cuda.current_stream()
    if args.tune_cache and os.path.exists(args.tune_cache):
        log("tune cache: %d entries from %s" % (native.bf_tune_load(args.tune_cache), args.tune_cache))

    plans = {}
    medians = {}

    def timed(prec, out, steps, warmup, use_graph=True):
        """Device time per step of one plan launch (graph replay by default)
        over all images; the plan (fits, job table upload, autotuning) is made
        once, outside the timed region."""
        plan = native.Plan(make_jobs(out), prec)
        nbytes = plan.workspace_bytes()
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        plan.upload(ws, nbytes, stream)
        if not args.no_tune:
            t0 = time.time()
            plan.tune(stream, reps=2)
            log("%s: tuned in %.2fs: %s" % (prec, time.time() - t0, plan.describe()["classes"]))
            if args.tune_cache:
                native.bf_tune_save(args.tune_cache)
        plans[prec] = plan.describe()
        for _ in range(warmup):
            plan.launch(stream, use_graph)
        torch.cuda.synchronize()
        # one event between consecutive steps: the total gives the mean, the
        # gaps give the per-step median
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        for i in range(steps):
            plan.launch(stream, use_graph)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        plan.destroy()
        per_step = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
        medians[prec] = per_step[steps // 2] if steps % 2 else 0.5 * (per_step[steps // 2 - 1] + per_step[steps // 2])
        return ev[0].elapsed_time(ev[steps]) / steps

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
    value = px / (ms * 1e-3) / 1e6
    log("%s planes: %.3f ms/step, %.1f Mpix/s (plan, graph replay)" % (args.precision, ms, value))

    extra = {"host_fit_ms_per_kernel": round(fit_ms, 3), "median_ms_per_step": round(medians[args.precision], 3)}
    ms_call = timed_call(args.precision, dst, max(2, args.steps // 2))
    log("%s planes: %.3f ms/step through bf_filter_batched" % (args.precision, ms_call))
    extra["batched_call_ms_per_step"] = round(ms_call, 3)
    outs = {args.precision: dst}
    if not args.no_bf16 and args.precision != "bf16":
        outs["bf16"] = [torch.empty_like(x) for x in srcs]
        msb = timed("bf16", outs["bf16"], args.steps, 1)
        vb = px / (msb * 1e-3) / 1e6
        log("bf16 planes: %.3f ms/step, %.1f Mpix/s" % (msb, vb))
        extra["bf16_value"] = round(vb, 1)
        extra["bf16_ms_per_step"] = round(msb, 3)
    if not args.no_fp32 and args.precision != "fp32":
        outs["fp32"] = [torch.empty_like(x) for x in srcs]
        ms32 = timed("fp32", outs["fp32"], max(2, args.steps // 4), 1)
        v32 = px / (ms32 * 1e-3) / 1e6
        log("fp32 planes: %.3f ms/step, %.1f Mpix/s" % (ms32, v32))
        extra["fp32_value"] = round(v32, 1)
        extra["fp32_ms_per_step"] = round(ms32, 3)
        extra["speedup_vs_fp32"] = round(value / v32, 3)
    if args.precision != "fp16" and not args.no_fp16_alongside:
        outs["fp16"] = [torch.empty_like(x) for x in srcs]
        ms16 = timed("fp16", outs["fp16"], args.steps, 1)
        extra["fp16_value"] = round(px / (ms16 * 1e-3) / 1e6, 1)
        extra["fp16_ms_per_step"] = round(ms16, 3)
        log("fp16 planes: %.3f ms/step, %.1f Mpix/s" % (ms16, extra["fp16_value"]))

    if args.calib_copy_mib > 0:
        a = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))
        del a, b

    # ---- roofline of the dominant kernel: with one kernel class (every image
    # with the same window class and kernel family) the plan is one launch per
    # step; with several, the launches share the step and the figure is their
    # average
    launches = len(plans[args.precision]["classes"])
    avg_launch_s = ms * 1e-3 / launches
    flops = alg_flops / launches   # algorithmic flops of one launch
    achieved = flops / avg_launch_s / 1e12
    # a box filter's algorithmic work is running sums on the vector ALUs: the
    # float32-plane box kernel runs them in float64 (priced against the fp64
    # vector peak); the 16-bit paths run the box as MFMA Toeplitz products
    # all the same (priced against the fp32 vector peak)
    main_family = max(plans[args.precision]["classes"], key=lambda c: c["items"])["family"]
    if all_box:
        peak = PEAK_FP64_VECTOR_TFLOPS if main_family == 3 else PEAK_FP32_VECTOR_TFLOPS
    else:
        peak = PEAK_TFLOPS[args.precision]
    fam = {1: "wave_batched_kernel", 2: "fused_batched_kernel", 0: "fused_batched_kernel (general phase)",
           3: "box_batched_kernel (float64 running sums)"}
    roof = {"bound": "alu" if all_box else "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": (measured_traffic(args.workload, args.precision, n,
                                         plans[args.precision]["classes"][0]["tile_rows"])
                        if launches == 1 else None),
            "kernel": fam[main_family] + (" (modulate + row/column running sums + demodulate + divide)"
                                          if main_family == 3 else
                                          " (modulate + row/column MFMA Toeplitz + demodulate + divide)"),
            "alg_flops_per_px": round(alg_flops / px, 1), "launches_per_step": launches,
            "plan": plans[args.precision]["classes"]}
    if launches == 1 and main_family == 1 and uniform:
        th = plans[args.precision]["classes"][0]["tile_rows"]
        ifl = issued_flops_per_px(params[0]["K"], params[0]["W"], th)
        roof["issued_flops_per_px"] = round(ifl, 1)
        roof["issued_frac"] = round(ifl * px / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[args.precision], 4)
    if roof["traffic"] is not None:
        roof["hbm_gbs"] = round(roof["traffic"] / avg_launch_s / 1e9, 1)
        roof["hbm_frac"] = round(roof["hbm_gbs"] / PEAK_HBM_GBS, 4)

    # ---- error against the FP64 oracle: every pixel of sampled rows (borders,
    # window edges, middle, seeded random) of the first and last image (and
    # two more for mixed batches)
    if not args.no_check:
        import oracle
        check = sorted({0, n - 1} if uniform else {0, n // 3, (2 * n) // 3, n - 1})
        errs = {k: [] for k in outs}
        errsd = []
        nrows = 0
        for fi in check:
            p = params[fi]
            H, Wd = imgs[fi].shape
            W = p["W"]
            rows = np.unique(np.array([0, 1, W - 1, W, H // 2, H - W - 1, H - 2, H - 1] +
                                      list(np.random.default_rng(fi).integers(0, H, 4))))
            nrows += len(rows)
            pix = (rows[:, None] * Wd + np.arange(Wd)[None, :]).ravel()
            ref = oracle.fourier(imgs[fi], p["spatial"], p["sigma_s"], W, p["d"], wl["T"], pixels=pix)
            dire = oracle.direct(imgs[fi], p["spatial"], p["sigma_s"], W, p["range_kind"], p["sigma_r"],
                                 T=wl["T"], table=phi_table, pixels=pix)
            for k, o in outs.items():
                got = o[fi].cpu().numpy().ravel()[pix]
                errs[k].append(float(np.abs(got - ref).max()))
                if k == args.precision:
                    errsd.append(float(np.abs(got - dire).max()))
        extra["max_err_vs_fourier_fp64"] = float("%.4g" % max(errs[args.precision]))
        extra["max_err_vs_direct_fp64"] = float("%.4g" % max(errsd))
        for k in outs:
            if k != args.precision:
                extra["%s_max_err_vs_fourier_fp64" % k] = float("%.4g" % max(errs[k]))
        if "bf16" in errs:
            extra["bf16_meets_0p5"] = bool(max(errs["bf16"]) < 0.5)
        extra["err_sample"] = "all pixels of %d rows of images %s" % (nrows, check)
        extra["meets_0p5"] = bool(max(errs[args.precision]) < 0.5)

    # ---- CPU baseline: the FP64 oracle of eq. (9) (all host threads) on a
    # bounded sample of the same workload: whole rows of image 0, then image
    # 1, ..., until about --cpu-seconds of work
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        def ora(i, pix):
            p = params[i]
            return oracle.fourier(imgs[i], p["spatial"], p["sigma_s"], p["W"], p["d"], wl["T"], pixels=pix)

        ora(0, np.arange(imgs[0].shape[1]))  # warm (threads, page-in)
        done_px, spent, used = 0, 0.0, []
        for i in range(n):
            Hi, Wi = imgs[i].shape
            t1 = time.time()
            ora(i, np.arange(2 * Wi))
            per_row = (time.time() - t1) / 2
            nr = int(max(1, min(Hi, (args.cpu_seconds - spent) / max(per_row, 1e-6))))
            pix = np.arange(((Hi - nr) // 2) * Wi, ((Hi - nr) // 2 + nr) * Wi)
            t1 = time.time()
            ora(i, pix)
            spent += time.time() - t1
            done_px += pix.size
            used.append("%d rows of image %d" % (nr, i))
            if spent >= args.cpu_seconds * 0.95:
                break
        # single-thread rate of the same oracle on the first rows of image 0
        nthreads = oracle.num_threads()
        prev = oracle.set_threads(1)
        W0 = imgs[0].shape[1]
        t1 = time.time()
        n1 = 0
        while time.time() - t1 < min(3.0, args.cpu_seconds / 5):
            ora(0, np.arange(n1 * W0, (n1 + 1) * W0))
            n1 += 1
        t_single = time.time() - t1
        oracle.set_threads(prev)
        cpu = {"value": round(done_px / spent / 1e6, 4), "unit": "Mpix/s", "cores": nthreads,
               "kind": "oracle", "cpu_model": cpu_model(),
               "single_thread_value": round(n1 * W0 / t_single / 1e6, 5),
               "sample": "eq. (9) in FP64 on %s (%d px), %.1f s; single thread: %d rows of image 0, %.1f s"
                         % (", ".join(used), done_px, spent, n1, t_single)}

    if uniform:
        H, Wd = imgs[0].shape
        config = {"workload": args.workload, "frames": n, "height": H, "width": Wd,
                  "spatial": wl["spatial"], "sigma_s": wl["sigma_s"], "W": wl["W"],
                  "range": wl.get("table", wl["range_kind"]), "sigma_r": wl["sigma_r"], "T": wl["T"],
                  "K": params[0]["K"],
                  "planes": args.precision, "accumulation": "fp32"}
    else:
        config = {"workload": args.workload, "images": n, "megapixels": round(px / 1e6, 2),
                  "sides": "round(exp U[ln 256, ln 4096]) each", "spatial": wl["spatial"],
                  "W": [min(p["W"] for p in params), max(p["W"] for p in params)],
                  "range": "gaussian or exponential per image",
                  "K": [min(p["K"] for p in params), max(p["K"] for p in params)], "T": wl["T"],
                  "eps": wl["eps"], "K_max": wl["K_max"], "planes": args.precision, "accumulation": "fp32"}
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic", "config": config,
        "roofline": roof, "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
