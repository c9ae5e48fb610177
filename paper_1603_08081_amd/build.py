"""Build libbf.so (gfx950) in-tree with hipcc.

The fused kernel is instantiated once per (plane precision, window-tile
count) in its own object, compiled in parallel from csrc/bf_fused_inst.hip.

    python -m paper_1603_08081_amd.build [--force] [--jobs N] [--save-temps]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libbf.so")
ROOT = os.path.dirname(PKG)

PRECS = (0, 1, 2)          # bf_planes: fp32, fp16, bf16
NTS = tuple(range(2, 10))  # window tiles (W <= 64)
HOST_SRCS = ("bf_api.cpp", "bf_batch.cpp", "bf_fit.cpp", "bf_dispatch.cpp")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _units():
    units = []
    for s in HOST_SRCS:
        units.append((os.path.join(CSRC, s), os.path.join(BUILD, s.replace(".cpp", ".o")), []))
    units.append((os.path.join(CSRC, "bf_range.hip"), os.path.join(BUILD, "bf_range.o"), []))
    units.append((os.path.join(CSRC, "bf_recursive.hip"), os.path.join(BUILD, "bf_recursive.o"), []))
    units.append((os.path.join(CSRC, "bf_noalloc.hip"), os.path.join(BUILD, "bf_noalloc.o"), []))
    units.append((os.path.join(CSRC, "bf_box.hip"), os.path.join(BUILD, "bf_box.o"), []))
    for p in PRECS:
        for nt in NTS:
            units.append((os.path.join(CSRC, "bf_fused_inst.hip"),
                          os.path.join(BUILD, "bf_fused_p%d_nt%d.o" % (p, nt)),
                          ["-DBF_INST_PREC=%d" % p, "-DBF_INST_NT=%d" % nt]))
    return units


def _newest_header():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(ROOT, "include", "bf.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(unit, force, save_temps):
    src, obj, defs = unit
    if not force and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t >= os.path.getmtime(src) and t >= _newest_header():
            return obj, False
    cmd = [HIPCC] + COMMON + defs + ["-c", src, "-o", obj + ".tmp"]
    if save_temps:
        cmd += ["-save-temps=obj"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    msgs = [ln for ln in r.stdout.splitlines() if "is not a recognized feature" not in ln]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s %s:\n%s" % (src, " ".join(defs), "\n".join(msgs)))
    os.replace(obj + ".tmp", obj)
    return obj, True


def build(force: bool = False, jobs: int | None = None, save_temps: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or int(os.environ.get("MAX_JOBS", 0)) or os.cpu_count() or 8
    jobs = max(1, min(jobs, 16))
    units = _units()
    rebuilt = 0
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, did in ex.map(lambda u: _compile(u, force, save_temps), units):
            rebuilt += int(did)
    if rebuilt or force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [u[1] for u in units]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    if verbose:
        print("libbf: %d/%d objects rebuilt -> %s" % (rebuilt, len(units), LIB), file=sys.stderr)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--save-temps", action="store_true")
    a = ap.parse_args()
    build(force=a.force, jobs=a.jobs, save_temps=a.save_temps)
