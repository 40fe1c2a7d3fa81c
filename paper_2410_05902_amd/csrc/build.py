"""Builds libmbkk.so (the HIP library behind include/mbkk.h) for gfx950.

Every translation unit is compiled with hipcc for gfx950 only, with packed
FP32 instructions disabled, and linked into paper_2410_05902_amd/libmbkk.so.
Run directly (python -m paper_2410_05902_amd.csrc.build) or via
__graft_entry__.build().
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
OUT = os.path.join(PKG, "libmbkk.so")
BUILD_DIR = os.path.join(PKG, "_build")
SOURCES = ["kernels_prep.hip", "kernels_cross.hip", "kernels_score.hip", "kernels_gram.hip", "kernels_init.hip", "kernels_grad.hip",
           "microbench.hip",
           "kernels_metrics.hip", "kernels_dp.hip", "mbkk_host.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          # no packed FP32 (v_pk_*_f32) generation
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # the MFMA kernels' k-step loops must unroll fully (register-resident
          # fragments and accumulators are indexed by the loop counters)
          "-mllvm", "-pragma-unroll-threshold=1000000",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    # keep real warnings visible, drop the host pass note about the feature flag
    msg = "\n".join(l for l in (r.stderr or "").splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if msg:
        print(msg, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
