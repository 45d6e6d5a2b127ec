"""Build the HIP library (gfx950) in-tree: paper_1907_13088_amd/libmx.so.

Each source is compiled to an object in parallel, then linked.  Usage:
    python -m paper_1907_13088_amd.build [--force]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmx.so")
OBJ = os.path.join(HERE, "_build")
# the long compile units first, so that the parallel build finishes early
SOURCES = ["k2fs_k6.hip", "k2fs_k5.hip", "k2small_f64.hip", "k2small_f32.hip", "k2fs_k4.hip", "k2fs_k3.hip", "k2s_f32_tm.hip", "k2s_f32d_tm.hip", "k2s_f32_te.hip", "k2s_f32d_te.hip", "k2s_f32_all.hip",
           "k2s_f32d_all.hip", "k2s_f64_tm.hip", "k2s_f64d_tm.hip", "k2s_f64_te.hip", "k2s_f64d_te.hip",
           "k2s_f64_all.hip", "k2s_f64d_all.hip", "k2s_f32c_te.hip", "k2s_f32c_tm.hip", "k2s_f32c_all.hip",
           "k2s_f64c_te.hip", "k2s_f64c_tm.hip", "k2s_f64c_all.hip", "k2fs.hip", "k2d.hip", "k2f.hip", "kbatch_f32.hip", "kbatch_f64.hip",
           "k3s.hip", "k3d.hip", "k3f.hip", "kpic.hip", "kadj.hip", "k2s.hip", "mx_api.cpp", "mx_batch.cpp", "mx_static.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # packed FP32 VALU forms stay off: plain FP32 VALU only
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # no automatic contraction: FMAs are written out where intended, so
         # every schedule of the same stencil rounds identically
         "-ffp-contract=off",
         "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC, *FLAGS, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libmx.so (always rebuilds
    when force is set)."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    deps = [os.path.join(CSRC, s) for s in srcs] + [os.path.join(CSRC, h) for h in ("mx_internal.h", "k2s_impl.h", "k2f_impl.h", "k2fs_impl.h", "kbatch_impl.h", "stencil2d.h", "k2tile.h", "k2small_impl.h", "gridbar.h")] + [
                                                    os.path.join(HERE, "..", "include", "mx.h")]
    if not force and os.path.exists(OUT) and all(os.path.getmtime(OUT) >= os.path.getmtime(d) for d in deps):
        return OUT
    os.makedirs(OBJ, exist_ok=True)
    jobs = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(force="--no-force" not in sys.argv, verbose=True)
