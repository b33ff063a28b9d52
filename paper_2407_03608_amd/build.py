"""Build libgpnufft.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2407_03608_amd.build   (or call build()).
Each translation unit under csrc/ is compiled in parallel, then linked.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgpnufft.so")
# (source, object, extra flags): gp_mode.hip is built once per precision
SOURCES = [
    ("gp_fft.hip", "gp_fft.o", []),
    ("gp_plan.hip", "gp_plan.o", []),
    ("gp_nufft.hip", "gp_nufft.o", []),
    ("gp_spread.hip", "gp_spread.o", []),
    ("gp_mode.hip", "gp_mode64.o", ["-DGP_MODE_FP64=1"]),
    ("gp_mode.hip", "gp_mode32.o", ["-DGP_MODE_FP64=0"]),
    ("gp_cg.hip", "gp_cg.o", []),
    ("gp_capi.hip", "gp_capi.o", []),
    ("gp_serve.hip", "gp_serve.o", []),
    ("gp_noalloc.hip", "gp_noalloc.o", []),
    ("gp_rules.cpp", "gp_rules.o", []),
]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("GP_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed fp32 instructions stay off (known-bad forms on this hardware)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _compile(job) -> str:
    src, objname, extra = job
    obj = os.path.join(OBJ, objname)
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
