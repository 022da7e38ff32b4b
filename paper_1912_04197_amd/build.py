"""Builds libbhx.so (HIP, gfx950) in-tree from csrc/*.hip, and
libbhx_checked.so, the same library with the device-side invariant checks of
csrc/checks.h compiled in (-DBHX_CHECKS).

Usage: python -m paper_1912_04197_amd.build  (or call build()).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBS = {  # variant: (object directory, library, extra flags)
    "release": (os.path.join(ROOT, "_build", "bhx"), os.path.join(PKG, "libbhx.so"), []),
    "checked": (os.path.join(ROOT, "_build", "bhx_checked"), os.path.join(PKG, "libbhx_checked.so"),
                ["-DBHX_CHECKS=1"]),
}
LIB = LIBS["release"][1]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 VALU ops are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(job) -> str:
    src, obj_dir, extra = job
    obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compiles every csrc/*.hip for gfx950 and links libbhx.so and
    libbhx_checked.so; returns the path of libbhx.so."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = []
    for obj_dir, _, extra in LIBS.values():
        os.makedirs(obj_dir, exist_ok=True)
        jobs += [(src, obj_dir, extra) for src in srcs]
    workers = min(len(jobs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        objs = list(ex.map(_compile, jobs))
    for k, (obj_dir, lib, _) in enumerate(LIBS.values()):
        mine = objs[k * len(srcs):(k + 1) * len(srcs)]
        tmp = lib + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *mine]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
        if verbose:
            print(f"built {lib}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
