"""Build libgsmi.so (hand-written HIP kernels for gfx950) in-tree with hipcc.

    python -m paper_2509_12138_amd.build          # build
    python -m paper_2509_12138_amd.build --force  # rebuild everything
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgsmi.so")

SOURCES = ["capi.hip", "project.hip", "binsort.hip", "raster.hip", "schedule.hip", "loss.hip", "adam.hip",
           "knn.hip", "mlp.hip", "density.hip", "peaks.hip"]

ARCH = os.environ.get("GSMI_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # hardware FP32 atomics (no CAS loops) for the rasteriser backward
    "-munsafe-fp-atomics",
    # no packed-FP32 instructions: write plain scalar/float2 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _sources():
    return [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _compile(src: str, force: bool) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    srcp = os.path.join(CSRC, src)
    deps = [srcp, os.path.join(CSRC, "gs_device.h"), os.path.join(INCLUDE, "gs.h"), __file__]
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= max(
            os.path.getmtime(d) for d in deps):
        return obj
    cmd = [HIPCC, *CFLAGS, "-c", srcp, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature; that warning is expected
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l
                     and "not a recognized feature" not in l and l.strip())
    if warn:
        sys.stderr.write(warn + "\n")
    return obj


def build(force: bool = False, verbose: bool = False) -> str:
    """Compile every kernel source for gfx950 and link libgsmi.so (always
    re-links; recompiles sources whose object is older than the source)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} sources for {ARCH}")
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
