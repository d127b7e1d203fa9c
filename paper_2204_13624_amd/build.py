"""Build libcombo.so (HIP kernels + C-ABI) for gfx950 in-tree.

Usage: python -m paper_2204_13624_amd.build   (or build() from Python).
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libcombo.so")
BUILD_DIR = os.path.join(HERE, "_build")

# (source, defines): the FFT kernel file is compiled once per part, in parallel
SOURCES = [("fft_kernels.hip", ["-DCOMBO_PART=%d" % k]) for k in range(1, 7)] + [
    ("material_kernels.hip", []), ("dfmg_kernels.hip", []), ("boxels.hip", []), ("setup_kernels.hip", []),
    ("solver.hip", [])]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


def _compile(item):
    src, defs = item
    tag = "".join(d.split("=")[-1] for d in defs)
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + (("_" + tag) if tag else "") + ".o")
    cmd = [HIPCC] + FLAGS + defs + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


def build(verbose=False):
    """Compile every source and link libcombo.so next to this file."""
    if not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found at %s" % HIPCC)
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    shutil.move(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
