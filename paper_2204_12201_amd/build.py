"""Compile the HIP library (csrc/*.hip) for gfx950 into libfhe.so, in-tree.

    python -m paper_2204_12201_amd.build

Each translation unit is compiled in parallel with hipcc, then linked into a
shared library next to this file.  Packed-FP32 instructions are disabled for
the device code (the feature flag is ignored by the host pass).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfhe.so")
CALIB_SRC = os.path.join(HERE, "calib", "valu_calib.cpp")
CALIB_BIN = os.path.join(HERE, "calib", "valu_calib")
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC,
]

SOURCES = ["host.hip", "kernels_conv.hip", "kernels_ntt.hip", "kernels_lin.hip", "kernels_mfma.hip"]

# Per-source device flags: the base conversions and the weighted sums on the
# matrix cores keep their int32 sums in ordinary VGPRs (no accumulator-register
# copies).
EXTRA = {
    "kernels_conv.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "kernels_lin.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    # roofline calibration probe (a separate executable, not part of the library)
    cmd = [HIPCC, *CFLAGS, "-x", "hip", CALIB_SRC, "-o", CALIB_BIN]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"calibration probe build failed:\n{r.stderr[-4000:]}")
    if verbose:
        print(f"built {LIB} and {CALIB_BIN}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
