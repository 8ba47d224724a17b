"""Build libslepian.so in-tree with hipcc for gfx950.

Each translation unit is compiled separately (in parallel) and then linked
into paper_1611_04950_amd/libslepian.so.  All device code is built with the
packed-FP32 instructions disabled (-Xclang -target-feature -Xclang
-packed-fp32-ops); hipcc's host pass warns that it does not know the feature,
which is harmless.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libslepian.so")

SOURCES = ["fft.hip", "fft2.hip", "eig.hip", "corr.hip", "corr_mfma.hip", "lsq.hip", "multiband.hip", "coeffs.hip", "factor.hip", "mbcg.hip",
           "capi.cpp",
           "trace.cpp"]
ARCH = os.environ.get("SLEPIAN_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # private arrays (register-staged loads) stay in registers rather than
    # being moved into LDS behind the kernel's back
    "-mllvm", "-disable-promote-alloca-to-lds",
    f"-I{INCLUDE}", f"-I{CSRC}",
    "-Wno-unused-result",
]


def source_digest() -> str:
    """Short hash of the library's sources (identifies which kernels a profile
    was taken with)."""
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-lrocsolver", "-lrocblas", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
