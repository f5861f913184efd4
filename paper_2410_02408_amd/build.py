"""Build libbjp.so (the HIP library) in-tree for gfx950, and
libbjp_calib.so (the benchmark's bandwidth references, calib/calib.hip).

    python -m paper_2410_02408_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "bjp.hip")
LIB = os.path.join(PKG, "libbjp.so")
CALIB_SRC = os.path.join(PKG, "calib", "calib.hip")
CALIB_LIB = os.path.join(PKG, "libbjp_calib.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def source_digest() -> str:
    """sha256 over the library sources and header (identifies a kernel build)."""
    import hashlib

    h = hashlib.sha256()
    files = [os.path.join(ROOT, "include", "bjp.h")]
    csrc = os.path.join(PKG, "csrc")
    files += [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def _hipcc(src: str, out: str, verbose: bool) -> str:
    tmp = out + ".tmp"
    res = subprocess.run([hipcc(), *HIPCC_FLAGS, "-o", tmp, src], capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    if verbose:
        sys.stdout.write(res.stdout)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Compile the library and the benchmark's calibration kernels (always
    recompiles)."""
    _hipcc(CALIB_SRC, CALIB_LIB, verbose)
    return _hipcc(SRC, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
