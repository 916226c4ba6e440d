"""Build of the in-tree HIP library liblbfd.so for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbfd.so")
SOURCES = [os.path.join(CSRC, "lbfd.hip")]
HEADERS = [os.path.join(CSRC, "lbfd_kernels.h"), os.path.join(CSRC, "lbfd_lattice_tables.h"),
           os.path.join(CSRC, "sg_conv.h"), os.path.join(ROOT, "include", "lbfd.h"),
           os.path.join(ROOT, "include", "lbfd_surrogate.h")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile the HIP sources for gfx950 into paper_2311_15242_amd/liblbfd.so."""
    cmd = [hipcc(), "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
           "-Wno-unused-result", "-Wno-unused-value",
           # no packed-FP32 (v_pk_*_f32) instructions are generated
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # FP32 division and square root use the hardware reciprocal and square
           # root (a few ulp) instead of the correctly rounded sequences; FP64 is unaffected
           "-fno-hip-fp32-correctly-rounded-divide-sqrt",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
