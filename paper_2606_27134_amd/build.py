"""Build libdmkloc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2606_27134_amd.build

Every build compiles from source; the result is
paper_2606_27134_amd/libdmkloc.so, loaded by the ctypes binding.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdmkloc.so")
SOURCES = ["dmk_bin.hip", "dmk_residual.hip", "dmk_far.hip", "dmk_cheb.hip", "dmk_pswf.cpp", "dmk_noalloc.hip"]
ARCH = os.environ.get("DMK_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
        # packed FP32 VALU ops are kept out of the generated code on purpose
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # matrix-core products accumulate in ordinary vector registers (the
        # accumulation-register form made the compiler copy loop-carried
        # accumulators out and back on every iteration of the leaf-grid
        # anterpolation: 15-28 % slower there, no change elsewhere)
        "-mllvm", "-amdgpu-mfma-vgpr-form=1",
        "-I", os.path.join(ROOT, "include"),
    ]


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    objs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(ROOT, "_build", os.path.splitext(s)[0] + ".o")
        cmd = [hipcc()] + flags() + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (s, msg))
        if verbose and msg.strip():
            print(msg)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
