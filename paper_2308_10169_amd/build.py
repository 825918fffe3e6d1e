"""Build libsepso.so in-tree: hipcc for gfx950 (device + host objects), then a
plain shared-library link against the HIP runtime.

Packed-FP32 instruction selection is disabled (`-packed-fp32-ops`): hipcc
would otherwise emit v_pk_{add,mul,fma}_f32 from ordinary float code.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsepso.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(HERE, "..", "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


DEVICE_SOURCES = ("kernels.hip", "mlp.hip", "bf.hip", "philox.hip", "fitness.hip", "rng.h", "common.h", "kernels.h", "mlp.h")


def kernels_id() -> str:
    """First 64 bits of a SHA-256 over the device-code sources (keys the
    autotuner's tile cache to these sources)."""
    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return "0x" + h.hexdigest()[:16] + "ull"


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    objs = []
    kid = kernels_id()
    for src in ("kernels.hip", "mlp.hip", "bf.hip", "philox.hip", "fitness.hip", "api.cpp", "lin.cpp"):
        obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        cmd = [hipcc] + HIPFLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip"] + HIPFLAGS + [f"-DSEPSO_KERNELS_ID={kid}", "-c",
                                                     os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-o", tmp] + objs + ["-L", os.path.join(ROCM, "lib"), "-lamdhip64"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
