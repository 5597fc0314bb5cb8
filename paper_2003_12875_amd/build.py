"""Build libnllmi.so for gfx950: hipcc for the device code, the host runtime
compiled as plain C++ against the HIP runtime API, linked by hipcc.

    python -m paper_2003_12875_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libnllmi.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

INCLUDES = ["-I", CSRC, "-I", os.path.join(ROOT, "include")]
# Packed FP32 instructions are disabled for all device code (never emitted).
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wall", "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
              "-I", os.path.join(ROCM, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the device-only target feature: harmless
    noise = ("packed-fp32-ops", "is not a recognized feature for this target")
    err = "\n".join(l for l in r.stderr.splitlines() if not any(n in l for n in noise))
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{err}")
    return err


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    units = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        units.append([HIPCC, *DEVICE_FLAGS, *INCLUDES, "-c", src, "-o", obj])
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        units.append(["g++", *HOST_FLAGS, *INCLUDES, "-c", src, "-o", obj])
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for msg in ex.map(_run, units):
            if verbose and msg:
                print(msg, file=sys.stderr)
    objs = [u[-1] for u in units]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp, "-lhiprtc"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
