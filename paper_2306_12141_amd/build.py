"""Build librecoil.so in-tree with hipcc for gfx950 only."""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librecoil.so")
BUILD = os.path.join(HERE, "_build")

HOST_SOURCES = ["host/codec.cpp", "host/plan.cpp", "host/batch.cpp", "host/server.cpp", "host/staging.cpp"]
DEVICE_SOURCES = ["device/decode.hip", "device/batch.hip", "device/unpack.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall"]
# Device code: gfx950 only; packed FP32 instructions are switched off.
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src.replace("/", "_") + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, *COMMON, "-D__HIP_PLATFORM_AMD__", "-pthread", "-c", path, "-o", obj]
    subprocess.check_call(cmd)
    return obj


def sources():
    return HOST_SOURCES + DEVICE_SOURCES


def build(verbose: bool = False) -> str:
    """Compile every source and link librecoil.so next to this file."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-pthread", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
