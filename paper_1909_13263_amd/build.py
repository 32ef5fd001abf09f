"""Build the HIP library (gfx950) and the CPU emulation library in-tree."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhjw.so")
EMU = os.path.join(PKG, "libhjw_emu.so")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC]


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(cand) or cand == "hipcc":
            return cand


def _run(cmd):
    subprocess.check_call(cmd)


def build_library(out: str = LIB) -> str:
    tmp = out + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", *COMMON, os.path.join(CSRC, "hjw.hip"), "-o", tmp])
    os.replace(tmp, out)
    return out


def build_emulator(out: str = EMU) -> str:
    tmp = out + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", "--offload-host-only", *COMMON,
          os.path.join(CSRC, "hjw_emulate.hip"), "-o", tmp])
    os.replace(tmp, out)
    return out


def build_all() -> None:
    build_library()
    build_emulator()


if __name__ == "__main__":
    build_all()
