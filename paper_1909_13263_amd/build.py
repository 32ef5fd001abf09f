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
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC]
# Translation units of the library: the single-grid API and the batched server.
LIB_SOURCES = ("hjw.hip", "hjw_server.hip")


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(cand) or cand == "hipcc":
            return cand


def _run(cmd):
    subprocess.check_call(cmd)


def build_library(out: str = LIB) -> str:
    """Compile the library's translation units in parallel, then link them."""
    objs, procs = [], []
    for src in LIB_SOURCES:
        obj = out + "." + os.path.splitext(src)[0] + ".o"
        objs.append(obj)
        procs.append((subprocess.Popen([_hipcc(), f"--offload-arch={ARCH}", *COMMON, "-c",
                                        os.path.join(CSRC, src), "-o", obj]), src))
    failed = [src for p, src in procs if p.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    tmp = out + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", "-shared", *objs, "-o", tmp])
    os.replace(tmp, out)
    for obj in objs:
        os.remove(obj)
    return out


def build_emulator(out: str = EMU) -> str:
    tmp = out + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", "--offload-host-only", "-shared", *COMMON,
          os.path.join(CSRC, "hjw_emulate.hip"), "-o", tmp])
    os.replace(tmp, out)
    return out


C_EXAMPLE_SRC = os.path.join(ROOT, "tests", "c", "hjw_c_example.c")
C_EXAMPLE = os.path.join(ROOT, "tests", "c", "hjw_c_example")


def build_c_example(out: str = C_EXAMPLE) -> str:
    """The C program that drives the C ABI without Python (test support): plain C99,
    linked against libhjw.so (found next to the package through its run path) and the
    HIP runtime."""
    rocm = "/opt/rocm"
    tmp = out + ".tmp"
    _run(["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE,
          "-I", os.path.join(rocm, "include"), C_EXAMPLE_SRC, "-o", tmp,
          "-L", PKG, "-lhjw", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
          "-Wl,-rpath,$ORIGIN/../../paper_1909_13263_amd", "-Wl,-rpath," + os.path.join(rocm, "lib")])
    os.replace(tmp, out)
    return out


def build_all() -> None:
    build_library()
    build_emulator()
    build_c_example()


if __name__ == "__main__":
    build_all()
