"""Build libswgpu.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_0808_2109_amd.build            # build the library
    python -m paper_0808_2109_amd.build --check    # build and list exported symbols
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswgpu.so")
SOURCES = ["sw_kernels.hip", "sw_runtime.hip", "sw_autotune.hip", "sw_server.hip", "sw_noalloc.hip"]
ARCH = os.environ.get("SW_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-DSW_BUILD_LIBRARY",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libswgpu.so")
    os.replace(tmp, LIB)
    return LIB


def exported_symbols(path: str = LIB) -> list:
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    return sorted(line.split()[-1] for line in out.splitlines() if " T " in line)


if __name__ == "__main__":
    lib = build(verbose=True)
    print("built", lib)
    if "--check" in sys.argv:
        print("\n".join(s for s in exported_symbols(lib) if s.startswith("sw_")))
