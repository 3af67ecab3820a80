"""Build libgaca.so for gfx950 with hipcc (in-tree: paper_2312_11219_amd/libgaca.so).

Host sources are compiled with -ffp-contract=off so that geometric decisions (tree
median order, admissibility, quadrature tier) use plain IEEE operations; HIP sources are
compiled with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libgaca.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HOST_SRC = ["host.cpp", "lib.cpp", "gcq_host.cpp"]
HIP_SRC = ["near.hip", "far_aca.hip", "apply.hip", "apply_mfma.hip", "gcq.hip", "far_recompress.hip",
           "near_aca.hip"]
COMMON = ["-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I" + CSRC,
          "-I" + os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        flags = ["-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-munsafe-fp-atomics"]
    else:
        flags = ["-O2", "-ffp-contract=off"]
    cmd = [HIPCC] + COMMON + flags + ["-c", path, "-o", obj]
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = HOST_SRC + HIP_SRC
    with ThreadPoolExecutor(max_workers=min(4, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs,
                   check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
