"""Compile the HIP sources for gfx950 into in-tree shared libraries.

    python paper_2009_10917_amd/build.py

builds ``paper_2009_10917_amd/libbs.so`` (the streaming-operation library)
and ``bsgen/libbsgen.so`` (the device form of the seeded input generator).
Objects go to ``_build/``; every call recompiles.

Run it as a file (or load it by path): importing it through the package
would first load the library it is about to rebuild, which fails when the
library is missing or older than the header.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2009_10917_amd")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed-FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit fused multiply-adds; the kernels write the ones they want
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]

LIBS = {
    os.path.join(PKG, "libbs.so"): [
        os.path.join(PKG, "csrc", f)
        for f in ("bs_host.hip", "bs_stream.hip", "bs_mesh.hip", "bs_plan.hip", "bs_gs.hip", "bs_cg.hip", "bs_batch.hip",
                  "bs_elem.hip", "bs_prim.hip", "bs_order.hip")
    ],
    os.path.join(ROOT, "bsgen", "libbsgen.so"): [os.path.join(ROOT, "bsgen", "csrc", "bsgen.hip")],
}


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout + p.stderr)
    return p


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    _run([HIPCC, *COMMON, "-c", src, "-o", obj])
    return obj


def build(verbose=False):
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for lib in LIBS.values() for s in lib]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    for lib, lib_srcs in LIBS.items():
        tmp = lib + ".tmp"
        _run([HIPCC, *COMMON, "-shared", "-o", tmp, *[objs[s] for s in lib_srcs], "-ldl"])
        os.replace(tmp, lib)
        if verbose:
            print("built", os.path.relpath(lib, ROOT))
    return list(LIBS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
