"""Build libhsg.so in-tree with hipcc for gfx950.

Flags: -O3; no FMA contraction (every fused multiply-add in the kernels is
written explicitly); packed-FP32 instructions disabled; position independent.
"""

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhsg.so")
SOURCES = ["api.hip", "kernels.hip", "sweep_stream.hip", "sweep_stream_s0.hip", "sweep_stream_s1.hip",
           "sweep_stream_s2.hip", "sweep_stream_s3.hip", "tile_chain.hip", "resident.hip"]
ARCH = os.environ.get("HSG_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def source_id() -> str:
    """Hash of the kernel and host sources (and the build flags) of libhsg.so."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    with open(os.path.join(HERE, "..", "include", "hsg.h"), "rb") as f:
        h.update(f.read())
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()[:16]


FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link libhsg.so."""
    import concurrent.futures
    import tempfile
    tmp = LIB + ".tmp"
    bid = source_id()
    with tempfile.TemporaryDirectory(prefix="hsg_build_") as work:
        def compile_one(src):
            obj = os.path.join(work, src + ".o")
            cmd = [hipcc(), f"--offload-arch={ARCH}"] + [f for f in FLAGS if f != "-shared"] + [
                f'-DHSG_BUILD_ID="{bid}"', "-I", os.path.join(HERE, "..", "include"), "-c",
                os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            return obj
        jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
