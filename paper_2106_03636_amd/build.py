"""Compile the HIP library (gfx950) in-tree: paper_2106_03636_amd/_tpctrack.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "tpc_track.hip")
SRC_REQUESTS = os.path.join(HERE, "csrc", "tpc_requests.hip")
SRC_SERVER = os.path.join(HERE, "csrc", "tpc_server.cpp")
SRC_COLLISIONS = os.path.join(HERE, "csrc", "tpc_collisions.hip")
SRC_CLUSTERIZE = os.path.join(HERE, "csrc", "tpc_clusterize.hip")
SRC_COMPRESS = os.path.join(HERE, "csrc", "tpc_compress.hip")
SRC_REFIT = os.path.join(HERE, "csrc", "tpc_refit.hip")
SRC_MERGE = os.path.join(HERE, "csrc", "tpc_merge.hip")
LIB = os.path.join(HERE, "_tpctrack.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-mcode-object-version=5",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp, SRC, SRC_REQUESTS, SRC_COLLISIONS, SRC_CLUSTERIZE, SRC_COMPRESS, SRC_REFIT, SRC_MERGE, SRC_SERVER, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
