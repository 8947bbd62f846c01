"""Build libavs.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "avs_api.hip")
OUT = os.path.join(HERE, "libavs.so")
# host objects under AddressSanitizer and UndefinedBehaviorSanitizer, for
# the host-only tests on a machine without a GPU (never loaded on a GPU)
SAN_OUT = os.path.join(HERE, "libavs_san.so")
SAN_FLAGS = [
    "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Wl,-rpath,/opt/rocm/lib",
]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 ops are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-variable",
    "-Wl,-rpath,/opt/rocm/lib",
]


def build(verbose=False, out=None, defines=(), sanitize=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = out or (SAN_OUT if sanitize else OUT)
    tmp = out + ".tmp"
    cmd = [hipcc, *(SAN_FLAGS if sanitize else FLAGS), *[f"-D{d}" for d in defines], SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "-v"]
    out = next((a.split("=", 1)[1] for a in args if a.startswith("--out=")), None)
    defs = [a[2:] for a in args if a.startswith("-D")]
    build(verbose="-v" in sys.argv, out=out, defines=defs, sanitize="--sanitize" in args)
