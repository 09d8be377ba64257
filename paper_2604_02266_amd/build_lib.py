"""Build libotfs.so (HIP, gfx950) in-tree with hipcc."""
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libotfs.so")
SOURCES = ["kernels.hip", "dzt.hip", "plan.cpp", "server.cpp"]
ARCH = os.environ.get("OTFS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 VALU ops stay off (compiler-generated v_pk_*_f32 are avoided)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I" + INCLUDE, "-I" + CSRC,
]


HEADERS = ["otfs_internal.h", "plan_internal.h"]


def source_sha(csrc: str = None, include: str = None) -> str:
    """SHA-256 (first 16 hex digits) over the library's sources and headers, in a fixed order:
    the stamp a build carries (otfs_build_info) and the loader compares."""
    csrc = csrc or CSRC
    include = include or INCLUDE
    h = hashlib.sha256()
    for p in [os.path.join(csrc, s) for s in SOURCES + HEADERS] + [os.path.join(include, "otfs.h")]:
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    stamp = ["OTFS_SOURCE_SHA=\"" + source_sha(CSRC) + "\"", "OTFS_BUILD_ARCH=\"" + ARCH + "\""]
    cmd = ([hipcc] + HIPCC_FLAGS + ["-D" + d for d in list(defines) + stamp] + srcs +
           ["-lpthread", "-o", tmp])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libotfs.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
