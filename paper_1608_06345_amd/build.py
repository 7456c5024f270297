"""Build the HIP libraries (gfx950) in-tree with hipcc.

liblbm.so     the solver library behind include/lbm.h.
libhbmprobe.so  the bench's HBM ceiling probes (a streaming copy and a
              read-only sweep of known size); not part of the solver.

Each source compiles to its own object in parallel (no device code crosses
translation units), then the objects are linked.

Usage: python -m paper_1608_06345_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liblbm.so")
PROBE_LIB = os.path.join(HERE, "libhbmprobe.so")
SOURCES = ["kernels.hip", "fd.hip", "api.hip", "pool.hip", "noalloc.hip", "lattice.cpp"]
PROBE_SOURCES = ["hbm_probe.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _up_to_date(src, obj):
    """The object is newer than its source and every header it may include."""
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + \
        [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(src, extra_flags, verbose, incremental=False):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if incremental and not extra_flags and _up_to_date(src, obj):
        return obj
    cmd = [HIPCC] + FLAGS + list(extra_flags) + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-FP32 feature and says so
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if out.strip():
        print(out, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)
    return obj


def _link(objs, target, verbose):
    tmp = target + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, target)
    return target


def build(verbose=False, extra_flags=(), incremental=False):
    """Compile every source (incremental: only those whose object is older
    than the source or a header) and link both libraries."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES + PROBE_SOURCES]
    with ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra_flags, verbose, incremental), srcs))
    _link(objs[:len(SOURCES)], LIB, verbose)
    _link(objs[len(SOURCES):], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    args = sys.argv[1:]
    inc = "--incremental" in args
    build(verbose=True, extra_flags=[a for a in args if a != "--incremental"], incremental=inc)
