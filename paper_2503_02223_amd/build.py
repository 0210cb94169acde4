"""Builds libdqo.so (all HIP sources in csrc/) for gfx950 with hipcc, in-tree.

Each source is compiled to an object of its own, in parallel (the kernels of
one source call no device code of another), then the objects are linked."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdqo.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "project.hip", "sort.hip", "render.hip", "loss.hip", "adam.hip", "quadric.hip",
           "net.hip", "init.hip", "learned_api.hip", "incremental.hip", "refine.hip", "assoc.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # no packed-FP32 instructions (v_pk_*_f32) anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _jobs():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n, len(SOURCES)))


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(OBJ, src.replace(".hip", ".o"))
        cmd = ["hipcc", *FLAGS, *extra, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, res

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = False
    for src, _, res in results:
        out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
        if out.strip() and (verbose or res.returncode):
            print(out, file=sys.stderr, flush=True)
        if res.returncode:
            print(f"compiling {src} failed", file=sys.stderr, flush=True)
            failed = True
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc")
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + [o for _, o, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
