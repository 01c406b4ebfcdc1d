"""Build the gfx950 shared library ``libboxscreen.so`` in-tree with hipcc.

Every HIP source is compiled to an object in its own hipcc process (in
parallel; the column-sweep variants are spread over several translation
units), then the objects are linked.  Objects go to a temporary directory, so
every call compiles everything."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libboxscreen.so")
CSRC = os.path.join(PKG, "csrc")


def sources() -> list[str]:
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


# Packed FP32 instructions are disabled for all device code.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _jobs() -> int:
    for k in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(k)
        if v and v.isdigit() and int(v) > 0:
            return min(int(v), 16)
    return min(os.cpu_count() or 4, 16)


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source of the library and link libboxscreen.so."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="bxs_build_") as tmpd:
        def compile_one(src: str):
            obj = os.path.join(tmpd, src[:-4] + ".o")
            cmd = [hipcc(), *HIPCC_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + res.stdout + res.stderr)
            return obj

        srcs = sources()
        # the largest units first
        srcs.sort(key=lambda s: (not s.startswith("sweep_"), s))
        with cf.ThreadPoolExecutor(max_workers=_jobs()) as ex:
            objs = list(ex.map(compile_one, srcs))
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
               "-Wl,-rpath,/opt/rocm/lib"]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
