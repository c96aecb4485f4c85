"""Build the HIP library ``libphoebe_gpu.so`` in-tree for gfx950.

    python -m paper_2111_14999_amd.build

Compiles every ``csrc/*.hip`` with hipcc to an object (in parallel, under
``_build/`` next to this file), then links them into one shared library next to
this file.  Packed FP32 instructions are disabled for all device code.
"""

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libphoebe_gpu.so")
OBJ_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("PHOEBE_GPU_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(16, n or (os.cpu_count() or 4)))


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    if not srcs:
        raise RuntimeError("no HIP sources")
    os.makedirs(OBJ_DIR, exist_ok=True)
    cc = hipcc()
    inc = ["-I", os.path.join(HERE, "csrc")]

    def compile_one(src):
        obj = os.path.join(OBJ_DIR, os.path.basename(src)[:-4] + ".o")
        cmd = [cc] + FLAGS + inc + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, res

    objs = []
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        for src, obj, res in ex.map(compile_one, srcs):
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
            warns = [l for l in res.stderr.splitlines() if "warning" in l and "packed-fp32-ops" not in l]
            if verbose and warns:
                sys.stderr.write("\n".join(warns) + "\n")
            objs.append(obj)
    tmp = LIB + ".tmp"
    # roctx: named ranges per entry point for tracing tools
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + [
        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
