"""Builds ``libmg.so`` (the C-ABI multigrid library) in-tree with hipcc for gfx950.

Each source is compiled to an object of its own, in parallel, under
``_build/`` at the repository root, and the objects are linked into the
library.  Every call recompiles every source.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmg.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("flat_row.hip", "var_row.hip", "kernels.hip", "tail.hip",
                                                    "visit.hip", "pcg.hip", "readout.hip", "noalloc.hip",
                                                    "mg_api.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay disabled in every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + os.path.join(HERE, "csrc"),
]
LINK = ["--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-rpath,/opt/rocm/lib"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source into ``libmg.so`` (always recompiles)."""
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.basename(src) + ".o") for src in SOURCES]
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        rcs = list(ex.map(lambda so: _run([HIPCC] + FLAGS + ["-c", so[0], "-o", so[1]], verbose),
                          zip(SOURCES, objs)))
    if any(rcs):
        bad = [os.path.basename(s) for s, rc in zip(SOURCES, rcs) if rc]
        raise RuntimeError("hipcc failed on " + ", ".join(bad))
    tmp = LIB + ".tmp"
    if _run([HIPCC] + LINK + objs + ["-o", tmp], verbose):
        raise RuntimeError("hipcc failed linking libmg.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
