"""Build libfd.so (all HIP sources, gfx950) in-tree.

Usage: python -m paper_2312_13094_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfd.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled (some of their forms are unreliable on
# this hardware generation); the compiler still vectorises everything else.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


PER_RADIUS = "fd-build: one object per stencil radius"


def _jobs(src: str):
    """(source, extra flags, object) for one file; sources marked per-radius
    are compiled once per stencil radius 1..8."""
    with open(src) as f:
        head = f.read(200)
    base = os.path.join(BUILD, os.path.basename(src))
    if PER_RADIUS in head:
        return [(src, ["-DFD_RADIUS=%d" % r], base + ".r%d.o" % r) for r in range(1, 9)]
    return [(src, [], base + ".o")]


def _compile(job) -> str:
    src, extra, obj = job
    subprocess.check_call([HIPCC, *FLAGS, *extra, "-c", src, "-o", obj])
    return obj


def _headers_mtime() -> float:
    hs = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(HERE, "..", "include", "*.h"))
    return max((os.path.getmtime(h) for h in hs), default=0.0)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental: only objects older than their
    source or any header) and link libfd.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = [j for s in srcs for j in _jobs(s)]
    every = [j[2] for j in jobs]
    if incremental:
        hdr = _headers_mtime()
        jobs = [j for j in jobs if not os.path.exists(j[2]) or
                os.path.getmtime(j[2]) < max(os.path.getmtime(j[0]), hdr)]
    # big objects first so the pool stays busy
    jobs.sort(key=lambda j: 0 if j[1] else 1)
    workers = max(1, min(16, os.cpu_count() or 1, max(len(jobs), 1)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(_compile, jobs))
    objs = every
    for stale in glob.glob(os.path.join(BUILD, "*.o")):
        if stale not in objs:
            os.remove(stale)
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
