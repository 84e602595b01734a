"""Build the HIP library libpss.so for gfx950 (hipcc, in-tree).

Every (dtype, nx, ny) implementation is its own object, compiled in parallel
from csrc/inst.hip; csrc/api.hip holds the C ABI.  Output:
paper_2207_00426_amd/libpss.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpss.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

DIMS = [(1, 1), (2, 1), (2, 3), (3, 2), (3, 3), (4, 2), (5, 2)]
DTYPES = ["float", "double"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE,
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout[-8000:])
    return r.stdout


def _deps(src: str, seen=None) -> set:
    """The source and every file it reaches through #include "..." lines."""
    import re
    seen = set() if seen is None else seen
    if src in seen or not os.path.exists(src):
        return seen
    seen.add(src)
    for inc in re.findall(r'^#include "([^"]+)"', open(src).read(), flags=re.M):
        _deps(os.path.normpath(os.path.join(os.path.dirname(src), inc)), seen)
    return seen


def _stale(src: str, obj: str) -> bool:
    # a unit is rebuilt when its source or a header it includes is newer
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in _deps(src))


def build(jobs: int | None = None, verbose: bool = False, extra_flags=(),
          incremental: bool = False) -> str:
    """Compile every unit (incremental: only units older than a source) and
    link libpss.so."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    units = [(os.path.join(CSRC, "api.hip"), os.path.join(BUILD, "api.o"), []),
             (os.path.join(CSRC, "persistent.hip"), os.path.join(BUILD, "persistent.o"), []),
             (os.path.join(CSRC, "ift_api.hip"), os.path.join(BUILD, "ift_api.o"), []),
             (os.path.join(CSRC, "noalloc.hip"), os.path.join(BUILD, "noalloc.o"), [])]
    # the fixed-point gradient's dual-number passes: one unit per precision
    # and half (they are the slowest units to compile)
    for t in DTYPES:
        for src in ("ift", "ift_smoother"):
            units.append((os.path.join(CSRC, src + ".hip"),
                          os.path.join(BUILD, "%s_%s.o" % (src, t[0])), ["-DPSS_IFT_T=%s" % t]))
    for t in DTYPES:
        for nx, ny in DIMS:
            obj = os.path.join(BUILD, "inst_%s_%d_%d.o" % (t[0], nx, ny))
            units.append((os.path.join(CSRC, "inst.hip"), obj,
                          ["-DPSS_T=%s" % t, "-DPSS_NX=%d" % nx, "-DPSS_NY=%d" % ny]))

    def compile_one(u):
        src, obj, defs = u
        if incremental and not _stale(src, obj):
            return obj
        out = _run([HIPCC, *FLAGS, *extra_flags, *defs, "-c", src, "-o", obj])
        if verbose and out.strip():
            print(out)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, units))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
