"""The operator flop counts bench.py uses for its roofline are reproducible:
tests/flop_count.cpp instantiates the library's register code on a counting
number type (host build with hipcc) and must print exactly bench.FLOPS."""
import os
import shutil
import subprocess
import tempfile

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def counted():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "flop_count")
        subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I" + os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "flop_count.cpp"), "-o", exe],
                       check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        out = subprocess.run([exe], check=True, stdout=subprocess.PIPE, text=True).stdout
    res = {}
    for line in out.split("\n"):
        if line.strip():
            name, fl, tr = line.split()
            res[name] = (int(fl), int(tr))
    return res


def test_bench_flop_constants_match_the_counting_harness():
    res = counted()
    assert {k: v[0] for k, v in res.items()} == bench.FLOPS
    assert res["slr_transition"][1] > 0 and res["slr_bearings"][1] > 0
