"""The transition SLR forms each sigma point's image of the coordinated-turn
map as phi(m) plus a deviation, whose sin(w dt)/w part needs
sinc(x + d) - sinc(x) without cancellation (dsinc in device_ops.hpp).
tests/dsinc_check.cpp builds that device function for the host in FP32 and
FP64; here it is checked against the same difference evaluated in 60-digit
decimal arithmetic from the Taylor series of sin, on a grid that takes all
three of its branches (both arguments small; a small step from a larger x;
a large step)."""
import decimal
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

decimal.getcontext().prec = 60
D = decimal.Decimal


def _sinc(x):
    """sin(x)/x from its power series, exact to the context precision."""
    if x == 0:
        return D(1)
    s, t, k = D(0), D(1), 0
    x2 = x * x
    while True:
        s += t
        k += 1
        t = -t * x2 / ((2 * k) * (2 * k + 1))
        if abs(t) < D(10) ** -70:
            return s + t


def _ref(x, d):
    x, d = D(repr(x)), D(repr(d))
    return float(_sinc(x + d) - _sinc(x))


XS = [0.0, 1e-6, -3e-4, 4e-3, 0.02, -0.05, 0.1, 0.33, 0.49, -0.6, 1.0, 2.0, -3.0]
DS = [1e-9, -1e-6, 3e-5, -1e-3, 1e-2, -0.1, 0.4, 1.5]


def test_dsinc_matches_extended_precision_difference():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    pairs = [(x, d) for x in XS for d in DS]
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "dsinc_check")
        subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I" + os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "dsinc_check.cpp"), "-o", exe],
                       check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        inp = "".join("%r %r\n" % p for p in pairs)
        out = subprocess.run([exe], input=inp, check=True, stdout=subprocess.PIPE,
                             text=True).stdout.split("\n")
    worst = {"f32": 0.0, "f64": 0.0}
    for (x, d), line in zip(pairs, out):
        f32, f64 = (float(v) for v in line.split())
        # FP32 is fed the FP32-rounded arguments: compare with their exact
        # difference
        x32, d32 = float(np.float32(x)), float(np.float32(d))
        r64, r32 = _ref(x, d), _ref(x32, d32)
        e64 = abs(f64 - r64) / abs(r64)
        e32 = abs(f32 - r32) / abs(r32)
        worst["f64"] = max(worst["f64"], e64)
        worst["f32"] = max(worst["f32"], e32)
        assert e64 < 64 * 2.2e-16, (x, d, f64, r64)
        assert e32 < 64 * 1.2e-7, (x, d, f32, r32)
    print("dsinc worst relative error: FP32 %.2e, FP64 %.2e" % (worst["f32"], worst["f64"]))


def test_dsinc_of_zero_step_is_zero():
    # the rules' centre point (no offset) has an exactly zero deviation
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "dsinc_check")
        subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I" + os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "dsinc_check.cpp"), "-o", exe],
                       check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        out = subprocess.run([exe], input="0 0\n0.3 0\n2.5 0\n", check=True,
                             stdout=subprocess.PIPE, text=True).stdout.split()
    assert [float(v) for v in out] == [0.0] * 6
