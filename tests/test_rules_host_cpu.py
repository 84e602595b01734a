"""Host-side check of the library's Gauss-Hermite rule construction
(csrc/rules_host.hpp: Golub-Welsch with Jacobi rotations, Newton polish):
compiled with g++ on the CPU, its nodes and weights for every order the ABI
accepts (2..20) equal numpy's hermegauss (normalised to the probability
measure) and integrate the Gaussian moments up to degree 2p - 1."""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2207_00426_amd", "csrc", "rules_host.hpp")

PROG = r'''
#include <cstdio>
#include "%s"
int main() {
    for (int p = 2; p <= 20; ++p) {
        double x[20], w[20];
        pss::gauss_hermite_1d(p, x, w);
        printf("%%d", p);
        for (int i = 0; i < p; ++i) printf(" %%.17g %%.17g", x[i], w[i]);
        printf("\n");
    }
}
'''


@pytest.fixture(scope="module")
def rules():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "gh.cpp")
        exe = os.path.join(d, "gh")
        with open(src, "w") as fh:
            fh.write(PROG % HDR)
        subprocess.run(["g++", "-O2", "-std=c++17", src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        v = line.split()
        p = int(v[0])
        a = np.array(v[1:], dtype=float).reshape(p, 2)
        res[p] = (a[:, 0], a[:, 1])
    return res


def test_nodes_and_weights_equal_numpy(rules):
    for p, (x, w) in rules.items():
        xr, wr = np.polynomial.hermite_e.hermegauss(p)
        wr = wr / wr.sum()
        np.testing.assert_allclose(x, xr, rtol=0, atol=1e-13)
        np.testing.assert_allclose(w, wr, rtol=1e-12, atol=1e-300)


def test_rules_integrate_gaussian_moments(rules):
    for p, (x, w) in rules.items():
        for k in range(2 * p):
            exact = 0.0 if k % 2 else float(math.prod(range(k - 1, 0, -2)) if k else 1)
            scale = w @ np.abs(x) ** k
            assert abs(w @ x ** k - exact) <= 1e-12 * max(1.0, exact) + 1e-13 * scale, (p, k)
