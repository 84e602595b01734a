"""Pins of the oracle's first-order Taylor linearisation (Section 4.2, the
iterated extended smoother) of the coordinated-turn model, against things
independent of its formulas:

* the analytic Jacobians of f and h equal central finite differences of the
  model functions themselves (also at w = 0 and on both sides of the switch
  from the closed form to the series of d/dw sin(w dt)/w, (1 - cos(w dt))/w);
* the cubature SLR of Section 4.3 at a nominal with covariance eps^2 I tends
  to the Taylor linearisation (slopes to the Jacobians, offsets to
  f(m) - J m) as eps -> 0, with error O(eps^2): two independent codes;
* the noise factors are those of the model (Lambda = Q, Omega = R);
* the iterated extended smoother reaches a fixed point on CT data.
"""
import numpy as np
import pytest

from paper_2207_00426_amd import workloads as wl


def _fd(fun, x, h=1e-6):
    x = np.asarray(x, dtype=np.float64)
    cols = []
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = h
        cols.append((fun(x + e) - fun(x - e)) / (2 * h))
    return np.stack(cols, axis=1)


XS = [np.array([0.3, -0.7, 1.2, 0.4, 0.0]), np.array([2.0, 1.5, -0.8, 0.9, 0.3]),
      np.array([-1.0, 3.0, 0.5, -1.5, 5.0]), np.array([0.1, 0.2, 1.0, 0.0, -2.0]),
      np.array([0.4, 0.1, -0.3, 0.7, 1e-5])]


@pytest.mark.parametrize("x", XS)
def test_transition_jacobian_equals_finite_differences(orc, x):
    prm = orc.ct_params()
    J = orc.ct_jac_f(prm, x)
    Jfd = _fd(lambda z: orc.ct_f(prm, z), x)
    # central differences of O(1) values with h = 1e-6 carry ~1e-10 rounding
    np.testing.assert_allclose(J, Jfd, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("x", XS)
def test_bearing_jacobian_equals_finite_differences(orc, x):
    prm = orc.ct_params()
    J = orc.ct_jac_h(prm, x)
    Jfd = _fd(lambda z: orc.ct_h(prm, z), x)
    np.testing.assert_allclose(J, Jfd, rtol=1e-7, atol=1e-9)


def test_transition_jacobian_is_continuous_at_the_series_switch(orc):
    prm = orc.ct_params()
    dt = prm[0]
    x = np.array([0.0, 0.0, 1.3, -0.6, 0.0])
    # two points 2e-12 apart in a = w dt around |a| = 1e-3: the Jacobian moves
    # by ~1e-9 relative; a jump between the series and the closed form (the
    # truncated terms are ~1e-13 relative there) would show above that
    for s in (1.0, -1.0):
        lo, hi = x.copy(), x.copy()
        lo[4] = s * (1e-3 - 1e-12) / dt
        hi[4] = s * (1e-3 + 1e-12) / dt
        np.testing.assert_allclose(orc.ct_jac_f(prm, lo), orc.ct_jac_f(prm, hi), rtol=1e-8,
                                   atol=1e-14)


def test_cubature_slr_tends_to_taylor_as_covariance_shrinks(orc):
    prm = orc.ct_params()
    rng = np.random.default_rng(3)
    n = 4
    ms = np.stack([np.array([0.5, -0.3, 1.0, 0.2, 0.4]) + 0.1 * rng.standard_normal(5)
                   for _ in range(n + 1)])
    y = np.stack([orc.ct_h(prm, ms[k + 1]) for k in range(n)])
    tay = orc.ct_linearize(prm, ms, np.repeat(np.eye(5)[None], n + 1, axis=0), y, method="taylor")
    errs = []
    for eps in (1e-2, 1e-3):
        Ns = np.repeat((eps * np.eye(5))[None], n + 1, axis=0)
        cub = orc.ct_linearize(prm, ms, Ns, y)
        e = max(np.max(np.abs(cub["F"] - tay["F"])), np.max(np.abs(cub["H"] - tay["H"])),
                np.max(np.abs(cub["c"] - tay["c"])), np.max(np.abs(cub["d"] - tay["d"])))
        errs.append(e)
    assert errs[1] < 1e-5
    assert errs[1] < 0.02 * errs[0]  # ~ eps^2 (ratio 1e-2)


def test_taylor_noise_factors_are_the_model_noise(orc):
    prm = orc.ct_params()
    n = 3
    ms = np.tile(np.array([0.5, -0.3, 1.0, 0.2, 0.4]), (n + 1, 1))
    y = np.zeros((n, 2))
    lin = orc.ct_linearize(prm, ms, np.repeat(np.eye(5)[None], n + 1, axis=0), y, method="taylor")
    Q = orc.ct_Q(prm)
    for j in range(n):
        np.testing.assert_allclose(lin["SL"][j] @ lin["SL"][j].T, Q, rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(lin["SO"][j] @ lin["SO"][j].T, prm[3] ** 2 * np.eye(2),
                                   rtol=1e-12)
        # the linearisation reproduces the model at the expansion point
        np.testing.assert_allclose(lin["F"][j] @ ms[j] + lin["c"][j], orc.ct_f(prm, ms[j]),
                                   rtol=1e-12, atol=1e-14)


def test_iterated_extended_smoother_reaches_a_fixed_point(orc):
    w = wl.ct_single(300, seed=7)
    prm = orc.ct_params()
    r = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, 25, history=True, method="taylor")
    hm = r["hist_ms"]
    steps = [np.max(np.abs(hm[i + 1] - hm[i])) for i in range(len(hm) - 1)]
    # linear convergence (about x0.3 per pass here) down to round-off
    assert steps[-1] < 1e-9 * max(1.0, np.max(np.abs(hm[-1])))
    assert all(b < 0.6 * a for a, b in zip(steps[4:], steps[5:]))
