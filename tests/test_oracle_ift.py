"""Pins of the oracle's total derivative of the pseudo-log-likelihood at the
IPLS fixed point (the quantity of eq. implicity_function_theorem and
Algorithm 4), which the oracle takes from its definition by extrapolated
central differences:

* the chain rule: the total derivative equals the frozen-nominal score
  (computed by Fisher's identity, a different code path) plus the
  nominal-sensitivity term lhat(theta, n*(theta +- h)) differenced at fixed
  theta;
* the extrapolated differences agree across step sizes;
* the correction over the frozen-nominal score is not negligible on the CT
  model (so the GPU test of it is not vacuous).
"""
import numpy as np

from paper_2207_00426_amd import workloads as wl


def _case():
    w = wl.ct_single(400, seed=3)
    return w, np.eye(5)


def test_total_derivative_is_frozen_score_plus_nominal_term(orc):
    w, N0 = _case()
    prm = orc.ct_params()
    l0, g_tot, ms, Ns = orc.ct_score_total(prm, w.model.m0, N0, w.y)
    ll, g_fro = orc.ct_score(prm, w.model.m0, N0, w.y, ms, Ns)
    assert abs(ll - l0) < 1e-9 * abs(l0)
    th = np.log(prm[1:4])
    h = 1e-4
    nom = np.zeros(3)
    for j in range(3):
        vals = []
        for s in (1.0, -1.0, 2.0, -2.0):
            t = th.copy()
            t[j] += s * h
            r = orc.ct_ipls(orc.ct_theta_params(t, prm), w.model.m0, N0, w.y, 60)
            vals.append(orc.ct_loglik(prm, w.model.m0, N0, w.y, r["ms"], r["Ns"]))
        d1 = (vals[0] - vals[1]) / (2 * h)
        d2 = (vals[2] - vals[3]) / (4 * h)
        nom[j] = (4 * d1 - d2) / 3
    np.testing.assert_allclose(g_tot, g_fro + nom, rtol=0, atol=1e-6 * max(1, np.max(np.abs(g_tot))))


def test_extrapolated_differences_agree_across_step_sizes(orc):
    w, N0 = _case()
    prm = orc.ct_params()
    _, g1, _, _ = orc.ct_score_total(prm, w.model.m0, N0, w.y, h=1e-4)
    _, g2, _, _ = orc.ct_score_total(prm, w.model.m0, N0, w.y, h=4e-4)
    assert np.max(np.abs(g1 - g2)) < 1e-7 * max(1.0, np.max(np.abs(g1)))


def test_fixed_point_correction_is_visible(orc):
    w, N0 = _case()
    prm = orc.ct_params()
    _, g_tot, ms, Ns = orc.ct_score_total(prm, w.model.m0, N0, w.y)
    _, g_fro = orc.ct_score(prm, w.model.m0, N0, w.y, ms, Ns)
    assert np.max(np.abs(g_tot - g_fro)) > 1e-3 * max(1.0, np.max(np.abs(g_tot)))
