"""Pin of the step-slot mapping of the oracle's linearisation.

Step slot j of a linearisation feeds step k = j + 1: its transition part is
the regression of x_k | x_{k-1} at the marginal of state k - 1 = j (the
transition SLR of Section 4.3 is taken around the previous state's
marginal, as eq. F-c-sigma-point-params states), and its measurement part
is the regression of y_k | x_k at the marginal of state k = j + 1.  Here
every state has its own random marginal, and each slot of
oracle.ct_linearize is recomputed from the oracle's single-marginal
primitives (the cubature SLR on model images at the sigma points, the
general rule SLR, the analytic Jacobians) at exactly those two marginals;
the slot-shifted alternatives are checked to differ, so an off-by-one in
either half of the mapping fails.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2207_00426_amd import workloads as wl

N_STEPS = 6


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(15)
    x, y = wl.simulate_ct(N_STEPS, rng)
    ms = x + 0.3 * rng.standard_normal(x.shape)
    Ns = np.tril(0.2 * rng.standard_normal((N_STEPS + 1, 5, 5)))
    for k in range(N_STEPS + 1):
        Ns[k][np.diag_indices(5)] = 0.2 + 0.5 * rng.random(5)
    return orc.ct_params(), ms, Ns, y


def gram(S):
    return S @ S.T


def _cubature(prm, m, N, g, Sn):
    Xp, Xm = orc.sigma_points(m, N)
    Zp = np.stack([g(x) for x in Xp])
    Zm = np.stack([g(x) for x in Xm])
    return orc.slr(m, N, Zp, Zm, Sn)


def _same(a, b):
    return np.allclose(a, b, rtol=1e-12, atol=1e-12)


def _check_slot(lin, j, trans, meas, method):
    F, c, SL = trans
    H, d, SO = meas
    ok_t = _same(lin["F"][j], F) and _same(lin["c"][j], c) and _same(gram(lin["SL"][j]), gram(SL))
    ok_m = _same(lin["H"][j], H) and _same(lin["d"][j], d) and _same(gram(lin["SO"][j]), gram(SO))
    return ok_t, ok_m


@pytest.mark.parametrize("method", ["cubature", "unscented", "taylor"])
def test_slot_j_uses_marginal_j_for_transition_and_j_plus_1_for_measurement(case, method):
    prm, ms, Ns, y = case
    lin = orc.ct_linearize(prm, ms, Ns, y, method=method, kappa=1.0)
    LQ = np.linalg.cholesky(orc.ct_Q(prm))
    SR = prm[3] * np.eye(2)

    def lin_at(kt, km, j):
        f = lambda x: orc.ct_f(prm, x)  # noqa: E731
        h = lambda x: orc.ct_h(prm, x, y[j])  # noqa: E731
        if method == "cubature":
            return _cubature(prm, ms[kt], Ns[kt], f, LQ), _cubature(prm, ms[km], Ns[km], h, SR)
        if method == "unscented":
            xi, w = orc.rule_unscented(5, 1.0)
            return (orc.slr_rule(xi, w, ms[kt], Ns[kt], f, Snoise=LQ),
                    orc.slr_rule(xi, w, ms[km], Ns[km], h, Snoise=SR))
        Ff = orc.ct_jac_f(prm, ms[kt])
        Hh = orc.ct_jac_h(prm, ms[km])
        return ((Ff, f(ms[kt]) - Ff @ ms[kt], LQ), (Hh, h(ms[km]) - Hh @ ms[km], SR))

    for j in range(N_STEPS):
        trans, meas = lin_at(j, j + 1, j)
        ok_t, ok_m = _check_slot(lin, j, trans, meas, method)
        assert ok_t, (method, j, "transition")
        assert ok_m, (method, j, "measurement")
        # the shifted readings are distinguishable on this case
        if j + 1 < N_STEPS + 1:
            trans2, meas2 = lin_at(j + 1, j, j)
            bad_t, bad_m = _check_slot(lin, j, trans2, meas2, method)
            assert not bad_t and not bad_m, (method, j)
