"""Pins of the oracle's general sigma-point rules and of the generalised SLR
(GSLR, Section 2.3 moments with the sigma-point forms of Section 4.3) on the
Ricker-Poisson model of Section 6.1, against facts independent of its code:

* each rule integrates the moments of N(0, I) it must (weights sum to one,
  zero mean, identity second moment; Gauss-Hermite of order p is exact to
  degree 2p - 1), and the unscented rule reduces to textbook rules in its
  special cases (kappa = 0: cubature; nx = 1, kappa = 2: 3-point
  Gauss-Hermite);
* the SLR of an affine map returns the map and the noise factor exactly;
* the residual form equals the printed Tria + DownDate form;
* on the Ricker model, a high-order Gauss-Hermite GSLR equals the closed
  forms of the lognormal moments (the E[V[y|x]] term of the Poisson counts
  included), the Taylor linearisation equals finite differences, every rule
  tends to the Taylor linearisation as the spread shrinks, and in one
  dimension the cubature regression residual vanishes;
* on the CT model, the rule path with the cubature rule reproduces the
  dedicated cubature code, and the unscented rule with kappa = 0 equals it.
"""
import math

import numpy as np
import pytest

from paper_2207_00426_amd import workloads as wl


def _dfact(k):
    return math.prod(range(k - 1, 0, -2)) if k > 0 else 1


RULES = [("cubature_rule", 1, {}), ("cubature_rule", 5, {}), ("unscented", 1, {}),
         ("unscented", 5, {}), ("unscented", 3, {"kappa": 0.5}),
         ("gauss_hermite", 1, {"gh_order": 7}), ("gauss_hermite", 2, {"gh_order": 4}),
         ("gauss_hermite", 5, {"gh_order": 3})]


@pytest.mark.parametrize("method,nx,kw", RULES)
def test_rules_integrate_gaussian_moments(orc, method, nx, kw):
    xi, w = orc.make_rule(method, nx, kw.get("kappa"), kw.get("gh_order"))
    assert np.all(w > 0)
    np.testing.assert_allclose(w.sum(), 1.0, rtol=1e-14)
    np.testing.assert_allclose(w @ xi, np.zeros(nx), atol=1e-14)
    np.testing.assert_allclose((xi * w[:, None]).T @ xi, np.eye(nx), atol=1e-13)
    if method == "gauss_hermite":
        p = kw["gh_order"]
        for k in range(2 * p):  # E[x^k] of N(0, 1): 0 for odd k, (k-1)!! for even
            exact = 0.0 if k % 2 else float(_dfact(k))
            scale = w @ np.abs(xi[:, 0]) ** k  # rounding of the sum
            np.testing.assert_allclose(w @ xi[:, 0] ** k, exact, rtol=1e-12, atol=1e-13 * scale)
        # degree 2p is not integrated exactly
        assert abs(w @ xi[:, 0] ** (2 * p) - _dfact(2 * p)) > 1e-6


def _as_set(xi, w):
    order = np.lexsort(xi.T[::-1])
    return xi[order], w[order]


def test_unscented_special_cases(orc):
    a = _as_set(*orc.rule_unscented(1, 2.0))
    b = _as_set(*orc.rule_gauss_hermite(1, 3))
    np.testing.assert_allclose(a[0], b[0], atol=1e-14)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-14)
    for nx in (1, 3, 5):
        a = _as_set(*orc.rule_unscented(nx, 0.0))
        b = _as_set(*orc.rule_cubature(nx))
        np.testing.assert_allclose(a[0], b[0], atol=1e-14)
        np.testing.assert_allclose(a[1], b[1], rtol=1e-14)


@pytest.mark.parametrize("method,nx,kw", RULES)
def test_slr_of_an_affine_map_is_exact(orc, method, nx, kw):
    rng = np.random.default_rng(nx + 7)
    nz = 2
    A = rng.standard_normal((nz, nx))
    bb = rng.standard_normal(nz)
    Sn = np.tril(rng.standard_normal((nz, nz)))
    Sn[np.diag_indices(nz)] = np.abs(Sn[np.diag_indices(nz)]) + 0.5
    m = rng.standard_normal(nx)
    N = np.tril(rng.standard_normal((nx, nx)))
    N[np.diag_indices(nx)] = np.abs(N[np.diag_indices(nx)]) + 0.3
    xi, w = orc.make_rule(method, nx, kw.get("kappa"), kw.get("gh_order"))
    for per_point in (False, True):
        if per_point:
            G, off, S = orc.slr_rule(xi, w, m, N, lambda x: A @ x + bb, Sg=lambda x: Sn)
        else:
            G, off, S = orc.slr_rule(xi, w, m, N, lambda x: A @ x + bb, Snoise=Sn)
        np.testing.assert_allclose(G, A, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(off, bb, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(S @ S.T, Sn @ Sn.T, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("method,kw", [("cubature_rule", {}), ("unscented", {}),
                                       ("gauss_hermite", {"gh_order": 3})])
def test_residual_form_equals_the_printed_downdate_form(orc, method, kw):
    prm = orc.ct_params()
    m = np.array([0.4, -0.2, 1.1, 0.3, 0.5])
    N = 0.3 * np.eye(5) + 0.05 * np.tril(np.ones((5, 5)), -1)
    xi, w = orc.make_rule(method, 5, kw.get("kappa"), kw.get("gh_order"))
    LQ = np.linalg.cholesky(orc.ct_Q(prm))
    y = orc.ct_h(prm, m)
    for g, Sn in ((lambda x: orc.ct_f(prm, x), LQ),
                  (lambda x: orc.ct_h(prm, x, y), prm[3] * np.eye(2))):
        G1, o1, S1 = orc.slr_rule(xi, w, m, N, g, Snoise=Sn)
        G2, o2, S2, bad = orc.slr_rule(xi, w, m, N, g, Snoise=Sn, literal=True)
        assert bad == 0
        np.testing.assert_allclose(G1, G2, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(o1, o2, rtol=1e-13, atol=1e-13)
        P1, P2 = S1 @ S1.T, S2 @ S2.T
        np.testing.assert_allclose(P1, P2, rtol=1e-7, atol=1e-9 * np.max(np.abs(P1)))


# ---------------------------------------------------------------------------
# Ricker-Poisson GSLR
# ---------------------------------------------------------------------------
def _closed_forms(prm, m, P):
    """GSLR of the Ricker model at N(m, P) from lognormal moments:
    mu = E[exp x] = exp(m + P/2), Cov(x, exp x) = P mu, V[exp x] = mu^2 (e^P - 1)."""
    a, b, Q = prm
    mu = math.exp(m + P / 2)
    F = 1.0 - mu
    c = (math.log(a) + m - mu) - F * m
    Lam = Q + mu * mu * (math.exp(P) - 1.0 - P)
    H = b * mu
    d = b * mu - H * m
    Om = b * mu + b * b * mu * mu * (math.exp(P) - 1.0 - P)  # E[V[y|x]] + V[E[y|x]] - H P H
    return F, c, Lam, H, d, Om


@pytest.mark.parametrize("m,s", [(-3.0, 0.1), (0.5, 0.5), (2.0, 1.0), (1.2, 0.05)])
def test_ricker_gslr_matches_lognormal_closed_forms(orc, m, s):
    prm = orc.ricker_params()
    g = orc.ricker_linearize(prm, [m, m], [s, s], [0.0], method="gauss_hermite", gh_order=40)
    F, c, Lam, H, d, Om = _closed_forms(prm, m, s * s)
    got = (g["F"][0], g["c"][0], g["SL"][0] ** 2, g["H"][0], g["d"][0], g["SO"][0] ** 2)
    for name, v, ref in zip(("F", "c", "Lam", "H", "d", "Om"), got, (F, c, Lam, H, d, Om)):
        assert abs(v - ref) <= 1e-10 * max(1.0, abs(ref)), (name, v, ref)
    # without the E[V[y|x]] term Omega would miss b mu
    assert g["SO"][0] ** 2 > prm[1] * math.exp(m + s * s / 2) * (1 - 1e-12)


def test_ricker_taylor_is_the_jacobian(orc):
    prm = orc.ricker_params()
    ms = np.array([-2.0, 0.3, 1.7, 2.9])
    g = orc.ricker_linearize(prm, ms, np.full(4, 0.2), np.zeros(3), method="taylor")
    h = 1e-6
    for j in range(3):
        m, m1 = ms[j], ms[j + 1]
        fd = (orc.ricker_f(prm, m + h) - orc.ricker_f(prm, m - h)) / (2 * h)
        np.testing.assert_allclose(g["F"][j], fd, rtol=1e-8, atol=1e-9)
        np.testing.assert_allclose(g["F"][j] * m + g["c"][j], orc.ricker_f(prm, m), rtol=1e-13)
        hd = prm[1] * (math.exp(m1 + h) - math.exp(m1 - h)) / (2 * h)
        np.testing.assert_allclose(g["H"][j], hd, rtol=1e-8)
        np.testing.assert_allclose(g["H"][j] * m1 + g["d"][j], prm[1] * math.exp(m1), rtol=1e-13)
        np.testing.assert_allclose(g["SO"][j] ** 2, prm[1] * math.exp(m1), rtol=1e-13)
        np.testing.assert_allclose(g["SL"][j] ** 2, prm[2], rtol=1e-13)


@pytest.mark.parametrize("method,kw", [("cubature", {}), ("unscented", {}),
                                       ("gauss_hermite", {"gh_order": 6})])
def test_ricker_rules_tend_to_taylor_as_the_spread_shrinks(orc, method, kw):
    prm = orc.ricker_params()
    ms = np.array([-1.0, 0.4, 2.2, 1.1])
    tay = orc.ricker_linearize(prm, ms, np.ones(4), np.zeros(3), method="taylor")
    errs = []
    for eps in (1e-2, 1e-3):
        g = orc.ricker_linearize(prm, ms, np.full(4, eps), np.zeros(3), method=method, **kw)
        e = max(np.max(np.abs(g[k] - tay[k]) / np.maximum(1.0, np.abs(tay[k])))
                for k in ("F", "c", "H", "d"))
        e = max(e, np.max(np.abs(g["SO"] ** 2 - tay["SO"] ** 2) / tay["SO"] ** 2),
                np.max(np.abs(g["SL"] ** 2 - tay["SL"] ** 2) / tay["SL"] ** 2))
        errs.append(e)
    assert errs[1] < 1e-4
    assert errs[1] < 0.02 * errs[0]  # O(eps^2)


def test_ricker_cubature_regression_residual_vanishes_in_one_dimension(orc):
    # two points determine the line: Lambda = Q and Omega = E[V[y|x]] exactly
    prm = orc.ricker_params()
    ms = np.array([0.3, -0.8, 2.4])
    Ns = np.array([0.4, 0.2, 0.7])
    g = orc.ricker_linearize(prm, ms, Ns, np.zeros(2), method="cubature")
    np.testing.assert_allclose(g["SL"], math.sqrt(prm[2]), rtol=1e-14)
    ev = prm[1] * 0.5 * (np.exp(ms[1:] + Ns[1:]) + np.exp(ms[1:] - Ns[1:]))
    np.testing.assert_allclose(g["SO"] ** 2, ev, rtol=1e-13)
    np.testing.assert_allclose(g["H"], prm[1] * 0.5 * (np.exp(ms[1:] + Ns[1:]) -
                                                      np.exp(ms[1:] - Ns[1:])) / Ns[1:],
                               rtol=1e-13)


def test_ricker_simulation_and_one_pass(orc):
    # the simulated counts follow the model's rate, and one pass from the
    # prior gives finite marginals with positive factors
    w = wl.ricker_single(400, seed=11)
    x = w.x_true[0].ravel()
    rate = 10.0 * np.exp(x[1:])
    z = (w.y.ravel() - rate) / np.sqrt(np.maximum(rate, 1e-12))
    assert abs(np.mean(z[rate > 5])) < 0.2 and 0.8 < np.std(z[rate > 5]) < 1.2
    r = orc.ricker_ipls(orc.ricker_params(), w.model.m0, math.sqrt(w.model.P0[0, 0]), w.y, 1)
    assert np.all(np.isfinite(r["ms"])) and np.all(r["Ns"] > 0)


# ---------------------------------------------------------------------------
# CT model through the rule path
# ---------------------------------------------------------------------------
def _ct_nominal(n, seed):
    rng = np.random.default_rng(seed)
    ms = np.array([0.5, -0.3, 1.0, 0.2, 0.4]) + 0.2 * rng.standard_normal((n + 1, 5))
    Ns = np.stack([0.2 * np.eye(5) + 0.03 * np.tril(rng.standard_normal((5, 5)), -1)
                   for _ in range(n + 1)])
    return ms, Ns


def test_ct_rule_path_reproduces_the_dedicated_cubature(orc):
    prm = orc.ct_params()
    ms, Ns = _ct_nominal(6, 2)
    y = np.stack([orc.ct_h(prm, ms[k + 1]) + 0.01 for k in range(6)])
    a = orc.ct_linearize(prm, ms, Ns, y, method="cubature")
    for meth, kw in (("cubature_rule", {}), ("unscented", {"kappa": 0.0})):
        b = orc.ct_linearize(prm, ms, Ns, y, method=meth, **kw)
        for k in ("F", "c", "H", "d"):
            np.testing.assert_allclose(b[k], a[k], rtol=1e-11, atol=1e-12)
        for k in ("SL", "SO"):
            Pa = a[k] @ np.swapaxes(a[k], -1, -2)
            Pb = b[k] @ np.swapaxes(b[k], -1, -2)
            np.testing.assert_allclose(Pb, Pa, rtol=1e-10, atol=1e-16)


def test_ct_gauss_hermite_tends_to_taylor(orc):
    prm = orc.ct_params()
    ms, _ = _ct_nominal(3, 4)
    y = np.stack([orc.ct_h(prm, ms[k + 1]) for k in range(3)])
    tay = orc.ct_linearize(prm, ms, np.repeat(np.eye(5)[None], 4, 0), y, method="taylor")
    errs = []
    for eps in (1e-2, 1e-3):
        g = orc.ct_linearize(prm, ms, np.repeat((eps * np.eye(5))[None], 4, 0), y,
                             method="gauss_hermite", gh_order=3)
        errs.append(max(np.max(np.abs(g[k] - tay[k])) for k in ("F", "c", "H", "d")))
    assert errs[1] < 1e-5 and errs[1] < 0.02 * errs[0]
