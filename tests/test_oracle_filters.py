"""Pins of the oracle's filters, smoothers, elements, operators and score.

* The sequential square-root KF/RTS (the algebra of Tables 1-2 and 4 applied
  as recursions) and the covariance KF/RTS equal a dense joint-Gaussian brute
  force over x_{0:n} (tests/bruteforce.py) for tiny n.
* Scalar random walk: the filter and smoother reach the closed-form Riccati
  steady state (q = r = 1 gives a smoothed variance of 1/sqrt(5)).
* The parallel-form elements (Tables 1, 2, 4) folded with the operators
  (Tables 3, 5) in any bracketing reproduce the brute-force marginals; the
  square-root operator's Grams equal the covariance operator (Table 3 left).
* Fisher-identity sensitivities equal central finite differences of the
  log-likelihood.
"""
import math

import numpy as np
import pytest

from paper_2207_00426_amd import workloads as wl
from tests import bruteforce as bf

CASES = [(1, 1, 5), (2, 1, 4), (3, 2, 6), (4, 2, 5), (5, 2, 6), (2, 3, 4), (3, 3, 3)]


def _model(nx, ny, n, seed, per_step=True):
    rng = np.random.default_rng(seed)
    G, m0, N0 = wl.random_linear_model(nx, ny, rng, n if per_step else None)
    y = wl.simulate_linear(G, m0, N0, n, rng)
    return G, m0, N0, y


def _cov(G):
    SL = np.asarray(G["SL"])
    SO = np.asarray(G["SO"])
    return dict(F=G["F"], c=G["c"], Lam=SL @ np.swapaxes(SL, -1, -2), H=G["H"], d=G["d"],
                Om=SO @ np.swapaxes(SO, -1, -2))


def _gram(N):
    return N @ np.swapaxes(N, -1, -2)


@pytest.mark.parametrize("nx,ny,n", CASES)
@pytest.mark.parametrize("per_step", [True, False])
def test_filters_and_smoothers_match_bruteforce(orc, nx, ny, n, per_step):
    G, m0, N0, y = _model(nx, ny, n, 10 * nx + ny + n, per_step)
    mf_b, Pf_b, ms_b, Ps_b, ll_b = bf.filter_smoother_loglik(m0, N0, G, y)
    mf, Nf, ell = orc.sqrt_filter(m0, N0, G, y)
    np.testing.assert_allclose(mf, mf_b, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(_gram(Nf), Pf_b, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(ell.sum(), ll_b, rtol=1e-11)
    ms, Ns, _ = orc.sqrt_smoother(G, mf, Nf)
    np.testing.assert_allclose(ms, ms_b, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(_gram(Ns), Ps_b, rtol=1e-9, atol=1e-10)
    Gc = _cov(G)
    mf2, Pf2, _, _, ell2 = orc.cov_filter(m0, N0 @ N0.T, Gc, y)
    np.testing.assert_allclose(mf2, mf_b, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(Pf2, Pf_b, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(ell2, ell, rtol=1e-10, atol=1e-12)
    ms2, Ps2, _ = orc.cov_smoother(Gc, mf2, Pf2)
    np.testing.assert_allclose(ms2, ms_b, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(Ps2, Ps_b, rtol=1e-9, atol=1e-10)


def test_scalar_random_walk_riccati_steady_state(orc):
    for q, r in [(1.0, 1.0), (0.3, 2.0), (4.0, 0.5)]:
        n = 400
        G = dict(F=np.eye(1), c=np.zeros(1), SL=np.sqrt(q) * np.eye(1), H=np.eye(1), d=np.zeros(1),
                 SO=np.sqrt(r) * np.eye(1))
        y = np.random.default_rng(1).standard_normal((n, 1))
        mf, Nf, _ = orc.sqrt_filter(np.zeros(1), np.eye(1), G, y)
        ms, Ns, _ = orc.sqrt_smoother(G, mf, Nf)
        Pm = (q + math.sqrt(q * q + 4 * q * r)) / 2
        Pf = Pm * r / (Pm + r)
        Ps = Pf / (1 + Pf / Pm)
        assert abs(Nf[n // 2, 0, 0] ** 2 - Pf) < 1e-12
        assert abs(Ns[n // 2, 0, 0] ** 2 - Ps) < 1e-12
        if q == 1.0 and r == 1.0:
            assert abs(Ns[n // 2, 0, 0] ** 2 - 1 / math.sqrt(5)) < 1e-12


def _fold(elems, op, order):
    """Combine a list of elements under a bracketing: 'left', 'right' or 'tree'."""
    if order == "left":
        acc = elems[0]
        for e in elems[1:]:
            acc = op(acc, e)
        return acc
    if order == "right":
        acc = elems[-1]
        for e in reversed(elems[:-1]):
            acc = op(e, acc)
        return acc
    if len(elems) == 1:
        return elems[0]
    h = len(elems) // 2
    return op(_fold(elems[:h], op, "tree"), _fold(elems[h:], op, "tree"))


@pytest.mark.parametrize("nx,ny,n", CASES)
def test_parallel_filter_elements_reproduce_marginals(orc, nx, ny, n):
    G, m0, N0, y = _model(nx, ny, n, 7 * nx + 3 * ny + n)
    mf_b, Pf_b, ms_b, Ps_b, _ = bf.filter_smoother_loglik(m0, N0, G, y)
    el = orc.filter_elements(m0, N0, G, y)
    for k in range(1, n + 1):
        for order in ("left", "right", "tree"):
            A, b, U, eta, Z = _fold(el[:k], orc.filter_combine, order)
            np.testing.assert_allclose(A, 0.0, atol=1e-12)
            np.testing.assert_allclose(b, mf_b[k], rtol=1e-9, atol=1e-10)
            np.testing.assert_allclose(U @ U.T, Pf_b[k], rtol=1e-9, atol=1e-10)
    # smoother: a_k (x) a_{k+1} (x) ... (x) a_n gives p(x_k | y_{1:n})
    mf, Nf, _ = orc.sqrt_filter(m0, N0, G, y)
    sel = orc.smoother_elements(G, mf, Nf)
    for k in range(n + 1):
        for order in ("left", "right", "tree"):
            E, g, D = _fold(sel[k:], orc.smoother_combine, order)
            np.testing.assert_allclose(E, 0.0, atol=1e-12)
            np.testing.assert_allclose(g, ms_b[k], rtol=1e-9, atol=1e-10)
            np.testing.assert_allclose(D @ D.T, Ps_b[k], rtol=1e-9, atol=1e-10)


def _rand_elem(rng, nx, full=True):
    A = rng.standard_normal((nx, nx)) * 0.5
    b = rng.standard_normal(nx)
    U = np.tril(rng.standard_normal((nx, nx))) * 0.5
    eta = rng.standard_normal(nx)
    Z = np.tril(rng.standard_normal((nx, nx))) * 0.5
    if not full:
        Z[:, 1:] = 0.0  # rank-deficient information factor, as in a leaf
    return A, b, U, eta, Z


@pytest.mark.parametrize("nx", [1, 2, 4, 5, 7])
def test_sqrt_operator_grams_equal_covariance_operator(orc, nx):
    rng = np.random.default_rng(nx)
    for full in (True, False):
        ei = _rand_elem(rng, nx, full)
        ej = _rand_elem(rng, nx, full)
        A, b, U, eta, Z = orc.filter_combine(ei, ej)
        ci = (ei[0], ei[1], _gram(ei[2]), ei[3], _gram(ei[4]))
        cj = (ej[0], ej[1], _gram(ej[2]), ej[3], _gram(ej[4]))
        A2, b2, C2, eta2, J2 = orc.filter_combine_cov(ci, cj)
        np.testing.assert_allclose(A, A2, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(b, b2, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(U @ U.T, C2, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(eta, eta2, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(Z @ Z.T, J2, rtol=1e-10, atol=1e-12)
        assert np.allclose(np.triu(U, 1), 0.0) and np.allclose(np.triu(Z, 1), 0.0)


@pytest.mark.parametrize("nx", [2, 5])
def test_operators_associative_with_identity(orc, nx):
    rng = np.random.default_rng(100 + nx)
    a, b, c = (_rand_elem(rng, nx) for _ in range(3))
    l = orc.filter_combine(orc.filter_combine(a, b), c)
    r = orc.filter_combine(a, orc.filter_combine(b, c))
    for i in (0, 1, 3):
        np.testing.assert_allclose(l[i], r[i], rtol=1e-9, atol=1e-11)
    for i in (2, 4):
        np.testing.assert_allclose(_gram(l[i]), _gram(r[i]), rtol=1e-9, atol=1e-11)
    e = (np.eye(nx), np.zeros(nx), np.zeros((nx, nx)), np.zeros(nx), np.zeros((nx, nx)))
    for x in (orc.filter_combine(e, a), orc.filter_combine(a, e)):
        np.testing.assert_allclose(x[0], a[0], atol=1e-13)
        np.testing.assert_allclose(x[1], a[1], atol=1e-13)
        np.testing.assert_allclose(_gram(x[2]), _gram(a[2]), atol=1e-13)
        np.testing.assert_allclose(x[3], a[3], atol=1e-13)
        np.testing.assert_allclose(_gram(x[4]), _gram(a[4]), atol=1e-13)
    s = [(rng.standard_normal((nx, nx)) * 0.5, rng.standard_normal(nx),
          np.tril(rng.standard_normal((nx, nx)))) for _ in range(3)]
    l = orc.smoother_combine(orc.smoother_combine(s[0], s[1]), s[2])
    r = orc.smoother_combine(s[0], orc.smoother_combine(s[1], s[2]))
    np.testing.assert_allclose(l[0], r[0], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(l[1], r[1], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(_gram(l[2]), _gram(r[2]), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("nx,ny,n", [(2, 1, 5), (4, 2, 6), (5, 2, 4)])
def test_fisher_sensitivities_equal_finite_differences(orc, nx, ny, n):
    G, m0, N0, y = _model(nx, ny, n, 55 + nx)
    Gc = _cov(G)
    rng = np.random.default_rng(9)
    # theta acts through Lam_j(t) = Lam_j + t1 V1_j and Om_j(t) = Om_j + t2 V2_j
    V1 = [(lambda X: X @ X.T)(rng.standard_normal((nx, nx))) * 0.1 for _ in range(n)]
    V2 = [(lambda X: X @ X.T)(rng.standard_normal((ny, ny))) * 0.1 for _ in range(n)]

    def ll(t1, t2):
        g = dict(Gc)
        g["Lam"] = np.stack([Gc["Lam"][j] + t1 * V1[j] for j in range(n)])
        g["Om"] = np.stack([Gc["Om"][j] + t2 * V2[j] for j in range(n)])
        return orc.cov_filter(m0, N0 @ N0.T, g, y)[4].sum()

    tot, Lb, Ob = orc.lgssm_score_terms(m0, N0 @ N0.T, Gc, y)
    np.testing.assert_allclose(tot, ll(0.0, 0.0), rtol=1e-12)
    g1 = sum(np.sum(Lb[j] * V1[j]) for j in range(n))
    g2 = sum(np.sum(Ob[j] * V2[j]) for j in range(n))
    h = 1e-5
    fd1 = (ll(h, 0.0) - ll(-h, 0.0)) / (2 * h)
    fd2 = (ll(0.0, h) - ll(0.0, -h)) / (2 * h)
    np.testing.assert_allclose(g1, fd1, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(g2, fd2, rtol=1e-6, atol=1e-8)
    for j in range(n):  # symmetric sensitivities
        np.testing.assert_allclose(Lb[j], Lb[j].T, atol=1e-10)
