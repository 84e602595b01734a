"""Pins of the oracle's iterated posterior linearisation, log-likelihood and score.

* Algorithm 3 is a fixed-point iteration: on the CT workload it converges and
  its limit satisfies n* = KS(n*) (the identity of Section 5.2).
* The downdate-free SLR and the paper's literal Tria + DownDate recipe give the
  same linearisation in FP64.
* The pseudo-log-likelihood of a linearised model equals the brute-force
  Gaussian log-density of the stacked measurements.
* The Fisher-identity score equals central finite differences (h = 1e-5) of the
  frozen-nominal pseudo-log-likelihood in theta = (log q1, log q2, log sigma).
* Batched entry points equal their single-sequence counterparts.
"""
import numpy as np
import pytest

from paper_2207_00426_amd import workloads as wl
from tests import bruteforce as bf


@pytest.fixture(scope="module")
def ct300():
    return wl.ct_single(300, 1)


def test_ipls_converges_to_a_fixed_point(orc, ct300):
    md = ct300.model
    prm = orc.ct_params()
    out = orc.ct_ipls(prm, md.m0, np.eye(5), ct300.y, 40, history=True)
    hm = out["hist_ms"]
    assert np.abs(hm[-1] - hm[-2]).max() < 1e-11
    # one more pass started from the limit returns it: n* = KS(n*)
    again = orc.ct_ipls(prm, md.m0, np.eye(5), ct300.y, 1, ms_init=out["ms"], Ns_init=out["Ns"])
    np.testing.assert_allclose(again["ms"], out["ms"], atol=1e-10)
    np.testing.assert_allclose(again["Ns"] @ np.swapaxes(again["Ns"], 1, 2),
                               out["Ns"] @ np.swapaxes(out["Ns"], 1, 2), atol=1e-12)
    # the smoothed positions track the truth far better than the prior does
    x = ct300.x_true[0]
    rmse = np.sqrt(((out["ms"][:, :2] - x[:, :2]) ** 2).mean())
    rmse_prior = np.sqrt(((md.m0[:2] - x[:, :2]) ** 2).mean())
    assert rmse < 0.5 * rmse_prior


def test_one_pass_is_linearise_filter_smooth(orc, ct300):
    md = ct300.model
    prm = orc.ct_params()
    n = len(ct300.y)
    ms0 = np.repeat(md.m0[None], n + 1, 0)
    Ns0 = np.repeat(np.eye(5)[None], n + 1, 0)
    G = orc.ct_linearize(prm, ms0, Ns0, ct300.y)
    mf, Nf, _ = orc.sqrt_filter(md.m0, np.eye(5), G, ct300.y)
    ms, Ns, _ = orc.sqrt_smoother(G, mf, Nf)
    out = orc.ct_ipls(prm, md.m0, np.eye(5), ct300.y, 1)
    np.testing.assert_array_equal(out["ms"], ms)
    np.testing.assert_array_equal(out["Ns"], Ns)


def test_literal_and_residual_slr_agree_along_ipls(orc, ct300):
    md = ct300.model
    prm = orc.ct_params()
    out = orc.ct_ipls(prm, md.m0, np.eye(5), ct300.y, 4, history=True)
    for i in range(4):
        ms, Ns = out["hist_ms"][i], out["hist_Ns"][i]
        a = orc.ct_linearize(prm, ms, Ns, ct300.y, literal=False)
        b = orc.ct_linearize(prm, ms, Ns, ct300.y, literal=True)
        assert b["bad"] == 0
        for k in ("F", "c", "H", "d"):
            np.testing.assert_allclose(a[k], b[k], rtol=1e-7, atol=1e-9)
        for k in ("SL", "SO"):
            Ga = a[k] @ np.swapaxes(a[k], 1, 2)
            Gb = b[k] @ np.swapaxes(b[k], 1, 2)
            np.testing.assert_allclose(Ga, Gb, rtol=1e-5, atol=1e-12)


def test_pseudo_loglik_is_gaussian_density_of_linearised_model(orc):
    w = wl.ct_single(6, 5)
    md = w.model
    prm = orc.ct_params()
    out = orc.ct_ipls(prm, md.m0, np.eye(5), w.y, 3)
    G = orc.ct_linearize(prm, out["ms"], out["Ns"], w.y)
    _, _, _, _, ll_b = bf.filter_smoother_loglik(md.m0, np.eye(5), G, w.y)
    tot, ell = orc.ct_loglik(prm, md.m0, np.eye(5), w.y, out["ms"], out["Ns"], per_step=True)
    np.testing.assert_allclose(tot, ll_b, rtol=1e-10)
    np.testing.assert_allclose(ell.sum(), tot, rtol=1e-14)


@pytest.mark.parametrize("n,seed,M", [(50, 11, 2), (400, 12, 6)])
def test_ct_score_equals_finite_differences(orc, n, seed, M):
    w = wl.ct_single(n, seed)
    md = w.model
    prm = orc.ct_params()
    out = orc.ct_ipls(prm, md.m0, np.eye(5), w.y, M)
    ms, Ns = out["ms"], out["Ns"]
    tot, g = orc.ct_score(prm, md.m0, np.eye(5), w.y, ms, Ns)
    np.testing.assert_allclose(tot, orc.ct_loglik(prm, md.m0, np.eye(5), w.y, ms, Ns), rtol=1e-12)
    th = md.theta
    h = 1e-5
    for i in range(3):
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (orc.ct_loglik(orc.ct_theta_params(tp), md.m0, np.eye(5), w.y, ms, Ns)
              - orc.ct_loglik(orc.ct_theta_params(tm), md.m0, np.eye(5), w.y, ms, Ns)) / (2 * h)
        np.testing.assert_allclose(g[i], fd, rtol=1e-6, atol=1e-6)


def test_batches_equal_single_sequences(orc):
    rng_w = wl.ct_batch(B=3, n=120, seed=21)
    md = rng_w.model
    prm = orc.ct_params()
    off = rng_w.y_off
    T_x = off[-1] + 3
    ms = np.repeat(md.m0[None], T_x, 0).copy()
    Ns = np.repeat(np.eye(5)[None], T_x, 0).copy()
    orc.ct_ipls_batch(prm, md.m0, np.eye(5), rng_w.y, off, 3, ms, Ns)
    ll = orc.ct_loglik_batch(prm, md.m0, np.eye(5), rng_w.y, off, ms, Ns)
    ll2, g2 = orc.ct_score_batch(prm, md.m0, np.eye(5), rng_w.y, off, ms, Ns)
    for b in range(3):
        yb = rng_w.y[off[b]:off[b + 1]]
        xo = off[b] + b
        n = off[b + 1] - off[b]
        one = orc.ct_ipls(prm, md.m0, np.eye(5), yb, 3)
        np.testing.assert_array_equal(ms[xo:xo + n + 1], one["ms"])
        np.testing.assert_array_equal(Ns[xo:xo + n + 1], one["Ns"])
        assert ll[b] == orc.ct_loglik(prm, md.m0, np.eye(5), yb, one["ms"], one["Ns"])
        t, g = orc.ct_score(prm, md.m0, np.eye(5), yb, one["ms"], one["Ns"])
        assert ll2[b] == t and np.array_equal(g2[b], g)
    cv = wl.CVModel()
    G = dict(F=cv.F(), c=np.zeros(4), SL=np.linalg.cholesky(cv.Q()), H=cv.H(), d=np.zeros(2),
             SO=np.linalg.cholesky(cv.R()))
    ys = [wl.simulate_cv(k, np.random.default_rng(k), cv)[1] for k in (5, 9)]
    yy = np.concatenate(ys)
    off = np.array([0, 5, 14])
    ms = np.zeros((16, 4)); Ns = np.zeros((16, 4, 4))
    orc.linear_smoother_batch(np.zeros(4), np.eye(4), G, yy, off, ms, Ns)
    for b in range(2):
        mf, Nf, _ = orc.sqrt_filter(np.zeros(4), np.eye(4), G, ys[b])
        m1, N1, _ = orc.sqrt_smoother(G, mf, Nf)
        xo = off[b] + b
        np.testing.assert_array_equal(ms[xo:xo + len(ys[b]) + 1], m1)
        np.testing.assert_array_equal(Ns[xo:xo + len(ys[b]) + 1], N1)
