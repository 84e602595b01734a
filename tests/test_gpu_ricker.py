"""GPU parity of the generalised SLR with positive-weight sigma-point rules:

* the Ricker-Poisson model of Section 6.1 (non-additive noise: the E[V[y|x]]
  term of the GSLR moments) with the cubature, unscented and Gauss-Hermite
  rules and the Taylor expansion: the linearisation itself, every pass of the
  iterated smoother (square-root and covariance forms) started from the
  oracle's previous nominal, the log-likelihood, the sequential comparator,
  and one pass at a 10^5-step sequence;
* the coordinated-turn model with the unscented and Gauss-Hermite rules: the
  linearisation, every pass, the log-likelihood and the frozen-nominal
  gradient.
Each pass is started from the oracle's nominal so that differences do not
compound through the iteration (on the chaotic Ricker map the iterated
smoother need not settle to a fixed point)."""
import math

import numpy as np
import pytest
import torch

import oracle as orc
from paper_2207_00426_amd import pss
from paper_2207_00426_amd import workloads as wl
from tests import parity as par

pytestmark = pytest.mark.gpu
DEV = "cuda"

LINS = [("cubature", {}), ("taylor", {}), ("unscented", {"ut_kappa": 2.0}),
        ("unscented", {"ut_kappa": 0.5}), ("gauss_hermite", {"gh_order": 5}),
        ("gauss_hermite", {"gh_order": 20})]


def _dt(tag):
    return torch.float64 if tag == "f64" else torch.float32


def _okw(kw):
    return dict(kappa=kw.get("ut_kappa"), gh_order=kw.get("gh_order"))


def _ricker_case(lengths, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    md = wl.RickerModel()
    seqs = [wl.simulate_ricker(int(n), rng, md) for n in lengths]
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return md, [s[1] for s in seqs], off


def _state_cat(per_seq):
    return np.concatenate(per_seq)


def _nominal_to_gpu(ms_list, Ns_list, dtype, cov):
    m = _state_cat(ms_list)
    N = _state_cat(Ns_list)
    if cov:
        N = N * N
    return (torch.tensor(m[None], dtype=dtype, device=DEV),
            torch.tensor(N[None], dtype=dtype, device=DEV))


def _split(a, off):
    return [a[off[s] + s:off[s + 1] + s + 1] for s in range(len(off) - 1)]


@pytest.mark.parametrize("tag", ["f64", "f32"])
@pytest.mark.parametrize("lin,kw", LINS)
def test_ricker_linearisation_matches_oracle(tag, lin, kw):
    md, ys, off = _ricker_case([600], 21)
    prm = orc.ricker_params()
    ref = orc.ricker_ipls(prm, md.m0, math.sqrt(md.P0[0, 0]), ys[0], 2, method=lin, **_okw(kw))
    b = pss.Batch.ricker(off, md, dtype=_dt(tag), device=DEV, linearization=lin, **kw)
    m, N = _nominal_to_gpu([ref["ms"]], [ref["Ns"]], _dt(tag), False)
    g = pss.slr_linearize(b, m, N, pss.to_soa(ys[0], _dt(tag), DEV))
    torch.cuda.synchronize()
    lr = orc.ricker_linearize(prm, ref["ms"], ref["Ns"], ys[0], method=lin, **_okw(kw))
    tol = 1e-10 if tag == "f64" else 2e-4
    for key in ("F", "c", "H", "d", "SL", "SO"):
        got = g[key][0].double().cpu().numpy()
        want = lr[key]
        if key in ("SL", "SO"):  # factors are unique up to sign: compare squares
            got, want = got * got, want * want
        err = np.max(np.abs(got - want) / np.maximum(np.abs(want), 1.0))
        assert err < tol, (key, err)


@pytest.mark.parametrize("form", ["sqrt", "cov"])
@pytest.mark.parametrize("lin,kw", LINS)
def test_ricker_every_pass_f64(form, lin, kw):
    lengths = [1, 333, 2000]
    md, ys, off = _ricker_case(lengths, 22)
    prm = orc.ricker_params()
    M = 5
    refs = [orc.ricker_ipls(prm, md.m0, math.sqrt(md.P0[0, 0]), y, M, history=True, method=lin,
                            **_okw(kw)) for y in ys]
    b = pss.Batch.ricker(off, md, dtype=torch.float64, device=DEV, linearization=lin, form=form,
                         **kw)
    yd = pss.to_soa(np.concatenate(ys), torch.float64, DEV)
    tol = par.TOL["f64"]
    for i in range(M):
        if i == 0:
            m, N = b.prior_nominal()
        else:
            m, N = _nominal_to_gpu([r["hist_ms"][i - 1] for r in refs],
                                   [r["hist_Ns"][i - 1] for r in refs], torch.float64,
                                   form == "cov")
        pss.ipls_iterate(b, yd, 1, m, N)
        torch.cuda.synchronize()
        ma = m[0].cpu().numpy()
        Pa = N[0].cpu().numpy() if form == "cov" else N[0].cpu().numpy() ** 2
        for s, r in enumerate(refs):
            mm, PP = _split(ma, off)[s], _split(Pa, off)[s]
            em = par.mean_err(mm[:, None], r["hist_ms"][i][:, None],
                              (r["hist_Ns"][i] ** 2)[:, None, None])
            eP = par.cov_err(PP[:, None, None], (r["hist_Ns"][i] ** 2)[:, None, None])
            assert em < tol["m"] and eP < tol["P"], (i, s, em, eP)


@pytest.mark.parametrize("lin,kw", [("cubature", {}), ("taylor", {}),
                                    ("gauss_hermite", {"gh_order": 7})])
def test_ricker_every_pass_f32(lin, kw):
    md, ys, off = _ricker_case([700], 23)
    prm = orc.ricker_params()
    M = 4
    r = orc.ricker_ipls(prm, md.m0, math.sqrt(md.P0[0, 0]), ys[0], M, history=True, method=lin,
                        **_okw(kw))
    b = pss.Batch.ricker(off, md, dtype=torch.float32, device=DEV, linearization=lin, **kw)
    yd = pss.to_soa(ys[0], torch.float32, DEV)
    tol = par.TOL["f32"]
    for i in range(M):
        if i == 0:
            m, N = b.prior_nominal()
        else:
            m, N = _nominal_to_gpu([r["hist_ms"][i - 1]], [r["hist_Ns"][i - 1]], torch.float32,
                                   False)
        pss.ipls_iterate(b, yd, 1, m, N)
        torch.cuda.synchronize()
        mm = m[0].double().cpu().numpy()
        PP = N[0].double().cpu().numpy() ** 2
        Pr = (r["hist_Ns"][i] ** 2)[:, None, None]
        em = par.mean_err(mm[:, None], r["hist_ms"][i][:, None], Pr)
        eP = par.cov_err(PP[:, None, None], Pr)
        assert em < tol["m"] and eP < tol["P"], (i, em, eP)


@pytest.mark.parametrize("form", ["sqrt", "cov"])
@pytest.mark.parametrize("lin,kw", [("cubature", {}), ("taylor", {}),
                                    ("unscented", {"ut_kappa": 2.0}),
                                    ("gauss_hermite", {"gh_order": 9})])
def test_ricker_loglik(form, lin, kw):
    lengths = [50, 1500]
    md, ys, off = _ricker_case(lengths, 24)
    prm = orc.ricker_params()
    refs = [orc.ricker_ipls(prm, md.m0, math.sqrt(md.P0[0, 0]), y, 3, method=lin, **_okw(kw))
            for y in ys]
    b = pss.Batch.ricker(off, md, dtype=torch.float64, device=DEV, linearization=lin, form=form,
                         **kw)
    m, N = _nominal_to_gpu([r["ms"] for r in refs], [r["Ns"] for r in refs], torch.float64,
                           form == "cov")
    ll = pss.loglik(b, pss.to_soa(np.concatenate(ys), torch.float64, DEV), m, N)
    torch.cuda.synchronize()
    for s, (y, r) in enumerate(zip(ys, refs)):
        want = orc.ricker_loglik(prm, md.m0, math.sqrt(md.P0[0, 0]), y, r["ms"], r["Ns"],
                                 method=lin, **_okw(kw))
        assert par.ll_err(float(ll[s]), want) < par.TOL["f64"]["ll"], (s, float(ll[s]), want)


@pytest.mark.parametrize("form", ["sqrt", "cov"])
@pytest.mark.parametrize("lin", ["taylor", "cubature"])
def test_ricker_sequential_comparator(form, lin):
    # the square-root recursions, or the standard Kalman filter and RTS
    # smoother in the covariance form (the paper's Section 6.1 comparator)
    md, ys, off = _ricker_case([400, 900], 25)
    prm = orc.ricker_params()
    b = pss.Batch.ricker(off, md, dtype=torch.float64, device=DEV, linearization=lin,
                         form=form)
    m, N = b.prior_nominal()
    pss.sequential_smoother(b, pss.to_soa(np.concatenate(ys), torch.float64, DEV), 2, m, N)
    torch.cuda.synchronize()
    ma, Na = m[0].cpu().numpy(), N[0].cpu().numpy()
    Pa = Na if form == "cov" else Na ** 2
    for s, y in enumerate(ys):
        r = orc.ricker_ipls(prm, md.m0, math.sqrt(md.P0[0, 0]), y, 2, method=lin)
        Pr = (r["Ns"] ** 2)[:, None, None]
        em = par.mean_err(_split(ma, off)[s][:, None], r["ms"][:, None], Pr)
        eP = par.cov_err(_split(Pa, off)[s][:, None, None], Pr)
        assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"], (s, em, eP)


@pytest.mark.parametrize("lin,kw", [("cubature", {}), ("gauss_hermite", {"gh_order": 5})])
def test_ricker_one_pass_at_1e5_steps(lin, kw):
    md, ys, off = _ricker_case([100000], 26)
    prm = orc.ricker_params()
    b = pss.Batch.ricker(off, md, dtype=torch.float64, device=DEV, linearization=lin, **kw)
    m, N = b.prior_nominal()
    pss.ipls_iterate(b, pss.to_soa(ys[0], torch.float64, DEV), 1, m, N)
    torch.cuda.synchronize()
    r = orc.ricker_ipls(prm, md.m0, math.sqrt(md.P0[0, 0]), ys[0], 1, method=lin, **_okw(kw))
    Pr = (r["Ns"] ** 2)[:, None, None]
    em = par.mean_err(m[0].cpu().numpy()[:, None], r["ms"][:, None], Pr)
    eP = par.cov_err((N[0].cpu().numpy() ** 2)[:, None, None], Pr)
    print("Ricker n=1e5 %s: mean err %.3e, cov err %.3e" % (lin, em, eP))
    assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"]


# ---------------------------------------------------------------------------
# CT model with the unscented and Gauss-Hermite rules
# ---------------------------------------------------------------------------
CT_RULES = [("unscented", {"ut_kappa": 1.0}), ("unscented", {"ut_kappa": 0.0}),
            ("gauss_hermite", {"gh_order": 3})]


@pytest.mark.parametrize("tag", ["f64", "f32"])
@pytest.mark.parametrize("lin,kw", CT_RULES + [("gauss_hermite", {"gh_order": 4})])
def test_ct_rule_linearisation_matches_oracle(tag, lin, kw):
    # gh_order 4 is the largest CT rule (4^5 = 1024 points)
    w = wl.ct_single(300, seed=12)
    prm = orc.ct_params()
    ref = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, 3, method=lin, **_okw(kw))
    b = pss.Batch.ct(w.y_off, w.model, dtype=_dt(tag), device=DEV, linearization=lin, **kw)
    m = pss.to_soa(ref["ms"], _dt(tag), DEV)
    N = pss.to_soa(pss.pack_lower(ref["Ns"]), _dt(tag), DEV)
    g = pss.slr_linearize(b, m, N, pss.to_soa(w.y, _dt(tag), DEV))
    torch.cuda.synchronize()
    lr = orc.ct_linearize(prm, ref["ms"], ref["Ns"], w.y, method=lin, **_okw(kw))
    tol = 1e-10 if tag == "f64" else 2e-4
    for key, shape in (("F", (5, 5)), ("c", (5,)), ("H", (2, 5)), ("d", (2,))):
        got = pss.from_soa(g[key], shape)
        scale = np.maximum(np.abs(lr[key]), 1.0)
        assert np.max(np.abs(got - lr[key]) / scale) < tol, key
    for key, n in (("SL", 5), ("SO", 2)):
        S = pss.unpack_lower(pss.from_soa(g[key], (n * (n + 1) // 2,)), n)
        Pg, Pr = par.gram(S), par.gram(lr[key])
        err = np.max(np.abs(Pg - Pr)) / np.max(np.abs(Pr))
        assert err < (1e-9 if tag == "f64" else 1e-4), (key, err)


@pytest.mark.parametrize("lin,kw", CT_RULES)
def test_ct_rule_every_pass_and_gradient(lin, kw):
    w = wl.ct_single(1000, seed=1)
    M = 4
    prm = orc.ct_params()
    ref = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, M, history=True, method=lin, **_okw(kw))
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float64, device=DEV, linearization=lin, **kw)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, N = b.prior_nominal()
    for i in range(M):
        if i > 0:  # start each pass from the oracle's nominal
            m = pss.to_soa(ref["hist_ms"][i - 1], torch.float64, DEV)
            N = pss.to_soa(pss.pack_lower(ref["hist_Ns"][i - 1]), torch.float64, DEV)
        pss.ipls_iterate(b, yd, 1, m, N)
        torch.cuda.synchronize()
        ma, Na = pss.marg_from_soa(m, N, 5)
        em, eP = par.marg_errs(ma, Na, ref["hist_ms"][i], ref["hist_Ns"][i])
        assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"], (i, em, eP)
    m = pss.to_soa(ref["ms"], torch.float64, DEV)
    N = pss.to_soa(pss.pack_lower(ref["Ns"]), torch.float64, DEV)
    ll, grad, _ = pss.loglik_grad(b, m, N, yd)
    ll_ref, g_ref = orc.ct_score(prm, w.model.m0, np.eye(5), w.y, ref["ms"], ref["Ns"],
                                 method=lin, **_okw(kw))
    assert par.ll_err(float(ll.item()), ll_ref) < par.TOL["f64"]["ll"]
    assert par.grad_err(grad[:, 0].cpu().numpy(), g_ref) < par.TOL["f64"]["g"]
