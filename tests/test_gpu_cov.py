"""GPU parity of the standard (covariance-form) parallel filter and smoother
(left columns of Tables 1-5), run through pss_ipls_iterate / pss_loglik with
form = PSS_FORM_COV, against the FP64 oracle (whose sequential recursions
give the same marginals in any form).  Covariances come back as packed
lower triangles of P."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2207_00426_amd import pss
from paper_2207_00426_amd import workloads as wl
from tests import parity as par
from tests.test_gpu_parity import DIMS, _linear_case, _oracle_linear, _split_states

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _cov_from_soa(m, P, nx):
    mm = pss.from_soa(m, (nx,))
    L = pss.unpack_lower(pss.from_soa(P, (pss.tri(nx),)), nx)
    full = L + np.swapaxes(L, -1, -2) - np.einsum("...ii->...i", L)[..., None] * np.eye(nx)
    return mm, full


def _errs(m, P, mr, Nr):
    Pr = par.gram(Nr)
    return par.mean_err(m, mr, Pr), par.cov_err(P, Pr)


@pytest.mark.parametrize("nx,ny", DIMS)
def test_cov_form_linear_multilevel(nx, ny):
    lengths = np.array([700, 1, 130, 2])
    G, m0, N0, y, y_off = _linear_case(nx, ny, lengths, 31 + nx)
    b = pss.Batch(pss.MODEL_LINEAR, torch.float64, nx, ny, y_off, m0, N0, device=DEV,
                  scan_threads=64, scan_elems=2, form="cov")
    g = b.gamma_from_numpy(G)
    yd = pss.to_soa(y, torch.float64, DEV)
    m, N = b.prior_nominal()
    pss.ipls_iterate(b, yd, 1, m, N, gamma=g)
    ll = pss.loglik(b, yd, m, N, gamma=g)
    torch.cuda.synchronize()
    ma, Pa = _cov_from_soa(m, N, nx)
    ref = _oracle_linear(G, m0, N0, y, y_off)
    for s, (ms_, Ps_) in enumerate(zip(_split_states(ma, y_off), _split_states(Pa, y_off))):
        em, eP = _errs(ms_, Ps_, ref[s]["ms"], ref[s]["Ns"])
        assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"], (s, em, eP)
        assert par.ll_err(float(ll[s]), ref[s]["ll"]) < par.TOL["f64"]["ll"]


def test_cov_form_ct_every_pass():
    w = wl.ct_single(1000, seed=1)
    M = 10
    ref = orc.ct_ipls(orc.ct_params(), w.model.m0, np.eye(5), w.y, M, history=True)
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float64, device=DEV, form="cov")
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, N = b.prior_nominal()  # (m0, P0) at every state
    for i in range(M):
        pss.ipls_iterate(b, yd, 1, m, N)
        torch.cuda.synchronize()
        ma, Pa = _cov_from_soa(m, N, 5)
        em, eP = _errs(ma, Pa, ref["hist_ms"][i], ref["hist_Ns"][i])
        assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"], (i, em, eP)
    ll = pss.loglik(b, yd, m, N)
    ll_ref = orc.ct_loglik(orc.ct_params(), w.model.m0, np.eye(5), w.y, ref["ms"], ref["Ns"])
    assert par.ll_err(float(ll.item()), ll_ref) < par.TOL["f64"]["ll"]


@pytest.mark.parametrize("lin", ["cubature", "taylor"])
def test_cov_form_ct_fp32_each_pass_from_its_own_nominal(lin):
    """FP32 covariance form (in FP32 the linearisation and the filter
    elements run as one kernel): every pass against one oracle pass taken
    from the GPU's own nominal before it, so FP32 error does not compound,
    within the FP32 bar; then the log-likelihood at the final nominal."""
    w = wl.ct_single(1000, seed=1)
    prm = orc.ct_params()
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float32, device=DEV, form="cov",
                     linearization=lin)
    yd = pss.to_soa(w.y, torch.float32, DEV)
    m, N = b.prior_nominal()
    tol = par.TOL["f32"]
    for i in range(5):
        m_in, P_in = _cov_from_soa(m, N, 5)
        ref = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, 1, ms_init=m_in,
                          Ns_init=np.linalg.cholesky(P_in.astype(np.float64)), method=lin)
        pss.ipls_iterate(b, yd, 1, m, N)
        torch.cuda.synchronize()
        ma, Pa = _cov_from_soa(m, N, 5)
        em, eP = _errs(ma, Pa, ref["ms"], ref["Ns"])
        assert em < tol["m"] and eP < tol["P"], (lin, i, em, eP)
    ma, Pa = _cov_from_soa(m, N, 5)
    ll = pss.loglik(b, yd, m, N)
    ll_ref = orc.ct_loglik(prm, w.model.m0, np.eye(5), w.y, ma,
                           np.linalg.cholesky(Pa.astype(np.float64)), method=lin)
    assert par.ll_err(float(ll.item()), ll_ref) < tol["ll"]


def test_fp32_square_root_form_does_not_diverge_where_covariance_form_does():
    # informative bearings (sigma 5e-4) and slow dynamics (q 1e-3): the
    # setting of the robustness comparison where the covariance form loses
    # positive definiteness in FP32
    md = wl.CTModel(q1=1e-3, q2=1e-3, sigma=5e-4)
    sets, n = 15, 4000
    rng = np.random.Generator(np.random.PCG64(7))
    ys = [wl.simulate_ct(n, rng, md)[1] for _ in range(sets)]
    off = np.arange(sets + 1, dtype=np.int64) * n
    bad = {}
    for form in ("sqrt", "cov"):
        b = pss.Batch.ct(off, md, dtype=torch.float32, device=DEV, form=form)
        yd = pss.to_soa(np.concatenate(ys), torch.float32, DEV)
        m, N = b.prior_nominal()
        pss.ipls_iterate(b, yd, 20, m, N)
        ll = pss.loglik(b, yd, m, N)
        torch.cuda.synchronize()
        bad[form] = int((~torch.isfinite(ll)).sum().item())
    print("FP32 non-finite log-likelihoods of 15: square root %d, covariance %d"
          % (bad["sqrt"], bad["cov"]))
    assert bad["sqrt"] == 0
    assert bad["cov"] > 0


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_sequential_covariance_comparator_ct(tag):
    # the standard Kalman filter / RTS smoother (one thread per sequence) on
    # the CT model, ragged batch, against the oracle's pass
    rng = np.random.default_rng(41)
    ct = wl.CTModel()
    lens = [300, 1, 800]
    ys = [wl.simulate_ct(n, rng, ct)[1] for n in lens]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    dt = torch.float64 if tag == "f64" else torch.float32
    b = pss.Batch.ct(off, ct, dtype=dt, device=DEV, form="cov")
    m, P = b.prior_nominal()
    pss.sequential_smoother(b, pss.to_soa(np.concatenate(ys), dt, DEV), 1, m, P)
    torch.cuda.synchronize()
    ma, Pa = _cov_from_soa(m.double(), P.double(), 5)
    for s, y in enumerate(ys):
        r = orc.ct_ipls(orc.ct_params(), ct.m0, np.eye(5), y, 1)
        a, z = off[s] + s, off[s + 1] + s + 1
        em, eP = _errs(ma[a:z], Pa[a:z], r["ms"], r["Ns"])
        assert em < par.TOL[tag]["m"] and eP < par.TOL[tag]["P"], (s, em, eP)
