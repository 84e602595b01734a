"""GPU parity at the benchmark's full size (one sequence of 10^6 steps) in the
launch configuration bench.py times (the library's default shapes).

* coordinated-turn bearings model: one IPLS pass from the prior, every
  smoothed state of the million against the oracle's pass, then the
  log-likelihood and the frozen-nominal gradient at that nominal;
* linear constant-velocity model: filter and smoother at every state
  against the oracle's sequential square-root recursions;
* FP32 at full size: one pass within the FP32 bar of the FP64 run at every
  state (each later pass linearises at the previous FP32 result, so the
  difference compounds: 1.0e-4 after two); after the 10 passes of the
  benchmark finite, with the bulk
  close (median) and the deviation percentiles reported: the fixed-count
  iteration amplifies FP32 round-off where bearings-only triangulation is
  ill-conditioned, so a few percent of the states separate by more than
  1e-2 (measured: 2.6%, steps 8e3 to 2.8e5).
"""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2207_00426_amd import pss
from paper_2207_00426_amd import workloads as wl
from tests import parity as par

pytestmark = pytest.mark.gpu
DEV = "cuda"
N = 10 ** 6


@pytest.fixture(scope="module")
def ct_long():
    return wl.ct_long(N, 2, M=10)


def test_ct_one_pass_and_gradient_full_size(ct_long):
    w = ct_long
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float64, device=DEV)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, Nn = pss.ipls_iterate(b, yd, 1)
    ll, grad, _ = pss.loglik_grad(b, m, Nn, yd)
    torch.cuda.synchronize()
    ma, Na = pss.marg_from_soa(m, Nn, 5)
    prm = orc.ct_params()
    r = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, 1)
    em, eP = par.marg_errs(ma, Na, r["ms"], r["Ns"])
    print("full-size CT pass: mean err %.3e, cov err %.3e" % (em, eP))
    assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"]
    ll_ref, g_ref = orc.ct_score(prm, w.model.m0, np.eye(5), w.y, r["ms"], r["Ns"])
    el = par.ll_err(float(ll.item()), ll_ref)
    eg = par.grad_err(grad[:, 0].cpu().numpy(), g_ref)
    print("full-size CT loglik err %.3e, gradient err %.3e" % (el, eg))
    assert el < par.TOL["f64"]["ll"] and eg < par.TOL["f64"]["g"]


def test_linear_filter_smoother_full_size():
    w = wl.cv_single(N, seed=5)
    md = w.model
    G = dict(F=md.F(), c=np.zeros(4), SL=np.linalg.cholesky(md.Q()), H=md.H(), d=np.zeros(2),
             SO=np.linalg.cholesky(md.R()))
    b = pss.Batch(pss.MODEL_LINEAR, torch.float64, 4, 2, w.y_off, md.m0, np.eye(4), device=DEV)
    g = b.gamma_from_numpy(G)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    el = pss.sqrt_filter_elements(b, g, yd)
    mf, Nf = pss.sqrt_filter_scan(b, el)
    ms, Ns = pss.sqrt_smoother_scan(b, g, mf, Nf)
    torch.cuda.synchronize()
    rmf, rNf, _ = orc.sqrt_filter(md.m0, np.eye(4), G, w.y)
    rms, rNs, _ = orc.sqrt_smoother(G, rmf, rNf)
    for (m, NN, rm, rN, what) in ((mf, Nf, rmf, rNf, "filter"), (ms, Ns, rms, rNs, "smoother")):
        ma, Na = pss.marg_from_soa(m, NN, 4)
        em, eP = par.marg_errs(ma, Na, rm, rN)
        print("full-size CV %s: mean err %.3e, cov err %.3e" % (what, em, eP))
        assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"], what


def _per_state_mean_err(m, N, mr, Nr):
    Pr = par.gram(Nr)
    den = np.maximum(np.linalg.norm(mr, axis=-1),
                     np.sqrt(np.maximum(np.trace(Pr, axis1=-2, axis2=-1), 0.0)))
    return np.linalg.norm(m - mr, axis=-1) / den


def test_fp32_full_size_per_pass_parity_and_ten_passes(ct_long):
    w = ct_long
    res = {}
    for passes in (1, 10):
        out = {}
        for dt in (torch.float64, torch.float32):
            b = pss.Batch.ct(w.y_off, w.model, dtype=dt, device=DEV)
            yd = pss.to_soa(w.y, dt, DEV)
            m, Nn = pss.ipls_iterate(b, yd, passes)
            ll, _, _ = pss.loglik_grad(b, m, Nn, yd)
            torch.cuda.synchronize()
            out[dt] = (pss.marg_from_soa(m.double(), Nn.double(), 5), float(ll.item()))
        (m32, N32), ll32 = out[torch.float32]
        (m64, N64), ll64 = out[torch.float64]
        assert np.isfinite(m32).all() and np.isfinite(N32).all() and np.isfinite(ll32)
        e = _per_state_mean_err(m32, N32, m64, N64)
        res[passes] = (par.marg_errs(m32, N32, m64, N64), np.percentile(e, [50, 99, 100]),
                       par.ll_err(ll32, ll64))
        print("full-size FP32 vs FP64, %d passes: (mean, cov) %s, mean-err percentiles "
              "50/99/100 %s, loglik %.3e" % (passes, res[passes][0], res[passes][1],
                                           res[passes][2]))
    # one pass (the same linearisation point for both): within the FP32 bar
    # at every one of the 10^6 states
    (em, eP), _, _ = res[1]
    assert em < par.TOL["f32"]["m"] and eP < par.TOL["f32"]["P"]
    # ten passes: the fixed-count iteration amplifies FP32 differences in the
    # ill-conditioned stretches of the trajectory; the bulk stays close
    (_, pct, el) = res[10]
    assert pct[0] < 1e-3 and el < 0.1
