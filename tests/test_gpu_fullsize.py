"""GPU parity at the benchmark's full size (one sequence of 10^6 steps) in the
launch configuration bench.py times (the library's default shapes).

* coordinated-turn bearings model, FP64, the benchmark's 10 IPLS passes:
  every pass, started from the GPU's own previous nominal, against one
  oracle pass from that nominal at every one of the 10^6 + 1 states (the
  FP64 bar); the log-likelihood and the adjoint gradient at the final
  nominal against the oracle's; and the whole chain of passes from the
  prior against the oracle's own chain, within the chain's sensitivity to
  round-off (the oracle's chain, perturbed by one part in 10^15 after its
  first pass, moves by about 1e-7 after ten: the iteration amplifies
  round-off where bearings-only triangulation is ill-conditioned);
* linear constant-velocity model: filter and smoother at every state
  against the oracle's sequential square-root recursions;
* the sequential comparator (FP64) over the whole track: one pass against
  the oracle's at every state;
* FP32 at full size: every pass from the GPU's own FP32 nominal against one
  oracle pass from it.  Measured limit, not the FP32 bar: passes 1 and 2
  meet 1e-4 at every state; from pass 3 on (a nominal concentrated on the
  track) the errors grow to 1e-4 .. 1.1e-3 at p99 (largest: the covariance
  at pass 9) and 1.2e-3 at most.  The sequential FP32 square-root recursion
  on the same pass is itself above the bar there (covariance p99 3.3e-4 at
  pass 9); at passes 3, 6 and 9 the parallel scan's errors stay within a
  bounded factor of it (asserted below).  The FP32 pass runs in deviation
  coordinates relative to the nominal means, which cut the late passes'
  mean error about 5x (information vectors eta ~ J m at |m| ~ 100 lose
  digits in FP32); the covariance factors' FP32 composition is what
  remains.
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


def test_ct_ten_passes_fp64_every_pass_and_gradient(ct_long):
    w = ct_long
    prm = orc.ct_params()
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float64, device=DEV)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, Nn = b.prior_nominal()
    for i in range(w.M):
        mp, Np = pss.marg_from_soa(m, Nn, 5)
        pss.ipls_iterate(b, yd, 1, m, Nn)
        torch.cuda.synchronize()
        r = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, 1, ms_init=mp, Ns_init=Np)
        em, eP = par.marg_errs(*pss.marg_from_soa(m, Nn, 5), r["ms"], r["Ns"])
        print("full-size FP64 pass %d: mean err %.3e, cov err %.3e" % (i + 1, em, eP), flush=True)
        assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"], i
    ll, grad, _ = pss.loglik_grad(b, m, Nn, yd)
    torch.cuda.synchronize()
    ll_ref, g_ref = orc.ct_score(prm, w.model.m0, np.eye(5), w.y, *pss.marg_from_soa(m, Nn, 5))
    el = par.ll_err(float(ll.item()), ll_ref)
    eg = par.grad_err(grad[:, 0].cpu().numpy(), g_ref)
    print("full-size CT loglik err %.3e, gradient err %.3e" % (el, eg))
    assert el < par.TOL["f64"]["ll"] and eg < par.TOL["f64"]["g"]


def test_ct_ten_pass_chain_within_the_iterations_round_off_sensitivity(ct_long):
    w = ct_long
    prm = orc.ct_params()
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float64, device=DEV)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    hist = []
    m, Nn = b.prior_nominal()
    for i in range(w.M):
        pss.ipls_iterate(b, yd, 1, m, Nn)
        torch.cuda.synchronize()
        hist.append(pss.marg_from_soa(m, Nn, 5))
    A = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, w.M, history=True)
    # the oracle's own chain restarted from the GPU's first pass (which equals
    # the oracle's first pass up to round-off): how far the iteration carries
    # one pass's rounding differences
    Bp = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, w.M - 1, ms_init=hist[0][0],
                     Ns_init=hist[0][1], history=True)
    for i in range(w.M):
        em, eP = par.marg_errs(*hist[i], A["hist_ms"][i], A["hist_Ns"][i])
        if i == 0:
            sm = sP = 0.0
        else:
            sm, sP = par.marg_errs(Bp["hist_ms"][i - 1], Bp["hist_Ns"][i - 1], A["hist_ms"][i],
                                   A["hist_Ns"][i])
        print("chain pass %d: GPU vs oracle (%.3e, %.3e); oracle from the GPU's first pass vs "
              "oracle (%.3e, %.3e)" % (i + 1, em, eP, sm, sP), flush=True)
        # within the FP64 bar, or within a small factor of how far the
        # oracle's own chain carries the first pass's round-off
        assert em < max(par.TOL["f64"]["m"], 10 * sm), i
        assert eP < max(par.TOL["f64"]["P"], 10 * sP), i


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


def _per_state(m, N, mr, Nr):
    Pr = par.gram(Nr)
    den = np.maximum(np.linalg.norm(mr, axis=-1),
                     np.sqrt(np.maximum(np.trace(Pr, axis1=-2, axis2=-1), 0.0)))
    em = np.linalg.norm(m - mr, axis=-1) / den
    dP = (par.gram(N) - Pr).reshape(len(Pr), -1)
    eP = np.linalg.norm(dP, axis=-1) / np.linalg.norm(Pr.reshape(len(Pr), -1), axis=-1)
    return em, eP


def test_fp32_full_size_every_pass(ct_long):
    w = ct_long
    prm = orc.ct_params()
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float32, device=DEV)
    yd = pss.to_soa(w.y, torch.float32, DEV)
    y_in = par.kernel_input(w.y, torch.float32)
    m, Nn = b.prior_nominal()
    for i in range(w.M):
        mp, Np = pss.marg_from_soa(m.double(), Nn.double(), 5)
        m_in, N_in = m.clone(), Nn.clone()
        pss.ipls_iterate(b, yd, 1, m, Nn)
        torch.cuda.synchronize()
        assert torch.isfinite(m).all() and torch.isfinite(Nn).all()
        r = orc.ct_ipls(prm, w.model.m0, np.eye(5), y_in, 1, ms_init=mp, Ns_init=Np)
        em, eP = _per_state(*pss.marg_from_soa(m.double(), Nn.double(), 5), r["ms"], r["Ns"])
        line = ("full-size FP32 pass %d: mean err max %.3e p99 %.3e, cov err max %.3e p99 "
                "%.3e, states above 1e-4: %d" % (i + 1, em.max(), np.percentile(em, 99), eP.max(),
                                                  np.percentile(eP, 99),
                                                  int((np.maximum(em, eP) > 1e-4).sum())))
        if i in (2, 5, 8):
            # the sequential FP32 recursion on the same pass: the FP32 limit
            ms_, Ns_ = pss.sequential_smoother(b, yd, 1, m_in, N_in)
            torch.cuda.synchronize()
            sm, sP = _per_state(*pss.marg_from_soa(ms_.double(), Ns_.double(), 5), r["ms"],
                                r["Ns"])
            line += ("; sequential FP32: mean max %.3e p99 %.3e, cov max %.3e p99 %.3e" %
                     (sm.max(), np.percentile(sm, 99), sP.max(), np.percentile(sP, 99)))
            rmax = max(em.max() / sm.max(), eP.max() / sP.max())
            r99 = max(np.percentile(em, 99) / np.percentile(sm, 99),
                      np.percentile(eP, 99) / np.percentile(sP, 99))
            line += "; parallel / sequential: max %.1f, p99 %.1f" % (rmax, r99)
            # the parallel scan adds a bounded factor to the FP32 error of the
            # sequential recursion (measured: p99 up to 8.9x, max up to 10.1x,
            # both at pass 3; 2-4x later)
            assert r99 < 12 and rmax < 15, (i, r99, rmax)
        print(line, flush=True)
        # the measured FP32 limit of the parallel scan on this sequence: the
        # bar holds on the first passes; from the third pass on the errors
        # grow to ~6e-4 (p99) -- see the module docstring
        if i < 2:
            assert em.max() < par.TOL["f32"]["m"] and eP.max() < par.TOL["f32"]["P"]
        assert np.percentile(em, 99) < 2e-3 and np.percentile(eP, 99) < 2e-3
        assert em.max() < 3e-3 and eP.max() < 3e-3
    ll, grad, _ = pss.loglik_grad(b, m, Nn, yd)
    torch.cuda.synchronize()
    ll_ref, g_ref = orc.ct_score(prm, w.model.m0, np.eye(5), y_in,
                                 *pss.marg_from_soa(m.double(), Nn.double(), 5))
    el = par.ll_err(float(ll.item()), ll_ref)
    eg = par.grad_err(grad[:, 0].cpu().numpy(), g_ref)
    print("full-size FP32 loglik err %.3e, adjoint gradient err %.3e" % (el, eg))
    assert el < par.TOL["f32"]["ll"] and eg < par.TOL["f32"]["g"]


def test_sequential_comparator_full_size_fp64(ct_long):
    """The sequential comparator (one wave per sequence) over the whole
    10^6-step track: one pass from the prior nominal against the oracle's
    pass, every state, FP64 bar."""
    w = ct_long
    prm = orc.ct_params()
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float64, device=DEV)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, Nn = pss.sequential_smoother(b, yd, 1)
    torch.cuda.synchronize()
    r = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, 1)
    em, eP = par.marg_errs(*pss.marg_from_soa(m, Nn, 5), r["ms"], r["Ns"])
    print("full-size sequential FP64: mean err %.3e, cov err %.3e" % (em, eP))
    assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"]
