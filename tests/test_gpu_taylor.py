"""GPU parity of the first-order Taylor linearisation (Section 4.2; the
square-root iterated extended smoother) against the FP64 oracle: the
linearisation itself, every pass of the iteration on the n = 1000
coordinated-turn configuration, the log-likelihood and gradient at its
nominal, and the persistent batched pass."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2207_00426_amd import pss
from paper_2207_00426_amd import workloads as wl
from tests import parity as par

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _dt(tag):
    return torch.float64 if tag == "f64" else torch.float32


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_taylor_linearisation_matches_oracle(tag):
    w = wl.ct_single(300, seed=12)
    prm = orc.ct_params()
    ref = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, 3, method="taylor")
    ms, Ns = ref["ms"], ref["Ns"]
    b = pss.Batch.ct(w.y_off, w.model, dtype=_dt(tag), device=DEV, linearization="taylor")
    m = pss.to_soa(ms, _dt(tag), DEV)
    N = pss.to_soa(pss.pack_lower(Ns), _dt(tag), DEV)
    g = pss.slr_linearize(b, m, N, pss.to_soa(w.y, _dt(tag), DEV))
    torch.cuda.synchronize()
    lin = orc.ct_linearize(prm, ms, Ns, w.y, method="taylor")
    tol = 1e-10 if tag == "f64" else 2e-4
    for key, shape in (("F", (5, 5)), ("c", (5,)), ("H", (2, 5)), ("d", (2,))):
        got = pss.from_soa(g[key], shape)
        scale = np.maximum(np.abs(lin[key]), 1.0)
        assert np.max(np.abs(got - lin[key]) / scale) < tol, key
    SL = pss.unpack_lower(pss.from_soa(g["SL"], (15,)), 5)
    np.testing.assert_allclose(par.gram(SL), par.gram(lin["SL"]), rtol=tol, atol=1e-14)


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_iterated_extended_smoother_every_pass(tag):
    """Every pass of the n = 1000 IEKS: each GPU pass, started from the GPU's
    own previous nominal, against one oracle pass from that same nominal at
    the fixed bar of its precision; in FP64 also the whole chain of passes
    against the oracle's own iteration from the prior."""
    w = wl.ct_single(1000, seed=1)
    M = 10
    prm = orc.ct_params()
    ref = orc.ct_ipls(prm, w.model.m0, np.eye(5), w.y, M, history=True, method="taylor")
    b = pss.Batch.ct(w.y_off, w.model, dtype=_dt(tag), device=DEV, linearization="taylor")
    yd = pss.to_soa(w.y, _dt(tag), DEV)
    m, N = b.prior_nominal()
    tol = par.TOL[tag]
    for i in range(M):
        m_prev, N_prev = pss.marg_from_soa(m.double(), N.double(), 5)
        pss.ipls_iterate(b, yd, 1, m, N)
        torch.cuda.synchronize()
        ma, Na = pss.marg_from_soa(m.double(), N.double(), 5)
        one = orc.ct_ipls(prm, w.model.m0, np.eye(5), par.kernel_input(w.y, tag), 1,
                          ms_init=m_prev, Ns_init=N_prev, method="taylor")
        em, eP = par.marg_errs(ma, Na, one["ms"], one["Ns"])
        assert em < tol["m"] and eP < tol["P"], (i, em, eP)
        if tag == "f64":
            em, eP = par.marg_errs(ma, Na, ref["hist_ms"][i], ref["hist_Ns"][i])
            assert em < tol["m"] and eP < tol["P"], (i, em, eP)
    ll, grad, _ = pss.loglik_grad(b, m, N, yd)
    ma, Na = pss.marg_from_soa(m.double(), N.double(), 5)
    ll_ref, g_ref = orc.ct_score(prm, w.model.m0, np.eye(5), w.y, ma, Na, method="taylor")
    assert par.ll_err(float(ll.item()), ll_ref) < tol["ll"]
    assert par.grad_err(grad[:, 0].cpu().numpy(), g_ref) < tol["g"]


def test_taylor_in_the_persistent_batched_pass():
    rng = np.random.default_rng(9)
    ct = wl.CTModel()
    lens = [50, 700, 300]
    ys = [wl.simulate_ct(n, rng, ct)[1] for n in lens]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    b = pss.Batch.ct(off, ct, dtype=torch.float64, device=DEV, scan_threads=64, scan_elems=2,
                     linearization="taylor")
    y = pss.to_soa(np.concatenate(ys), torch.float64, DEV)
    m, N = b.prior_nominal()
    status = pss.ipls_batched([(b, y, m, N, None)], 4)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    ma, Na = pss.marg_from_soa(m, N, 5)
    for s, yy in enumerate(ys):
        r = orc.ct_ipls(orc.ct_params(), ct.m0, np.eye(5), yy, 4, method="taylor")
        a, z = off[s] + s, off[s + 1] + s + 1
        em, eP = par.marg_errs(ma[a:z], Na[a:z], r["ms"], r["Ns"])
        assert em < par.TOL["f64"]["m"] and eP < par.TOL["f64"]["P"], (s, em, eP)
