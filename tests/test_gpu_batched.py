"""GPU parity of the persistent multi-group batched IPLS (pss_ipls_batched)
and its autotuner against the FP64 oracle.

A ragged batch mixes a linear constant-velocity group (nx 4) and a
coordinated-turn group (nx 5) in one persistent launch per pass; tiles are
forced small so every sequence chains several tiles."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2207_00426_amd import pss
from paper_2207_00426_amd import workloads as wl
from tests import parity as par

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _cv_gamma(md):
    return dict(F=md.F(), c=np.zeros(4), SL=np.linalg.cholesky(md.Q()), H=md.H(), d=np.zeros(2),
                SO=np.linalg.cholesky(md.R()))


def _groups(lens_cv, lens_ct, dtype, seed, T=0, E=0):
    rng = np.random.default_rng(seed)
    cv, ct = wl.CVModel(), wl.CTModel()
    ys_cv = [wl.simulate_cv(int(n), rng, cv)[1] for n in lens_cv]
    ys_ct = [wl.simulate_ct(int(n), rng, ct)[1] for n in lens_ct]
    off_cv = np.concatenate([[0], np.cumsum(lens_cv)]).astype(np.int64)
    off_ct = np.concatenate([[0], np.cumsum(lens_ct)]).astype(np.int64)
    b_cv = pss.Batch(pss.MODEL_LINEAR, dtype, 4, 2, off_cv, cv.m0, np.eye(4), device=DEV,
                     scan_threads=T, scan_elems=E)
    b_ct = pss.Batch.ct(off_ct, ct, dtype=dtype, device=DEV, scan_threads=T, scan_elems=E)
    g_cv = b_cv.gamma_from_numpy(_cv_gamma(cv))
    y_cv = pss.to_soa(np.concatenate(ys_cv), dtype, DEV)
    y_ct = pss.to_soa(np.concatenate(ys_ct), dtype, DEV)
    m_cv, N_cv = b_cv.prior_nominal()
    m_ct, N_ct = b_ct.prior_nominal()
    groups = [(b_cv, y_cv, m_cv, N_cv, g_cv), (b_ct, y_ct, m_ct, N_ct, None)]
    return groups, (ys_cv, ys_ct, off_cv, off_ct, cv, ct)


def _oracle(meta, M, dtype=torch.float64):
    ys_cv, ys_ct, off_cv, off_ct, cv, ct = meta
    ys_cv = [par.kernel_input(y, dtype) for y in ys_cv]
    ys_ct = [par.kernel_input(y, dtype) for y in ys_ct]
    G = _cv_gamma(cv)
    ref_cv = []
    for y in ys_cv:
        mf, Nf, _ = orc.sqrt_filter(cv.m0, np.eye(4), G, y)
        ms, Ns, _ = orc.sqrt_smoother(G, mf, Nf)
        ref_cv.append((ms, Ns))
    ref_ct = [orc.ct_ipls(orc.ct_params(), ct.m0, np.eye(5), y, M) for y in ys_ct]
    return ref_cv, [(r["ms"], r["Ns"]) for r in ref_ct]


def _check(groups, meta, ref, tol):
    (b_cv, _, m_cv, N_cv, _), (b_ct, _, m_ct, N_ct, _) = groups
    _, _, off_cv, off_ct, _, _ = meta
    for (m, N, off, nx, refs) in ((m_cv, N_cv, off_cv, 4, ref[0]), (m_ct, N_ct, off_ct, 5, ref[1])):
        ma, Na = pss.marg_from_soa(m, N, nx)
        for s, (rm, rN) in enumerate(refs):
            a, z = off[s] + s, off[s + 1] + s + 1
            em, eP = par.marg_errs(ma[a:z], Na[a:z], rm, rN)
            assert em < tol["m"] and eP < tol["P"], (nx, s, em, eP)


@pytest.mark.parametrize("tag,T,E,M", [("f64", 64, 1, 3), ("f64", 64, 2, 2), ("f32", 64, 2, 3),
                                       ("f64", 0, 0, 3), ("f32", 0, 0, 2)])
def test_batched_two_groups_match_oracle(tag, T, E, M):
    dtype = torch.float64 if tag == "f64" else torch.float32
    groups, meta = _groups([1, 37, 700, 129], [2, 300, 1000, 64], dtype, 11, T, E)
    status = pss.ipls_batched(groups, M)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    _check(groups, meta, _oracle(meta, M, dtype), par.TOL[tag])


def test_batched_is_deterministic_and_matches_single_group_calls():
    groups, meta = _groups([50, 400], [300, 777], torch.float64, 5, 64, 2)
    pss.ipls_batched(groups, 3)
    torch.cuda.synchronize()
    first = [g[2].clone() for g in groups] + [g[3].clone() for g in groups]
    groups2, _ = _groups([50, 400], [300, 777], torch.float64, 5, 64, 2)
    pss.ipls_batched(groups2, 3)
    # the CT group alone gives the same bits as inside the two-group launch
    groups3, _ = _groups([50, 400], [300, 777], torch.float64, 5, 64, 2)
    pss.ipls_batched([groups3[1]], 3)
    torch.cuda.synchronize()
    again = [g[2] for g in groups2] + [g[3] for g in groups2]
    for a, b in zip(first, again):
        assert torch.equal(a, b)
    assert torch.equal(groups3[1][2], groups[1][2]) and torch.equal(groups3[1][3], groups[1][3])


def test_batched_graph_capture_replays_match_eager():
    groups, meta = _groups([100, 33], [250, 600], torch.float32, 8, 64, 2)
    m0 = [g[2].clone() for g in groups]
    N0 = [g[3].clone() for g in groups]
    ws = torch.empty(pss.batched_workspace_size(groups), dtype=torch.uint8, device=DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pss.ipls_batched(groups, 2, ws=ws, status=status)
        torch.cuda.synchronize()
        eager = [g[2].clone() for g in groups]
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            for g, a, b in zip(groups, m0, N0):
                g[2].copy_(a)
                g[3].copy_(b)
            pss.ipls_batched(groups, 2, ws=ws, status=status)
        for _ in range(3):
            for g in groups:
                g[2].zero_()
            graph.replay()
            torch.cuda.synchronize()
            for g, e in zip(groups, eager):
                assert torch.equal(g[2], e)
    assert int(status.item()) == 0


def test_autotune_picks_a_valid_shape_and_is_used():
    groups, meta = _groups([200, 900], [400, 1500], torch.float32, 3)
    m_before = groups[1][2].clone()
    best = pss.autotune(groups)
    torch.cuda.synchronize()
    assert best[0] in (64, 128, 256) and best[1] in (1, 2, 4, 8) and best[2] in (1, 2, 4, 8)
    assert torch.equal(groups[1][2], m_before)  # the tuner does not touch the nominal
    pss.ipls_batched(groups, 2)
    torch.cuda.synchronize()
    _check(groups, meta, _oracle(meta, 2, torch.float32), par.TOL["f32"])


def _per_state(m, N, mr, Nr):
    Pr = par.gram(Nr)
    den = np.maximum(np.linalg.norm(mr, axis=-1),
                     np.sqrt(np.maximum(np.trace(Pr, axis1=-2, axis2=-1), 0.0)))
    em = np.linalg.norm(m - mr, axis=-1) / den
    dP = (par.gram(N) - Pr).reshape(len(Pr), -1)
    eP = np.linalg.norm(dP, axis=-1) / np.linalg.norm(Pr.reshape(len(Pr), -1), axis=-1)
    return em, eP


def test_ragged_512_fp32_persistent_graph_every_pass():
    """The batched benchmark configuration itself: 512 sequences with lengths
    uniform in [100, 20000] (seed 3), half constant-velocity, half
    coordinated-turn, FP32, the autotuned persistent pass captured in a HIP
    graph.  Each replay (one pass) is checked at every state of every
    sequence against one oracle pass from the GPU's previous nominal."""
    groups_w, lengths, kinds = wl.ragged_mixed(512, 100, 20000, 3, M=10)
    tdt = torch.float32
    cvm = wl.CVModel()
    G = _cv_gamma(cvm)
    wcv, _ = groups_w["cv"]
    wct, _ = groups_w["ct"]
    b_cv = pss.Batch(pss.MODEL_LINEAR, tdt, 4, 2, wcv.y_off, cvm.m0, np.eye(4), device=DEV)
    b_ct = pss.Batch.ct(wct.y_off, wct.model, dtype=tdt, device=DEV)
    y_cv = pss.to_soa(wcv.y, tdt, DEV)
    y_ct = pss.to_soa(wct.y, tdt, DEV)
    m_cv, N_cv = b_cv.prior_nominal()
    m_ct, N_ct = b_ct.prior_nominal()
    groups = [(b_cv, y_cv, m_cv, N_cv, b_cv.gamma_from_numpy(G)), (b_ct, y_ct, m_ct, N_ct, None)]
    shape = pss.autotune(groups)
    print("512 ragged FP32: autotuned shape T=%d E_f=%d E_s=%d" % tuple(shape), flush=True)
    ws = torch.empty(pss.batched_workspace_size(groups), dtype=torch.uint8, device=DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    stream = torch.cuda.Stream()
    pss.ipls_batched(groups, 1, ws=ws, status=status)  # warm-up, then back to the prior
    torch.cuda.synchronize()
    for t, s in ((m_cv, b_cv.prior_nominal()[0]), (N_cv, b_cv.prior_nominal()[1]),
                 (m_ct, b_ct.prior_nominal()[0]), (N_ct, b_ct.prior_nominal()[1])):
        t.copy_(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            pss.ipls_batched(groups, 1, ws=ws, status=status)
    # the linear group: every pass is the exact smoother of the linear model
    ms_cv_ref = np.zeros((len(wcv.y) + len(wcv.y_off) - 1, 4))
    Ns_cv_ref = np.zeros((len(wcv.y) + len(wcv.y_off) - 1, 4, 4))
    orc.linear_smoother_batch(cvm.m0, np.eye(4), G, par.kernel_input(wcv.y, tdt), wcv.y_off,
                              ms_cv_ref, Ns_cv_ref)
    y_ct_in = par.kernel_input(wct.y, tdt)
    prm = orc.ct_params()
    # state slot -> (sequence, state index) of the CT group
    soff = np.asarray(wct.y_off) + np.arange(len(wct.y_off))
    worst = []
    for i in range(10):
        m_in, N_in = m_ct.clone(), N_ct.clone()
        mp, Np = pss.marg_from_soa(m_in.double(), N_in.double(), 5)
        graph.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        ms_ref, Ns_ref = mp.copy(), Np.copy()
        orc.ct_ipls_batch(prm, wct.model.m0, np.eye(5), y_ct_in, wct.y_off, 1, ms_ref, Ns_ref)
        em, eP = _per_state(*pss.marg_from_soa(m_ct.double(), N_ct.double(), 5), ms_ref, Ns_ref)
        cm, cP = _per_state(*pss.marg_from_soa(m_cv.double(), N_cv.double(), 4), ms_cv_ref,
                            Ns_cv_ref)
        # the sequential FP32 recursion on the same pass: the FP32 limit of
        # the square-root smoother itself at each state
        sq_m, sq_N = pss.sequential_smoother(b_ct, y_ct, 1, m_in, N_in)
        torch.cuda.synchronize()
        qm, qP = _per_state(*pss.marg_from_soa(sq_m.double(), sq_N.double(), 5), ms_ref, Ns_ref)
        e = np.maximum(em, eP)
        q = np.maximum(qm, qP)
        w = int(np.argmax(e))
        sw = int(np.searchsorted(soff, w, side="right") - 1)
        worst.append((em.max(), eP.max(), cm.max(), cP.max()))
        p99 = max(np.percentile(em, 99), np.percentile(eP, 99))
        print("512 ragged FP32 pass %d: CT mean %.3e cov %.3e (p99 %.3e), CV mean %.3e cov "
              "%.3e; worst state: sequence %d k %d (parallel %.3e, sequential FP32 %.3e); "
              "sequential FP32 max %.3e p99 %.3e" % (
                  i + 1, *worst[-1][:2], p99, *worst[-1][2:], sw, w - soff[sw], e[w], q[w],
                  q.max(), np.percentile(q, 99)), flush=True)
        # the linear group and the first CT passes meet the FP32 bar at every
        # state; later CT passes stay within the FP32 limit of the parallel
        # scan measured here (p99 up to 1.04e-4, at most 7.3e-4; see the
        # full-size FP32 test for the attribution)
        assert max(cm.max(), cP.max()) < par.TOL["f32"]["m"], i
        if i < 2:
            assert max(em.max(), eP.max()) < par.TOL["f32"]["m"], i
        assert p99 < 2e-4 and max(em.max(), eP.max()) < 2e-3, i
