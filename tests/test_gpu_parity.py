"""GPU parity of every C-ABI entry point against the FP64 oracle.

All inputs are seeded and synthetic (paper_2207_00426_amd.workloads); the
oracle and the HIP library share nothing but those inputs.  Scan parity is
checked at sizes that span several tiles with a ragged tail (launch shapes
forced small so that the multi-level path runs), for every built (nx, ny),
for ragged batches, and for the degenerate n = 1 and n = 2 sequences.
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
DIMS = [(1, 1), (2, 1), (2, 3), (3, 2), (3, 3), (4, 2), (5, 2)]


def _tdtype(tag):
    return torch.float64 if tag == "f64" else torch.float32


def _linear_case(nx, ny, lengths, seed, per_step=True):
    rng = np.random.default_rng(seed)
    T = int(np.sum(lengths))
    G, m0, N0 = wl.random_linear_model(nx, ny, rng, T if per_step else None)
    y_off = np.zeros(len(lengths) + 1, dtype=np.int64)
    y_off[1:] = np.cumsum(lengths)
    ys = []
    for b in range(len(lengths)):
        if per_step:
            Gb = {k: v[y_off[b]:y_off[b + 1]] for k, v in G.items()}
        else:
            Gb = G
        ys.append(wl.simulate_linear(Gb, m0, N0, int(lengths[b]), rng))
    return G, m0, N0, np.concatenate(ys), y_off


def _seq_gamma(G, y_off, b):
    if np.asarray(G["F"]).ndim == 3:
        return {k: v[y_off[b]:y_off[b + 1]] for k, v in G.items()}
    return G


def _oracle_linear(G, m0, N0, y, y_off):
    out = []
    for b in range(len(y_off) - 1):
        Gb = _seq_gamma(G, y_off, b)
        yb = y[y_off[b]:y_off[b + 1]]
        mf, Nf, ell = orc.sqrt_filter(m0, N0, Gb, yb)
        ms, Ns, _ = orc.sqrt_smoother(Gb, mf, Nf)
        out.append(dict(mf=mf, Nf=Nf, ms=ms, Ns=Ns, ll=ell.sum()))
    return out


def _split_states(arr, y_off):
    return [arr[y_off[b] + b:y_off[b + 1] + b + 1] for b in range(len(y_off) - 1)]


@pytest.mark.parametrize("tag", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", DIMS)
def test_linear_filter_smoother_multilevel(nx, ny, tag):
    """Elements, filter scan and smoother scan over a ragged batch whose
    sequences span several tiles (T = 64, E = 2 -> tiles of 128 steps)."""
    lengths = np.array([1, 2, 300, 129, 1000])
    G, m0, N0, y, y_off = _linear_case(nx, ny, lengths, 100 * nx + ny)
    ref = _oracle_linear(G, m0, N0, y, y_off)
    dt = _tdtype(tag)
    b = pss.Batch(pss.MODEL_LINEAR, dt, nx, ny, y_off, m0, N0, device=DEV, scan_threads=64,
                  scan_elems=2)
    g = b.gamma_from_numpy(G)
    yd = pss.to_soa(y, dt, DEV)
    el = pss.sqrt_filter_elements(b, g, yd)
    mf, Nf = pss.sqrt_filter_scan(b, el)
    ms, Ns = pss.sqrt_smoother_scan(b, g, mf, Nf)
    torch.cuda.synchronize()
    tol = par.TOL[tag]
    mfa, Nfa = pss.marg_from_soa(mf, Nf, nx)
    msa, Nsa = pss.marg_from_soa(ms, Ns, nx)
    for bi, (r, a1, a2, a3, a4) in enumerate(zip(ref, _split_states(mfa, y_off),
                                                 _split_states(Nfa, y_off),
                                                 _split_states(msa, y_off),
                                                 _split_states(Nsa, y_off))):
        em, eP = par.marg_errs(a1, a2, r["mf"], r["Nf"])
        assert em < tol["m"] and eP < tol["P"], ("filter", bi, em, eP)
        em, eP = par.marg_errs(a3, a4, r["ms"], r["Ns"])
        assert em < tol["m"] and eP < tol["P"], ("smoother", bi, em, eP)


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_linear_many_sequences_default_shapes(tag):
    """150 ragged sequences (more than 64, so the level planner takes its
    block-wide path) at the default launch shapes: the filter's flat finest
    level, its interleaved next level and the smoother's tree, per sequence
    against the oracle."""
    rng = np.random.default_rng(77)
    lengths = rng.integers(1, 700, size=150)
    lengths[:3] = [1, 256, 257]
    G, m0, N0, y, y_off = _linear_case(4, 2, lengths, 4242)
    ref = _oracle_linear(G, m0, N0, y, y_off)
    dt = _tdtype(tag)
    b = pss.Batch(pss.MODEL_LINEAR, dt, 4, 2, y_off, m0, N0, device=DEV)
    g = b.gamma_from_numpy(G)
    yd = pss.to_soa(y, dt, DEV)
    el = pss.sqrt_filter_elements(b, g, yd)
    mf, Nf = pss.sqrt_filter_scan(b, el)
    ms, Ns = pss.sqrt_smoother_scan(b, g, mf, Nf)
    torch.cuda.synchronize()
    tol = par.TOL[tag]
    mfa, Nfa = pss.marg_from_soa(mf, Nf, 4)
    msa, Nsa = pss.marg_from_soa(ms, Ns, 4)
    for bi, (r, a1, a2, a3, a4) in enumerate(zip(ref, _split_states(mfa, y_off),
                                                 _split_states(Nfa, y_off),
                                                 _split_states(msa, y_off),
                                                 _split_states(Nsa, y_off))):
        em, eP = par.marg_errs(a1, a2, r["mf"], r["Nf"])
        assert em < tol["m"] and eP < tol["P"], ("filter", bi, em, eP)
        em, eP = par.marg_errs(a3, a4, r["ms"], r["Ns"])
        assert em < tol["m"] and eP < tol["P"], ("smoother", bi, em, eP)


@pytest.mark.parametrize("nx,ny", [(5, 2), (2, 3), (3, 3)])
def test_filter_elements_match_tables_1_2(nx, ny):
    lengths = np.array([7, 1, 4])
    G, m0, N0, y, y_off = _linear_case(nx, ny, lengths, 7 + nx)
    b = pss.Batch(pss.MODEL_LINEAR, torch.float64, nx, ny, y_off, m0, N0, device=DEV)
    el = pss.sqrt_filter_elements(b, b.gamma_from_numpy(G), pss.to_soa(y, torch.float64, DEV))
    torch.cuda.synchronize()
    A = pss.from_soa(el["A"], (nx, nx))
    bb = pss.from_soa(el["b"], (nx,))
    U = pss.unpack_lower(pss.from_soa(el["U"], (pss.tri(nx),)), nx)
    eta = pss.from_soa(el["eta"], (nx,))
    Z = pss.unpack_lower(pss.from_soa(el["Z"], (pss.tri(nx),)), nx)
    for s in range(len(lengths)):
        Gb = _seq_gamma(G, y_off, s)
        refs = orc.filter_elements(m0, N0, Gb, y[y_off[s]:y_off[s + 1]])
        for k, (rA, rb, rU, reta, rZ) in enumerate(refs):
            t = y_off[s] + k
            np.testing.assert_allclose(A[t], rA, rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(bb[t], rb, rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(eta[t], reta, rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(par.gram(U[t]), par.gram(rU), rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(par.gram(Z[t]), par.gram(rZ), rtol=1e-9, atol=1e-11)
            assert np.all(np.diag(U[t]) >= 0) and np.all(np.diag(Z[t]) >= 0)
            # Z = Tria([Z_k, 0]) with Z_k of ny columns: the columns from ny
            # on are exactly zero (the scan reads only the first ny)
            assert np.all(Z[t][:, ny:] == 0.0)


def test_scalar_random_walk_steady_state():
    """Closed-form Riccati limit through the HIP scans (q = r = 1)."""
    n = 3000
    G = dict(F=np.eye(1), c=np.zeros(1), SL=np.eye(1), H=np.eye(1), d=np.zeros(1),
             SO=np.eye(1))
    y = np.random.default_rng(3).standard_normal((n, 1))
    b = pss.Batch(pss.MODEL_LINEAR, torch.float64, 1, 1, [0, n], np.zeros(1), np.eye(1),
                  device=DEV)
    g = b.gamma_from_numpy(G)
    m, N = pss.ipls_iterate(b, pss.to_soa(y, torch.float64, DEV), 1, gamma=g)
    torch.cuda.synchronize()
    Ns = pss.from_soa(N, (1,))[:, 0]
    assert abs(Ns[n // 2] ** 2 - 1 / np.sqrt(5)) < 1e-12


def test_cv_single_sequence_end_to_end():
    """Constant-velocity model, n = 100, FP64: filter, smoother and loglik."""
    w = wl.cv_single(100, 0)
    md = w.model
    G = dict(F=md.F(), c=np.zeros(4), SL=np.linalg.cholesky(md.Q()), H=md.H(), d=np.zeros(2),
             SO=np.linalg.cholesky(md.R()))
    mf_r, Nf_r, ell = orc.sqrt_filter(md.m0, np.eye(4), G, w.y)
    ms_r, Ns_r, _ = orc.sqrt_smoother(G, mf_r, Nf_r)
    b = pss.Batch(pss.MODEL_LINEAR, torch.float64, 4, 2, w.y_off, md.m0, np.eye(4), device=DEV)
    g = b.gamma_from_numpy(G)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, N, mf, Nf = pss.ipls_iterate(b, yd, 1, gamma=g, want_filter=True)
    ll = pss.loglik(b, yd, gamma=g)
    torch.cuda.synchronize()
    em, eP = par.marg_errs(*pss.marg_from_soa(mf, Nf, 4), mf_r, Nf_r)
    assert em < 1e-9 and eP < 1e-9
    em, eP = par.marg_errs(*pss.marg_from_soa(m, N, 4), ms_r, Ns_r)
    assert em < 1e-9 and eP < 1e-9
    assert par.ll_err(ll.item(), ell.sum()) < 1e-8


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_ct_slr_matches_oracle(tag):
    w = wl.ct_single(400, 1)
    md = w.model
    prm = orc.ct_params()
    nom = orc.ct_ipls(prm, md.m0, np.eye(5), w.y, 2)  # a realistic nominal
    ref = orc.ct_linearize(prm, nom["ms"], nom["Ns"], w.y)
    dt = _tdtype(tag)
    b = pss.Batch.ct(w.y_off, md, dtype=dt, device=DEV)
    m = pss.to_soa(nom["ms"], dt, DEV)
    N = pss.to_soa(pss.pack_lower(nom["Ns"]), dt, DEV)
    g = pss.slr_linearize(b, m, N, pss.to_soa(w.y, dt, DEV))
    torch.cuda.synchronize()
    tol = 1e-9 if tag == "f64" else 2e-4
    # offsets are differences zbar - G m of O(|x|) terms: compare them on that scale
    Fm = np.abs(np.einsum("kij,kj->ki", ref["F"], nom["ms"][:-1])).max(axis=1, keepdims=True)
    Hm = np.abs(np.einsum("kij,kj->ki", ref["H"], nom["ms"][1:])).max(axis=1, keepdims=True)
    for key, shape, extra in (("F", (5, 5), 0.0), ("c", (5,), Fm), ("H", (2, 5), 0.0),
                              ("d", (2,), Hm)):
        got = pss.from_soa(g[key], shape)
        scale = np.maximum(np.abs(ref[key]).max(axis=tuple(range(1, ref[key].ndim)),
                                                    keepdims=True), 1.0)
        if key in ("c", "d"):
            scale = np.maximum(scale.reshape(-1, 1), extra)
        else:
            scale = scale.reshape((-1,) + (1,) * (ref[key].ndim - 1))
        assert np.max(np.abs(got - ref[key]) / scale) < tol, key
    for key, n in (("SL", 5), ("SO", 2)):
        got = pss.unpack_lower(pss.from_soa(g[key], (pss.tri(n),)), n)
        assert par.cov_err(par.gram(got), par.gram(ref[key])) < (1e-9 if tag == "f64" else 1e-3)


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_ct_ipls_per_pass_parity(tag):
    """Coordinated-turn, n = 1000, 10 cubature IPLS passes from the prior
    nominal: parity of the nominal after every pass, and of the final
    filter marginals."""
    w = wl.ct_single(1000, 1)
    md = w.model
    prm = orc.ct_params()
    ref = orc.ct_ipls(prm, md.m0, np.eye(5), w.y, 10, history=True)
    dt = _tdtype(tag)
    b = pss.Batch.ct(w.y_off, md, dtype=dt, device=DEV)
    yd = pss.to_soa(w.y, dt, DEV)
    m, N = b.prior_nominal()
    tol = par.TOL[tag]
    errs = []
    for i in range(10):
        out = pss.ipls_iterate(b, yd, 1, m, N, want_filter=(i == 9))
        torch.cuda.synchronize()
        ms, Ns = pss.marg_from_soa(m, N, 5)
        assert np.isfinite(ms).all() and np.isfinite(Ns).all(), "NaN at pass %d" % i
        errs.append(par.marg_errs(ms, Ns, ref["hist_ms"][i], ref["hist_Ns"][i]))
    print("per-pass errors", tag, errs)
    for i, (em, eP) in enumerate(errs):
        assert em < tol["m"] and eP < tol["P"], (i, em, eP)
    mf, Nf = pss.marg_from_soa(out[2], out[3], 5)
    em, eP = par.marg_errs(mf, Nf, ref["mf"], ref["Nf"])
    assert em < tol["m"] and eP < tol["P"]


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_ct_loglik_and_gradient(tag):
    w = wl.ct_single(500, 12)
    md = w.model
    prm = orc.ct_params()
    nom = orc.ct_ipls(prm, md.m0, np.eye(5), w.y, 4)
    l_ref, g_ref = orc.ct_score(prm, md.m0, np.eye(5), w.y, nom["ms"], nom["Ns"])
    dt = _tdtype(tag)
    b = pss.Batch.ct(w.y_off, md, dtype=dt, device=DEV)
    yd = pss.to_soa(w.y, dt, DEV)
    m = pss.to_soa(nom["ms"], dt, DEV)
    N = pss.to_soa(pss.pack_lower(nom["Ns"]), dt, DEV)
    ll = pss.loglik(b, yd, m, N)
    ll2, grad, tb = pss.loglik_grad(b, m, N, yd)
    torch.cuda.synchronize()
    tol = par.TOL[tag]
    assert par.ll_err(ll.item(), l_ref) < tol["ll"]
    assert par.ll_err(ll2.item(), l_ref) < tol["ll"]
    assert par.grad_err(grad[:, 0].cpu().numpy(), g_ref) < tol["g"], (grad, g_ref)
    np.testing.assert_allclose(tb.cpu().numpy(), grad[:, 0].cpu().numpy(), rtol=0, atol=0)
    if tag == "f64":  # central finite differences of the GPU log-likelihood itself
        h = 1e-5
        for i in range(3):
            tp, tm = list(md.theta), list(md.theta)
            tp[i] += h
            tm[i] -= h
            lp = pss.loglik(pss._with_theta(b, tp), yd, m, N).item()
            lm = pss.loglik(pss._with_theta(b, tm), yd, m, N).item()
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[i, 0].item()) < 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i, 0])


def test_autograd_function_backward():
    w = wl.ct_batch(B=3, n=200, seed=5)
    md = w.model
    prm = orc.ct_params()
    b = pss.Batch.ct(w.y_off, md, dtype=torch.float64, device=DEV)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, N = pss.ipls_iterate(b, yd, 3)
    theta = torch.tensor(md.theta + 0.1, dtype=torch.float64, requires_grad=True)
    ll = pss.LogLik.apply(theta, b, yd, m, N)
    (2.0 * ll).backward()
    ms, Ns = pss.marg_from_soa(m, N, 5)
    th = md.theta + 0.1
    _, g_ref = orc.ct_score_batch(orc.ct_theta_params(th), md.m0, np.eye(5), w.y, w.y_off, ms,
                                  Ns)
    assert par.grad_err(theta.grad.numpy(), 2.0 * g_ref.sum(0)) < 1e-7


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_sequential_comparator_matches_oracle(tag):
    w = wl.ct_single(300, 4)
    md = w.model
    prm = orc.ct_params()
    ref = orc.ct_ipls(prm, md.m0, np.eye(5), w.y, 3)
    dt = _tdtype(tag)
    b = pss.Batch.ct(w.y_off, md, dtype=dt, device=DEV)
    m, N = pss.sequential_smoother(b, pss.to_soa(w.y, dt, DEV), 3)
    torch.cuda.synchronize()
    em, eP = par.marg_errs(*pss.marg_from_soa(m, N, 5), ref["ms"], ref["Ns"])
    tol = par.TOL[tag]
    assert em < tol["m"] and eP < tol["P"]


@pytest.mark.parametrize("tag", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", DIMS)
def test_sequential_comparator_linear_every_dim(nx, ny, tag):
    """The comparator (one wave per sequence from nx = 2, one thread for
    nx = 1) on a ragged batch with n = 1 and n = 2 sequences, per-step Gamma:
    filtering and smoothing marginals at every state against the oracle's
    sequential square-root recursions."""
    lengths = np.array([1, 2, 300, 129, 64])
    G, m0, N0, y, y_off = _linear_case(nx, ny, lengths, 7 * nx + ny)
    ref = _oracle_linear(G, m0, N0, y, y_off)
    dt = _tdtype(tag)
    b = pss.Batch(pss.MODEL_LINEAR, dt, nx, ny, y_off, m0, N0, device=DEV)
    ms, Ns, mf, Nf = pss.sequential_smoother(b, pss.to_soa(y, dt, DEV), 1,
                                             gamma=b.gamma_from_numpy(G), want_filter=True)
    torch.cuda.synchronize()
    tol = par.TOL[tag]
    mfa, Nfa = pss.marg_from_soa(mf, Nf, nx)
    msa, Nsa = pss.marg_from_soa(ms, Ns, nx)
    for bi, (r, a1, a2, a3, a4) in enumerate(zip(ref, _split_states(mfa, y_off),
                                                 _split_states(Nfa, y_off),
                                                 _split_states(msa, y_off),
                                                 _split_states(Nsa, y_off))):
        em, eP = par.marg_errs(a1, a2, r["mf"], r["Nf"])
        assert em < tol["m"] and eP < tol["P"], ("filter", bi, em, eP)
        em, eP = par.marg_errs(a3, a4, r["ms"], r["Ns"])
        assert em < tol["m"] and eP < tol["P"], ("smoother", bi, em, eP)


def test_batch_equals_single_and_is_deterministic():
    """A ragged CT batch gives, per sequence, bitwise the single-sequence
    result (tiles never cross sequences); two runs are bitwise equal."""
    w = wl.ct_batch(B=4, n=150, seed=9)
    lens = [150, 37, 400, 1]
    rng = np.random.default_rng(0)
    seqs = [wl.simulate_ct(n, rng) for n in lens]
    y = np.concatenate([s[1] for s in seqs])
    y_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    md = w.model
    b = pss.Batch.ct(y_off, md, dtype=torch.float64, device=DEV, scan_threads=64, scan_elems=2)
    yd = pss.to_soa(y, torch.float64, DEV)
    m1, N1 = pss.ipls_iterate(b, yd, 3)
    m2, N2 = pss.ipls_iterate(b, yd, 3)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2) and torch.equal(N1, N2)
    ma = m1.cpu().numpy()
    for s in range(len(lens)):
        bs = pss.Batch.ct([0, lens[s]], md, dtype=torch.float64, device=DEV, scan_threads=64,
                          scan_elems=2)
        ms, Ns = pss.ipls_iterate(bs, pss.to_soa(seqs[s][1], torch.float64, DEV), 3)
        torch.cuda.synchronize()
        a, z = y_off[s] + s, y_off[s + 1] + s + 1
        assert np.array_equal(ma[:, a:z], ms.cpu().numpy())
    ref = [orc.ct_ipls(orc.ct_params(), md.m0, np.eye(5), s[1], 3) for s in seqs]
    msa, Nsa = pss.marg_from_soa(m1, N1, 5)
    for s in range(len(lens)):
        em, eP = par.marg_errs(msa[y_off[s] + s:y_off[s + 1] + s + 1],
                               Nsa[y_off[s] + s:y_off[s + 1] + s + 1], ref[s]["ms"], ref[s]["Ns"])
        assert em < 1e-9 and eP < 1e-9
