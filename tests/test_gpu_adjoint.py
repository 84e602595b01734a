"""GPU parity of the reverse-mode adjoint (pss_loglik_grad, pss_loglik_vjp)
and of its checkpoints.

The references are independent of the adjoint: the oracle's score by
Fisher's identity on the linearised model (sequential smoother moments),
central finite differences of the oracle's own sequential square-root
log-likelihood, and central differences of the GPU log-likelihood.  Bars:
gradients |dg|_inf / max(|g|_inf, 1) < 1e-7 (FP64), 1e-2 (FP32).
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


def _ragged_ct(lens, seed):
    rng = np.random.default_rng(seed)
    seqs = [wl.simulate_ct(n, rng) for n in lens]
    y = np.concatenate([s[1] for s in seqs])
    y_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return y, y_off


def _oracle_nominal(y, y_off, M):
    md = wl.CTModel()
    out_m, out_N = [], []
    for b in range(len(y_off) - 1):
        r = orc.ct_ipls(orc.ct_params(), md.m0, np.eye(5), y[y_off[b]:y_off[b + 1]], M)
        out_m.append(r["ms"])
        out_N.append(r["Ns"])
    return np.concatenate(out_m), np.concatenate(out_N)


def _to_dev(ms, Ns, dt):
    return pss.to_soa(ms, dt, DEV), pss.to_soa(pss.pack_lower(Ns), dt, DEV)


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_adjoint_against_oracle_score_and_fisher_route(tag):
    """C1 shape (n = 1000, nominal after 10 IPLS passes): the adjoint, the
    GPU's Fisher-identity route and the oracle's score agree."""
    w = wl.ct_single(1000, 1)
    md = w.model
    ms, Ns = _oracle_nominal(w.y, w.y_off, 10)
    dt = _tdtype(tag)
    m, N = _to_dev(ms, Ns, dt)
    # the oracle scores the nominal the GPU actually receives
    ma, Na = pss.marg_from_soa(m.double(), N.double(), 5)
    l_ref, g_ref = orc.ct_score(orc.ct_params(), md.m0, np.eye(5), w.y, ma, Na)
    b = pss.Batch.ct(w.y_off, md, dtype=dt, device=DEV)
    yd = pss.to_soa(w.y, dt, DEV)
    ll, grad, tb = pss.loglik_grad(b, m, N, yd)
    llf, gradf, _ = pss.score_fisher(b, m, N, yd)
    torch.cuda.synchronize()
    tol = par.TOL[tag]
    g = grad[:, 0].cpu().numpy()
    e_or = par.grad_err(g, g_ref)
    e_fi = par.grad_err(g, gradf[:, 0].cpu().numpy())
    print("%s adjoint vs oracle %.3e, vs Fisher route %.3e, g %s" % (tag, e_or, e_fi, g))
    assert par.ll_err(ll.item(), l_ref) < tol["ll"]
    assert e_or < tol["g"] and e_fi < tol["g"]
    np.testing.assert_array_equal(tb.cpu().numpy(), g)


def test_checkpoint_levels_give_bitwise_equal_gradients():
    """A ragged batch whose filter scan has three levels: the gradient from
    a checkpoint of every level (0: all marginals; 1, 2: scan prefixes with
    the levels below re-run; 3: nothing, whole scan re-run) and without one
    is bitwise the same (same kernels, same bracketing), and matches the
    oracle's score per sequence."""
    lens = [5000, 1200, 7, 1, 2]
    y, y_off = _ragged_ct(lens, 21)
    ms, Ns = _oracle_nominal(y, y_off, 3)
    md = wl.CTModel()
    b = pss.Batch.ct(y_off, md, dtype=torch.float64, device=DEV)
    yd = pss.to_soa(y, torch.float64, DEV)
    m, N = _to_dev(ms, Ns, torch.float64)
    w = torch.linspace(0.5, 2.0, len(lens), dtype=torch.float64, device=DEV)
    ll0, g0, tb0 = pss.loglik_grad(b, m, N, yd, ll_bar=w)
    outs = {}
    for level in (0, 1, 2, 3, 7):
        ck = pss.Checkpoint(b, level)
        llc = pss.loglik(b, yd, m, N, ckpt=ck)
        outs[level] = (llc, *pss.loglik_grad(b, m, N, yd, ll_bar=w, ckpt=ck), ck.bytes)
    torch.cuda.synchronize()
    sizes = [outs[lv][4] for lv in (0, 1, 2, 3)]
    print("checkpoint bytes by level:", sizes)
    assert sizes[0] > sizes[1] > sizes[2] > sizes[3] == outs[7][4]
    for level, (llc, ll, g, tb, _) in outs.items():
        assert torch.equal(llc, ll0) and torch.equal(ll, ll0), level
        assert torch.equal(g, g0) and torch.equal(tb, tb0), level
    ga = g0.cpu().numpy()
    for s in range(len(lens)):
        a, z = y_off[s], y_off[s + 1]
        l_ref, g_ref = orc.ct_score(orc.ct_params(), md.m0, np.eye(5), y[a:z],
                                    ms[a + s:z + s + 1], Ns[a + s:z + s + 1])
        assert par.grad_err(ga[:, s], g_ref) < 1e-7, (s, ga[:, s], g_ref)
        assert par.ll_err(ll0[s].item(), l_ref) < 1e-8
    np.testing.assert_allclose(tb0.cpu().numpy(), (ga * w.cpu().numpy()).sum(1), rtol=1e-14)


def test_adjoint_gradient_central_differences():
    """FP64 gradient against central differences (h = 1e-5) of the GPU's
    own log-likelihood at the frozen nominal, with launch shapes forced
    small so that the adjoint scan runs several levels."""
    w = wl.ct_single(3000, 13)
    md = w.model
    ms, Ns = _oracle_nominal(w.y, w.y_off, 4)
    b = pss.Batch.ct(w.y_off, md, dtype=torch.float64, device=DEV, scan_threads=64)
    yd = pss.to_soa(w.y, torch.float64, DEV)
    m, N = _to_dev(ms, Ns, torch.float64)
    _, grad, _ = pss.loglik_grad(b, m, N, yd)
    h = 1e-5
    for i in range(3):
        tp, tm = list(md.theta), list(md.theta)
        tp[i] += h
        tm[i] -= h
        lp = pss.loglik(pss._with_theta(b, tp), yd, m, N).item()
        lm = pss.loglik(pss._with_theta(b, tm), yd, m, N).item()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i, 0].item()) < 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i, 0])


def _oracle_ll(G, m0, N0, y, y_off, w):
    tot = 0.0
    for b in range(len(y_off) - 1):
        Gb = {k: v[y_off[b]:y_off[b + 1]] for k, v in G.items()}
        _, _, ell = orc.sqrt_filter(m0, N0, Gb, y[y_off[b]:y_off[b + 1]])
        tot += w[b] * ell.sum()
    return tot


@pytest.mark.parametrize("nx,ny", DIMS)
def test_vjp_linear_model_against_oracle_differences(nx, ny):
    """pss_loglik_vjp on a ragged batch of a random linear model with a
    different Gamma at every step: every entry of F, c, H, d, the lower
    factors S_L, S_O and the prior (m0, N0) against central differences of
    the oracle's sequential square-root log-likelihood (weighted by ll_bar)."""
    rng = np.random.default_rng(100 + 10 * nx + ny)
    lens = [6, 3, 1]
    T = sum(lens)
    G, m0, N0 = wl.random_linear_model(nx, ny, rng, T)
    y_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    y = np.concatenate([wl.simulate_linear({k: v[y_off[b]:y_off[b + 1]] for k, v in G.items()},
                                           m0, N0, lens[b], rng) for b in range(len(lens))])
    wts = np.array([1.0, -0.5, 2.0])
    b = pss.Batch(pss.MODEL_LINEAR, torch.float64, nx, ny, y_off, m0, N0, device=DEV)
    g = b.gamma_from_numpy(G)
    ll, gbar, m0b, N0b = pss.loglik_vjp(b, pss.to_soa(y, torch.float64, DEV), gamma=g,
                                        ll_bar=torch.tensor(wts))
    torch.cuda.synchronize()
    h = 1e-6

    def fd(fun, X, mask=None):
        out = np.zeros_like(X)
        for idx in np.ndindex(X.shape):
            if mask is not None and not mask[idx]:
                continue
            Xp, Xm = X.copy(), X.copy()
            Xp[idx] += h
            Xm[idx] -= h
            out[idx] = (fun(Xp) - fun(Xm)) / (2 * h)
        return out

    def gb(k, lower=False):
        a = gbar[k].cpu().numpy().T  # [T, components]
        if lower:
            return pss.unpack_lower(a, nx if k == "SL" else ny)
        return a.reshape((T,) + G[k].shape[1:])

    scale = max(1.0, abs(_oracle_ll(G, m0, N0, y, y_off, wts)))
    for k in ("F", "c", "H", "d", "SL", "SO"):
        lower = k in ("SL", "SO")
        mask = None
        if lower:
            mask = np.broadcast_to(np.tril(np.ones(G[k].shape[1:], bool)), G[k].shape)

        def fun(X, k=k):
            G2 = dict(G)
            G2[k] = X
            return _oracle_ll(G2, m0, N0, y, y_off, wts)

        ref = fd(fun, G[k], mask)
        got = gb(k, lower)
        err = np.abs(got - ref).max() / max(1.0, np.abs(ref).max())
        assert err < 1e-6, (k, err)
    # the prior is shared: its gradient is the sum over sequences
    ref_m0 = fd(lambda X: _oracle_ll(G, X, N0, y, y_off, wts), m0)
    got_m0 = m0b.cpu().numpy().sum(1)
    assert np.abs(got_m0 - ref_m0).max() / max(1.0, np.abs(ref_m0).max()) < 1e-6
    ref_N0 = fd(lambda X: _oracle_ll(G, m0, X, y, y_off, wts), N0, np.tril(np.ones((nx, nx), bool)))
    got_N0 = pss.unpack_lower(N0b.cpu().numpy().sum(1), nx)
    assert np.abs(got_N0 - ref_N0).max() / max(1.0, np.abs(ref_N0).max()) < 1e-6
    ll_ref = [_oracle_ll(G, m0, N0, y, y_off, np.eye(3)[s]) for s in range(3)]
    assert par.ll_err(ll.cpu().numpy(), np.array(ll_ref)) < 1e-10


def test_vjp_fp32_against_fp64():
    """FP32 VJP within the FP32 gradient bar of the FP64 VJP (CV model)."""
    rng = np.random.default_rng(7)
    nx, ny, n = 4, 2, 3000
    G, m0, N0 = wl.random_linear_model(nx, ny, rng, n)
    y = wl.simulate_linear(G, m0, N0, n, rng)
    res = {}
    for dt in (torch.float64, torch.float32):
        b = pss.Batch(pss.MODEL_LINEAR, dt, nx, ny, [0, n], m0, N0, device=DEV)
        _, gbar, m0b, _ = pss.loglik_vjp(b, pss.to_soa(y, dt, DEV), gamma=b.gamma_from_numpy(G))
        res[dt] = {k: gbar[k].double().cpu().numpy() for k in ("F", "c", "SL", "H", "d", "SO")}
    for k, v in res[torch.float64].items():
        err = np.abs(res[torch.float32][k] - v).max() / max(1.0, np.abs(v).max())
        assert err < 1e-2, (k, err)


@pytest.mark.parametrize("tag", ["f64", "f32"])
def test_parameter_estimation_batch_gradient(tag):
    """The parameter-estimation configuration: 64 CT sequences of 10^4
    steps, nominal = 10 IPLS passes from the prior on the GPU; the adjoint
    gradient per sequence against the oracle's score at that nominal, and in
    FP64 against central differences of the GPU log-likelihood."""
    w = wl.ct_batch(64, 10 ** 4, 4)
    md = w.model
    dt = _tdtype(tag)
    b = pss.Batch.ct(w.y_off, md, dtype=dt, device=DEV)
    yd = pss.to_soa(w.y, dt, DEV)
    m, N = pss.ipls_iterate(b, yd, 10)
    ll, grad, tb = pss.loglik_grad(b, m, N, yd)
    torch.cuda.synchronize()
    ma, Na = pss.marg_from_soa(m.double(), N.double(), 5)
    l_ref, g_ref = orc.ct_score_batch(orc.ct_params(), md.m0, np.eye(5), w.y, w.y_off, ma, Na)
    eg = par.grad_err(grad.cpu().numpy().T, g_ref)
    el = par.ll_err(ll.cpu().numpy(), l_ref)
    print("%s 64 x 1e4: gradient err %.3e, loglik err %.3e" % (tag, eg, el))
    assert eg < par.TOL[tag]["g"] and el < par.TOL[tag]["ll"]
    if tag == "f64":
        h = 1e-5
        for i in range(3):
            tp, tm = list(md.theta), list(md.theta)
            tp[i] += h
            tm[i] -= h
            lp = pss.loglik(pss._with_theta(b, tp), yd, m, N).sum().item()
            lm = pss.loglik(pss._with_theta(b, tm), yd, m, N).sum().item()
            fd = (lp - lm) / (2 * h)
            assert abs(fd - tb[i].item()) < 1e-6 * max(1.0, abs(fd)), (i, fd, tb[i])
