"""FP64 CPU oracle (test infrastructure only).

Plain sequential reference for the parallel square-root iterated smoother of
Yaghoobi, Corenflos, Hassan and Sarkka.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the HIP library
never does, and the two share no code.

Layout: numpy arrays, one row-major block per step/state, e.g. ``Nf`` has
shape ``(n+1, nx, nx)`` and the linearisation parameters of step slot ``j``
(transition x_j -> x_{j+1}, measurement of y_{j+1}) are ``F[j], c[j], SL[j],
H[j], d[j], SO[j]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over sequences)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.or_ct_loglik.restype = ctypes.c_double
        _lib.or_ct_score.restype = ctypes.c_double
        _lib.or_lgssm_score_terms.restype = ctypes.c_double
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


I = ctypes.c_int
L = ctypes.c_long


def max_threads() -> int:
    return int(_load().or_max_threads())


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------
def tria(A):
    """Tria(A) of Section 2.2: lower r x r with Tria(A) Tria(A)^T = A A^T."""
    A = _f64(A)
    r, c = A.shape
    Lo = np.zeros((r, r))
    _load().or_tria(I(r), I(c), _p(A), _p(Lo))
    return Lo


def downdate(A, B):
    """DownDate(A, B) of Section 2.2 via rank-1 Cholesky downdates."""
    A = _f64(A)
    B = _f64(B)
    n, m = B.shape
    Lo = np.zeros((n, n))
    bad = _load().or_downdate(I(n), I(m), _p(A), _p(B), _p(Lo))
    return Lo, int(bad)


def cholesky(P):
    P = _f64(P)
    n = P.shape[0]
    Lo = np.zeros((n, n))
    rc = _load().or_cholesky(I(n), _p(P), _p(Lo))
    if rc != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return Lo


def sigma_points(m, N):
    m = _f64(m)
    N = _f64(N)
    nx = m.shape[0]
    Xp = np.zeros((nx, nx))
    Xm = np.zeros((nx, nx))
    _load().or_sigma_points(I(nx), _p(m), _p(N), _p(Xp), _p(Xm))
    return Xp, Xm


def slr(m, N, Zp, Zm, Snoise, literal=False):
    """Cubature SLR from the images Zp[i] = g(X+_i), Zm[i] = g(X-_i).

    Returns (G, offset, S) with the affine fit g(x) ~ G x + offset and the
    lower factor S of the noise-plus-linearisation-error covariance.
    """
    m = _f64(m)
    N = _f64(N)
    Zp = _f64(Zp)
    Zm = _f64(Zm)
    Snoise = _f64(Snoise)
    nx = m.shape[0]
    nz = Zp.shape[1]
    G = np.zeros((nz, nx))
    off = np.zeros(nz)
    S = np.zeros((nz, nz))
    fn = _load().or_slr_literal if literal else _load().or_slr_residual
    bad = fn(I(nx), I(nz), _p(m), _p(N), _p(Zp), _p(Zm), _p(Snoise), _p(G), _p(off), _p(S))
    if literal:
        return G, off, S, int(bad)
    return G, off, S


# --------------------------------------------------------------------------
# CT model
# --------------------------------------------------------------------------
def ct_params(dt=0.01, q1=0.1, q2=0.1, sigma=0.05, sensors=((-1.5, 0.5), (1.0, 1.0))):
    return np.array([dt, q1, q2, sigma, sensors[0][0], sensors[0][1], sensors[1][0],
                     sensors[1][1]], dtype=np.float64)


def ct_f(prm, x):
    prm = _f64(prm)
    x = _f64(x)
    out = np.zeros(5)
    _load().or_ct_f(_p(prm), _p(x), _p(out))
    return out


def ct_h(prm, x, yref=None):
    prm = _f64(prm)
    x = _f64(x)
    out = np.zeros(2)
    if yref is None:
        _load().or_ct_h(_p(prm), _p(x), None, _p(out))
    else:
        yr = _f64(yref)
        _load().or_ct_h(_p(prm), _p(x), _p(yr), _p(out))
    return out


def ct_Q(prm):
    prm = _f64(prm)
    Q = np.zeros((5, 5))
    _load().or_ct_Q(_p(prm), _p(Q))
    return Q


METHODS = {"cubature": 0, "cubature_literal": 1, "taylor": 2}


def ct_linearize(prm, ms, Ns, y, literal=False, method=None):
    """Per-step linearisation of the CT model at the nominal (ms, Ns):
    method "cubature" (residual SLR, Section 4.3), "cubature_literal" (the
    printed Tria + DownDate form) or "taylor" (first-order, Section 4.2)."""
    if method is None:
        method = "cubature_literal" if literal else "cubature"
    prm = _f64(prm)
    ms = _f64(ms)
    Ns = _f64(Ns)
    y = _f64(y)
    n = y.shape[0]
    F = np.zeros((n, 5, 5)); c = np.zeros((n, 5)); SL = np.zeros((n, 5, 5))
    H = np.zeros((n, 2, 5)); d = np.zeros((n, 2)); SO = np.zeros((n, 2, 2))
    bad = _load().or_ct_linearize(I(n), _p(prm), _p(ms), _p(Ns), _p(y), I(METHODS[method]), _p(F),
                                  _p(c), _p(SL), _p(H), _p(d), _p(SO))
    return dict(F=F, c=c, SL=SL, H=H, d=d, SO=SO, bad=int(bad))


def ct_ipls(prm, m0, N0, y, M, ms_init=None, Ns_init=None, history=False, method="cubature"):
    """Algorithm 3 (sequential reference).  Initial nominal: the prior at every k.
    method "taylor": the iterated extended smoother (Section 4.2)."""
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y)
    n = y.shape[0]
    ms = np.repeat(m0[None], n + 1, axis=0) if ms_init is None else _f64(ms_init).copy()
    Ns = np.repeat(N0[None], n + 1, axis=0) if Ns_init is None else _f64(Ns_init).copy()
    hm = np.zeros((M, n + 1, 5)) if history else None
    hN = np.zeros((M, n + 1, 5, 5)) if history else None
    mf = np.zeros((n + 1, 5)); Nf = np.zeros((n + 1, 5, 5))
    rc = _load().or_ct_ipls(I(n), _p(prm), _p(m0), _p(N0), _p(y), I(M), _p(ms), _p(Ns),
                            _p(hm) if history else None, _p(hN) if history else None,
                            _p(mf), _p(Nf), I(METHODS[method]))
    if rc != 0:
        raise RuntimeError("oracle IPLS failed")
    out = dict(ms=ms, Ns=Ns, mf=mf, Nf=Nf)
    if history:
        out["hist_ms"] = hm
        out["hist_Ns"] = hN
    return out


def ct_loglik(prm, m0, N0, y, ms, Ns, per_step=False, method="cubature"):
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y); ms = _f64(ms); Ns = _f64(Ns)
    n = y.shape[0]
    ell = np.zeros(n)
    tot = _load().or_ct_loglik(I(n), _p(prm), _p(m0), _p(N0), _p(y), _p(ms), _p(Ns), _p(ell),
                               I(METHODS[method]))
    return (tot, ell) if per_step else tot


def ct_score(prm, m0, N0, y, ms, Ns, method="cubature"):
    """(loglik, d loglik / d (log q1, log q2, log sigma)) at a frozen nominal."""
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y); ms = _f64(ms); Ns = _f64(Ns)
    n = y.shape[0]
    g = np.zeros(3)
    tot = _load().or_ct_score(I(n), _p(prm), _p(m0), _p(N0), _p(y), _p(ms), _p(Ns), _p(g),
                              I(METHODS[method]))
    return tot, g


def ct_jac_f(prm, x):
    J = np.zeros((5, 5))
    _load().or_ct_jac_f(_p(_f64(prm)), _p(_f64(x)), _p(J))
    return J


def ct_jac_h(prm, x):
    J = np.zeros((2, 5))
    _load().or_ct_jac_h(_p(_f64(prm)), _p(_f64(x)), _p(J))
    return J


def ct_theta_params(theta, base=None):
    """prm vector for theta = (log q1, log q2, log sigma)."""
    prm = ct_params() if base is None else _f64(base).copy()
    prm[1] = np.exp(theta[0])
    prm[2] = np.exp(theta[1])
    prm[3] = np.exp(theta[2])
    return prm


# --------------------------------------------------------------------------
# linear(ised) models
# --------------------------------------------------------------------------
def _gamma(G, n, nx, ny):
    """Per-step arrays (stride 1) or one shared set (stride 0)."""
    F = _f64(G["F"])
    stride = 0 if F.ndim == 2 else 1
    return stride, F, _f64(G["c"]), _f64(G["SL"]), _f64(G["H"]), _f64(G["d"]), _f64(G["SO"])


def sqrt_filter(m0, N0, G, y):
    """Sequential square-root Kalman filter; returns (mf, Nf, ell)."""
    m0 = _f64(m0); N0 = _f64(N0); y = _f64(y)
    n, ny = y.shape
    nx = m0.shape[0]
    s, F, c, SL, H, d, SO = _gamma(G, n, nx, ny)
    mf = np.zeros((n + 1, nx)); Nf = np.zeros((n + 1, nx, nx)); ell = np.zeros(n)
    _load().or_sqrt_filter(I(n), I(nx), I(ny), _p(m0), _p(N0), _p(F), _p(c), _p(SL), _p(H),
                           _p(d), _p(SO), L(s), _p(y), _p(mf), _p(Nf), _p(ell))
    return mf, Nf, ell


def sqrt_smoother(G, mf, Nf):
    """Sequential square-root RTS smoother; returns (ms, Ns, E)."""
    mf = _f64(mf); Nf = _f64(Nf)
    n = mf.shape[0] - 1
    nx = mf.shape[1]
    F = _f64(G["F"])
    s = 0 if F.ndim == 2 else 1
    c = _f64(G["c"]); SL = _f64(G["SL"])
    ms = np.zeros_like(mf); Ns = np.zeros_like(Nf); E = np.zeros((max(n, 1), nx, nx))
    _load().or_sqrt_smoother(I(n), I(nx), _p(F), _p(c), _p(SL), L(s), _p(mf), _p(Nf), _p(ms),
                             _p(Ns), _p(E))
    return ms, Ns, E[:n]


def cov_filter(m0, P0, Gc, y):
    """Covariance-form KF. Gc holds F, c, Lam, H, d, Om. Returns (mf, Pf, mp, Pp, ell)."""
    m0 = _f64(m0); P0 = _f64(P0); y = _f64(y)
    n, ny = y.shape
    nx = m0.shape[0]
    F = _f64(Gc["F"])
    s = 0 if F.ndim == 2 else 1
    c = _f64(Gc["c"]); Lam = _f64(Gc["Lam"]); H = _f64(Gc["H"]); d = _f64(Gc["d"]); Om = _f64(Gc["Om"])
    mf = np.zeros((n + 1, nx)); Pf = np.zeros((n + 1, nx, nx))
    mp = np.zeros((n, nx)); Pp = np.zeros((n, nx, nx)); ell = np.zeros(n)
    rc = _load().or_cov_filter(I(n), I(nx), I(ny), _p(m0), _p(P0), _p(F), _p(c), _p(Lam), _p(H),
                               _p(d), _p(Om), L(s), _p(y), _p(mf), _p(Pf), _p(mp), _p(Pp), _p(ell))
    if rc != 0:
        raise np.linalg.LinAlgError("covariance filter failed")
    return mf, Pf, mp, Pp, ell


def cov_smoother(Gc, mf, Pf):
    mf = _f64(mf); Pf = _f64(Pf)
    n = mf.shape[0] - 1
    nx = mf.shape[1]
    F = _f64(Gc["F"])
    s = 0 if F.ndim == 2 else 1
    c = _f64(Gc["c"]); Lam = _f64(Gc["Lam"])
    ms = np.zeros_like(mf); Ps = np.zeros_like(Pf); G = np.zeros((max(n, 1), nx, nx))
    rc = _load().or_cov_smoother(I(n), I(nx), _p(F), _p(c), _p(Lam), L(s), _p(mf), _p(Pf), _p(ms),
                                 _p(Ps), _p(G))
    if rc != 0:
        raise np.linalg.LinAlgError("covariance smoother failed")
    return ms, Ps, G[:n]


def lgssm_score_terms(m0, P0, Gc, y):
    """(loglik, Lbar[n], Obar[n]): Fisher-identity sensitivities per step slot."""
    m0 = _f64(m0); P0 = _f64(P0); y = _f64(y)
    n, ny = y.shape
    nx = m0.shape[0]
    F = _f64(Gc["F"])
    s = 0 if F.ndim == 2 else 1
    c = _f64(Gc["c"]); Lam = _f64(Gc["Lam"]); H = _f64(Gc["H"]); d = _f64(Gc["d"]); Om = _f64(Gc["Om"])
    Lb = np.zeros((n, nx, nx)); Ob = np.zeros((n, ny, ny))
    tot = _load().or_lgssm_score_terms(I(n), I(nx), I(ny), _p(m0), _p(P0), _p(F), _p(c), _p(Lam),
                                       _p(H), _p(d), _p(Om), L(s), _p(y), _p(Lb), _p(Ob))
    return tot, Lb, Ob


# --------------------------------------------------------------------------
# parallel-form elements and operators (Lemmas 1-4)
# --------------------------------------------------------------------------
def filter_element_first(m0, N0, F0, c0, SL0, H1, d1, SO1, y1):
    nx = len(m0); ny = len(y1)
    A = np.zeros((nx, nx)); b = np.zeros(nx); U = np.zeros((nx, nx)); eta = np.zeros(nx); Z = np.zeros((nx, nx))
    args = [_f64(a) for a in (m0, N0, F0, c0, SL0, H1, d1, SO1, y1)]
    _load().or_filter_element_first(I(nx), I(ny), *[_p(a) for a in args], _p(A), _p(b), _p(U), _p(eta), _p(Z))
    return A, b, U, eta, Z


def filter_element(F, c, SL, H, d, SO, y):
    nx = F.shape[0]; ny = len(y)
    A = np.zeros((nx, nx)); b = np.zeros(nx); U = np.zeros((nx, nx)); eta = np.zeros(nx); Z = np.zeros((nx, nx))
    args = [_f64(a) for a in (F, c, SL, H, d, SO, y)]
    _load().or_filter_element(I(nx), I(ny), *[_p(a) for a in args], _p(A), _p(b), _p(U), _p(eta), _p(Z))
    return A, b, U, eta, Z


def filter_combine(ei, ej):
    """Square-root filtering operator (Lemma 2): ei (x) ej, each (A, b, U, eta, Z)."""
    nx = ei[1].shape[0]
    out = [np.zeros((nx, nx)), np.zeros(nx), np.zeros((nx, nx)), np.zeros(nx), np.zeros((nx, nx))]
    a = [_f64(x) for x in ei] + [_f64(x) for x in ej]
    _load().or_filter_combine(I(nx), *[_p(x) for x in a], *[_p(x) for x in out])
    return tuple(out)


def filter_combine_cov(ei, ej):
    """Standard operator (Table 3 left), each element (A, b, C, eta, J)."""
    nx = ei[1].shape[0]
    out = [np.zeros((nx, nx)), np.zeros(nx), np.zeros((nx, nx)), np.zeros(nx), np.zeros((nx, nx))]
    a = [_f64(x) for x in ei] + [_f64(x) for x in ej]
    _load().or_filter_combine_cov(I(nx), *[_p(x) for x in a], *[_p(x) for x in out])
    return tuple(out)


def smoother_element(F, c, SL, mf, Nf):
    nx = F.shape[0]
    E = np.zeros((nx, nx)); g = np.zeros(nx); D = np.zeros((nx, nx))
    a = [_f64(x) for x in (F, c, SL, mf, Nf)]
    _load().or_smoother_element(I(nx), *[_p(x) for x in a], _p(E), _p(g), _p(D))
    return E, g, D


def smoother_combine(ei, ej):
    nx = ei[1].shape[0]
    E = np.zeros((nx, nx)); g = np.zeros(nx); D = np.zeros((nx, nx))
    a = [_f64(x) for x in ei] + [_f64(x) for x in ej]
    _load().or_smoother_combine(I(nx), *[_p(x) for x in a], _p(E), _p(g), _p(D))
    return E, g, D


def filter_elements(m0, N0, G, y):
    """All filter elements a_1..a_n of Algorithm 1 (Tables 1-2)."""
    y = _f64(y)
    n = y.shape[0]
    s = 0 if np.asarray(G["F"]).ndim == 2 else 1
    pick = (lambda key, j: np.asarray(G[key])[j] if s else np.asarray(G[key]))
    out = []
    for j in range(n):
        if j == 0:
            out.append(filter_element_first(m0, N0, pick("F", 0), pick("c", 0), pick("SL", 0),
                                            pick("H", 0), pick("d", 0), pick("SO", 0), y[0]))
        else:
            # a_{j+1}: transition x_j -> x_{j+1} and measurement y_{j+1} share slot j
            out.append(filter_element(pick("F", j), pick("c", j), pick("SL", j),
                                      pick("H", j), pick("d", j), pick("SO", j), y[j]))
    return out


def smoother_elements(G, mf, Nf):
    """All smoother elements a_0..a_n of Algorithm 2 (Table 4)."""
    mf = _f64(mf); Nf = _f64(Nf)
    n = mf.shape[0] - 1
    nx = mf.shape[1]
    s = 0 if np.asarray(G["F"]).ndim == 2 else 1
    pick = (lambda key, j: np.asarray(G[key])[j] if s else np.asarray(G[key]))
    out = []
    for k in range(n):
        out.append(smoother_element(pick("F", k), pick("c", k), pick("SL", k), mf[k], Nf[k]))
    out.append((np.zeros((nx, nx)), mf[n].copy(), Nf[n].copy()))
    return out


# --------------------------------------------------------------------------
# batches
# --------------------------------------------------------------------------
def ct_ipls_batch(prm, m0, N0, y, y_off, M, ms, Ns):
    """In-place IPLS over a batch (ms, Ns hold the initial nominal)."""
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y)
    y_off = np.ascontiguousarray(np.asarray(y_off, dtype=np.int64))
    assert ms.dtype == np.float64 and ms.flags.c_contiguous
    assert Ns.dtype == np.float64 and Ns.flags.c_contiguous
    B = len(y_off) - 1
    rc = _load().or_ct_ipls_batch(I(B), _lp(y_off), _p(prm), _p(m0), _p(N0), _p(y), I(M), _p(ms), _p(Ns))
    if rc != 0:
        raise RuntimeError("oracle batch IPLS failed")


def linear_smoother_batch(m0, N0, G, y, y_off, ms, Ns):
    m0 = _f64(m0); N0 = _f64(N0); y = _f64(y)
    y_off = np.ascontiguousarray(np.asarray(y_off, dtype=np.int64))
    nx = m0.shape[0]; ny = y.shape[1]
    B = len(y_off) - 1
    a = [_f64(G[k]) for k in ("F", "c", "SL", "H", "d", "SO")]
    rc = _load().or_linear_smoother_batch(I(B), _lp(y_off), I(nx), I(ny), _p(m0), _p(N0),
                                          *[_p(x) for x in a], _p(y), _p(ms), _p(Ns))
    if rc != 0:
        raise RuntimeError("oracle batch smoother failed")


def ct_loglik_batch(prm, m0, N0, y, y_off, ms, Ns):
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y); ms = _f64(ms); Ns = _f64(Ns)
    y_off = np.ascontiguousarray(np.asarray(y_off, dtype=np.int64))
    B = len(y_off) - 1
    ll = np.zeros(B)
    _load().or_ct_loglik_batch(I(B), _lp(y_off), _p(prm), _p(m0), _p(N0), _p(y), _p(ms), _p(Ns), _p(ll))
    return ll


def ct_score_batch(prm, m0, N0, y, y_off, ms, Ns):
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y); ms = _f64(ms); Ns = _f64(Ns)
    y_off = np.ascontiguousarray(np.asarray(y_off, dtype=np.int64))
    B = len(y_off) - 1
    ll = np.zeros(B)
    g = np.zeros((B, 3))
    _load().or_ct_score_batch(I(B), _lp(y_off), _p(prm), _p(m0), _p(N0), _p(y), _p(ms), _p(Ns), _p(ll), _p(g))
    return ll, g
