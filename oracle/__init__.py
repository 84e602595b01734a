"""FP64 CPU oracle (test infrastructure only).

Plain sequential reference for the parallel square-root iterated smoother of
Yaghoobi, Corenflos, Hassan and Sarkka.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import this package; the HIP library
never does, and the two share no code.

Models: the coordinated-turn bearings model (Section 6.2), the Ricker
population model with Poisson counts (Section 6.1) and linear-Gaussian
models; linearisations: first-order Taylor (Section 4.2) and the
sigma-point GSLR of Section 4.3 with the cubature, unscented or
Gauss-Hermite rule.

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
_LIB_NATIVE = os.path.join(_HERE, "liboracle_native.so")

_lib = None


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over sequences), -O3.
    native=True builds a separate copy with -march=native for the machine it
    runs on (the CPU-baseline timing) and makes it the library this module
    calls."""
    global _LIB, _lib
    target = _LIB_NATIVE if native else _LIB
    if force or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O3", *(["-march=native"] if native else []), "-std=c11",
               "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", _SRC, "-o", target + ".tmp",
               "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(target + ".tmp", target)
    if native and _LIB != _LIB_NATIVE:
        _LIB = _LIB_NATIVE
        _lib = None
    return target


def build_flags() -> str:
    """The compiler flags of the library this module calls."""
    return "gcc -O3%s -fopenmp" % (" -march=native" if _LIB == _LIB_NATIVE else "")


def host_info() -> dict:
    """Core count and CPU model of the host (for the baseline record)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.or_ct_loglik.restype = ctypes.c_double
        _lib.or_ct_score.restype = ctypes.c_double
        _lib.or_lgssm_score_terms.restype = ctypes.c_double
        _lib.or_ricker_loglik.restype = ctypes.c_double
        _lib.or_ricker_f.restype = ctypes.c_double
        _lib.or_ricker_f.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double]
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
RULE_METHODS = ("cubature_rule", "unscented", "gauss_hermite")
_RULE = 3


# --------------------------------------------------------------------------
# sigma-point rules (Section 4.3): unit points xi [np, nx] and positive
# weights w [np] (sum 1) integrating the moments of N(0, I) up to order 2
# --------------------------------------------------------------------------
def rule_cubature(nx):
    """Third-degree spherical-radial rule: +-sqrt(nx) e_i, weights 1/(2 nx)."""
    xi = np.concatenate([np.sqrt(nx) * np.eye(nx), -np.sqrt(nx) * np.eye(nx)])
    return xi, np.full(2 * nx, 1.0 / (2 * nx))


def default_kappa(nx):
    """Unscented spread kappa used when none is given: Julier's n + kappa = 3
    where that keeps the centre weight positive, else 1."""
    return float(max(3 - nx, 1))


def rule_unscented(nx, kappa=None):
    """Unscented transform with alpha = 1, beta = 0 (mean and covariance
    weights equal, all positive for kappa >= 0): the centre with weight
    kappa / (nx + kappa) and +-sqrt(nx + kappa) e_i with 1 / (2 (nx + kappa)).
    A zero centre weight drops the centre point."""
    k = default_kappa(nx) if kappa is None else float(kappa)
    if not k >= 0:
        raise ValueError("kappa must be >= 0 for positive weights")
    s = np.sqrt(nx + k)
    pts = [s * np.eye(nx), -s * np.eye(nx)]
    ws = [np.full(2 * nx, 1.0 / (2 * (nx + k)))]
    if k > 0:
        pts.insert(0, np.zeros((1, nx)))
        ws.insert(0, np.array([k / (nx + k)]))
    return np.concatenate(pts), np.concatenate(ws)


def rule_gauss_hermite(nx, order=3):
    """Tensor product of the order-point Gauss-Hermite rule for N(0, 1)
    (numpy's hermegauss: nodes of He_order, weights normalised to sum 1);
    point index i = sum_j digit_j order^j, digit_0 the first coordinate."""
    x1, w1 = np.polynomial.hermite_e.hermegauss(int(order))
    w1 = w1 / w1.sum()
    np_ = int(order) ** nx
    xi = np.zeros((np_, nx))
    w = np.ones(np_)
    for i in range(np_):
        r = i
        for j in range(nx):
            dgt = r % order
            r //= order
            xi[i, j] = x1[dgt]
            w[i] *= w1[dgt]
    return xi, w


def make_rule(method, nx, kappa=None, gh_order=None):
    if method == "cubature_rule" or method == "cubature":
        return rule_cubature(nx)
    if method == "unscented":
        return rule_unscented(nx, kappa)
    if method == "gauss_hermite":
        return rule_gauss_hermite(nx, 3 if gh_order is None else gh_order)
    raise ValueError(method)


def set_rule(xi, w):
    xi = _f64(xi)
    w = _f64(w)
    if _load().or_set_rule(I(xi.shape[1]), I(xi.shape[0]), _p(xi), _p(w)) != 0:
        raise ValueError("rule too large")


def _code(method, nx, kappa=None, gh_order=None, rule_for_cubature=False):
    """Method code for the C linearisations; installs the rule if needed."""
    if method in RULE_METHODS or (rule_for_cubature and method == "cubature"):
        set_rule(*make_rule(method, nx, kappa, gh_order))
        return _RULE
    return METHODS[method]


def slr_rule(xi, w, m, N, g, Snoise=None, Sg=None, literal=False):
    """GSLR of a conditional model with mean g(x) (x [nx] -> [nz]) and
    covariance factor Snoise (additive) or Sg(x) (per point) at N(m, N N^T)
    with the rule (xi, w).  Returns (G, offset, S) (and the downdate
    breakdown count when literal)."""
    m = _f64(m); N = _f64(N); xi = _f64(xi); w = _f64(w)
    nx = m.shape[0]
    X = m[None, :] + xi @ N.T
    Z = _f64(np.stack([np.atleast_1d(g(x)) for x in X]))
    nz = Z.shape[1]
    np_ = X.shape[0]
    SgA = None
    if Sg is not None:
        SgA = _f64(np.stack([np.atleast_2d(Sg(x)) for x in X]))
    Sn = None if Snoise is None else _f64(np.atleast_2d(Snoise))
    G = np.zeros((nz, nx)); off = np.zeros(nz); S = np.zeros((nz, nz))
    bad = _load().or_slr_rule(I(nx), I(nz), I(np_), _p(_f64(X)), _p(w), _p(m), _p(N), _p(Z),
                              _p(SgA) if SgA is not None else None,
                              _p(Sn) if Sn is not None else None, I(1 if literal else 0),
                              _p(G), _p(off), _p(S))
    return (G, off, S, int(bad)) if literal else (G, off, S)


def ct_linearize(prm, ms, Ns, y, literal=False, method=None, kappa=None, gh_order=None):
    """Per-step linearisation of the CT model at the nominal (ms, Ns):
    method "cubature" (residual SLR, Section 4.3), "cubature_literal" (the
    printed Tria + DownDate form), "taylor" (first-order, Section 4.2), or a
    general positive-weight rule: "cubature_rule", "unscented" (kappa),
    "gauss_hermite" (gh_order points per coordinate)."""
    if method is None:
        method = "cubature_literal" if literal else "cubature"
    prm = _f64(prm)
    ms = _f64(ms)
    Ns = _f64(Ns)
    y = _f64(y)
    n = y.shape[0]
    F = np.zeros((n, 5, 5)); c = np.zeros((n, 5)); SL = np.zeros((n, 5, 5))
    H = np.zeros((n, 2, 5)); d = np.zeros((n, 2)); SO = np.zeros((n, 2, 2))
    code = _code(method, 5, kappa, gh_order)
    bad = _load().or_ct_linearize(I(n), _p(prm), _p(ms), _p(Ns), _p(y), I(code), _p(F),
                                  _p(c), _p(SL), _p(H), _p(d), _p(SO))
    return dict(F=F, c=c, SL=SL, H=H, d=d, SO=SO, bad=int(bad))


def ct_ipls(prm, m0, N0, y, M, ms_init=None, Ns_init=None, history=False, method="cubature",
            kappa=None, gh_order=None):
    """Algorithm 3 (sequential reference).  Initial nominal: the prior at every k.
    method "taylor": the iterated extended smoother (Section 4.2)."""
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y)
    n = y.shape[0]
    ms = np.repeat(m0[None], n + 1, axis=0) if ms_init is None else _f64(ms_init).copy()
    Ns = np.repeat(N0[None], n + 1, axis=0) if Ns_init is None else _f64(Ns_init).copy()
    hm = np.zeros((M, n + 1, 5)) if history else None
    hN = np.zeros((M, n + 1, 5, 5)) if history else None
    mf = np.zeros((n + 1, 5)); Nf = np.zeros((n + 1, 5, 5))
    code = _code(method, 5, kappa, gh_order)
    rc = _load().or_ct_ipls(I(n), _p(prm), _p(m0), _p(N0), _p(y), I(M), _p(ms), _p(Ns),
                            _p(hm) if history else None, _p(hN) if history else None,
                            _p(mf), _p(Nf), I(code))
    if rc != 0:
        raise RuntimeError("oracle IPLS failed")
    out = dict(ms=ms, Ns=Ns, mf=mf, Nf=Nf)
    if history:
        out["hist_ms"] = hm
        out["hist_Ns"] = hN
    return out


def ct_loglik(prm, m0, N0, y, ms, Ns, per_step=False, method="cubature", kappa=None,
              gh_order=None):
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y); ms = _f64(ms); Ns = _f64(Ns)
    n = y.shape[0]
    ell = np.zeros(n)
    code = _code(method, 5, kappa, gh_order)
    tot = _load().or_ct_loglik(I(n), _p(prm), _p(m0), _p(N0), _p(y), _p(ms), _p(Ns), _p(ell),
                               I(code))
    return (tot, ell) if per_step else tot


def ct_score(prm, m0, N0, y, ms, Ns, method="cubature", kappa=None, gh_order=None):
    """(loglik, d loglik / d (log q1, log q2, log sigma)) at a frozen nominal."""
    prm = _f64(prm); m0 = _f64(m0); N0 = _f64(N0); y = _f64(y); ms = _f64(ms); Ns = _f64(Ns)
    n = y.shape[0]
    g = np.zeros(3)
    code = _code(method, 5, kappa, gh_order)
    tot = _load().or_ct_score(I(n), _p(prm), _p(m0), _p(N0), _p(y), _p(ms), _p(Ns), _p(g),
                              I(code))
    return tot, g


def ct_score_total(prm, m0, N0, y, M=60, h=1e-4, method="cubature", kappa=None,
                   gh_order=None):
    """Total derivative of the pseudo-log-likelihood at the IPLS fixed point,
    l(theta) = lhat(theta, n*(theta)) with n* = KS(n*, theta) (the quantity
    that eq. implicity_function_theorem / Algorithm 4 reach through a linear
    fixed point), taken here from its definition: central differences in
    theta = (log q1, log q2, log sigma) at steps 2h and h, combined by
    Richardson extrapolation (error O(h^4)); every evaluation runs its own
    M-pass IPLS from the prior (M = 60 converges the CT iteration to
    round-off).  Returns (l(theta), gradient [3], n*(theta) as (ms, Ns))."""
    prm = _f64(prm)
    th = np.log(prm[1:4])
    kw = dict(method=method, kappa=kappa, gh_order=gh_order)

    def L(t):
        p = ct_theta_params(t, prm)
        r = ct_ipls(p, m0, N0, y, M, **kw)
        return ct_loglik(p, m0, N0, y, r["ms"], r["Ns"], **kw), r

    l0, r0 = L(th)
    g = np.zeros(3)
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1.0
        d1 = (L(th + h * e)[0] - L(th - h * e)[0]) / (2 * h)
        d2 = (L(th + 2 * h * e)[0] - L(th - 2 * h * e)[0]) / (4 * h)
        g[j] = (4.0 * d1 - d2) / 3.0
    return l0, g, r0["ms"], r0["Ns"]


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
# Ricker population model with Poisson counts (Section 6.1); nx = ny = 1
# --------------------------------------------------------------------------
def ricker_params(a=44.7, b=10.0, Q=0.3 ** 2):
    return np.array([a, b, Q], dtype=np.float64)


def ricker_f(prm, x):
    return float(_load().or_ricker_f(_p(_f64(prm)), ctypes.c_double(float(x))))


def ricker_linearize(prm, ms, Ns, y, method="cubature", kappa=None, gh_order=None):
    """Per-step GSLR of the Ricker model at the nominal (ms [n+1], Ns [n+1]
    scalar factors): "taylor" (Section 4.2) or a rule ("cubature",
    "unscented", "gauss_hermite"; Section 4.3).  Arrays of shape [n]."""
    prm = _f64(prm); ms = _f64(np.ravel(ms)); Ns = _f64(np.ravel(Ns)); y = _f64(np.ravel(y))
    n = y.shape[0]
    out = {k: np.zeros(n) for k in ("F", "c", "SL", "H", "d", "SO")}
    code = _code(method, 1, kappa, gh_order, rule_for_cubature=True)
    rc = _load().or_ricker_linearize(I(n), _p(prm), _p(ms), _p(Ns), _p(y), I(code),
                                     *[_p(out[k]) for k in ("F", "c", "SL", "H", "d", "SO")])
    if rc != 0:
        raise RuntimeError("oracle Ricker linearisation failed")
    return out


def ricker_ipls(prm, m0, N0, y, M, ms_init=None, Ns_init=None, history=False,
                method="cubature", kappa=None, gh_order=None):
    """Algorithm 3 on the Ricker model (sequential reference); initial
    nominal: the prior (m0, N0) at every state.  Arrays of shape [n+1]."""
    prm = _f64(prm); y = _f64(np.ravel(y))
    n = y.shape[0]
    m0a = _f64(np.ravel(m0)); N0a = _f64(np.ravel(N0))
    ms = np.full(n + 1, m0a[0]) if ms_init is None else _f64(np.ravel(ms_init)).copy()
    Ns = np.full(n + 1, N0a[0]) if Ns_init is None else _f64(np.ravel(Ns_init)).copy()
    hm = np.zeros((M, n + 1)) if history else None
    hN = np.zeros((M, n + 1)) if history else None
    mf = np.zeros(n + 1); Nf = np.zeros(n + 1)
    code = _code(method, 1, kappa, gh_order, rule_for_cubature=True)
    rc = _load().or_ricker_ipls(I(n), _p(prm), _p(m0a), _p(N0a), _p(y), I(M), _p(ms), _p(Ns),
                                _p(hm) if history else None, _p(hN) if history else None,
                                _p(mf), _p(Nf), I(code))
    if rc != 0:
        raise RuntimeError("oracle Ricker IPLS failed")
    out = dict(ms=ms, Ns=Ns, mf=mf, Nf=Nf)
    if history:
        out["hist_ms"] = hm
        out["hist_Ns"] = hN
    return out


def ricker_loglik(prm, m0, N0, y, ms, Ns, per_step=False, method="cubature", kappa=None,
                  gh_order=None):
    prm = _f64(prm); y = _f64(np.ravel(y)); ms = _f64(np.ravel(ms)); Ns = _f64(np.ravel(Ns))
    m0a = _f64(np.ravel(m0)); N0a = _f64(np.ravel(N0))
    n = y.shape[0]
    ell = np.zeros(n)
    code = _code(method, 1, kappa, gh_order, rule_for_cubature=True)
    tot = _load().or_ricker_loglik(I(n), _p(prm), _p(m0a), _p(N0a), _p(y), _p(ms), _p(Ns),
                                   _p(ell), I(code))
    return (tot, ell) if per_step else tot


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
