"""Dense joint-Gaussian brute force for tiny linear-Gaussian state-space models.

Stacks x_{0:n} into one vector s with (I - M) s = u + e, where M holds the
transition matrices, u the offsets and prior mean, e the independent noises;
then y = Hbig s + dvec + v.  Filtering, smoothing and the log-likelihood follow
from textbook Gaussian conditioning (numpy.linalg), independent of any Kalman
recursion.
"""
import numpy as np


def _pick(G, key, j):
    a = np.asarray(G[key])
    base = {"F": 2, "c": 1, "SL": 2, "H": 2, "d": 1, "SO": 2}[key]
    return a[j] if a.ndim == base + 1 else a


def joint(m0, N0, G, n):
    nx = len(m0)
    ny = np.asarray(G["H"]).shape[-2]
    S = (n + 1) * nx
    M = np.zeros((S, S))
    u = np.zeros(S)
    D = np.zeros((S, S))
    u[:nx] = m0
    D[:nx, :nx] = N0 @ N0.T
    Hb = np.zeros((n * ny, S))
    dv = np.zeros(n * ny)
    Om = np.zeros((n * ny, n * ny))
    for j in range(n):
        r = slice((j + 1) * nx, (j + 2) * nx)
        M[r, j * nx:(j + 1) * nx] = _pick(G, "F", j)
        u[r] = _pick(G, "c", j)
        SL = _pick(G, "SL", j)
        D[r, r] = SL @ SL.T
        ry = slice(j * ny, (j + 1) * ny)
        Hb[ry, r] = _pick(G, "H", j)
        dv[ry] = _pick(G, "d", j)
        SO = _pick(G, "SO", j)
        Om[ry, ry] = SO @ SO.T
    Tm = np.linalg.inv(np.eye(S) - M)
    mu = Tm @ u
    Sig = Tm @ D @ Tm.T
    return mu, Sig, Hb, dv, Om


def condition(mu, Sig, Hb, dv, Om, y, upto):
    """Posterior of s given y_{1:upto}."""
    ny = y.shape[1]
    if upto == 0:
        return mu, Sig
    rows = slice(0, upto * ny)
    Hs = Hb[rows]
    Sy = Hs @ Sig @ Hs.T + Om[rows, rows]
    K = np.linalg.solve(Sy, Hs @ Sig).T
    r = y[:upto].reshape(-1) - (Hs @ mu + dv[rows])
    return mu + K @ r, Sig - K @ Sy @ K.T


def filter_smoother_loglik(m0, N0, G, y):
    n, ny = y.shape
    nx = len(m0)
    mu, Sig, Hb, dv, Om = joint(m0, N0, G, n)
    mf = np.zeros((n + 1, nx))
    Pf = np.zeros((n + 1, nx, nx))
    for k in range(n + 1):
        m, P = condition(mu, Sig, Hb, dv, Om, y, k)
        b = slice(k * nx, (k + 1) * nx)
        mf[k] = m[b]
        Pf[k] = P[b, b]
    m, P = condition(mu, Sig, Hb, dv, Om, y, n)
    ms = np.stack([m[k * nx:(k + 1) * nx] for k in range(n + 1)])
    Ps = np.stack([P[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] for k in range(n + 1)])
    Sy = Hb @ Sig @ Hb.T + Om
    r = y.reshape(-1) - (Hb @ mu + dv)
    sign, logdet = np.linalg.slogdet(Sy)
    ll = -0.5 * (len(r) * np.log(2 * np.pi) + logdet + r @ np.linalg.solve(Sy, r))
    return mf, Pf, ms, Ps, ll
