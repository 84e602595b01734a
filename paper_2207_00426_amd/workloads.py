"""Seeded synthetic workloads shaped like the paper's tracking experiments.

This module only *simulates* data (states and measurements) from the two
state-space models used by the library; it contains none of the filtering,
smoothing or linearisation arithmetic, and it is the only code shared by the
HIP path's callers and the oracle's callers.

Models
  * CT  - coordinated-turn target with two bearings-only sensors
          (the paper's Section 6.2 experiment), x = (px, py, vx, vy, w),
          nx = 5, ny = 2.
  * CV  - linear constant-velocity target with noisy position fixes,
          x = (px, py, vx, vy), nx = 4, ny = 2.
  * RP  - stochastic Ricker population model with Poisson counts (the
          paper's Section 6.1 experiment), nx = ny = 1.

Simulation protocol (CT and CV): ``rng = numpy.random.Generator(PCG64(seed))``;
x_0 = m0 + chol(P0) e_0; then a single (n, nx + ny) block of standard normals
whose row k-1 holds the process noise of step k followed by its measurement
noise; x_k = f(x_{k-1}) + chol(Q) e, y_k = h(x_k) + noise (bearings wrapped to
[-pi, pi)).  RP: x_0 = log c exactly (the paper's point-mass prior), then
per step one standard normal for the process noise and one Poisson draw,
x_k = log a + x_{k-1} - exp(x_{k-1}) + sqrt(Q) e_k, y_k ~ Poisson(b exp(x_k)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


def _wrap(a):
    return np.mod(np.asarray(a) + math.pi, TWO_PI) - math.pi


# ---------------------------------------------------------------------------
# model parameters
# ---------------------------------------------------------------------------
@dataclass
class CTModel:
    dt: float = 0.01
    q1: float = 0.1
    q2: float = 0.1
    sigma: float = 0.05
    sensors: tuple = ((-1.5, 0.5), (1.0, 1.0))
    m0: np.ndarray = field(default_factory=lambda: np.array([0.1, 0.2, 1.0, 0.0, 0.0]))
    P0: np.ndarray = field(default_factory=lambda: np.eye(5))
    nx: int = 5
    ny: int = 2

    @property
    def theta(self):
        return np.array([math.log(self.q1), math.log(self.q2), math.log(self.sigma)])

    def with_theta(self, theta):
        return CTModel(dt=self.dt, q1=math.exp(theta[0]), q2=math.exp(theta[1]),
                       sigma=math.exp(theta[2]), sensors=self.sensors, m0=self.m0.copy(),
                       P0=self.P0.copy())

    def Q(self):
        dt, q1, q2 = self.dt, self.q1, self.q2
        Q = np.zeros((5, 5))
        Q[0, 0] = Q[1, 1] = q1 * dt ** 3 / 3.0
        Q[0, 2] = Q[2, 0] = Q[1, 3] = Q[3, 1] = q1 * dt ** 2 / 2.0
        Q[2, 2] = Q[3, 3] = q1 * dt
        Q[4, 4] = q2 * dt
        return Q


@dataclass
class CVModel:
    dt: float = 0.1
    q: float = 1.0
    r: float = 0.5
    m0: np.ndarray = field(default_factory=lambda: np.zeros(4))
    P0: np.ndarray = field(default_factory=lambda: np.eye(4))
    nx: int = 4
    ny: int = 2

    def F(self):
        F = np.eye(4)
        F[0, 2] = F[1, 3] = self.dt
        return F

    def Q(self):
        dt, q = self.dt, self.q
        Q = np.zeros((4, 4))
        Q[0, 0] = Q[1, 1] = q * dt ** 3 / 3.0
        Q[0, 2] = Q[2, 0] = Q[1, 3] = Q[3, 1] = q * dt ** 2 / 2.0
        Q[2, 2] = Q[3, 3] = q * dt
        return Q

    def H(self):
        H = np.zeros((2, 4))
        H[0, 0] = H[1, 1] = 1.0
        return H

    def R(self):
        return self.r ** 2 * np.eye(2)


@dataclass
class RickerModel:
    """Ricker map with Poisson counts; parameters of the paper's Section 6.1.
    The filter prior is N(log c, s0^2): the paper's point mass at log c
    widened by s0 so that a sigma-point rule can regress around it."""
    a: float = 44.7
    b: float = 10.0
    c: float = 7.0
    Q: float = 0.3 ** 2
    s0: float = 0.01
    nx: int = 1
    ny: int = 1

    @property
    def m0(self):
        return np.array([math.log(self.c)])

    @property
    def P0(self):
        return np.array([[self.s0 ** 2]])

    @property
    def theta(self):
        return np.array([math.log(self.a), math.log(self.b), math.log(self.Q)])


# ---------------------------------------------------------------------------
# simulators
# ---------------------------------------------------------------------------
def simulate_ct(n: int, rng: np.random.Generator, model: CTModel | None = None):
    """Simulate one CT trajectory; returns (x[n+1, 5], y[n, 2])."""
    md = CTModel() if model is None else model
    LQ = np.linalg.cholesky(md.Q())
    LP = np.linalg.cholesky(md.P0)
    x = np.zeros((n + 1, 5))
    x[0] = md.m0 + LP @ rng.standard_normal(5)
    e = rng.standard_normal((n, 7))
    proc = e[:, :5] @ LQ.T
    meas = md.sigma * e[:, 5:]
    dt = md.dt
    (s1x, s1y), (s2x, s2y) = md.sensors
    y = np.zeros((n, 2))
    px, py, vx, vy, w = (float(v) for v in x[0])
    for k in range(n):
        a = w * dt
        if abs(a) < 1e-4:
            s1 = dt * (1.0 - a * a / 6.0)
            s2 = dt * a / 2.0 * (1.0 - a * a / 24.0) ** 2
        else:
            s1 = math.sin(a) / w
            s2 = (1.0 - math.cos(a)) / w
        ca, sa = math.cos(a), math.sin(a)
        p = proc[k]
        px, py, vx, vy, w = (px + s1 * vx - s2 * vy + p[0], py + s2 * vx + s1 * vy + p[1],
                             ca * vx - sa * vy + p[2], sa * vx + ca * vy + p[3], w + p[4])
        x[k + 1] = (px, py, vx, vy, w)
        y[k, 0] = math.atan2(py - s1y, px - s1x) + meas[k, 0]
        y[k, 1] = math.atan2(py - s2y, px - s2x) + meas[k, 1]
    return x, _wrap(y)


def simulate_cv(n: int, rng: np.random.Generator, model: CVModel | None = None):
    """Simulate one CV trajectory; returns (x[n+1, 4], y[n, 2]).

    The recursion v_k = v_{k-1} + w^v_k, p_k = p_{k-1} + dt v_{k-1} + w^p_k is
    evaluated with cumulative sums (same draws as the step-by-step form).
    """
    md = CVModel() if model is None else model
    LQ = np.linalg.cholesky(md.Q())
    LP = np.linalg.cholesky(md.P0)
    x0 = md.m0 + LP @ rng.standard_normal(4)
    e = rng.standard_normal((n, 6))
    w = e[:, :4] @ LQ.T
    x = np.zeros((n + 1, 4))
    x[0] = x0
    v = x0[2:] + np.cumsum(w[:, 2:], axis=0)
    v_prev = np.vstack([x0[2:][None], v[:-1]])
    p = x0[:2] + np.cumsum(md.dt * v_prev + w[:, :2], axis=0)
    x[1:, :2] = p
    x[1:, 2:] = v
    y = p + md.r * e[:, 4:]
    return x, y


def simulate_ricker(n: int, rng: np.random.Generator, model: RickerModel | None = None):
    """Simulate one Ricker trajectory; returns (x[n+1, 1], y[n, 1]) (counts
    as float64)."""
    md = RickerModel() if model is None else model
    e = rng.standard_normal(n)
    x = np.zeros(n + 1)
    x[0] = math.log(md.c)
    la, sq = math.log(md.a), math.sqrt(md.Q)
    for k in range(n):
        x[k + 1] = la + x[k] - math.exp(x[k]) + sq * e[k]
    y = rng.poisson(md.b * np.exp(x[1:])).astype(np.float64)
    return x[:, None], y[:, None]


# ---------------------------------------------------------------------------
# the benchmark configurations
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    model: object
    y: np.ndarray            # [T_y, ny] concatenated measurements
    y_off: np.ndarray        # [B+1] int64 offsets
    kinds: np.ndarray        # [B] 0 = CV, 1 = CT
    x_true: list             # per-sequence true states (for reference only)
    M: int = 10

    @property
    def B(self):
        return len(self.y_off) - 1

    @property
    def lengths(self):
        return np.diff(self.y_off)


def _pack(seqs):
    lens = [len(y) for _, y in seqs]
    y_off = np.zeros(len(seqs) + 1, dtype=np.int64)
    y_off[1:] = np.cumsum(lens)
    y = np.concatenate([y for _, y in seqs], axis=0) if seqs else np.zeros((0, 2))
    return y, y_off


def cv_single(n: int = 100, seed: int = 0) -> Workload:
    """Linear constant-velocity model, one sequence (dt 0.1, q 1, R 0.5^2 I)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    md = CVModel()
    x, y = simulate_cv(n, rng, md)
    yy, off = _pack([(x, y)])
    return Workload("cv_n%d_seed%d" % (n, seed), md, yy, off, np.zeros(1, np.int64), [x], M=1)


def ct_single(n: int = 1000, seed: int = 1, M: int = 10) -> Workload:
    """Coordinated-turn bearings-only model, one sequence."""
    rng = np.random.Generator(np.random.PCG64(seed))
    md = CTModel()
    x, y = simulate_ct(n, rng, md)
    yy, off = _pack([(x, y)])
    return Workload("ct_n%d_seed%d" % (n, seed), md, yy, off, np.ones(1, np.int64), [x], M=M)


def ct_long(n: int = 10 ** 6, seed: int = 2, M: int = 10) -> Workload:
    return ct_single(n, seed, M)


def ragged_mixed(B: int = 512, lo: int = 100, hi: int = 20000, seed: int = 3, M: int = 10):
    """Ragged batch: lengths uniform in [lo, hi], half CV and half CT.

    Returns two workloads (the CV group and the CT group) plus the index map
    from group position to batch position.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = rng.integers(lo, hi + 1, size=B)
    kinds = np.array([0] * (B // 2) + [1] * (B - B // 2), dtype=np.int64)[rng.permutation(B)]
    cvm, ctm = CVModel(), CTModel()
    seqs = []
    for b in range(B):
        if kinds[b] == 0:
            seqs.append(simulate_cv(int(lengths[b]), rng, cvm))
        else:
            seqs.append(simulate_ct(int(lengths[b]), rng, ctm))
    groups = {}
    for kind, md, nm in ((0, cvm, "cv"), (1, ctm, "ct")):
        idx = np.nonzero(kinds == kind)[0]
        part = [seqs[i] for i in idx]
        yy, off = _pack(part)
        groups[nm] = (Workload("ragged_%s_B%d_seed%d" % (nm, len(idx), seed), md, yy, off,
                               np.full(len(idx), kind), [p[0] for p in part], M=M), idx)
    return groups, lengths, kinds


def ct_batch(B: int = 64, n: int = 10 ** 4, seed: int = 4, theta=None, M: int = 10) -> Workload:
    """Batch of equal-length CT sequences simulated at theta (parameter estimation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    md = CTModel() if theta is None else CTModel().with_theta(theta)
    seqs = [simulate_ct(n, rng, md) for _ in range(B)]
    yy, off = _pack(seqs)
    return Workload("ct_B%d_n%d_seed%d" % (B, n, seed), md, yy, off, np.ones(B, np.int64),
                    [s[0] for s in seqs], M=M)


def random_linear_model(nx: int, ny: int, rng: np.random.Generator, n: int | None = None,
                        scale: float = 0.9):
    """A random stable linear-Gaussian model in square-root form.

    Returns dict with F, c, SL, H, d, SO (shared, or per step slot when n is
    given) and a prior (m0, N0).  Lower factors have positive diagonals.
    """
    def lower(k):
        Lm = np.tril(rng.standard_normal((k, k))) * 0.3
        Lm[np.diag_indices(k)] = 0.5 + rng.random(k)
        return Lm

    def one():
        A = rng.standard_normal((nx, nx))
        A *= scale / max(1e-9, np.max(np.abs(np.linalg.eigvals(A))))
        return dict(F=A, c=rng.standard_normal(nx) * 0.1, SL=lower(nx),
                    H=rng.standard_normal((ny, nx)), d=rng.standard_normal(ny) * 0.1, SO=lower(ny))

    if n is None:
        G = one()
    else:
        parts = [one() for _ in range(n)]
        G = {k: np.stack([p[k] for p in parts]) for k in parts[0]}
    m0 = rng.standard_normal(nx)
    N0 = lower(nx)
    return G, m0, N0


def simulate_linear(G, m0, N0, n: int, rng: np.random.Generator):
    """Simulate measurements from a linear-Gaussian model given in factor form."""
    nx = len(m0)
    ny = (G["H"].shape[-2])
    per = np.asarray(G["F"]).ndim == 3
    pick = (lambda k, j: G[k][j]) if per else (lambda k, j: G[k])
    x = m0 + N0 @ rng.standard_normal(nx)
    y = np.zeros((n, ny))
    for j in range(n):
        x = pick("F", j) @ x + pick("c", j) + pick("SL", j) @ rng.standard_normal(nx)
        y[j] = pick("H", j) @ x + pick("d", j) + pick("SO", j) @ rng.standard_normal(ny)
    return y


def ricker_single(n: int = 1000, seed: int = 5, M: int = 10) -> Workload:
    """Ricker-Poisson model, one sequence."""
    rng = np.random.Generator(np.random.PCG64(seed))
    md = RickerModel()
    x, y = simulate_ricker(n, rng, md)
    yy, off = _pack([(x, y)])
    return Workload("ricker_n%d_seed%d" % (n, seed), md, yy, off, np.full(1, 2, np.int64), [x],
                    M=M)


def ricker_batch(B: int = 100, n: int = 1000, seed: int = 6, M: int = 100) -> Workload:
    """Batch of B equal-length Ricker sequences (the paper repeats each
    configuration 100 times)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    md = RickerModel()
    seqs = [simulate_ricker(n, rng, md) for _ in range(B)]
    yy, off = _pack(seqs)
    return Workload("ricker_B%d_n%d_seed%d" % (B, n, seed), md, yy, off, np.full(B, 2, np.int64),
                    [s[0] for s in seqs], M=M)
