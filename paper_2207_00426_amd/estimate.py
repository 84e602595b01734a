"""Likelihood-based parameter estimation for the coordinated-turn model.

theta = (log q1, log q2, log sigma) is fitted by maximising the pseudo
log-likelihood of Section 5.1, summed over a batch.  Every objective
evaluation first recomputes the nominal trajectory by IPLS (Algorithm 3) at
the current theta, so the objective is the likelihood of the model
linearised where IPLS puts it for that theta.  Two gradients:

* "frozen": the library's frozen-nominal one (the nominal's own dependence
  on theta through the iterated linearisation is not differentiated), an
  approximation of the objective's derivative (pss.LogLik);
* "fixed_point": the total derivative at the IPLS fixed point (Algorithm 4,
  pss_loglik_grad_ift through pss.LogLikFixedPoint), exact for the
  objective once IPLS has converged.

Holding one nominal fixed over many steps instead is not a usable objective:
linearised at a poor starting theta it can prefer parameters far from the
generating ones.  The optimiser is a limited-memory BFGS with an Armijo
backtracking line search (which needs only a descent direction, so it also
works with the approximate gradient) and a cap on the step length.  Only
argument marshalling happens here; every pass is a library call.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import pss


def lbfgs(fg, x0, n_steps=50, history=10, max_step=1.0, c1=1e-4, max_backtracks=30,
          gtol=1e-10):
    """Minimise f with f, g = fg(x) (g may approximate the gradient).

    Two-loop recursion for the direction (initial inverse Hessian scaled by
    s.y / y.y of the latest pair), Armijo backtracking from step 1 with the
    step length capped at max_step, curvature pairs with s.y <= 0 skipped; a
    direction whose search fails is replaced once by the scaled negative
    gradient (memory cleared) before the run stops.
    Returns (x, f, trace) with trace a list of (f, |g|_inf, evaluations)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    f, g = fg(x)
    evals = 1
    S, Y = [], []
    trace = [(f, float(np.max(np.abs(g))), evals)]
    for _ in range(n_steps):
        if not np.all(np.isfinite(g)) or np.max(np.abs(g)) <= gtol:
            break
        # two-loop recursion
        q = g.copy()
        alphas = []
        for s, y in zip(reversed(S), reversed(Y)):
            a = s.dot(q) / y.dot(s)
            alphas.append(a)
            q -= a * y
        if S:
            q *= S[-1].dot(Y[-1]) / Y[-1].dot(Y[-1])
        else:
            q /= max(np.max(np.abs(g)), 1e-300)  # first step: unit max-norm
        for (s, y), a in zip(zip(S, Y), reversed(alphas)):
            b = y.dot(q) / y.dot(s)
            q += (a - b) * s
        d = -q
        slope = g.dot(d)
        if not slope < 0:  # not a descent direction: restart from -g
            S, Y = [], []
            d = -g / max(np.max(np.abs(g)), 1e-300)
            slope = g.dot(d)
        accepted = False
        for attempt in range(2):
            nd = np.linalg.norm(d)
            t = min(1.0, max_step / nd) if nd > 0 else 1.0
            for _ in range(max_backtracks):
                xn = x + t * d
                fn, gn = fg(xn)
                evals += 1
                if np.isfinite(fn) and fn <= f + c1 * t * slope:
                    accepted = True
                    break
                t *= 0.5
            if accepted or attempt == 1:
                break
            # the quasi-Newton direction failed (with an approximate gradient
            # it need not descend): forget the curvature pairs and retry along
            # the scaled negative gradient
            S, Y = [], []
            d = -g / max(np.max(np.abs(g)), 1e-300)
            slope = g.dot(d)
        if not accepted:
            break
        s, y = xn - x, gn - g
        if s.dot(y) > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
            S.append(s)
            Y.append(y)
            if len(S) > history:
                S.pop(0)
                Y.pop(0)
        x, f, g = xn, fn, gn
        trace.append((f, float(np.max(np.abs(g))), evals))
    return x, f, trace


def fit_theta_lbfgs(batch, y, theta0, n_steps=50, passes=10, history=10, max_step=1.0,
                    gradient="frozen", ift_iter=30):
    """Returns a dict: final theta, the objective (mean negative
    log-likelihood per step) at the start and end and after every step, the
    number of L-BFGS iterations and objective evaluations, and timings (IPLS
    and loglik + gradient separately).  gradient: "frozen" or "fixed_point"
    (ift_iter tangent iterations; FP64 only)."""
    if gradient not in ("frozen", "fixed_point"):
        raise ValueError(gradient)
    pss._require_gpu()
    n_total = float(batch.y_off_host[-1])
    times = {"ipls": 0.0, "eval": 0.0}

    def fg(th):
        t0 = time.perf_counter()
        b = pss._with_theta(batch, th)
        m_nom, N_nom = pss.ipls_iterate(b, y, passes)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # objective and gradient through the autograd binding
        tt = torch.tensor(np.asarray(th, dtype=np.float64), requires_grad=True)
        if gradient == "frozen":
            loss = -pss.LogLik.apply(tt, batch, y, m_nom, N_nom) / n_total
        else:
            loss = -pss.LogLikFixedPoint.apply(tt, batch, y, m_nom, N_nom, ift_iter) / n_total
        loss.backward()
        f = float(loss.detach())
        g = tt.grad.numpy().copy()
        times["ipls"] += t1 - t0
        times["eval"] += time.perf_counter() - t1
        return f, g

    th, f, trace = lbfgs(fg, theta0, n_steps=n_steps, history=history, max_step=max_step)
    n_ev = trace[-1][2]
    return {"theta": th.tolist(), "iterations": len(trace) - 1, "evaluations": n_ev,
            "loss_start": trace[0][0], "loss_final": f,
            "loss_trace": [t[0] for t in trace], "grad_inf_trace": [t[1] for t in trace],
            "ipls_s": times["ipls"], "eval_s": times["eval"],
            "ms_per_evaluation": 1e3 * times["eval"] / max(n_ev, 1),
            "ms_ipls_per_evaluation": 1e3 * times["ipls"] / max(n_ev, 1)}
