"""Parity metrics between the HIP path and the FP64 oracle.

Relative errors follow one fixed reading of "relative":
  means        max_k |m_k - m^_k|_2 / max(|m^_k|_2, sqrt(tr P^_k))
  covariances  max_k |P_k - P^_k|_F / |P^_k|_F   (P = N N^T: factors are unique
               only up to column signs, so factors are compared via Grams)
  log-lik      |l - l^| / max(|l^|, 1)
  gradients    |g - g^|_inf / max(|g^|_inf, 1)
Tolerances: FP64 1e-9 (moments), 1e-8 (log-lik), 1e-7 (gradient);
FP32 1e-4, 1e-3, 1e-2.
"""
import numpy as np

TOL = {
    "f64": dict(m=1e-9, P=1e-9, ll=1e-8, g=1e-7),
    "f32": dict(m=1e-4, P=1e-4, ll=1e-3, g=1e-2),
}


def kernel_input(x, dtype):
    """x as the kernel reads it: rounded to the kernel's precision (an FP32
    kernel receives FP32 measurements), returned in FP64 for the oracle, so
    that both sides solve the same problem.  This matters where the inputs
    decide an integer: a bearing whose sigma-point images straddle the
    wrap-around cut takes its branch from y, and the FP32 rounding of y can
    move an image across the cut."""
    import torch
    if dtype in ("f32", torch.float32, np.float32):
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


def gram(N):
    return N @ np.swapaxes(N, -1, -2)


def mean_err(m, m_ref, P_ref):
    num = np.linalg.norm(m - m_ref, axis=-1)
    den = np.maximum(np.linalg.norm(m_ref, axis=-1),
                     np.sqrt(np.maximum(np.trace(P_ref, axis1=-2, axis2=-1), 0.0)))
    den = np.maximum(den, 1e-300)
    return float(np.max(num / den))


def cov_err(P, P_ref):
    num = np.linalg.norm((P - P_ref).reshape(P.shape[0], -1), axis=-1)
    den = np.maximum(np.linalg.norm(P_ref.reshape(P.shape[0], -1), axis=-1), 1e-300)
    return float(np.max(num / den))


def marg_errs(m, N, m_ref, N_ref):
    P, P_ref = gram(N), gram(N_ref)
    return mean_err(m, m_ref, P_ref), cov_err(P, P_ref)


def ll_err(l, l_ref):
    l = np.asarray(l, dtype=np.float64)
    l_ref = np.asarray(l_ref, dtype=np.float64)
    return float(np.max(np.abs(l - l_ref) / np.maximum(np.abs(l_ref), 1.0)))


def grad_err(g, g_ref):
    g = np.asarray(g, dtype=np.float64)
    g_ref = np.asarray(g_ref, dtype=np.float64)
    return float(np.max(np.abs(g - g_ref)) / max(np.max(np.abs(g_ref)), 1.0))
