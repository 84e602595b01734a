"""Thin Python binding of libpss.so (the C ABI declared in include/pss.h).

Argument marshalling only: every computation runs in the HIP library.  PyTorch
provides device memory and the current HIP stream.  There is no fallback: if
the library or a GPU is missing, calls raise.

Layouts follow the C ABI: structure-of-arrays, component-major.
  y      [ny, T_y]          measurements (step slots)
  m      [nx, T_x]          means (state slots)
  N      [nx(nx+1)/2, T_x]  packed lower factors, row-major
  Gamma  dict F [nx*nx, S], c [nx, S], SL [P, S], H [ny*nx, S], d [ny, S],
         SO [Py, S] with S = T_y (stride 1) or 1 (stride 0)
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpss.so")

PSS_F32, PSS_F64 = 0, 1
MODEL_LINEAR, MODEL_CT, MODEL_RICKER = 0, 1, 2
LIN_CUBATURE, LIN_TAYLOR, LIN_UNSCENTED, LIN_GAUSS_HERMITE = 0, 1, 2, 3
LINEARIZATIONS = {"cubature": LIN_CUBATURE, "taylor": LIN_TAYLOR, "unscented": LIN_UNSCENTED,
                  "gauss_hermite": LIN_GAUSS_HERMITE}
FORM_SQRT, FORM_COV = 0, 1
FORMS = {"sqrt": FORM_SQRT, "cov": FORM_COV}
OPS = dict(slr=0, filter_elements=1, filter_scan=2, smoother_scan=3, ipls=4, loglik=5,
           loglik_grad=6, sequential=7, loglik_grad_ift=8, loglik_vjp=9, score_fisher=10)
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported", -3: "workspace too small",
          -4: "HIP error"}
EXPORTS = ["pss_workspace_size", "pss_slr_linearize", "pss_sqrt_filter_elements",
           "pss_sqrt_filter_scan", "pss_sqrt_smoother_scan", "pss_ipls_iterate", "pss_loglik",
           "pss_loglik_grad", "pss_sequential_smoother", "pss_validate", "pss_last_error",
           "pss_version", "pss_batched_workspace_size", "pss_ipls_batched",
           "pss_autotune_workspace_size", "pss_autotune", "pss_kernel_timing",
           "pss_kernel_times", "pss_loglik_grad_ift", "pss_ckpt_size", "pss_loglik_vjp",
           "pss_score_fisher", "pss_noalloc_max_bytes", "pss_ipls_iterate_noalloc",
           "pss_nan_status"]


class PssError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pss error %d (%s): %s" % (code, STATUS.get(code, "?"), msg))
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("dtype", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("B", ctypes.c_int32),
                ("y_off", ctypes.c_void_p), ("y_off_host", ctypes.c_void_p),
                ("m0", ctypes.c_void_p), ("N0", ctypes.c_void_p),
                ("dt", ctypes.c_double), ("theta", ctypes.c_double * 3),
                ("sensors", ctypes.c_double * 4),
                ("scan_threads", ctypes.c_int32), ("scan_elems", ctypes.c_int32),
                ("linearization", ctypes.c_int32), ("form", ctypes.c_int32),
                ("gh_order", ctypes.c_int32), ("ut_kappa", ctypes.c_double)]


class GroupC(ctypes.Structure):
    _fields_ = [("p", ctypes.POINTER(Problem)), ("g", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("m_nom", ctypes.c_void_p), ("N_nom", ctypes.c_void_p)]


class GammaC(ctypes.Structure):
    _fields_ = [("F", ctypes.c_void_p), ("c", ctypes.c_void_p), ("SL", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("d", ctypes.c_void_p), ("SO", ctypes.c_void_p),
                ("stride", ctypes.c_int64)]


class FElemC(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("U", ctypes.c_void_p),
                ("eta", ctypes.c_void_p), ("Z", ctypes.c_void_p)]


class CkptC(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("buf", ctypes.c_void_p), ("bytes", ctypes.c_size_t),
                ("tag", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libpss.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpss.so not built: run __graft_entry__.build() "
                               "(or python paper_2207_00426_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        P = ctypes.POINTER(Problem)
        L.pss_workspace_size.restype = sz
        L.pss_workspace_size.argtypes = [P, i32]
        L.pss_validate.argtypes = [P]
        L.pss_last_error.restype = ctypes.c_char_p
        L.pss_version.restype = ctypes.c_char_p
        L.pss_slr_linearize.argtypes = [P, vp, vp, vp, ctypes.POINTER(GammaC), vp]
        L.pss_sqrt_filter_elements.argtypes = [P, ctypes.POINTER(GammaC), vp,
                                               ctypes.POINTER(FElemC), vp]
        L.pss_sqrt_filter_scan.argtypes = [P, ctypes.POINTER(FElemC), vp, vp, vp, sz, vp]
        L.pss_sqrt_smoother_scan.argtypes = [P, ctypes.POINTER(GammaC), vp, vp, vp, vp, vp, sz,
                                             vp]
        L.pss_ipls_iterate.argtypes = [P, ctypes.POINTER(GammaC), vp, i32, vp, vp, vp, vp, vp,
                                       sz, vp]
        CK = ctypes.POINTER(CkptC)
        L.pss_ckpt_size.restype = sz
        L.pss_ckpt_size.argtypes = [P, i32]
        L.pss_loglik.argtypes = [P, ctypes.POINTER(GammaC), vp, vp, vp, vp, CK, vp, sz, vp]
        L.pss_loglik_grad.argtypes = [P, vp, vp, vp, vp, CK, vp, vp, vp, vp, sz, vp]
        L.pss_loglik_vjp.argtypes = [P, ctypes.POINTER(GammaC), vp, vp, vp, vp, CK, vp,
                                     ctypes.POINTER(GammaC), vp, vp, vp, sz, vp]
        L.pss_score_fisher.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.pss_nan_status.argtypes = [P, vp, vp, i32, vp, i32, vp, vp]
        L.pss_nan_status.restype = ctypes.c_int
        L.pss_noalloc_max_bytes.restype = sz
        L.pss_noalloc_max_bytes.argtypes = []
        L.pss_ipls_iterate_noalloc.argtypes = [P, ctypes.POINTER(GammaC), vp, i32, vp, vp, vp,
                                               vp, vp]
        L.pss_sequential_smoother.argtypes = [P, ctypes.POINTER(GammaC), vp, i32, vp, vp, vp, vp,
                                              vp, sz, vp]
        L.pss_loglik_grad_ift.argtypes = [P, vp, vp, vp, i32, vp, vp, vp, vp, sz, vp]
        G = ctypes.POINTER(GroupC)
        L.pss_batched_workspace_size.restype = sz
        L.pss_batched_workspace_size.argtypes = [G, i32]
        L.pss_autotune_workspace_size.restype = sz
        L.pss_autotune_workspace_size.argtypes = [G, i32]
        L.pss_ipls_batched.argtypes = [G, i32, i32, vp, vp, sz, vp]
        L.pss_autotune.argtypes = [G, i32, vp, sz, ctypes.c_char_p, vp, vp]
        L.pss_ipls_batched.restype = ctypes.c_int
        L.pss_autotune.restype = ctypes.c_int
        L.pss_kernel_timing.argtypes = [i32]
        L.pss_kernel_timing.restype = ctypes.c_int
        L.pss_kernel_times.argtypes = [ctypes.c_char_p, sz]
        L.pss_kernel_times.restype = ctypes.c_int64
        for name in ("pss_slr_linearize", "pss_sqrt_filter_elements", "pss_sqrt_filter_scan",
                     "pss_sqrt_smoother_scan", "pss_ipls_iterate", "pss_loglik",
                     "pss_loglik_grad", "pss_sequential_smoother", "pss_validate",
                     "pss_loglik_grad_ift", "pss_loglik_vjp", "pss_score_fisher",
                     "pss_ipls_iterate_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().pss_last_error().decode()


def version() -> str:
    return lib().pss_version().decode()


def kernel_timing(enable: bool) -> None:
    """Switch per-launch HIP-event timing of the library's kernels on or off."""
    _check(lib().pss_kernel_timing(1 if enable else 0))


def kernel_times() -> dict:
    """Collect the launches timed since the last call:
    {(kernel, level): (launches, total_ms)}; waits for the recorded events."""
    L = lib()
    need = L.pss_kernel_times(None, 0)
    if need < 0:
        _check(int(need))
    buf = ctypes.create_string_buffer(int(need) + 256)
    got = L.pss_kernel_times(buf, len(buf))
    if got < 0:
        _check(int(got))
    out = {}
    for line in buf.value.decode().splitlines():
        name, level, calls, ms = line.split()
        out[(name, int(level))] = (int(calls), float(ms))
    return out


def _check(rc):
    if rc != 0:
        raise PssError(rc, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("the pss library needs a GPU (gfx950); none is visible")


def tri(n):
    return n * (n + 1) // 2


# ---------------------------------------------------------------------------
# layout helpers (numpy AoS <-> torch SoA)
# ---------------------------------------------------------------------------
def pack_lower(N):
    """[..., n, n] -> [..., n(n+1)/2] row-major lower triangle."""
    N = np.asarray(N)
    n = N.shape[-1]
    ii, jj = np.tril_indices(n)
    return N[..., ii, jj]


def unpack_lower(P, n):
    P = np.asarray(P)
    ii, jj = np.tril_indices(n)
    out = np.zeros(P.shape[:-1] + (n, n), dtype=P.dtype)
    out[..., ii, jj] = P
    return out


def to_soa(a, dtype, device):
    """numpy [T, ...] -> torch [prod(...), T] on device."""
    a = np.asarray(a, dtype=np.float64)
    a2 = a.reshape(a.shape[0], -1).T
    return torch.tensor(np.ascontiguousarray(a2), dtype=dtype, device=device)


def from_soa(t, shape):
    """torch [C, T] -> numpy [T, *shape]."""
    a = t.detach().double().cpu().numpy()
    return a.T.reshape((a.shape[1],) + tuple(shape))


def marg_from_soa(m, N, nx):
    """(m [nx, T], N [P, T]) -> numpy means [T, nx] and factors [T, nx, nx]."""
    return from_soa(m, (nx,)), unpack_lower(from_soa(N, (tri(nx),)), nx)


# ---------------------------------------------------------------------------
# problem
# ---------------------------------------------------------------------------
class Batch:
    """A batch of B sequences of one model, plus the device buffers the C ABI reads."""

    def __init__(self, model, dtype, nx, ny, y_off, m0, N0, device="cuda", dt=0.0,
                 theta=(0.0, 0.0, 0.0), sensors=(0.0, 0.0, 0.0, 0.0), scan_threads=0,
                 scan_elems=0, linearization="cubature", form="sqrt", gh_order=3, ut_kappa=None):
        self.model = model
        self.torch_dtype = dtype
        self.nx, self.ny = nx, ny
        self.y_off_host = np.ascontiguousarray(np.asarray(y_off, dtype=np.int64))
        self.B = len(self.y_off_host) - 1
        self.T_y = int(self.y_off_host[-1])
        self.T_x = self.T_y + self.B
        self.device = device
        self.y_off = torch.tensor(self.y_off_host, dtype=torch.int64, device=device)
        self.m0 = torch.tensor(np.asarray(m0, dtype=np.float64), dtype=dtype, device=device)
        self.N0 = torch.tensor(pack_lower(np.asarray(N0, dtype=np.float64)), dtype=dtype,
                               device=device)
        self.dt = float(dt)
        self.theta = tuple(float(v) for v in theta)
        self.sensors = tuple(float(v) for v in sensors)
        self.scan_threads = int(scan_threads)
        self.scan_elems = int(scan_elems)
        self.linearization = LINEARIZATIONS[linearization]
        self.form = FORMS[form]
        self.gh_order = int(gh_order)
        # unscented spread: Julier's nx + kappa = 3 where the centre weight
        # stays positive, else 1
        self.ut_kappa = float(max(3 - nx, 1) if ut_kappa is None else ut_kappa)

    @classmethod
    def ct(cls, y_off, model, dtype=torch.float64, device="cuda", theta=None, **kw):
        """Coordinated-turn bearings model (workloads.CTModel)."""
        th = model.theta if theta is None else theta
        s = model.sensors
        return cls(MODEL_CT, dtype, 5, 2, y_off, model.m0, np.linalg.cholesky(model.P0),
                   device=device, dt=model.dt, theta=th,
                   sensors=(s[0][0], s[0][1], s[1][0], s[1][1]), **kw)

    @classmethod
    def ricker(cls, y_off, model, dtype=torch.float64, device="cuda", theta=None, **kw):
        """Ricker-Poisson model (workloads.RickerModel): theta = (log a,
        log b, log Q); prior N(log c, s0^2)."""
        th = model.theta if theta is None else theta
        return cls(MODEL_RICKER, dtype, 1, 1, y_off, model.m0, np.sqrt(model.P0),
                   device=device, theta=th, **kw)

    @property
    def pss_dtype(self):
        return PSS_F64 if self.torch_dtype == torch.float64 else PSS_F32

    def struct(self):
        p = Problem()
        p.model = self.model
        p.dtype = self.pss_dtype
        p.nx, p.ny, p.B = self.nx, self.ny, self.B
        p.y_off = self.y_off.data_ptr() if self.y_off is not None else None
        p.y_off_host = self.y_off_host.ctypes.data
        p.m0 = self.m0.data_ptr() if self.m0 is not None else None
        p.N0 = self.N0.data_ptr() if self.N0 is not None else None
        p.dt = self.dt
        p.theta = (ctypes.c_double * 3)(*self.theta)
        p.sensors = (ctypes.c_double * 4)(*self.sensors)
        p.scan_threads = self.scan_threads
        p.scan_elems = self.scan_elems
        p.linearization = getattr(self, "linearization", LIN_CUBATURE)
        p.form = getattr(self, "form", FORM_SQRT)
        p.gh_order = getattr(self, "gh_order", 3)
        p.ut_kappa = getattr(self, "ut_kappa", 1.0)
        return p

    # buffers -------------------------------------------------------------
    def empty(self, rows, cols):
        return torch.empty((rows, cols), dtype=self.torch_dtype, device=self.device)

    def new_marg(self):
        return self.empty(self.nx, self.T_x), self.empty(tri(self.nx), self.T_x)

    def prior_nominal(self):
        """Nominal trajectory with the prior at every state (the initial IPLS
        nominal); in the covariance form its second part holds P0 = N0 N0^T."""
        m = self.m0[:, None].repeat(1, self.T_x).contiguous()
        N0 = self.N0
        if getattr(self, "form", FORM_SQRT) == FORM_COV:
            L = unpack_lower(self.N0.double().cpu().numpy(), self.nx)
            N0 = torch.tensor(pack_lower(L @ L.T), dtype=self.torch_dtype, device=self.device)
        N = N0[:, None].repeat(1, self.T_x).contiguous()
        return m, N

    def new_gamma(self, stride=1):
        S = self.T_y if stride else 1
        nx, ny = self.nx, self.ny
        return dict(F=self.empty(nx * nx, S), c=self.empty(nx, S), SL=self.empty(tri(nx), S),
                    H=self.empty(ny * nx, S), d=self.empty(ny, S), SO=self.empty(tri(ny), S),
                    stride=stride)

    def gamma_from_numpy(self, G):
        """numpy linear model (shared or per step) -> SoA Gamma dict."""
        F = np.asarray(G["F"])
        stride = 1 if F.ndim == 3 else 0
        dt, dev = self.torch_dtype, self.device

        def conv(a, lower=False):
            a = np.asarray(a, dtype=np.float64)
            if lower:
                a = pack_lower(a)
            if stride == 0:
                a = a[None]
            return to_soa(a, dt, dev)

        return dict(F=conv(G["F"]), c=conv(G["c"]), SL=conv(G["SL"], True), H=conv(G["H"]),
                    d=conv(G["d"]), SO=conv(G["SO"], True), stride=stride)

    def new_felem(self):
        nx = self.nx
        return dict(A=self.empty(nx * nx, self.T_y), b=self.empty(nx, self.T_y),
                    U=self.empty(tri(nx), self.T_y), eta=self.empty(nx, self.T_y),
                    Z=self.empty(tri(nx), self.T_y))

    def workspace(self, op):
        n = workspace_size(self, op)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.device), n


def _gamma_c(g):
    if g is None:
        return None
    s = GammaC()
    for k in ("F", "c", "SL", "H", "d", "SO"):
        setattr(s, k, g[k].data_ptr())
    s.stride = g["stride"]
    return ctypes.byref(s)


def _felem_c(e):
    s = FElemC()
    for k in ("A", "b", "U", "eta", "Z"):
        setattr(s, k, e[k].data_ptr())
    return ctypes.byref(s)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def validate(batch: Batch) -> int:
    p = batch.struct()
    return lib().pss_validate(ctypes.byref(p))


def workspace_size(batch: Batch, op) -> int:
    p = batch.struct()
    code = OPS[op] if isinstance(op, str) else int(op)
    return int(lib().pss_workspace_size(ctypes.byref(p), code))


def slr_linearize(batch, m_nom, N_nom, y, out=None):
    _require_gpu()
    out = batch.new_gamma(1) if out is None else out
    p = batch.struct()
    _check(lib().pss_slr_linearize(ctypes.byref(p), _ptr(m_nom), _ptr(N_nom), _ptr(y),
                                   _gamma_c(out), _stream()))
    return out


def sqrt_filter_elements(batch, gamma, y, out=None):
    _require_gpu()
    out = batch.new_felem() if out is None else out
    p = batch.struct()
    _check(lib().pss_sqrt_filter_elements(ctypes.byref(p), _gamma_c(gamma), _ptr(y),
                                          _felem_c(out), _stream()))
    return out


def sqrt_filter_scan(batch, felem, m_f=None, N_f=None):
    _require_gpu()
    if m_f is None:
        m_f, N_f = batch.new_marg()
    ws, n = batch.workspace("filter_scan")
    p = batch.struct()
    _check(lib().pss_sqrt_filter_scan(ctypes.byref(p), _felem_c(felem), _ptr(m_f), _ptr(N_f),
                                      _ptr(ws), n, _stream()))
    return m_f, N_f


def sqrt_smoother_scan(batch, gamma, m_f, N_f, m_s=None, N_s=None):
    _require_gpu()
    if m_s is None:
        m_s, N_s = batch.new_marg()
    ws, n = batch.workspace("smoother_scan")
    p = batch.struct()
    _check(lib().pss_sqrt_smoother_scan(ctypes.byref(p), _gamma_c(gamma), _ptr(m_f), _ptr(N_f),
                                        _ptr(m_s), _ptr(N_s), _ptr(ws), n, _stream()))
    return m_s, N_s


def ipls_iterate(batch, y, n_iter, m_nom=None, N_nom=None, gamma=None, want_filter=False,
                 ws=None):
    """Algorithm 3 in place on (m_nom, N_nom); returns (m_nom, N_nom[, m_f, N_f])."""
    _require_gpu()
    if m_nom is None:
        m_nom, N_nom = batch.prior_nominal()
    m_f = N_f = None
    if want_filter:
        m_f, N_f = batch.new_marg()
    if ws is None:
        ws, n = batch.workspace("ipls")
    else:
        n = ws.numel()
    p = batch.struct()
    _check(lib().pss_ipls_iterate(ctypes.byref(p), _gamma_c(gamma), _ptr(y), int(n_iter),
                                  _ptr(m_nom), _ptr(N_nom), _ptr(m_f), _ptr(N_f), _ptr(ws), n,
                                  _stream()))
    return (m_nom, N_nom, m_f, N_f) if want_filter else (m_nom, N_nom)


def sequential_smoother(batch, y, n_iter, m_nom=None, N_nom=None, gamma=None, want_filter=False,
                        ws=None):
    _require_gpu()
    if m_nom is None:
        m_nom, N_nom = batch.prior_nominal()
    m_f = N_f = None
    if want_filter:
        m_f, N_f = batch.new_marg()
    if ws is None:
        ws, n = batch.workspace("sequential")
    else:
        n = ws.numel()
    p = batch.struct()
    _check(lib().pss_sequential_smoother(ctypes.byref(p), _gamma_c(gamma), _ptr(y), int(n_iter),
                                         _ptr(m_nom), _ptr(N_nom), _ptr(m_f), _ptr(N_f),
                                         _ptr(ws), n, _stream()))
    return (m_nom, N_nom, m_f, N_f) if want_filter else (m_nom, N_nom)


class Checkpoint:
    """A pss_ckpt: device buffer (torch uint8) plus the C struct.  level 0
    keeps every filtering marginal, level l >= 1 the filter scan's level-l
    prefixes (the gradient re-runs the levels below), a level at or above the
    scan's top only the log-likelihoods."""

    def __init__(self, batch, level=0):
        self.level = int(level)
        self.bytes = ckpt_size(batch, self.level)
        self.buf = torch.empty(max(self.bytes, 1), dtype=torch.uint8, device=batch.device)
        self.c = CkptC()
        self.c.level = self.level
        self.c.buf = self.buf.data_ptr()
        self.c.bytes = self.bytes
        self.c.tag = 0

    def ref(self):
        return ctypes.byref(self.c)


def ckpt_size(batch, level) -> int:
    p = batch.struct()
    return int(lib().pss_ckpt_size(ctypes.byref(p), int(level)))


def _ckpt_ref(ckpt):
    return None if ckpt is None else ckpt.ref()


def loglik(batch, y, m_nom=None, N_nom=None, gamma=None, ws=None, ckpt=None):
    """Pseudo-log-likelihood per sequence (float64 [B]); fills ckpt if given."""
    _require_gpu()
    ll = torch.empty(batch.B, dtype=torch.float64, device=batch.device)
    if ws is None:
        ws, n = batch.workspace("loglik")
    else:
        n = ws.numel()
    p = batch.struct()
    _check(lib().pss_loglik(ctypes.byref(p), _gamma_c(gamma), _ptr(m_nom), _ptr(N_nom), _ptr(y),
                            _ptr(ll), _ckpt_ref(ckpt), _ptr(ws), n, _stream()))
    return ll


def loglik_grad(batch, m_nom, N_nom, y, ll_bar=None, ws=None, ckpt=None):
    """(ll [B], grad [3, B], theta_bar [3]) at the frozen nominal, by the
    reverse-mode adjoint (from ckpt when given)."""
    _require_gpu()
    dev = batch.device
    ll = torch.empty(batch.B, dtype=torch.float64, device=dev)
    grad = torch.empty((3, batch.B), dtype=torch.float64, device=dev)
    tb = torch.empty(3, dtype=torch.float64, device=dev)
    if ws is None:
        ws, n = batch.workspace("loglik_grad")
    else:
        n = ws.numel()
    if ll_bar is not None:
        ll_bar = ll_bar.to(device=dev, dtype=torch.float64).contiguous()
    p = batch.struct()
    _check(lib().pss_loglik_grad(ctypes.byref(p), _ptr(m_nom), _ptr(N_nom), _ptr(y),
                                 _ptr(ll_bar), _ckpt_ref(ckpt), _ptr(ll), _ptr(grad), _ptr(tb),
                                 _ptr(ws), n, _stream()))
    return ll, grad, tb


def score_fisher(batch, m_nom, N_nom, y, ll_bar=None, ws=None):
    """The same gradient by Fisher's identity from the smoother (cross-check)."""
    _require_gpu()
    dev = batch.device
    ll = torch.empty(batch.B, dtype=torch.float64, device=dev)
    grad = torch.empty((3, batch.B), dtype=torch.float64, device=dev)
    tb = torch.empty(3, dtype=torch.float64, device=dev)
    if ws is None:
        ws, n = batch.workspace("score_fisher")
    else:
        n = ws.numel()
    if ll_bar is not None:
        ll_bar = ll_bar.to(device=dev, dtype=torch.float64).contiguous()
    p = batch.struct()
    _check(lib().pss_score_fisher(ctypes.byref(p), _ptr(m_nom), _ptr(N_nom), _ptr(y),
                                  _ptr(ll_bar), _ptr(ll), _ptr(grad), _ptr(tb), _ptr(ws), n,
                                  _stream()))
    return ll, grad, tb


def loglik_vjp(batch, y, m_nom=None, N_nom=None, gamma=None, ll_bar=None, ws=None, ckpt=None,
               prior=True):
    """VJP of the log-likelihood with respect to every step's linearisation
    and the prior: (ll [B], g_bar (stride-1 Gamma dict of cotangents),
    m0_bar [nx, B], N0_bar [P, B]) -- the prior parts None if not prior."""
    _require_gpu()
    dev = batch.device
    ll = torch.empty(batch.B, dtype=torch.float64, device=dev)
    gbar = batch.new_gamma(1)
    m0b = N0b = None
    if prior:
        m0b = batch.empty(batch.nx, batch.B)
        N0b = batch.empty(tri(batch.nx), batch.B)
    if ws is None:
        ws, n = batch.workspace("loglik_vjp")
    else:
        n = ws.numel()
    if ll_bar is not None:
        ll_bar = ll_bar.to(device=dev, dtype=torch.float64).contiguous()
    p = batch.struct()
    _check(lib().pss_loglik_vjp(ctypes.byref(p), _gamma_c(gamma), _ptr(m_nom), _ptr(N_nom),
                                _ptr(y), _ptr(ll_bar), _ckpt_ref(ckpt), _ptr(ll), _gamma_c(gbar),
                                _ptr(m0b), _ptr(N0b), _ptr(ws), n, _stream()))
    return ll, gbar, m0b, N0b


STATUS_FILTER, STATUS_SMOOTHER, STATUS_LOGLIK = 1, 2, 4


def nan_status(batch, m=None, N=None, marg_bit=STATUS_SMOOTHER, ll=None,
               ll_bit=STATUS_LOGLIK, status=None):
    """Per-sequence int32 bitmask of non-finite results (ORed into status)."""
    _require_gpu()
    if status is None:
        status = torch.zeros(batch.B, dtype=torch.int32, device=batch.device)
    p = batch.struct()
    _check(lib().pss_nan_status(ctypes.byref(p), _ptr(m), _ptr(N), int(marg_bit), _ptr(ll),
                                int(ll_bit), _ptr(status), _stream()))
    return status


class LogLik(torch.autograd.Function):
    """Pseudo-log-likelihood summed over the batch as a function of theta =
    (log q1, log q2, log sigma) at a frozen nominal.  The forward pass keeps
    a checkpoint of its filter pass (level ckpt_level); backward runs the
    library's reverse-mode adjoint from it with the incoming cotangent."""

    @staticmethod
    def forward(ctx, theta, batch, y, m_nom, N_nom, ckpt_level=0):
        th = tuple(float(v) for v in theta.detach().cpu().tolist())
        b2 = _with_theta(batch, th)
        ck = Checkpoint(b2, ckpt_level)
        ll = loglik(b2, y, m_nom, N_nom, ckpt=ck)
        ctx.save_for_backward(theta)
        ctx.stuff = (b2, y, m_nom, N_nom, ck)
        return ll.sum().to(theta.dtype)

    @staticmethod
    def backward(ctx, g):
        (theta,) = ctx.saved_tensors
        b2, y, m_nom, N_nom, ck = ctx.stuff
        w = torch.full((b2.B,), 1.0, dtype=torch.float64, device=b2.device) * g.to(
            device=b2.device, dtype=torch.float64)
        _, _, tb = loglik_grad(b2, m_nom, N_nom, y, ll_bar=w, ckpt=ck)
        return tb.to(device=theta.device, dtype=theta.dtype), None, None, None, None, None


def loglik_grad_ift(batch, m_nom, N_nom, y, n_iter=30, ws=None, with_delta=False):
    """(ll [B], grad [3, B][, delta [B]]): the total derivative of the
    pseudo-log-likelihood at the IPLS fixed point (m_nom, N_nom) (Algorithm
    4), CT model; delta is the per-sequence tangent change of the last
    iteration (a convergence check)."""
    _require_gpu()
    dev = batch.device
    ll = torch.empty(batch.B, dtype=torch.float64, device=dev)
    grad = torch.empty((3, batch.B), dtype=torch.float64, device=dev)
    delta = torch.empty(batch.B, dtype=torch.float64, device=dev) if with_delta else None
    if ws is None:
        ws, n = batch.workspace("loglik_grad_ift")
    else:
        n = ws.numel()
    p = batch.struct()
    _check(lib().pss_loglik_grad_ift(ctypes.byref(p), _ptr(m_nom), _ptr(N_nom), _ptr(y),
                                     int(n_iter), _ptr(ll), _ptr(grad), _ptr(delta), _ptr(ws), n,
                                     _stream()))
    return (ll, grad, delta) if with_delta else (ll, grad)


class LogLikFixedPoint(torch.autograd.Function):
    """sum_b l_b(theta) at the IPLS fixed point (m_nom, N_nom) computed for
    theta; backward returns the total derivative (Algorithm 4) through
    pss_loglik_grad_ift."""

    @staticmethod
    def forward(ctx, theta, batch, y, m_nom, N_nom, n_iter=30):
        th = tuple(float(v) for v in theta.detach().cpu().tolist())
        b2 = _with_theta(batch, th)
        ll, grad = loglik_grad_ift(b2, m_nom, N_nom, y, n_iter=n_iter)
        ctx.save_for_backward(theta)
        ctx.grad = grad.sum(dim=1)
        return ll.sum().to(theta.dtype)

    @staticmethod
    def backward(ctx, g):
        (theta,) = ctx.saved_tensors
        tb = ctx.grad * g.to(device=ctx.grad.device, dtype=torch.float64)
        return tb.to(device=theta.device, dtype=theta.dtype), None, None, None, None, None


def _with_theta(batch, theta):
    b = Batch.__new__(Batch)
    b.__dict__.update(batch.__dict__)
    b.theta = tuple(float(v) for v in theta)
    return b


# ---------------------------------------------------------------------------
# ragged multi-group batches (one persistent launch per pass)
# ---------------------------------------------------------------------------
class _Groups:
    """ctypes array of pss_group plus the objects it points into (kept alive)."""

    def __init__(self, groups):
        self.keep = []
        arr = (GroupC * len(groups))()
        for i, (batch, y, m, N, gamma) in enumerate(groups):
            p = batch.struct()
            self.keep.append(p)
            arr[i].p = ctypes.pointer(p)
            if gamma is not None:
                gc = GammaC()
                for k in ("F", "c", "SL", "H", "d", "SO"):
                    setattr(gc, k, gamma[k].data_ptr())
                gc.stride = gamma["stride"]
                self.keep.append(gc)
                arr[i].g = ctypes.addressof(gc)
            else:
                arr[i].g = None
            arr[i].y = y.data_ptr()
            arr[i].m_nom = m.data_ptr()
            arr[i].N_nom = N.data_ptr()
        self.arr = arr
        self.n = len(groups)


def batched_workspace_size(groups) -> int:
    g = _Groups(groups)
    return int(lib().pss_batched_workspace_size(g.arr, g.n))


def ipls_batched(groups, n_iter, ws=None, status=None):
    """Algorithm 3 over several groups; groups = [(batch, y, m_nom, N_nom, gamma|None)].
    The nominals are updated in place.  Returns the device status tensor."""
    _require_gpu()
    g = _Groups(groups)
    if ws is None:
        n = int(lib().pss_batched_workspace_size(g.arr, g.n))
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=groups[0][0].device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=groups[0][0].device)
    _check(lib().pss_ipls_batched(g.arr, g.n, int(n_iter), _ptr(status), _ptr(ws), ws.numel(),
                                  _stream()))
    return status


def autotune(groups, cache_path=None):
    """Time the candidate launch shapes on these groups; returns (T, E_f, E_s)."""
    _require_gpu()
    g = _Groups(groups)
    n = int(lib().pss_autotune_workspace_size(g.arr, g.n))
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device=groups[0][0].device)
    best = (ctypes.c_int32 * 3)()
    _check(lib().pss_autotune(g.arr, g.n, _ptr(ws), n,
                              cache_path.encode() if cache_path else None,
                              ctypes.cast(best, ctypes.c_void_p), _stream()))
    return tuple(best)
