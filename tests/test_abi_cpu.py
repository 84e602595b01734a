"""Host-side checks of the C ABI (no GPU, no compute calls).

* libpss.so loads and exports every entry point include/pss.h declares;
* pss_validate / pss_workspace_size reject malformed problems before any HIP
  call, and the entry points return the documented status codes;
* workspace sizes and the scan level plan behave as documented.
"""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

from paper_2207_00426_amd import pss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "pss.h")).read()
    decl = r"^(?:int|int64_t|size_t|const char \*)\s*(pss_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    return pss.lib()


def test_library_exports_every_declared_symbol(L):
    syms = _header_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(L, s), s
    assert set(pss.EXPORTS) == set(syms)
    assert "gfx950" in pss.version()


def _cpu_batch(**kw):
    args = dict(model=pss.MODEL_LINEAR, dtype=torch.float64, nx=4, ny=2,
                y_off=np.array([0, 10, 25]), m0=np.zeros(4), N0=np.eye(4), device="cpu")
    args.update(kw)
    return pss.Batch(**args)


def test_validation_accepts_and_rejects(L):
    assert pss.validate(_cpu_batch()) == 0
    b = _cpu_batch()
    b.y_off_host = np.array([0, 10, 10], dtype=np.int64)  # empty sequence
    assert pss.validate(b) == -1
    b = _cpu_batch()
    b.y_off_host = np.array([1, 10, 25], dtype=np.int64)
    assert pss.validate(b) == -1
    assert pss.validate(_cpu_batch(nx=9, ny=2, m0=np.zeros(9), N0=np.eye(9))) == -1
    assert pss.validate(_cpu_batch(nx=6, ny=2, m0=np.zeros(6), N0=np.eye(6))) == -2
    assert pss.validate(_cpu_batch(model=pss.MODEL_CT)) == -1  # CT needs nx=5, ny=2
    b = _cpu_batch(model=pss.MODEL_CT, nx=5, m0=np.zeros(5), N0=np.eye(5), dt=0.0)
    assert pss.validate(b) == -1  # dt must be > 0
    b = _cpu_batch(scan_threads=100)
    assert pss.validate(b) == -1
    assert "scan_threads" in pss.last_error()
    b = _cpu_batch()
    b.model = 7
    assert pss.validate(b) == -1


def test_null_arguments_rejected_before_any_hip_call(L):
    b = _cpu_batch()
    p = b.struct()
    rc = L.pss_sqrt_filter_scan(ctypes.byref(p), None, None, None, None, 0, None)
    assert rc == -1
    rc = L.pss_slr_linearize(ctypes.byref(p), None, None, None, None, None)
    assert rc == -2  # a linear model has no SLR
    rc = L.pss_loglik_grad(ctypes.byref(p), None, None, None, None, None, None, None, None,
                           None, 0, None)
    assert rc == -2
    rc = L.pss_score_fisher(ctypes.byref(p), None, None, None, None, None, None, None, None, 0,
                            None)
    assert rc == -2
    rc = L.pss_loglik_vjp(ctypes.byref(p), None, None, None, None, None, None, None, None, None,
                          None, None, 0, None)
    assert rc == -1
    assert L.pss_validate(None) == -1


def test_workspace_sizes_and_too_small_workspace(L):
    b = _cpu_batch()
    for op in pss.OPS:
        n = pss.workspace_size(b, op)
        assert n >= 0 and n % 256 == 0
    assert pss.workspace_size(b, "slr") == 0
    big = _cpu_batch(y_off=np.array([0, 100000]))
    assert pss.workspace_size(big, "ipls") > pss.workspace_size(b, "ipls")
    # a workspace that is too small is refused with its own status
    p = b.struct()
    fe = pss.FElemC()
    for k in ("A", "b", "U", "eta", "Z"):
        setattr(fe, k, 8)  # non-null dummies; nothing is dereferenced
    rc = L.pss_sqrt_filter_scan(ctypes.byref(p), ctypes.byref(fe), ctypes.c_void_p(8),
                                ctypes.c_void_p(8), ctypes.c_void_p(8), 1, None)
    assert rc == -3
    assert "workspace" in pss.last_error()


def test_scan_levels_grow_logarithmically(L):
    # forcing tiny tiles makes the plan deeper; the workspace grows with it
    small = _cpu_batch(y_off=np.array([0, 5000]), scan_threads=64, scan_elems=1)
    large = _cpu_batch(y_off=np.array([0, 5000]), scan_threads=256, scan_elems=8)
    assert pss.workspace_size(small, "filter_scan") > pss.workspace_size(large, "filter_scan")


def test_layout_helpers_roundtrip():
    rng = np.random.default_rng(0)
    N = np.tril(rng.standard_normal((7, 5, 5)))
    P = pss.pack_lower(N)
    assert P.shape == (7, 15)
    np.testing.assert_array_equal(pss.unpack_lower(P, 5), N)
    t = pss.to_soa(N.reshape(7, 25), torch.float64, "cpu")
    assert t.shape == (25, 7)
    np.testing.assert_array_equal(pss.from_soa(t, (5, 5)), N)


def test_compute_calls_refuse_without_gpu():
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    b = _cpu_batch()
    with pytest.raises(RuntimeError):
        pss.ipls_iterate(b, torch.zeros(2, 25, dtype=torch.float64), 1,
                         gamma=b.new_gamma(0))


def test_kernel_timing_switch_without_launches(L):
    # no launch was timed: the report is empty and the switch round-trips
    pss.kernel_timing(True)
    pss.kernel_timing(False)
    assert pss.kernel_times() == {}


def test_form_and_linearization_fields_are_validated(L):
    b = _cpu_batch()
    b.form = 2
    assert pss.validate(b) == -1
    b = _cpu_batch()
    b.linearization = 4
    assert pss.validate(b) == -1
    assert pss.validate(_cpu_batch(form="cov")) == 0
    # the covariance form is refused by the square-root-only entry points
    # before anything is dereferenced or enqueued
    p = _cpu_batch(form="cov").struct()
    fe = pss.FElemC()
    for k in ("A", "b", "U", "eta", "Z"):
        setattr(fe, k, 8)
    rc = L.pss_sqrt_filter_scan(ctypes.byref(p), ctypes.byref(fe), ctypes.c_void_p(8),
                                ctypes.c_void_p(8), ctypes.c_void_p(8), 1, None)
    assert rc == -2 and "square-root" in pss.last_error()


def _ricker_cpu(**kw):
    args = dict(model=pss.MODEL_RICKER, dtype=torch.float64, nx=1, ny=1,
                y_off=np.array([0, 10, 25]), m0=np.array([np.log(7.0)]),
                N0=np.array([[0.01]]), device="cpu", theta=(np.log(44.7), np.log(10.0),
                                                           np.log(0.09)))
    args.update(kw)
    return pss.Batch(**args)


def test_ricker_model_and_sigma_point_rules_are_validated(L):
    for lin in ("cubature", "taylor", "unscented", "gauss_hermite"):
        assert pss.validate(_ricker_cpu(linearization=lin)) == 0, lin
        assert pss.validate(_ricker_cpu(linearization=lin, form="cov")) == 0, lin
    # the Ricker model is scalar
    assert pss.validate(_ricker_cpu(nx=2, m0=np.zeros(2), N0=np.eye(2))) == -1
    b = _ricker_cpu()
    b.theta = (float("nan"), 0.0, 0.0)
    assert pss.validate(b) == -1
    # unscented: kappa >= 0 keeps every weight positive
    assert pss.validate(_ricker_cpu(linearization="unscented", ut_kappa=-0.5)) == -1
    assert "kappa" in pss.last_error()
    assert pss.validate(_ricker_cpu(linearization="unscented", ut_kappa=0.0)) == 0
    # Gauss-Hermite: order 2..20 and at most 1024 points
    assert pss.validate(_ricker_cpu(linearization="gauss_hermite", gh_order=1)) == -1
    assert pss.validate(_ricker_cpu(linearization="gauss_hermite", gh_order=20)) == 0
    assert pss.validate(_ricker_cpu(linearization="gauss_hermite", gh_order=21)) == -1
    ct = dict(model=pss.MODEL_CT, nx=5, ny=2, m0=np.zeros(5), N0=np.eye(5), dt=0.01)
    assert pss.validate(_cpu_batch(linearization="gauss_hermite", gh_order=4, **ct)) == 0
    assert pss.validate(_cpu_batch(linearization="gauss_hermite", gh_order=5, **ct)) == -1
    assert "1024" in pss.last_error()
    # the gradient is defined for the CT model only; refused before any HIP call
    p = _ricker_cpu().struct()
    rc = L.pss_loglik_grad(ctypes.byref(p), None, None, None, None, None, None, None, None,
                           None, 0, None)
    assert rc == -2
    rc = L.pss_score_fisher(ctypes.byref(p), None, None, None, None, None, None, None, None, 0,
                            None)
    assert rc == -2
    rc = L.pss_loglik_vjp(ctypes.byref(p), None, None, None, None, None, None, None, None, None,
                          None, None, 0, None)
    assert rc == -1
    # the persistent pass fuses the cubature / Taylor CT SLR only
    y = ctypes.c_void_p(8)
    for bad in (_ricker_cpu(), _cpu_batch(linearization="unscented", **ct)):
        pb = bad.struct()
        g = pss.GroupC(ctypes.pointer(pb), None, y, y, y)
        assert L.pss_batched_workspace_size(ctypes.byref(g), 1) == 0
        rc = L.pss_ipls_batched(ctypes.byref(g), 1, 1, None, None, 0, None)
        assert rc == -2, pss.last_error()


def test_fixed_point_gradient_is_validated_before_any_hip_call(L):
    # (refusals before any HIP call)
    ct = dict(model=pss.MODEL_CT, nx=5, ny=2, m0=np.zeros(5), N0=np.eye(5), dt=0.01)
    b = _cpu_batch(**ct)
    assert pss.workspace_size(b, "loglik_grad_ift") > pss.workspace_size(b, "loglik_grad")
    d = ctypes.c_void_p(8)
    # FP32 is built too; non-CT models are refused
    assert pss.workspace_size(_cpu_batch(dtype=torch.float32, **ct), "loglik_grad_ift") > 0
    for bad in (_ricker_cpu(), _cpu_batch()):
        p = bad.struct()
        assert pss.workspace_size(bad, "loglik_grad_ift") == 0
        rc = L.pss_loglik_grad_ift(ctypes.byref(p), d, d, d, 5, d, d, None, d, 1 << 40, None)
        assert rc == -2, pss.last_error()
    p = b.struct()
    # n_iter >= 1, non-null buffers, a large enough workspace
    assert L.pss_loglik_grad_ift(ctypes.byref(p), d, d, d, 0, d, d, None, d, 1 << 40, None) == -1
    assert L.pss_loglik_grad_ift(ctypes.byref(p), None, d, d, 5, d, d, None, d, 1 << 40,
                                 None) == -1
    assert L.pss_loglik_grad_ift(ctypes.byref(p), d, d, d, 5, d, d, None, d, 16, None) == -3
    assert "workspace" in pss.last_error()


def _scan_ws_bytes(plan, B, NE, NP, esz):
    """Workspace of one scan as the library carves it: tile offsets of every
    level; element offsets, elements and exclusive prefixes of every level
    above the finest; the LDS-tree copies of the lower tree levels (each
    piece 256-byte aligned)."""
    al = lambda x: (x + 255) // 256 * 256
    used = 0
    for l, (T, E, elems, tiles, threads, flat) in enumerate(plan):
        used += al((B + 1) * 8)
        if l > 0:
            used += al((B + 1) * 8) + al(NE * elems * esz) + al(NP * elems * esz)
        if l + 1 < len(plan) and not flat:
            used += al(NE * tiles * T * esz)
    return used


@pytest.mark.parametrize("lengths", [[1], [255], [256], [257], [10 ** 6], [150, 37, 400, 1],
                                     [3000] * 70])
@pytest.mark.parametrize("T,E", [(0, 0), (128, 1), (256, 8)])
def test_bench_scan_plan_mirrors_the_library(L, lengths, T, E):
    """bench.py prices every scan kernel from its own mirror of the level plan
    (flat finest filter level, tree levels above, the smoother's tree): the
    workspace that mirror implies is exactly what the library asks for."""
    import bench
    y_off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    b = _cpu_batch(nx=5, ny=2, m0=np.zeros(5), N0=np.eye(5), y_off=y_off, scan_threads=T,
                   scan_elems=E)
    B = len(lengths)
    fplan = bench.scan_plan(lengths, *bench.shapes("f64", T, E, False))
    assert fplan[0][5] and not any(lv[5] for lv in fplan[1:])
    assert pss.workspace_size(b, "filter_scan") == _scan_ws_bytes(fplan, B, 65, 20, 8)
    splan = bench.scan_plan([n + 1 for n in lengths], *bench.shapes("f64", T, E, True))
    assert not any(lv[5] for lv in splan)
    T_x = int(y_off[-1]) + B
    stash = (45 * T_x * 8 + 255) // 256 * 256
    assert pss.workspace_size(b, "smoother_scan") == _scan_ws_bytes(splan, B, 45, 20, 8) + stash


def test_checkpoint_sizes_and_validation(L):
    """pss_ckpt_size follows the level plan: level 0 keeps every filtering
    marginal, level l the filter scan's level-l prefixes, levels at or above
    the top only the log-likelihoods; a wrong tag, a short buffer or the
    covariance form are refused before any HIP call."""
    n = 10 ** 5
    b = pss.Batch(pss.MODEL_CT, torch.float64, 5, 2, np.array([0, n]), np.zeros(5), np.eye(5),
                  device="cpu", dt=0.01, theta=(0.0, 0.0, 0.0))
    s0, s1, s2, s9 = (pss.ckpt_size(b, lv) for lv in (0, 1, 2, 9))
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    assert s0 == al(8) + al(20 * 8 * (n + 1))
    # flat level 0 folds 4 per thread: n / 4 prefixes at level 1
    assert s1 == al(8) + al(20 * 8 * (n // 4))
    assert s2 == al(8) + al(20 * 8 * -(-n // (4 * 256)))
    assert s9 == al(8)
    assert s0 > s1 > s2 > s9
    assert pss.ckpt_size(b, -1) == 0
    p = b.struct()
    ck = pss.CkptC()
    ck.level = 0
    ck.buf = 1
    ck.bytes = s0 - 1
    ck.tag = 0
    ws = ctypes.c_void_p(1)
    big = 1 << 40
    # consuming: short buffer, then a tag of another problem
    rc = L.pss_loglik_grad(ctypes.byref(p), ws, ws, ws, None, ctypes.byref(ck), ws, ws, ws, ws,
                           big, None)
    assert rc == -3 and "checkpoint" in pss.last_error()
    ck.bytes = s0
    rc = L.pss_loglik_grad(ctypes.byref(p), ws, ws, ws, None, ctypes.byref(ck), ws, ws, ws, ws,
                           big, None)
    assert rc == -1 and "another problem" in pss.last_error()
    b.form = pss.FORM_COV
    p = b.struct()
    rc = L.pss_loglik(ctypes.byref(p), None, ws, ws, ws, ws, ctypes.byref(ck), ws, big, None)
    assert rc == -2
