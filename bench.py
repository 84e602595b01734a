"""Benchmark of the parallel square-root iterated smoother on one MI355X.

Main workload: coordinated-turn bearings-only tracking, one long sequence of
n = 10^6 steps (the long-sequence configuration), 10 cubature IPLS passes
(SLR, filter elements, filter scan, smoother scan), then the
pseudo-log-likelihood and its gradient at the final nominal (one gradient
pass returns both), FP64.  One
"step" is that whole hot path over the sequence, captured in a HIP graph and
replayed; inputs are synthetic (seeded simulation) and already in HBM.

value = smoothed time steps per second = n * passes / seconds per step.

Also in the line (same run):
  fp32            the same step in FP32
  ieks_taylor     the same step with the first-order Taylor linearisation
                  (the iterated extended smoother) instead of cubature SLR
  sequential      time per IPLS pass of the parallel scans (with their
                  algorithmic GB/s) vs the sequential square-root kernel (one
                  wavefront walks the sequence, each step's Tria rows on its
                  lanes) at n = 10^4 and 10^5 (prefixes of
                  the same sequence, both precisions) and n = 10^6 (FP64)
  loglik_grad_ms  one loglik + gradient evaluation (the reverse-mode
                  adjoint) on 64 CT sequences of 10^4 steps (the parameter-
                  estimation configuration), with the checkpointed split
                  (forward with a checkpoint of each level, backward from it,
                  bytes kept) and the Fisher-identity route beside it, and 50
                  L-BFGS steps on theta from theta* + 0.5 on that batch (IPLS
                  re-run at every evaluation); ipls_next_pass_change: how far
                  the nominal still moves in one more pass after those
                  passes, per sequence (whether IPLS reached a fixed point)
  kernels         every scan kernel of one filter and one smoother scan,
                  timed per launch with HIP events on its stream, with the
                  counted flops it executes
  roofline        the kernel with the largest time among those: its counted
                  flops and algorithmic bytes per launch over its time, against
                  78.6 TFLOP/s (vector ALU) and 8 TB/s (HBM); bound = the larger
                  of the two lower bounds; traffic = counter HBM bytes per
                  launch from the committed rocprofv3 summary, when it was
                  taken on these kernels
  pass            one IPLS pass (its kernels once each): time, flops, the
                  algorithmic bytes and the counter bytes against the fused
                  minimum (the nominal and y in, the nominal out)
  fp32_divergence share of FP32 runs whose log-likelihood is NaN, square-root
                  vs standard covariance form (15 CT sequences per length,
                  20 passes; FP64 as a control)
  cpu_baseline    the FP64 oracle on the host, on a bounded prefix of the
                  same sequence
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2207_00426_amd import estimate  # noqa: E402
from paper_2207_00426_amd import pss  # noqa: E402
from paper_2207_00426_amd import workloads as wl  # noqa: E402

# Counted floating-point operations of the nx = 5, ny = 2 operators (add,
# multiply, divide, reciprocal, square root = 1; fused multiply-add = 2;
# transcendentals apart), from tests/flop_count.cpp, which instantiates the
# library's register code on a counting number type
# (tests/test_flop_counts_cpu.py keeps these equal to its output).  "_leaf":
# the filter operator with a finest-level element on the right, whose Z has
# only ny non-zero columns.  adjoint_element: the Kalman step and its map
# T_k; adjoint_cotangents: the Gram cotangents and the theta contraction.
FLOPS = dict(filter_combine=3371, filter_combine_leaf=2516, filter_apply=1912,
             filter_apply_leaf=1396, smoother_combine=732, smoother_apply=503,
             filter_element=1248, smoother_element=1510, slr_transition=1971, slr_bearings=437,
             adjoint_element=1469, adjoint_combine=740, adjoint_apply=515,
             adjoint_cotangents=966)
PEAK = {"f64": 78.6, "f32": 78.6}  # TFLOP/s vector ALU (FP32 without packed instructions)
HBM_GBPS = 8000.0  # MI355X HBM3E peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10 ** 6)
    ap.add_argument("--passes", type=int, default=10)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--scan-threads", type=int, default=0)
    ap.add_argument("--scan-elems", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="main line only (profiling)")
    ap.add_argument("--batched-only", action="store_true",
                    help="the ragged 512-sequence batch alone (profiling its persistent pass)")
    return ap.parse_args()


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def scan_plan(lengths, T0, E0, Tup, E1, Eup, flat0):
    """Mirror of the library's level plan: per level (T, E, elements, tiles,
    active threads, flat).  With flat0 the finest level is flat (never the
    top): its threads' aggregates are the next level's elements."""
    cnt = np.asarray(lengths, dtype=np.int64)
    levels = []
    for l in range(8):
        T, E = (T0, E0) if l == 0 else (Tup, E1 if l == 1 else Eup)
        TS = T * E
        tiles = -(-cnt // TS)
        last = cnt - (tiles - 1) * TS
        threads = (tiles - 1) * T + (-(-last // E))
        flat = flat0 and l == 0
        top = cnt.max() <= TS and not flat
        levels.append((T, E, int(cnt.sum()), int(tiles.sum()), int(threads.sum()), flat))
        if top:
            break
        cnt = -(-cnt // E) if flat else tiles
    return levels


def scan_kernel_flops(op, lengths, T0, E0, Tup, E1, Eup, flat0):
    """Counted flops of each kernel of one scan, keyed (kernel, level).

    Up-sweep (and the first half of the top kernel): the fold and the tile
    tree combine every element but the first of each tile, elems - tiles
    combines.  Down-sweep: the tree applies threads - tiles times and every
    element is applied once.  A flat level has no tree: elems - threads
    combines up, elems applies down.  The smoother's level-0 up-sweep also
    builds its elements (one per state)."""
    comb, app = FLOPS[op + "_combine"], FLOPS[op + "_apply"]
    if op == "adjoint":
        comb, app = FLOPS["adjoint_combine"], FLOPS["adjoint_apply"]
    # the filter's finest level folds and applies leaf elements (elements -
    # threads fold combines, elements applies); its trees use the general form
    lcomb = FLOPS.get(op + "_combine_leaf", comb)
    lapp = FLOPS.get(op + "_apply_leaf", app)
    plan = scan_plan(lengths, T0, E0, Tup, E1, Eup, flat0)
    out = {}
    for l, (T, E, elems, tiles, threads, flat) in enumerate(plan):
        if flat:
            up = (elems - threads) * lcomb
            down = elems * lapp
        elif l == 0:
            up = (elems - threads) * lcomb + (threads - tiles) * comb
            down = elems * lapp + (threads - tiles) * app
        else:
            up = (elems - tiles) * comb
            down = (elems + threads - tiles) * app
        if op == "smoother" and l == 0:
            up += elems * FLOPS["smoother_element"]
        if op == "adjoint" and l == 0:
            # the map of every step is built in the up-sweep and again in the
            # down-sweep, which also forms the step's cotangents
            up += elems * FLOPS["adjoint_element"]
            down += elems * (FLOPS["adjoint_element"] + FLOPS["adjoint_cotangents"])
        if l == len(plan) - 1:
            out[(op + "_top", l)] = up + down
        else:
            out[(op + "_up", l)] = up
            out[(op + "_down", l)] = down
    return out


# numbers per object (CT, nx = 5, ny = 2): marginal (m, packed N), filter
# element, smoother element / adjoint map, linearisation parts
NUM = dict(marg=20, felem=65, selem=45, gam_trans=45, gam_obs=15, y=2)


def scan_kernel_bytes(op, lengths, T0, E0, Tup, E1, Eup, flat0, esz, B=1):
    """Algorithmic HBM bytes of each kernel of one scan, keyed (kernel,
    level): every input the kernel's contract needs read once and every
    output written once, in the library's storage design (elements of the
    level, the tile's saved LDS tree, tile aggregates, exclusive prefixes).
    Level-0 inputs: filter elements (filter); the filtering marginal and the
    transition part of Gamma per state, plus the element stash written in
    the up-sweep and read in the down-sweep (smoother); the marginal, Gamma
    and y per step, and 3 FP64 theta terms written per step (adjoint)."""
    plan = scan_plan(lengths, T0, E0, Tup, E1, Eup, flat0)
    ne = NUM["felem"] if op == "filter" else NUM["selem"]
    npre = NUM["marg"]
    out = {}
    for l, (T, E, elems, tiles, threads, flat) in enumerate(plan):
        top = l == len(plan) - 1
        tree = 0 if (flat or top) else tiles * T * ne
        if l == 0 and op == "smoother":
            src_up = elems * npre + (elems - B) * NUM["gam_trans"] + elems * NUM["selem"]
            src_down = elems * NUM["selem"]
        elif l == 0 and op == "adjoint":
            src_up = src_down = elems * (npre + NUM["gam_trans"] + NUM["gam_obs"] + NUM["y"])
        else:
            src_up = src_down = elems * ne
        agg = threads * ne if flat else tiles * ne
        pre_in = threads * npre if flat else tiles * npre
        outs = elems * npre * esz
        if l == 0 and op == "adjoint":
            outs = elems * 3 * 8
        if top:
            out[(op + "_top", l)] = src_up * esz + outs
        else:
            out[(op + "_up", l)] = (src_up + tree + agg) * esz
            out[(op + "_down", l)] = (src_down + tree + pre_in) * esz + outs
    return out


def kernel_source_hash():
    """Hash of the HIP sources and build flags: a counter summary taken from
    other kernels than the ones built here is not used."""
    import hashlib
    from paper_2207_00426_amd import build as hipbuild
    # build flags without include paths (those differ between machines)
    h = hashlib.sha256(" ".join(f for f in hipbuild.FLAGS if not f.startswith("-I")).encode())
    csrc = os.path.join(ROOT, "paper_2207_00426_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    with open(os.path.join(ROOT, "include", "pss.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, level, dtype, n, summary=None):
    """HBM bytes per launch of (kernel, level) from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload, each scaled by what the
    same counter reads for a copy of known size; None when there is no
    summary for the kernels built here."""
    name = summary or "hbm_traffic_ct_n%d_%s.md" % (n, dtype)
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic:"):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                rec[(kv["kernel"], int(kv["level"]))] = kv
    kv = rec.get((kernel, level))
    if kv is None or kv.get("src") != kernel_source_hash():
        return None
    return int(float(kv["bytes"]))


def pass_alg_bytes(n, dtype, T_req=0, E_req=0):
    """Algorithmic HBM bytes of one IPLS pass of one sequence of n steps
    (the kernels of the multi-launch pass: linearisation, filter elements,
    every filter and smoother scan kernel)."""
    esz = 8 if dtype == "f64" else 4
    by = scan_kernel_bytes("filter", [n], *shapes(dtype, T_req, E_req), esz)
    by.update(scan_kernel_bytes("smoother", [n + 1], *shapes(dtype, T_req, E_req, True), esz))
    gam = NUM["gam_trans"] + NUM["gam_obs"]
    tot = sum(by.values())
    if dtype == "f32":  # linearisation fused with the elements
        tot += ((n + 1) * NUM["marg"] + n * (NUM["y"] + NUM["gam_trans"] + NUM["felem"])) * esz
    else:
        tot += ((n + 1) * NUM["marg"] + n * (NUM["y"] + gam)) * esz
        tot += n * (gam + NUM["y"] + NUM["felem"]) * esz
    return tot


def copy_probe(stream, dev, reps=5):
    """Plain streaming copy of known size (1 GiB read + 1 GiB written, an
    elementwise negate): HBM bandwidth reference, and the calibration kernel
    for the FETCH_SIZE / WRITE_SIZE counters."""
    x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    ms = timed(stream, lambda: torch.neg(x, out=y), reps)
    gbps = 2 * x.numel() * 8 / (ms * 1e-3) / 1e9
    del x, y
    return gbps


def shapes(dtype, T_req, E_req, smoother=False):
    """Mirror of the library's default launch shapes (T0, E0, Tup, E1 of level
    1, Eup of the levels above, flat finest level)."""
    T0 = T_req or 64
    E0 = E_req or (2 if smoother else 4)
    return T0, E0, min(T0, 64), 2 if smoother else 4, 2, not smoother


class Runner:
    """Device-resident buffers and a captured step for one batch."""

    def __init__(self, w, dtype, dev, stream, T=0, E=0, graph=True, linearization="cubature"):
        self.tdt = torch.float64 if dtype == "f64" else torch.float32
        self.w = w
        self.b = pss.Batch.ct(w.y_off, w.model, dtype=self.tdt, device=dev, scan_threads=T,
                              scan_elems=E, linearization=linearization)
        self.yd = pss.to_soa(w.y, self.tdt, dev)
        self.m0, self.N0 = self.b.prior_nominal()
        self.m, self.N = self.m0.clone(), self.N0.clone()
        self.ws_ipls, _ = self.b.workspace("ipls")
        self.ws_grad, _ = self.b.workspace("loglik_grad")
        self.stream = stream
        self.graph = None
        self.want_graph = graph

    def step(self):
        self.m.copy_(self.m0)
        self.N.copy_(self.N0)
        pss.ipls_iterate(self.b, self.yd, self.w.M, self.m, self.N, ws=self.ws_ipls)
        # the gradient pass also returns the log-likelihood
        return pss.loglik_grad(self.b, self.m, self.N, self.yd, ws=self.ws_grad)

    def prepare(self, warmup):
        for _ in range(max(1, warmup)):
            out = self.step()
        torch.cuda.synchronize()
        if self.want_graph:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph, stream=self.stream):
                out = self.step()
            for _ in range(2):  # replays agree with an eager run, bitwise
                self.graph.replay()
                torch.cuda.synchronize()
                g_ll = out[0].clone()
                e_ll = self.step()[0]
                torch.cuda.synchronize()
                # bitwise (NaN-safe) comparison
                assert torch.equal(g_ll.view(torch.int64), e_ll.view(torch.int64)), \
                    "graph replay differs from eager run"
        return out

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self.step()

    def time_steps(self, steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(self.stream)
        for _ in range(steps):
            self.run()
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, 1e3 * (time.perf_counter() - t0) / steps


def timed(stream, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batched(stream, dev, M, B=512, seed=3, graph=True):
    """Ragged batch: B sequences, lengths uniform in [100, 20000], half linear
    constant-velocity, half coordinated-turn, FP32; each IPLS pass is one
    persistent launch over both groups (autotuned shape, graph-captured)."""
    log("simulating ragged batch of %d sequences" % B)
    groups_w, lengths, kinds = wl.ragged_mixed(B, 100, 20000, seed, M=M)
    tdt = torch.float32
    cvm = wl.CVModel()
    G = dict(F=cvm.F(), c=np.zeros(4), SL=np.linalg.cholesky(cvm.Q()), H=cvm.H(), d=np.zeros(2),
             SO=np.linalg.cholesky(cvm.R()))
    wcv, _ = groups_w["cv"]
    wct, _ = groups_w["ct"]
    b_cv = pss.Batch(pss.MODEL_LINEAR, tdt, 4, 2, wcv.y_off, cvm.m0, np.eye(4), device=dev)
    b_ct = pss.Batch.ct(wct.y_off, wct.model, dtype=tdt, device=dev)
    g_cv = b_cv.gamma_from_numpy(G)
    y_cv = pss.to_soa(wcv.y, tdt, dev)
    y_ct = pss.to_soa(wct.y, tdt, dev)
    m_cv0, N_cv0 = b_cv.prior_nominal()
    m_ct0, N_ct0 = b_ct.prior_nominal()
    m_cv, N_cv, m_ct, N_ct = m_cv0.clone(), N_cv0.clone(), m_ct0.clone(), N_ct0.clone()
    groups = [(b_cv, y_cv, m_cv, N_cv, g_cv), (b_ct, y_ct, m_ct, N_ct, None)]
    steps = int(lengths.sum())
    best = pss.autotune(groups)
    log("batched: autotuned shape T=%d E_f=%d E_s=%d" % best)
    ws = torch.empty(pss.batched_workspace_size(groups), dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)

    def step():
        m_cv.copy_(m_cv0)
        N_cv.copy_(N_cv0)
        m_ct.copy_(m_ct0)
        N_ct.copy_(N_ct0)
        pss.ipls_batched(groups, M, ws=ws, status=status)

    step()
    torch.cuda.synchronize()
    if graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            step()
        g.replay()
        torch.cuda.synchronize()
        t_batched = timed(stream, g.replay, 3)
    else:  # eager launches (counter collection)
        t_batched = timed(stream, step, 3)
    ok = int(status.item()) == 0
    nan = int(torch.isnan(m_ct).any().item() or torch.isnan(m_cv).any().item())
    log("batched: %.3f ms for %d step-passes (status %s)" % (t_batched, steps * M, ok))
    # HBM: the fused minimum of a pass (every nominal and measurement read
    # once, every nominal written once) and, from the committed rocprofv3
    # summary of this batch, the persistent kernel's counter bytes per launch
    esz = 4
    n_ct, n_cv = len(wct.y), len(wcv.y)
    nseq_ct, nseq_cv = len(wct.y_off) - 1, len(wcv.y_off) - 1
    min_bytes = esz * (2 * NUM["marg"] * (n_ct + nseq_ct) + NUM["y"] * n_ct +
                       2 * 14 * (n_cv + nseq_cv) + NUM["y"] * n_cv)
    min_gbps = min_bytes * M / (t_batched * 1e-3) / 1e9
    ctr = counter_traffic("ipls_persistent", 0, "f32", B,
                          summary="hbm_traffic_batched_ragged512_f32.md")
    ctr_gbps = None if ctr is None else ctr * M / (t_batched * 1e-3) / 1e9
    log("batched: fused-minimum bytes per pass %.3g (%.0f GB/s), counter bytes per pass %s" %
        (min_bytes, min_gbps, ctr))
    # comparators: the multi-launch path per group, and one call per sequence
    wsi_cv, _ = b_cv.workspace("ipls")
    wsi_ct, _ = b_ct.workspace("ipls")

    def multi_launch():
        m_cv.copy_(m_cv0)
        N_cv.copy_(N_cv0)
        m_ct.copy_(m_ct0)
        N_ct.copy_(N_ct0)
        pss.ipls_iterate(b_cv, y_cv, M, m_cv, N_cv, gamma=g_cv, ws=wsi_cv)
        pss.ipls_iterate(b_ct, y_ct, M, m_ct, N_ct, ws=wsi_ct)

    t_multi = timed(stream, multi_launch, 2)
    singles = []
    for wgrp, bgrp, ygrp, gam in ((wcv, b_cv, y_cv, g_cv), (wct, b_ct, y_ct, None)):
        for s in range(len(wgrp.y_off) - 1):
            a, z = int(wgrp.y_off[s]), int(wgrp.y_off[s + 1])
            bs = pss.Batch(bgrp.model, tdt, bgrp.nx, 2, [0, z - a], bgrp.m0.cpu().numpy(),
                           pss.unpack_lower(bgrp.N0.cpu().numpy(), bgrp.nx), device=dev,
                           dt=bgrp.dt, theta=bgrp.theta, sensors=bgrp.sensors)
            ys = ygrp[:, a:z].contiguous()
            mm, NN = bs.prior_nominal()
            wsi, _ = bs.workspace("ipls")
            singles.append((bs, ys, mm, NN, gam, wsi))

    def loop_singles():
        for bs, ys, mm, NN, gam, wsi in singles:
            pss.ipls_iterate(bs, ys, M, mm, NN, gamma=gam, ws=wsi)

    t_loop = timed(stream, loop_singles, 1)
    log("batched: multi-launch %.3f ms, %d single-sequence calls %.3f ms" % (t_multi, B, t_loop))
    return {"B": B, "total_steps": steps, "passes": M, "dtype": "f32",
            "autotuned_shape": {"threads": best[0], "filter_elems": best[1],
                                "smoother_elems": best[2]},
            "persistent_graph_ms": round(t_batched, 4),
            "fused_min_bytes_per_pass": int(min_bytes),
            "fused_min_GBps": round(min_gbps, 1),
            "counter_bytes_per_pass": ctr,
            "counter_GBps": None if ctr_gbps is None else round(ctr_gbps, 1),
            "counter_hbm_frac": None if ctr_gbps is None else round(ctr_gbps / HBM_GBPS, 4),
            "value": round(steps * M / (t_batched * 1e-3), 1),
            "unit": "smoothed time steps/s",
            "multi_launch_ms": round(t_multi, 4),
            "looped_single_sequence_ms": round(t_loop, 4),
            "speedup_vs_looped": round(t_loop / t_batched, 2),
            "status_ok": ok, "nan": nan}


def bench_divergence(stream, dev, sets=15, passes=20, lengths=(100, 1000, 4000, 8000),
                     settings=((0.05, 0.1), (5e-4, 0.1), (5e-4, 1e-3))):
    """FP32 robustness of the two forms: for each (bearing noise sigma,
    process noise q1 = q2) setting and length, `sets` CT sequences (one
    batch), `passes` IPLS passes, then the log-likelihood; the share of
    sequences whose log-likelihood is not finite, square-root vs covariance
    form (FP64 as a control).  The first setting is the tracking model used
    everywhere else; the others make the measurements far more informative
    than the dynamics, which is where the covariance form loses positive
    definiteness in FP32."""
    out = {}
    for sigma, q in settings:
        md = wl.CTModel(q1=q, q2=q, sigma=sigma)
        key = "sigma%g_q%g" % (sigma, q)
        out[key] = {}
        for n in lengths:
            rng = np.random.Generator(np.random.PCG64(100 + n))
            ys = [wl.simulate_ct(n, rng, md)[1] for _ in range(sets)]
            off = np.arange(sets + 1, dtype=np.int64) * n
            row = {}
            for dt in ("f32", "f64"):
                tdt = torch.float32 if dt == "f32" else torch.float64
                yd = pss.to_soa(np.concatenate(ys), tdt, dev)
                for form in ("sqrt", "cov"):
                    b = pss.Batch.ct(off, md, dtype=tdt, device=dev, form=form)
                    m, N = b.prior_nominal()
                    pss.ipls_iterate(b, yd, passes, m, N)
                    ll = pss.loglik(b, yd, m, N)
                    torch.cuda.synchronize()
                    bad = int((~torch.isfinite(ll)).sum().item())
                    row["%s_%s" % (form, dt)] = round(bad / sets, 4)
            out[key]["n%d" % n] = row
            log("divergence %s n=%d: FP32 non-finite share sqrt %.2f, cov %.2f" % (
                key, n, row["sqrt_f32"], row["cov_f32"]))
    return {"sets": sets, "passes": passes, "nonfinite_share": out}


def bench_ricker(stream, dev, lengths=(10 ** 2, 10 ** 3, 10 ** 4, 10 ** 5), M=100, seed=8):
    """The Ricker-Poisson experiment of Section 6.1 on one sequence per
    length: M = 100 passes of the iterated extended (Taylor) and cubature
    smoothers, covariance and square-root forms, FP64, parallel (eager and
    graph-captured); the sequential comparator of the same form (the
    standard Kalman filter / RTS smoother for the covariance form, as in the
    paper's comparison) timed over 2 passes (per pass)."""
    out = {}
    for n in lengths:
        rng = np.random.Generator(np.random.PCG64(seed))
        md = wl.RickerModel()
        _, y = wl.simulate_ricker(n, rng, md)
        off = np.array([0, n], dtype=np.int64)
        yd = pss.to_soa(y, torch.float64, dev)
        row = {}
        for lin in ("taylor", "cubature"):
            for form in ("cov", "sqrt"):
                b = pss.Batch.ricker(off, md, dtype=torch.float64, device=dev, linearization=lin,
                                     form=form)
                m0, N0 = b.prior_nominal()
                mm, NN = m0.clone(), N0.clone()
                wi, _ = b.workspace("ipls")

                def run():
                    mm.copy_(m0)
                    NN.copy_(N0)
                    pss.ipls_iterate(b, yd, M, mm, NN, ws=wi)

                t_par = timed(stream, run, 2)
                eager = mm.clone()
                # the same 100 passes captured in one HIP graph (replay checked
                # bitwise against the eager run)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=stream):
                    run()
                g.replay()
                torch.cuda.synchronize()
                assert torch.equal(mm.view(torch.int64), eager.view(torch.int64))
                t_graph = timed(stream, g.replay, 3)
                r = {"parallel_ms_M%d" % M: round(t_par, 3),
                     "parallel_ms_per_pass": round(t_par / M, 4),
                     "graph_ms_M%d" % M: round(t_graph, 3),
                     "graph_ms_per_pass": round(t_graph / M, 4)}
                wsq, _ = b.workspace("sequential")
                t_seq = timed(stream, lambda: (mm.copy_(m0), NN.copy_(N0),
                                               pss.sequential_smoother(b, yd, 2, mm, NN,
                                                                       ws=wsq)), 1) / 2
                r["sequential_ms_per_pass"] = round(t_seq, 4)
                r["speedup_per_pass"] = round(t_seq / (t_par / M), 2)
                row["%s_%s" % (lin, form)] = r
                log("ricker n=%d %s %s: %d passes %.3f ms (graph %.3f ms), sequential %.3f "
                    "ms/pass" % (n, lin, form, M, t_par, t_graph, t_seq))
        out["n%d" % n] = row
    return {"model": "ricker_poisson a=44.7 b=10 c=7 Q=0.09", "passes": M, "dtype": "f64",
            "timings": out}


def bench_fixed_point(stream, dev, n=1000, seed=1, passes=40, ift_iter=30):
    """Gradient at the IPLS fixed point (Algorithm 4) on one CT sequence
    whose IPLS converges: time per call against the frozen-nominal
    gradient, their difference, the tangent iteration's last change, and
    L-BFGS from theta* + 0.5 with either gradient (IPLS re-run to
    convergence at every evaluation); the true gradient at each end point
    is the fixed-point one."""
    w = wl.ct_single(n, seed=seed)
    b = pss.Batch.ct(w.y_off, w.model, dtype=torch.float64, device=dev)
    yd = pss.to_soa(w.y, torch.float64, dev)
    m, N = pss.ipls_iterate(b, yd, passes)
    wi, _ = b.workspace("loglik_grad_ift")
    wg, _ = b.workspace("loglik_grad")
    t_ift = timed(stream, lambda: pss.loglik_grad_ift(b, m, N, yd, n_iter=ift_iter, ws=wi), 2)
    t_fro = timed(stream, lambda: pss.loglik_grad(b, m, N, yd, ws=wg), 10)
    _, g_ift, delta = pss.loglik_grad_ift(b, m, N, yd, n_iter=ift_iter, ws=wi, with_delta=True)
    _, g_fro, _ = pss.loglik_grad(b, m, N, yd, ws=wg)
    torch.cuda.synchronize()
    b32 = pss.Batch.ct(w.y_off, w.model, dtype=torch.float32, device=dev)
    y32 = pss.to_soa(w.y, torch.float32, dev)
    m32, N32 = pss.ipls_iterate(b32, y32, passes)
    wi32, _ = b32.workspace("loglik_grad_ift")
    t_ift32 = timed(stream, lambda: pss.loglik_grad_ift(b32, m32, N32, y32, n_iter=ift_iter,
                                                        ws=wi32), 2)
    out = {"n": n, "ift_iter": ift_iter, "ms_fixed_point_gradient": round(t_ift, 3),
           "ms_fixed_point_gradient_f32": round(t_ift32, 3),
           "ms_frozen_gradient": round(t_fro, 4),
           "gradient_fixed_point": [round(v, 6) for v in g_ift[:, 0].tolist()],
           "gradient_frozen": [round(v, 6) for v in g_fro[:, 0].tolist()],
           "tangent_change_last_iteration": float(delta[0])}
    log("fixed-point gradient n=%d: %.2f ms (%d iterations), frozen %.3f ms; g %s vs frozen %s" % (
        n, t_ift, ift_iter, t_fro, out["gradient_fixed_point"], out["gradient_frozen"]))
    th_star = [float(v) for v in w.model.theta]
    fits = {}
    for grad in ("fixed_point", "frozen"):
        t0 = time.perf_counter()
        fit = estimate.fit_theta_lbfgs(b, yd, [v + 0.5 for v in th_star], n_steps=40,
                                       passes=passes, gradient=grad, ift_iter=ift_iter)
        dt = time.perf_counter() - t0
        b2 = pss._with_theta(b, fit["theta"])
        m2, N2 = pss.ipls_iterate(b2, yd, passes)
        _, gt = pss.loglik_grad_ift(b2, m2, N2, yd, n_iter=ift_iter, ws=wi)
        torch.cuda.synchronize()
        fits[grad] = {"iterations": fit["iterations"], "evaluations": fit["evaluations"],
                      "theta_final": [round(v, 5) for v in fit["theta"]],
                      "loss_final": fit["loss_final"],
                      "true_gradient_inf_at_end": float(gt.abs().max()) / n,
                      "total_s": round(dt, 3)}
        log("L-BFGS with the %s gradient: %d iterations, %d evaluations, theta %s, |true grad| "
            "%.2e, %.1f s" % (grad, fit["iterations"], fit["evaluations"],
                              fits[grad]["theta_final"], fits[grad]["true_gradient_inf_at_end"],
                              dt))
    out["lbfgs"] = fits
    out["theta_true"] = [round(v, 5) for v in th_star]
    return out


def bench_ct_rules(stream, dev, full, n=10 ** 5):
    """Per-pass time of the CT smoother (square-root form) with each
    linearisation on a 10^5-step prefix of the main sequence."""
    out = {}
    wsub_y = full.y[:n]
    off = np.array([0, n], dtype=np.int64)
    for dt in ("f64", "f32"):
        tdt = torch.float64 if dt == "f64" else torch.float32
        yd = pss.to_soa(wsub_y, tdt, dev)
        for lin, kw in (("cubature", {}), ("taylor", {}), ("unscented", {}),
                        ("gauss_hermite", {"gh_order": 3})):
            b = pss.Batch.ct(off, full.model, dtype=tdt, device=dev, linearization=lin, **kw)
            m0, N0 = b.prior_nominal()
            mm, NN = m0.clone(), N0.clone()
            wi, _ = b.workspace("ipls")
            t = timed(stream, lambda: (mm.copy_(m0), NN.copy_(N0),
                                       pss.ipls_iterate(b, yd, 1, mm, NN, ws=wi)), 5)
            key = lin if lin != "gauss_hermite" else "gauss_hermite3"
            out["%s_%s" % (key, dt)] = round(t, 4)
            log("CT n=%d %s %s: %.3f ms/pass" % (n, key, dt, t))
    return {"n": n, "ms_per_pass": out}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    n, M = args.n, args.passes
    if args.batched_only:
        with torch.cuda.stream(stream):
            log("copy probe: %.1f GB/s" % copy_probe(stream, dev))
            print(json.dumps(bench_batched(stream, dev, M, graph=not args.no_graph)), flush=True)
        return
    log("simulating CT n=%d" % n)
    full = wl.ct_long(n, 2, M=M)
    extras = {}
    with torch.cuda.stream(stream):
        copy_gbps = copy_probe(stream, dev)
        log("copy probe: %.1f GB/s" % copy_gbps)
        log("main: CT n=%d passes=%d %s" % (n, M, args.dtype))
        R = Runner(full, args.dtype, dev, stream, args.scan_threads, args.scan_elems,
                   graph=not args.no_graph)
        out = R.prepare(args.warmup)
        nan = int(torch.isnan(out[0]).sum().item())
        ms_step, wall_step = R.time_steps(args.steps)
        log("main: %.3f ms/step (wall %.3f)" % (ms_step, wall_step))
        # stage timings on the final nominal
        b, yd, m, N = R.b, R.yd, R.m, R.N
        gam = pss.slr_linearize(b, m, N, yd)
        fel = pss.sqrt_filter_elements(b, gam, yd)
        mf, Nf = b.new_marg()
        ws_f, nf = b.workspace("filter_scan")
        ws_s, ns = b.workspace("smoother_scan")
        ms_, Ns_ = b.new_marg()
        prob = b.struct()
        L = pss.lib()

        def fscan():
            rc = L.pss_sqrt_filter_scan(ctypes.byref(prob), pss._felem_c(fel), pss._ptr(mf),
                                        pss._ptr(Nf), pss._ptr(ws_f), nf, pss._stream())
            assert rc == 0, pss.last_error()

        def sscan():
            rc = L.pss_sqrt_smoother_scan(ctypes.byref(prob), pss._gamma_c(gam), pss._ptr(mf),
                                          pss._ptr(Nf), pss._ptr(ms_), pss._ptr(Ns_),
                                          pss._ptr(ws_s), ns, pss._stream())
            assert rc == 0, pss.last_error()

        reps = 5 if n >= 10 ** 5 else 20
        # per-kernel durations inside the step itself (eager, same launches as
        # the captured graph), HIP events on the launch stream
        pss.kernel_timing(True)
        for _ in range(2):
            R.step()
        torch.cuda.synchronize()
        ktimes = pss.kernel_times()
        pss.kernel_timing(False)
        stage = {
            "slr": timed(stream, lambda: pss.slr_linearize(b, m, N, yd, out=gam), reps),
            "filter_elements": timed(stream, lambda: pss.sqrt_filter_elements(b, gam, yd, out=fel),
                                     reps),
            "filter_scan": timed(stream, fscan, reps),
            "smoother_scan": timed(stream, sscan, reps),
            "loglik_grad": timed(stream, lambda: pss.loglik_grad(b, m, N, yd, ws=R.ws_grad), reps),
        }
        log("stages (ms): " + ", ".join("%s %.3f" % kv for kv in stage.items()))
        fshape = shapes(args.dtype, args.scan_threads, args.scan_elems)
        sshape = shapes(args.dtype, args.scan_threads, args.scan_elems, True)
        ashape = (fshape[0], 2, min(fshape[0], 64), 2, 2, False)  # adjoint scan
        T0, E0 = fshape[0], fshape[1]
        esz = 8 if args.dtype == "f64" else 4
        kflops = scan_kernel_flops("filter", [n], *fshape)
        kflops.update(scan_kernel_flops("smoother", [n + 1], *sshape))
        kflops.update(scan_kernel_flops("adjoint", [n], *ashape))
        kbytes = scan_kernel_bytes("filter", [n], *fshape, esz)
        kbytes.update(scan_kernel_bytes("smoother", [n + 1], *sshape, esz))
        kbytes.update(scan_kernel_bytes("adjoint", [n], *ashape, esz))
        E0s = sshape[1]
        kflops[("slr", 0)] = n * (FLOPS["slr_transition"] + FLOPS["slr_bearings"])
        kflops[("filter_elements", 0)] = n * FLOPS["filter_element"]
        kflops[("slr_felem", 0)] = n * (FLOPS["slr_transition"] + FLOPS["slr_bearings"] +
                                         FLOPS["filter_element"])
        gam = NUM["gam_trans"] + NUM["gam_obs"]
        kbytes[("slr", 0)] = ((n + 1) * NUM["marg"] + n * (NUM["y"] + gam)) * esz
        kbytes[("filter_elements", 0)] = n * (gam + NUM["y"] + NUM["felem"]) * esz
        kbytes[("slr_felem", 0)] = ((n + 1) * NUM["marg"] +
                                    n * (NUM["y"] + NUM["gam_trans"] + NUM["felem"])) * esz
        kbytes[("loglik_terms", 0)] = n * (NUM["marg"] + gam + NUM["y"]) * esz + n * 8
        kernels = {}
        for key, (calls, tot) in sorted(ktimes.items()):
            avg = tot / calls
            fl_k, by_k = kflops.get(key), kbytes.get(key)
            kernels["%s_L%d" % key] = {
                "launches": calls, "avg_ms": round(avg, 5),
                "flops_per_launch": fl_k, "alg_bytes_per_launch": by_k,
                "tflops": None if fl_k is None else round(fl_k / (avg * 1e-3) / 1e12, 4),
                "alg_GBps": None if by_k is None else round(by_k / (avg * 1e-3) / 1e9, 1)}
        dom = max((k for k in ktimes if k in kflops and k in kbytes),
                  key=lambda k: ktimes[k][1])
        dom_ms = ktimes[dom][1] / ktimes[dom][0]
        fl, by = kflops[dom], kbytes[dom]
        t_dom = dom_ms * 1e-3
        alu_frac = fl / t_dom / 1e12 / PEAK[args.dtype]
        hbm_frac = by / t_dom / 1e9 / HBM_GBPS
        # the bound is the larger of the two lower bounds on the launch time
        bound = "hbm" if by / (HBM_GBPS * 1e9) >= fl / (PEAK[args.dtype] * 1e12) else "alu"
        traffic = counter_traffic(dom[0], dom[1], args.dtype, n)
        log("dominant kernel %s level %d: %.4f ms, %.3f TFLOP/s (ALU %.3f), %.0f GB/s "
            "algorithmic (HBM %.3f) -> %s bound" % (dom[0], dom[1], dom_ms, fl / t_dom / 1e12,
                                                   alu_frac, by / t_dom / 1e9, hbm_frac, bound))
        # one IPLS pass as a whole: its kernels once each
        pass_keys = [k for k in ktimes if k[0] in ("slr", "filter_elements", "slr_felem") or
                     k[0].startswith(("filter_up", "filter_down", "filter_top", "smoother_up",
                                      "smoother_down", "smoother_top"))]
        pass_ms = sum(ktimes[k][1] / ktimes[k][0] for k in pass_keys)
        pass_fl = sum(kflops.get(k, 0) for k in pass_keys)
        pass_by = sum(kbytes.get(k, 0) for k in pass_keys)
        pass_tr = [counter_traffic(k[0], k[1], args.dtype, n) for k in pass_keys]
        pass_tr = None if any(v is None for v in pass_tr) else sum(pass_tr)
        fused_min = n * 102 * esz  # nominal + y in, nominal + filter marginals out
        pass_info = {
            "kernels": ["%s_L%d" % k for k in sorted(pass_keys)],
            "ms": round(pass_ms, 4), "steps_per_s": round(n / (pass_ms * 1e-3), 1),
            "flops": int(pass_fl), "tflops": round(pass_fl / (pass_ms * 1e-3) / 1e12, 3),
            "alu_frac": round(pass_fl / (pass_ms * 1e-3) / 1e12 / PEAK[args.dtype], 4),
            "alg_bytes": int(pass_by), "fused_min_bytes": fused_min,
            "counter_bytes": pass_tr,
            "counter_hbm_frac": None if pass_tr is None else round(
                pass_tr / (pass_ms * 1e-3) / 1e9 / HBM_GBPS, 4),
            "counter_over_fused_min": None if pass_tr is None else round(pass_tr / fused_min, 2)}
        log("pass: %.3f ms, %.2f TFLOP/s, counter bytes %s" % (pass_ms, pass_info["tflops"],
                                                               pass_tr))
        del R, gam, fel, mf, Nf, ms_, Ns_, ws_f, ws_s
        torch.cuda.empty_cache()

        if not args.no_extras:
            # FP32 of the same step
            other = "f32" if args.dtype == "f64" else "f64"
            R2 = Runner(full, other, dev, stream, graph=not args.no_graph)
            out2 = R2.prepare(1)
            ms2, _ = R2.time_steps(max(2, args.steps // 2))
            extras[other] = {"ms_per_step": round(ms2, 4),
                             "value": round(n * M / (ms2 * 1e-3), 1),
                             "nan_loglik": int(torch.isnan(out2[0]).sum().item())}
            log("%s: %.3f ms/step" % (other, ms2))
            del R2
            torch.cuda.empty_cache()
            # the iterated extended smoother (first-order Taylor linearisation,
            # Section 4.2) on the same step, both precisions
            ieks = {}
            for dt in ("f64", "f32"):
                R3 = Runner(full, dt, dev, stream, graph=not args.no_graph,
                            linearization="taylor")
                out3 = R3.prepare(1)
                ms3, _ = R3.time_steps(max(2, args.steps // 2))
                ieks[dt] = {"ms_per_step": round(ms3, 4), "value": round(n * M / (ms3 * 1e-3), 1),
                            "nan_loglik": int(torch.isnan(out3[0]).sum().item())}
                log("IEKS %s: %.3f ms/step" % (dt, ms3))
                del R3
                torch.cuda.empty_cache()
            extras["ieks_taylor"] = ieks
            # parallel vs sequential square-root kernel, per IPLS pass
            seq = {}
            for nn in (10 ** 4, 10 ** 5):
                if nn > n:
                    continue
                wsub = wl.Workload("prefix", full.model, full.y[:nn], np.array([0, nn]),
                                   np.ones(1, np.int64), [], M=M)
                for dt in ("f64", "f32"):
                    tdt = torch.float64 if dt == "f64" else torch.float32
                    bb = pss.Batch.ct(wsub.y_off, full.model, dtype=tdt, device=dev)
                    yy = pss.to_soa(wsub.y, tdt, dev)
                    m0, N0 = bb.prior_nominal()
                    mm, NN = m0.clone(), N0.clone()
                    wi, _ = bb.workspace("ipls")
                    wsq, _ = bb.workspace("sequential")
                    t_par = timed(stream, lambda: (mm.copy_(m0), NN.copy_(N0),
                                                   pss.ipls_iterate(bb, yy, 1, mm, NN, ws=wi)), 5)
                    t_seq = timed(stream, lambda: (mm.copy_(m0), NN.copy_(N0),
                                                   pss.sequential_smoother(bb, yy, 1, mm, NN,
                                                                           ws=wsq)),
                                  1 if nn >= 10 ** 5 else 3)
                    ab = pass_alg_bytes(nn, dt)
                    seq["n%d_%s" % (nn, dt)] = {"parallel_ms_per_pass": round(t_par, 4),
                                                "sequential_ms_per_pass": round(t_seq, 4),
                                                "speedup": round(t_seq / t_par, 2),
                                                "parallel_alg_GBps": round(ab / (t_par * 1e-3) / 1e9,
                                                                           1)}
                    log("n=%d %s: parallel %.3f ms/pass (%.0f GB/s algorithmic), sequential "
                        "%.3f ms/pass" % (nn, dt, t_par, ab / (t_par * 1e-3) / 1e9, t_seq))
            # the long sequence itself: one sequential FP64 pass (about 10 s),
            # against the parallel pass measured in the main line
            if n >= 10 ** 6:
                bb = pss.Batch.ct(full.y_off, full.model, dtype=torch.float64, device=dev)
                yy = pss.to_soa(full.y, torch.float64, dev)
                mm, NN = bb.prior_nominal()
                wsq, _ = bb.workspace("sequential")
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                pss.sequential_smoother(bb, yy, 1, mm, NN, ws=wsq)
                e1.record(stream)
                torch.cuda.synchronize()
                t_seq = e0.elapsed_time(e1)
                t_par = pass_info["ms"]
                seq["n%d_f64" % n] = {"parallel_ms_per_pass": round(t_par, 4),
                                      "sequential_ms_per_pass": round(t_seq, 4),
                                      "speedup": round(t_seq / t_par, 2),
                                      "parallel_alg_GBps": round(pass_info["alg_bytes"] /
                                                                 (t_par * 1e-3) / 1e9, 1)}
                log("n=%d f64: parallel %.3f ms/pass (the main line's kernels), sequential "
                    "%.3f ms/pass" % (n, t_par, t_seq))
                del bb, yy, mm, NN, wsq
                torch.cuda.empty_cache()
            extras["sequential"] = seq
            # parameter-estimation configuration: loglik + gradient, 64 x 10^4
            log("simulating CT 64 x 10^4")
            wb = wl.ct_batch(64, 10 ** 4, 4, M=M)
            lg = {}
            for dt in ("f64", "f32"):
                tdt = torch.float64 if dt == "f64" else torch.float32
                bb = pss.Batch.ct(wb.y_off, wb.model, dtype=tdt, device=dev)
                yy = pss.to_soa(wb.y, tdt, dev)
                mm, NN = pss.ipls_iterate(bb, yy, M)
                wg, _ = bb.workspace("loglik_grad")
                t_g = timed(stream, lambda: pss.loglik_grad(bb, mm, NN, yy, ws=wg), 10)
                wf, _ = bb.workspace("score_fisher")
                t_f = timed(stream, lambda: pss.score_fisher(bb, mm, NN, yy, ws=wf), 10)
                wl_, _ = bb.workspace("loglik")
                t_l = timed(stream, lambda: pss.loglik(bb, yy, mm, NN, ws=wl_), 10)
                # checkpoint depth: bytes kept between the forward and the
                # backward call, and the backward's time from it
                ck = {}
                for level in (0, 1, 2, 9):
                    cp = pss.Checkpoint(bb, level)
                    t_fw = timed(stream, lambda: pss.loglik(bb, yy, mm, NN, ws=wl_, ckpt=cp), 5)
                    t_bw = timed(stream, lambda: pss.loglik_grad(bb, mm, NN, yy, ws=wg, ckpt=cp),
                                 5)
                    ck["level%d" % level] = {"bytes": cp.bytes, "forward_ms": round(t_fw, 4),
                                             "backward_ms": round(t_bw, 4)}
                    del cp
                wi, _ = bb.workspace("ipls")
                m0, N0 = bb.prior_nominal()
                t_i = timed(stream, lambda: (mm.copy_(m0), NN.copy_(N0),
                                             pss.ipls_iterate(bb, yy, M, mm, NN, ws=wi)), 3)
                # how far IPLS is from a fixed point after the M passes every
                # objective evaluation runs: the change one more pass makes,
                # per sequence (max over its states and components)
                m_prev = mm.clone()
                pss.ipls_iterate(bb, yy, 1, mm, NN, ws=wi)
                dmax = (mm - m_prev).abs().amax(dim=0).double().cpu().numpy()
                off = np.asarray(wb.y_off)
                dseq = np.array([dmax[off[i] + i:off[i + 1] + i + 1].max()
                                 for i in range(len(off) - 1)])
                lg[dt] = {"loglik_plus_grad_ms": round(t_g, 4), "loglik_ms": round(t_l, 4),
                          "fisher_route_ms": round(t_f, 4), "ipls_ms": round(t_i, 4),
                          "checkpoints": ck, "workspace_bytes_grad": pss.workspace_size(
                              bb, "loglik_grad"),
                          "ipls_next_pass_change": {
                              "max": float(dseq.max()),
                              "sequences_above_1e-6": int((dseq > 1e-6).sum()),
                              "sequences": int(len(dseq))}}
                log("64x1e4 %s: one more IPLS pass after %d moves the means by up to %.3g; "
                    "%d of %d sequences by more than 1e-6" % (dt, M, dseq.max(),
                                                             int((dseq > 1e-6).sum()), len(dseq)))
                log("64x1e4 %s: loglik+grad %.3f ms (loglik %.3f, Fisher route %.3f), IPLS %.3f "
                    "ms, checkpoints %s" % (dt, t_g, t_l, t_f, t_i, ck))
                # 50 L-BFGS steps from theta* + 0.5 (IPLS re-run at every
                # evaluation, frozen-nominal gradient)
                th_star = [float(v) for v in wb.model.theta]
                t0 = time.perf_counter()
                fit = estimate.fit_theta_lbfgs(bb, yy, [v + 0.5 for v in th_star], n_steps=50,
                                               passes=M)
                t_fit = time.perf_counter() - t0
                lg[dt]["lbfgs"] = {
                    "iterations": fit["iterations"], "evaluations": fit["evaluations"],
                    "theta_true": [round(v, 5) for v in th_star],
                    "theta_start": [round(v + 0.5, 5) for v in th_star],
                    "theta_final": [round(v, 5) for v in fit["theta"]],
                    "loss_start": fit["loss_start"], "loss_final": fit["loss_final"],
                    "ms_per_loglik_grad_evaluation": round(fit["ms_per_evaluation"], 3),
                    "ms_ipls_per_evaluation": round(fit["ms_ipls_per_evaluation"], 3),
                    "total_s": round(t_fit, 3)}
                log("64x1e4 %s: L-BFGS %d steps, %d evaluations, theta %s -> %s (true %s), "
                    "%.2f s" % (dt, fit["iterations"], fit["evaluations"],
                                [round(v + 0.5, 3) for v in th_star],
                                [round(v, 3) for v in fit["theta"]],
                                [round(v, 3) for v in th_star], t_fit))
            extras["param_estimation_64x1e4"] = lg

        if not args.no_extras:
            extras["batched_ragged_512"] = bench_batched(stream, dev, M)
            extras["fp32_divergence"] = bench_divergence(stream, dev)
            extras["ricker_poisson"] = bench_ricker(stream, dev)
            extras["ct_linearisations_1e5"] = bench_ct_rules(stream, dev, full)
            if args.dtype == "f64":
                extras["fixed_point_gradient"] = bench_fixed_point(stream, dev)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        try:  # a copy tuned for this host's CPU; the portable build otherwise
            oracle.build(force=True, native=True)
        except Exception as ex:  # noqa: BLE001
            log("native oracle build failed (%s); portable build" % ex)
            oracle.build(force=False)
        prm = oracle.ct_params()
        ns = min(n, 100000)
        log("cpu baseline: oracle on the first %d steps" % ns)
        t0 = time.perf_counter()
        reps = 0
        while True:
            r = oracle.ct_ipls(prm, full.model.m0, np.eye(5), full.y[:ns], M)
            oracle.ct_loglik(prm, full.model.m0, np.eye(5), full.y[:ns], r["ms"], r["Ns"])
            oracle.ct_score(prm, full.model.m0, np.eye(5), full.y[:ns], r["ms"], r["Ns"])
            reps += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        dt_cpu = (time.perf_counter() - t0) / reps
        cpu = {"value": round(ns * M / dt_cpu, 1), "unit": "smoothed time steps/s", "cores": 1,
               "kind": "oracle",
               "sample": "first %d steps of the same sequence, %d repeat(s) of the whole step "
                         "(IPLS %d passes + loglik + score), FP64, sequential in k, one core"
                         % (ns, reps, M),
               "build": oracle.build_flags(), **oracle.host_info()}

    peak = PEAK[args.dtype]
    line = {
        "metric": "smoothed time steps/s (sqrt filter+smoother scan) nx=5; loglik+grad ms",
        "value": round(n * M / (ms_step * 1e-3), 1),
        "unit": "smoothed time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded CT bearings-only simulation)",
        "config": {"workload": "ct_bearings_long_n%d_M%d_cubature" % (n, M), "B": 1, "n": n,
                   "passes": M, "nx": 5, "ny": 2, "graph": not args.no_graph,
                   "scan_threads": T0, "filter_elems": E0, "smoother_elems": E0s},
        "loglik_grad_ms": extras.get("param_estimation_64x1e4", {}).get(args.dtype, {}).get(
            "loglik_plus_grad_ms"),
        "nan_loglik": nan,
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "roofline": {"bound": bound, "kernel": "%s level %d" % dom,
                     "achieved": round(by / t_dom / 1e9, 1) if bound == "hbm"
                     else round(fl / t_dom / 1e12, 4),
                     "peak": HBM_GBPS if bound == "hbm" else peak,
                     "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
                     "frac": round(max(hbm_frac, alu_frac), 6), "traffic": traffic,
                     "hbm_frac": round(hbm_frac, 6), "alu_frac": round(alu_frac, 6),
                     "counter_hbm_frac": None if traffic is None else round(
                         traffic / t_dom / 1e9 / HBM_GBPS, 6),
                     "alg_bytes_per_launch": int(by), "flops_per_launch": int(fl),
                     "avg_launch_ms": round(dom_ms, 5)},
        "pass": pass_info,
        "kernels": kernels,
        "copy_probe_GBps": round(copy_gbps, 1),
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
