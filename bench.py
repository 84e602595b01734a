"""Benchmark of the parallel square-root iterated smoother on one MI355X.

Workload (default): coordinated-turn bearings-only tracking, one sequence of
n = 1000 steps, 10 cubature IPLS passes (SLR, filter elements, filter scan,
smoother scan), then the pseudo-log-likelihood and its gradient at the final
nominal, in FP64.  One "step" is that whole hot path; the step is captured
in a HIP graph and replayed.  Inputs are synthetic (seeded simulation) and
resident in HBM before timing starts.

The output is one JSON line.  value = smoothed time steps per second =
n * passes / (seconds per step).  Beside it:
  roofline     the dominant kernel (the filter-scan tile kernel) timed with
               HIP events on its own stream, against the FP64 vector peak;
               its work is the counted flops of the operators it executes;
  cpu_baseline the FP64 oracle on the host for the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2207_00426_amd import pss  # noqa: E402
from paper_2207_00426_amd import workloads as wl  # noqa: E402

# Counted floating-point operations of the nx = 5, ny = 2 operators (one add,
# multiply, divide or square root = 1, a fused multiply-add = 2), obtained by
# instantiating the register code on a counting number type.
FLOPS = dict(filter_combine=3328, filter_apply=2280, smoother_combine=730, smoother_apply=505,
             filter_element=1251, smoother_element=1502, slr_transition=937, slr_bearings=487)
PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64
PEAK_FP32_TFLOPS = 78.6   # vector FP32 without packed-FP32 instructions (kept off)
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--passes", type=int, default=10)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--scan-threads", type=int, default=0)
    ap.add_argument("--scan-elems", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def scan_tile_flops(n, T, E):
    """Counted flops of the filter-scan kernels for one sequence of n steps.

    Every element is folded once (E - 1 combines per thread plus the tree's
    T - 1 combines per tile ~ one combine per element) and applied once, and
    the down-sweep applies once per tree node.
    """
    tiles = -(-n // (T * E))
    combines = n - tiles + (tiles - 1)  # thread folds + trees, levels >= 1 included
    applies = n + n // max(E, 1)
    return combines * FLOPS["filter_combine"] + applies * FLOPS["filter_apply"]


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    n, M = args.n, args.passes
    w = wl.ct_single(n, 1, M=M)
    md = w.model
    b = pss.Batch.ct(w.y_off, md, dtype=tdt, device=dev, scan_threads=args.scan_threads,
                     scan_elems=args.scan_elems)
    yd = pss.to_soa(w.y, tdt, dev)
    m0, N0 = b.prior_nominal()
    m, N = m0.clone(), N0.clone()
    ws_ipls, _ = b.workspace("ipls")
    ws_grad, _ = b.workspace("loglik_grad")
    stream = torch.cuda.Stream()

    def step():
        m.copy_(m0)
        N.copy_(N0)
        pss.ipls_iterate(b, yd, M, m, N, ws=ws_ipls)
        return pss.loglik_grad(b, m, N, yd, ws=ws_grad)

    print("bench: CT n=%d passes=%d %s, warmup %d, steps %d" % (n, M, args.dtype, args.warmup,
                                                                 args.steps), file=sys.stderr,
          flush=True)
    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            out = step()
        torch.cuda.synchronize()
        graph = None
        if not args.no_graph:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                out = step()
            graph.replay()
            torch.cuda.synchronize()
        run = graph.replay if graph is not None else step
        # graph replays must equal eager results (checked once)
        ll_g = out[0].clone()
        if graph is not None:
            ll_e = step()[0]
            torch.cuda.synchronize()
            assert torch.equal(ll_e, ll_g), "graph replay differs from eager run"
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            run()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_step = ev0.elapsed_time(ev1) / args.steps
        print("bench: %.3f ms/step (wall %.3f ms/step)" % (ms_step, 1e3 * wall / args.steps),
              file=sys.stderr, flush=True)

        # component timings (eager, events on the same stream)
        def timed(fn, reps=10):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        mi, Ni = m0.clone(), N0.clone()
        t_ipls = timed(lambda: (mi.copy_(m0), Ni.copy_(N0),
                                pss.ipls_iterate(b, yd, M, mi, Ni, ws=ws_ipls)))
        t_grad = timed(lambda: pss.loglik_grad(b, m, N, yd, ws=ws_grad))
        gam = pss.slr_linearize(b, m, N, yd)
        fel = pss.sqrt_filter_elements(b, gam, yd)
        mf, Nf = b.new_marg()
        ws_f, nf = b.workspace("filter_scan")
        t_fscan = timed(lambda: pss.lib().pss_sqrt_filter_scan(
            pss.ctypes.byref(b.struct()), pss._felem_c(fel), pss._ptr(mf), pss._ptr(Nf),
            pss._ptr(ws_f), nf, pss._stream()), reps=20)
        t_slr = timed(lambda: pss.slr_linearize(b, m, N, yd, out=gam), reps=20)
        t_fel = timed(lambda: pss.sqrt_filter_elements(b, gam, yd, out=fel), reps=20)
        ms_s, Ns_s = b.new_marg()
        t_sscan = timed(lambda: pss.sqrt_smoother_scan(b, gam, mf, Nf, ms_s, Ns_s), reps=20)

    T0 = args.scan_threads or (128 if args.dtype == "f64" else 256)
    E0 = args.scan_elems or 4
    fl = scan_tile_flops(n, T0, E0)
    achieved = fl / (t_fscan * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if args.dtype == "f64" else PEAK_FP32_TFLOPS
    value = n * M / (ms_step * 1e-3)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        prm = oracle.ct_params()
        t0 = time.perf_counter()
        reps = 0
        while True:
            r = oracle.ct_ipls(prm, md.m0, np.eye(5), w.y, M)
            oracle.ct_score(prm, md.m0, np.eye(5), w.y, r["ms"], r["Ns"])
            reps += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        dt_cpu = (time.perf_counter() - t0) / reps
        cpu = {"value": n * M / dt_cpu, "unit": "smoothed time steps/s", "cores": 1,
               "kind": "oracle",
               "sample": "%d repeats of the whole step (IPLS %d passes + loglik + score) on "
                         "the same CT n=%d sequence, FP64, sequential in k on one core"
                         % (reps, M, n)}

    line = {
        "metric": "smoothed time steps/s (sqrt filter+smoother scan) nx=5; loglik+grad ms",
        "value": round(value, 1),
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
        "config": {"workload": "ct_bearings_n%d_M%d_cubature" % (n, M), "B": 1, "n": n,
                   "passes": M, "nx": 5, "ny": 2, "graph": graph is not None,
                   "scan_threads": T0, "scan_elems": E0},
        "loglik_grad_ms": round(t_grad, 4),
        "ipls_ms": round(t_ipls, 4),
        "stage_ms": {"slr": round(t_slr, 4), "filter_elements": round(t_fel, 4),
                     "filter_scan": round(t_fscan, 4), "smoother_scan": round(t_sscan, 4)},
        "roofline": {"bound": "alu", "kernel": "filter scan (k_plan + k_scan_* tiles)",
                     "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 6), "traffic": None,
                     "flops_per_launch": fl},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
