"""Benchmark: implicit filament steps on one MI355X.

Workload: the sedimenting suspension of 100 filaments x 20 segments (2,000
segments), every segment under gravity, steric barrier on, RPY hydrodynamics,
BDF2 steps solved by bad Broyden with the explicit block-diagonal J0 to a
1e-6 residual.  One "step" is one full implicit time step (warm start, J0 and
its inverse, every Broyden iteration with its mobility apply, finalisation).

Prints one JSON line: value = RPY pair-interactions per second of whole-step
wall time (mobility applies x S^2 / elapsed), ms_per_step, the roofline of the
mobility pair kernel (its duration measured with HIP events on the stream it
runs on, inside the timed steps) and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 85          # algorithmic flops of one ordered (target, source) RPY pair
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector peak
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector peak (packed)
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rpy_sweep(sizes=(2000, 16000, 32000), reps=10):
    """Stand-alone mobility applies (pairs/s) at the paper-workload sizes."""
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth
    out = []
    for S in sizes:
        Y, F, T = synth.rpy_throughput_inputs(S, seed=7)
        d = lambda a: torch.from_numpy(a.T.copy()).cuda()
        Yd, Fd, Td = d(Y), d(F), d(T)
        for prec in ("f64", "f32tile"):
            V, W = torch.empty_like(Yd), torch.empty_like(Yd)
            work = torch.empty(fil.rpy_workspace_bytes(S, prec), dtype=torch.uint8, device="cuda")
            for _ in range(3):
                fil.rpy_mobility_apply(Yd, Fd, Td, 1.0, 1.0, prec, V, W, work)
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(st)
            for _ in range(reps):
                fil.rpy_mobility_apply(Yd, Fd, Td, 1.0, 1.0, prec, V, W, work)
            e1.record(st)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / reps
            pairs = float(S) * S
            peak = PEAK_FP64_TFLOPS if prec == "f64" else PEAK_FP32_TFLOPS
            out.append(dict(S=S, prec=prec, ms=round(t * 1e3, 4), pairs_per_s=pairs / t,
                            tflops=FLOP_PER_PAIR * pairs / t / 1e12,
                            frac_of_peak=FLOP_PER_PAIR * pairs / t / 1e12 / peak))
            log("rpy apply", out[-1])
    return out


def cpu_baseline(w, steps=2):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload."""
    import oracle
    nthreads = len(os.sched_getaffinity(0))
    sim = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=nthreads, **w.params)
    applies = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, rep = sim.step()
        applies += rep.applies
    dt = time.perf_counter() - t0
    return dict(value=applies * float(w.S) ** 2 / dt, unit="pairs/s", cores=nthreads, kind="oracle",
                sample="%d implicit steps (%d mobility applies) of the %d-segment suspension, %.1f s" %
                       (steps, applies, w.S, dt), ms_per_step=dt / steps * 1e3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32tile"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth

    w = synth.sediment_suspension(M=100, N=20, side=200.0, seed=1002, dt_over_T=1 / 30)
    S = w.S
    sim = fil.Sim(w.fil_off, w.Y, w.q, w.params, prec=args.prec)
    for _ in range(args.warmup):
        sim.step()
    torch.cuda.synchronize()
    sim.set_timing(True)
    applies, iters = 0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = sim.step()[0]
        applies += r["applies"]
        iters += r["iters"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rpy_ms, nl = sim.timing()[args.prec]
    pairs = applies * float(S) ** 2
    kern_s = rpy_ms * 1e-3 / max(nl, 1)
    peak = PEAK_FP64_TFLOPS if args.prec == "f64" else PEAK_FP32_TFLOPS
    achieved = FLOP_PER_PAIR * float(S) ** 2 / kern_s / 1e12
    res = {
        "metric": "RPY pair-interactions/s (fp64 vs fp32) + ms/step to tol, plain vs learned",
        "value": pairs / el,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "f64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "sedimenting suspension, 100 filaments x 20 segments (S=2000), B=1e3, "
                               "dt=T/30, tol 1e-6, steric on, unbounded RPY", "segments": S,
                   "precision": args.prec},
        "iters_per_step": iters / args.steps,
        "mobility_applies_per_step": applies / args.steps,
        "roofline": {"bound": "alu", "kernel": "rpy_%s_kernel" % ("f64" if args.prec == "f64" else "f32"),
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None, "avg_kernel_us": kern_s * 1e6, "launches": nl,
                     "flop_per_launch": FLOP_PER_PAIR * float(S) ** 2},
    }
    if not args.no_sweep:
        res["rpy_apply"] = rpy_sweep()
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
