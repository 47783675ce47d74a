"""Benchmark: the RPY mobility apply and the implicit filament steps on one MI355X.

Headline workload: the mobility apply of the active array's size and layout, 1000
filaments x 32 segments (S = 32,000) on a 40 x 25 lattice of spacing 20a, bent as planar
arcs, F, T ~ N(0, 1), with FP32 pair tiles and FP64 per-target accumulation.  One "step"
is one apply (source packing, the pair kernel over all S^2 ordered pairs, the fixed-order
reduction of the split-K partials), inputs resident on the GPU.

Prints one JSON line: value = pair interactions per second of the FP32-tile apply
(S^2 / wall time per apply), ms_per_step = wall ms per apply, the roofline of the pair
kernel (its duration stamped by HIP events at the kernel's own start and end, on the
stream it runs on, in every timed apply), the same apply in FP64 beside it, and, unless
switched off: the implicit steps of the sedimenting suspension (100 x 20) in FP64 and
with FP32 tiles, stand-alone applies at other sizes and the ragged 256-suspension batch,
the 256-suspension ensemble's implicit steps, the force-coupling and wall mobilities,
the solver comparison, the learned warm start against plain Broyden, and the CPU
oracle's rate on a bounded sample of the headline apply (all host cores and one core)
with the GPU results' error against it.
"""
from __future__ import annotations

import argparse
import hashlib
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
GRAPH_ITERS = 32            # Broyden iterations per captured graph block (at most)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rpy_f32_active32000_traffic.json")
HEADLINE_WORKLOAD = ("RPY mobility apply, active-array layout: 1000 filaments x 32 segments (S=32000) on a 40 x 25 "
                     "lattice of spacing 20a, planar arcs (bend <= 0.05 rad per segment), F, T ~ N(0,1); FP32 pair "
                     "tiles with FP64 per-target accumulation")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _time_applies(fn, reps):
    import torch
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def apply_headline(steps, warmup):
    """K timed applies (after W untimed ones) of the active array's mobility in FP32 tiles
    and in FP64: wall time per apply between synchronisations, and the pair kernel's own
    duration from HIP events the library stamps at its start and end."""
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth
    Y, F, T = synth.active_array_mobility_inputs()
    S = Y.shape[0]
    d = lambda a: torch.from_numpy(a.T.copy()).cuda()
    Yd, Fd, Td = d(Y), d(F), d(T)
    out = {}
    for prec in ("f32tile", "f64"):
        V, W = torch.empty_like(Yd), torch.empty_like(Yd)
        work = torch.empty(fil.rpy_workspace_bytes(S, prec), dtype=torch.uint8, device="cuda")
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for _ in range(warmup):
            fil.rpy_mobility_apply(Yd, Fd, Td, 1.0, 1.0, prec, V, W, work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            fil.rpy_mobility_apply(Yd, Fd, Td, 1.0, 1.0, prec, V, W, work, events=evs[i])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kern_ms = [a.elapsed_time(b) for a, b in evs]
        out[prec] = dict(S=S, wall_s=el, ms_per_apply=el / steps * 1e3, pairs_per_s=float(S) ** 2 * steps / el,
                         kernel_avg_us=sum(kern_ms) / steps * 1e3, kernel_min_us=min(kern_ms) * 1e3,
                         V=V.cpu().numpy().T.copy(), W=W.cpu().numpy().T.copy())
        log("headline apply", prec, {k: v for k, v in out[prec].items() if k not in ("V", "W")})
    return out, (Y, F, T)


def rpy_sweep(sizes=(2000, 16000, 32000), reps=10):
    """Stand-alone mobility applies (pairs/s) at the workload sizes."""
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
            t = _time_applies(lambda: fil.rpy_mobility_apply(Yd, Fd, Td, 1.0, 1.0, prec, V, W, work), reps)
            pairs = float(S) * S
            peak = PEAK_FP64_TFLOPS if prec == "f64" else PEAK_FP32_TFLOPS
            out.append(dict(S=S, prec=prec, ms=round(t * 1e3, 4), pairs_per_s=pairs / t,
                            tflops=FLOP_PER_PAIR * pairs / t / 1e12,
                            frac_of_peak=FLOP_PER_PAIR * pairs / t / 1e12 / peak))
            log("rpy apply", out[-1])
    return out


def rpy_batched(reps=5):
    """One apply over the 256 ragged suspensions (filaments U{1..64} x N U{10..50})."""
    import numpy as np
    import torch
    import paper_1903_12609_amd as fil
    rng = np.random.default_rng(1004)
    sizes = [int(rng.integers(1, 65)) * int(rng.integers(10, 51)) for _ in range(256)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    S = int(off[-1])
    Y = np.concatenate([rng.uniform(0, 200.0 * (n / 2000.0) ** (1 / 3), (n, 3)) for n in sizes])
    F, T = rng.standard_normal((S, 3)), rng.standard_normal((S, 3))
    d = lambda a: torch.from_numpy(a.T.copy()).cuda()
    Yd, Fd, Td = d(Y), d(F), d(T)
    out = []
    pairs = float(sum(n * n for n in sizes))
    for prec in ("f64", "f32tile"):
        V, W = torch.empty_like(Yd), torch.empty_like(Yd)
        plan = fil.RpyBatch(off, prec)     # the work list is built once; applies only enqueue
        work = torch.empty(max(plan.work_bytes, 1), dtype=torch.uint8, device="cuda")
        t = _time_applies(lambda: plan.apply(Yd, Fd, Td, 1.0, 1.0, V, W, work), reps)
        plan.close()
        peak = PEAK_FP64_TFLOPS if prec == "f64" else PEAK_FP32_TFLOPS
        out.append(dict(suspensions=256, segments=S, pairs=pairs, prec=prec, ms=round(t * 1e3, 4),
                        pairs_per_s=pairs / t, tflops=FLOP_PER_PAIR * pairs / t / 1e12,
                        frac_of_peak=FLOP_PER_PAIR * pairs / t / 1e12 / peak))
        log("rpy batched apply", out[-1])
    return out


def run_steps(w, prec, steps, warmup, graph):
    """Timed implicit steps; returns (elapsed s, applies, iters, kernel timing)."""
    import torch
    import paper_1903_12609_amd as fil
    sim = fil.Sim(w.fil_off, w.Y, w.q, w.params, prec=prec, graph=graph)
    for _ in range(warmup):
        sim.step()
    torch.cuda.synchronize()
    sim.set_timing(True)
    applies, iters = 0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        r = sim.step()[0]
        applies += r["applies"]
        iters += r["iters"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = sim.timing()
    sim.close()
    return el, applies, iters, tm


def suspension_steps(steps=10, warmup=3, graph=GRAPH_ITERS):
    """Implicit steps of the 500 x 32 sedimenting suspension (S = 16000, cube of side 400a,
    dt = T/30) in FP64 and with FP32 tiles (FP64 finish): ms per step, iterations, mobility
    applies and how many of them ran in FP64."""
    from paper_1903_12609_amd import synth
    w = synth.sediment_suspension(M=500, N=32, side=400.0, seed=1005, dt_over_T=1 / 30)
    out = {"workload": "sedimenting suspension 500 x 32 (S=16000), side 400a, dt=T/30, tol 1e-6, graph blocks of %d"
                       % graph}
    for prec in ("f64", "f32tile"):
        import torch
        import paper_1903_12609_amd as fil
        sim = fil.Sim(w.fil_off, w.Y, w.q, w.params, prec=prec, graph=graph)
        for _ in range(warmup):
            sim.step()
        torch.cuda.synchronize()
        its = aps = a64 = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            r = sim.step()[0]
            its += r["iters"]
            aps += r["applies"]
            a64 += r["applies_f64"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sim.close()
        out[prec] = {"ms_per_step": el / steps * 1e3, "iters_per_step": its / steps,
                     "mobility_applies_per_step": aps / steps, "fp64_applies_per_step": a64 / steps}
        log("500x32 steps", prec, out[prec])
    out["f32tile_over_f64_speed"] = out["f64"]["ms_per_step"] / out["f32tile"]["ms_per_step"]
    return out


def ensemble_steps(steps=4, warmup=1, graph=GRAPH_ITERS):
    """The batched ensemble: 256 independent suspensions of U{1..64} filaments x U{10..50}
    segments (about 2.6e5 segments), each at its own dt = T/100 and gravity, in one
    simulation (one persistent mobility launch per evaluation, Broyden iterations in graph
    blocks, per-suspension convergence), in FP64 and with FP32 tiles."""
    import numpy as np
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth
    t0 = time.perf_counter()
    ws = synth.batched_ensemble(n_susp=256, seed=1004, dt_over_T=1 / 100)
    fil_off = [0]
    for w in ws:
        fil_off += list(fil_off[-1] + w.fil_off[1:])
    sfo = np.concatenate([[0], np.cumsum([w.M for w in ws])])
    Y, q = np.concatenate([w.Y for w in ws]), np.concatenate([w.q for w in ws])
    S = int(fil_off[-1])
    pairs = float(sum(w.S ** 2 for w in ws))
    out = {"workload": "256 suspensions, filaments U{1..64} x segments U{10..50} (S=%d, sum S_i^2=%.3g), "
                       "dt=T_i/100, tol 1e-6, graph blocks of %d" % (S, pairs, graph),
           "setup_s": time.perf_counter() - t0}
    for prec in ("f64", "f32tile"):
        sim = fil.Sim(fil_off, Y, q, ws[0].params, susp_fil_off=sfo, prec=prec, graph=graph)
        sim.set_suspension_params(dt=[w.params["dt"] for w in ws], grav=[w.params["grav"] for w in ws],
                                  FS=[w.params["FS"] for w in ws])
        for _ in range(warmup):
            sim.step()
        torch.cuda.synchronize()
        its, mx = [], 0
        t0 = time.perf_counter()
        for _ in range(steps):
            reps = sim.step()
            its += [r["iters"] for r in reps]
            mx = max(mx, max(r["iters"] for r in reps))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sim.close()
        out[prec] = {"ms_per_step": el / steps * 1e3, "mean_iters_per_suspension": float(np.mean(its)),
                     "max_iters": mx}
        log("ensemble steps", prec, out[prec])
    return out


def learned_gain(log_fn):
    """Learned warm start vs plain Broyden on the 500 x 32 sedimenting suspension (40 steps
    after 5).  The network (608-256-256-256-192 SiLU, BF16 MFMA) predicts the converged
    unknowns around a base guess, the extrapolation plus the last step's own correction; it
    is trained here, on the GPU, from pairs the method generates: (a) from another 500 x 32
    suspension at the same density (in-distribution), the headline factor; (b) from single
    filaments at N = 32, the config-1-style source.  (c) A network whose output is zero
    starts every step from the base alone, which separates the base's share of the gain."""
    import numpy as np
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import learned, synth
    w = synth.sediment_suspension(M=500, N=32, side=400.0, seed=1005, dt_over_T=1 / 30)
    out = {"workload": "sedimenting suspension 500 x 32 (S=16000), dt=T/30, tol 1e-6, 40 steps after 5"}
    for name, src, seed in (("suspension_trained", "dense", 21), ("single_filament_trained", "single", 2024)):
        t0 = time.perf_counter()
        feat, targ = learned.generate(n_fil=500, N=32, steps=100, source=src, seed=seed)
        t1 = time.perf_counter()
        m = fil.MLP(32, width=256, depth=3, max_batch=1024, seed=0)
        hist = learned.train(m, feat, targ, epochs=60, batch=1024, lr=1e-3)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = learned.compare(w, m, steps=45, skip=5, log=log_fn)
        res.update(train_samples=int(feat.shape[0]), data_s=t1 - t0, train_s=t2 - t1,
                   final_validation_loss=hist[-1][1],
                   source="one 500 x 32 suspension at the same density (another seed), 100 steps" if src == "dense"
                   else "500 single filaments of N=32, B log-uniform in [1e2, 1e4], 100 steps")
        out[name] = res
        m.close()
    m = fil.MLP(32, width=256, depth=3, max_batch=1024, seed=0)
    P = m.get_params()
    n_last = m.layer_dims[-1][0] * m.layer_dims[-1][1] + m.layer_dims[-1][1]
    P[len(P) - n_last:] = 0.0  # output layer zero: the prediction is exactly zero
    m.set_params(P)
    out["base_only"] = learned.compare(w, m, steps=45, skip=5, log=log_fn)
    m.close()
    out["time_ratio"] = out["suspension_trained"]["time_ratio"]
    out["iteration_ratio"] = out["suspension_trained"]["iteration_ratio"]
    return out


def solver_comparison(w, steps=5, warmup=2, names=("ejb_b", "jfnk_j0", "jfnk_none", "jfb_g_j0"), periodic=None,
                      workload="sedimenting suspension 100 x 20 (S=2000), dt=T/30, tolerances 1e-4 (paper's comparison)"):
    """Bad Broyden with the explicit J0 against Jacobian-free Newton-Krylov (J0 left
    preconditioner, the time-step right preconditioner, none) and the Jacobian-free good
    Broyden method (J0 left preconditioner), at the tolerances of the paper's comparisons
    (Newton/Broyden 1e-4, GMRES 1e-4, finite-difference delta 1e-7), on the same
    suspension and GPU; periodic = (box, grid, cut) puts it in a periodic box with the
    force-coupling mobility."""
    import torch
    import paper_1903_12609_amd as fil
    out = {}
    for name in names:
        # the Krylov methods get at most 30 outer iterations of at most 400 GMRES iterations
        # each per step, so that a stagnating step ends in bounded time
        kmax = w.params["kmax"] if name == "ejb_b" else min(w.params["kmax"], 30)
        sim = fil.Sim(w.fil_off, w.Y, w.q, dict(w.params, tol=1e-4, kmax=kmax), graph=GRAPH_ITERS)
        if periodic is not None:
            sim.set_periodic_fcm(*periodic)
        if name == "ejb_b":
            run = lambda: sim.step()[0]
        elif name.startswith("jfnk"):
            run = lambda: sim.jfnk_step(precond=name[5:], krylov_tol=1e-4, fd_delta=1e-7, krylov_max=400,
                                        raise_on_fail=False)
        else:
            run = lambda: sim.jfb_step(precond=name[6:], krylov_tol=1e-4, fd_delta=1e-7, krylov_max=400,
                                       raise_on_fail=False)
        failed = 0
        for _ in range(warmup):
            failed += isinstance(run(), tuple)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        applies = krylov = 0
        for j in range(steps):
            t1 = time.perf_counter()
            r = run()
            if isinstance(r, tuple):  # (error code, report): the step did not converge
                failed += 1
                r = r[1]
            applies += r["applies"]
            krylov += r.get("krylov", 0)
            if periodic is not None:
                torch.cuda.synchronize()
                log("solver %s step %d: %.1f ms, %d applies" % (name, j, (time.perf_counter() - t1) * 1e3,
                                                               r["applies"]))
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": (time.perf_counter() - t0) / steps * 1e3, "mobility_applies_per_step": applies / steps}
        if name != "ejb_b":
            out[name]["krylov_iters_per_step"] = krylov / steps
        if failed:
            out[name]["steps_not_converged"] = failed
        sim.close()
        log("solver", name, out[name])
    for name in names:
        if name != "ejb_b":
            out[name + "_over_ejb_b_time"] = out[name]["ms_per_step"] / out["ejb_b"]["ms_per_step"]
    out["workload"] = workload
    return out


def fcm_monolayer_steps(steps=4, warmup=1, cut=4.5):
    """The paper's solver test bed with its own mobility: a monolayer of 256 filaments of
    N = 15 segments in the centre plane of a periodic 141 dL x 141 dL x 8.8 dL box, the
    force-coupling method on a 1024 x 1024 x 64 grid (Gaussians truncated at 4.5 widths,
    where their tails fall below the 1e-4 tolerance), B = 1000, dt = T/300, gravity in the
    plane; bad Broyden against JFNK (J0, time-step preconditioners) and JFB-g (J0)."""
    from paper_1903_12609_amd import synth
    w = synth.periodic_monolayer(M=256, N=15, seed=1006)
    per = (w.extra["box"], w.extra["grid"], cut)
    return solver_comparison(w, steps=steps, warmup=warmup, names=("ejb_b", "jfnk_j0", "jfnk_pdt", "jfb_g_j0"),
                             periodic=per,
                             workload="periodic monolayer 256 x 15 (S=3840), FCM 1024x1024x64 over 141dL x 141dL x "
                                      "8.8dL, cut 4.5 widths, B=1e3, dt=T/300, tolerances 1e-4")


def fcm_apply_bench(reps=5):
    """Force-coupling-method applies on the paper's FCM grid (1024 x 1024 x 64 points over
    141 dL x 141 dL x 8.8 dL, a monolayer of M filaments of N = 15 segments): M = 1024
    (S = 15360 segments at random positions in the box), Gaussians truncated at 4 and 7.5
    widths."""
    import numpy as np
    import torch
    import paper_1903_12609_amd as fil
    dL = 2.2
    box = (141 * dL, 141 * dL, 8.8 * dL)
    grid = (1024, 1024, 64)
    S = 1024 * 15
    rng = np.random.default_rng(13)
    Y = torch.from_numpy(np.ascontiguousarray((rng.uniform(0, 1, (S, 3)) * np.array(box)).T)).cuda()
    F = torch.from_numpy(np.ascontiguousarray(rng.standard_normal((3, S)))).cuda()
    T = torch.from_numpy(np.ascontiguousarray(rng.standard_normal((3, S)))).cuda()
    out = []
    for cut in (4.0, 7.5):
        m = fil.FCM(box, grid, a=1.0, eta=1.0, cut=cut)
        V, W = m.apply(Y, F, T)
        ms = _time_applies(lambda: m.apply(Y, F, T, V, W), reps) * 1e3
        npts = grid[0] * grid[1] * grid[2]
        out.append(dict(grid=list(grid), box=list(box), segments=S, cut_widths=cut, ms=ms,
                        grid_points_per_s=npts / (ms * 1e-3), segments_per_s=S / (ms * 1e-3)))
        log("fcm apply", out[-1])
        m.close()
    return out


# FP64 flops of one pair of the wall kernel (FMA = 2): the free-space blocks as in the unbounded
# count (85), R and 1/|R| (14), the 18 image coefficients (153) and their application to F and
# T (98), as written in wall_image.h
WALL_FLOP_PER_PAIR = 350


def wall_mobility_bench(reps=5):
    """The RPY mobility above a no-slip wall: applies at S = 2000, 16000, 32000 (lattices of
    32-segment filaments standing on the wall, bases one segment spacing above it), and the
    implicit steps of the paper's cilia-array size (6 x 6 clamped filaments of N = 20 at
    spacing 20a, curvature-driven, dt = period/100) with the wall; without it the same
    array's first step does not converge."""
    import numpy as np
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth
    out = {"apply": []}
    for S in (2000, 16000, 32000):
        Y, F, T = synth.rpy_throughput_inputs(S)
        Y = Y.copy()
        Y[:, 2] += synth.DL
        d = lambda x: torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
        Yd, Fd, Td = d(Y), d(F), d(T)
        for prec in ("f64", "f32tile"):
            V, W = fil.rpy_wall_apply(Yd, Fd, Td, prec=prec)
            ms = _time_applies(lambda: fil.rpy_wall_apply(Yd, Fd, Td, prec=prec, V=V, W=W),
                               reps if S > 10000 else 20) * 1e3
            tf = WALL_FLOP_PER_PAIR * float(S) ** 2 / (ms * 1e-3) / 1e12
            pk = PEAK_FP64_TFLOPS if prec == "f64" else PEAK_FP32_TFLOPS
            out["apply"].append(dict(S=S, prec=prec, ms=ms, pairs_per_s=float(S) ** 2 / (ms * 1e-3), tflops=tf,
                                     frac_of_peak=tf / pk))
            log("wall apply", out["apply"][-1])
    w = synth.active_array(nx=6, ny=6, N=20, spacing=20.0, seed=1003, base_z=synth.DL)
    res = {}
    for wall in (True, False):
        sim = fil.Sim(w.fil_off, w.Y, w.q, w.params, graph=GRAPH_ITERS)
        if wall:
            sim.set_wall()
        its, t0, ok = [], time.perf_counter(), True
        for _ in range(10):
            r = sim.step(raise_on_fail=False)
            rep = r[1][0] if isinstance(r, tuple) else r[0]
            its.append(rep["iters"])
            if not rep["converged"]:
                ok = False
                break
        torch.cuda.synchronize()
        res["wall" if wall else "unbounded"] = dict(converged=ok, iters=its,
                                                    ms_per_step=(time.perf_counter() - t0) / len(its) * 1e3)
        sim.close()
        log("cilia-size array", res)
    out["array_6x6x20_steps"] = res
    out["cilia_6x6x20_switch"] = cilia_array_steps()
    return out


def cilia_array_steps(steps=40, dt=25000.0, n_tr=10, tau=0.02):
    """Model cilia of Sec. 5.2.2 at the paper's array size: 6 x 6 pinned filaments of N = 20
    on the wall (base-to-base spacing L in both directions, bases one segment spacing
    above the wall), each driven by the geometric switch about y (theta_max = 2 pi / 5,
    torque ratio 3: tau_pos = 3 tau, tau_neg = tau = 0.02 K_B, 10-step transition),
    dt = 25000, tol 1e-6; all start upright and in phase.  (tau = 0.05 needs dt <= 5000:
    at larger steps the reversal's first step does not converge.)"""
    import math
    import numpy as np
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth
    N, nc = 20, 6
    L = N * synth.DL
    qz = np.array([math.cos(-math.pi / 4), 0.0, math.sin(-math.pi / 4), 0.0])
    bases = np.array([[i * L, j * L, synth.DL] for i in range(nc) for j in range(nc)])
    Y = np.concatenate([b + np.outer(np.arange(N) * synth.DL, [0, 0, 1.0]) for b in bases])
    q = np.tile(qz, (nc * nc * N, 1))
    fo = np.arange(0, nc * nc * N + 1, N, dtype=np.int64)
    p = dict(a=1.0, eta=1.0, dL=synth.DL, KB=1.0, KT=1.0, chi=1.1, FS=1e3 / L ** 2, grav=(0.0, 0.0, 0.0),
             dt=dt, tol=1e-6, kmax=100, tether=np.full(nc * nc, 2, dtype=np.int32), base=bases)
    sim = fil.Sim(fo, Y, q, p, graph=GRAPH_ITERS)
    sim.set_wall()
    sim.set_geometric_switch((0.0, 1.0, 0.0), (0.0, 0.0, 1.0), 2 * math.pi / 5, 3 * tau, tau, n_tr)
    its, flips, ok = [], 0, True
    prev = sim.read_switch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = sim.step(raise_on_fail=False)
        rep = r[1][0] if isinstance(r, tuple) else r[0]
        its.append(rep["iters"])
        if not rep["converged"]:
            ok = False
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d = sim.read_switch()
    Yf = sim.read_state()[0]
    sim.close()
    res = dict(converged=ok, steps=len(its), ms_per_step=el / len(its) * 1e3, iters_per_step=float(np.mean(its)),
               drive_down=int((d < 0).sum()), min_height=float(Yf[:, 2].min()),
               workload="6 x 6 pinned cilia of N = 20 on a wall, geometric switch (theta_max 2 pi/5, tau_neg %g, "
                        "ratio 3, %d-step transition), dt = %g, tol 1e-6" % (tau, n_tr, dt))
    log("cilia array", res)
    return res


def array_wall_sweep(steps=10, beats=(100, 300, 1000)):
    """The full active array above a no-slip wall: 40 x 25 base-clamped filaments of N = 32
    (spacing 20a, bases one segment spacing above the wall), driven by the swimmers'
    travelling curvature wave from straight, dt = period/100, /300, /1000; up to `steps`
    steps each, a dt stopping at its first step that does not converge.  Reports the
    iterations, applies and time of every step tried."""
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth
    out = []
    for spb in beats:
        w = synth.active_array(nx=40, ny=25, N=32, spacing=20.0, seed=1003, base_z=synth.DL, steps_per_beat=spb)
        sim = fil.Sim(w.fil_off, w.Y, w.q, w.params, graph=GRAPH_ITERS)
        sim.set_wall()
        rec = dict(steps_per_beat=spb, dt=w.params["dt"], iters=[], applies=[], ms=[], converged=True)
        for j in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sim.step(raise_on_fail=False)
            torch.cuda.synchronize()
            rep = r[1][0] if isinstance(r, tuple) else r[0]
            rec["iters"].append(rep["iters"])
            rec["applies"].append(rep["applies"])
            rec["ms"].append((time.perf_counter() - t0) * 1e3)
            log("wall array dt = period/%d, step %d: %d iterations, converged %s, residual %.2e" %
                (spb, j, rep["iters"], rep["converged"], rep["resid"]))
            if not rep["converged"]:
                rec["converged"] = False
                rec["final_residual"] = rep["resid"]
                break
        sim.close()
        out.append(rec)
    return {"workload": "40 x 25 clamped filaments, N = 32, spacing 20a, bases 2.2a above a no-slip wall, "
                        "travelling curvature wave from straight, tol 1e-6", "sweep": out}


def array_wall_steps(steps=200, spacing=40.0, spb=100, prec="f32tile"):
    """The 40 x 25 array of base-clamped filaments of N = 32 (32,000 segments) above a no-slip
    wall at lattice spacing 40a (at 20a the first step diverges: the coupling of neighbouring
    filaments through the fluid, which the block-diagonal J0 does not carry, is too strong for
    filaments of this length), driven by the travelling curvature wave from straight,
    dt = period/spb, tol 1e-6, FP32 tiles with an FP64 finish (or FP64): iterations,
    mobility applies and wall time of every step."""
    import numpy as np
    import torch
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import synth
    w = synth.active_array(nx=40, ny=25, N=32, spacing=spacing, seed=1003, base_z=synth.DL, steps_per_beat=spb)
    sim = fil.Sim(w.fil_off, w.Y, w.q, w.params, graph=GRAPH_ITERS, prec=prec)
    sim.set_wall()
    rec = dict(iters=[], applies=[], applies_f64=[], ms=[], converged=True)
    for j in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sim.step(raise_on_fail=False)
        torch.cuda.synchronize()
        rep = r[1][0] if isinstance(r, tuple) else r[0]
        rec["iters"].append(rep["iters"])
        rec["applies"].append(rep["applies"])
        rec["applies_f64"].append(rep["applies_f64"])
        rec["ms"].append((time.perf_counter() - t0) * 1e3)
        if not rep["converged"]:
            rec["converged"] = False
            log("array on the wall (%s): step %d did not converge (residual %.2e)" % (prec, j, rep["resid"]))
            break
        if (j + 1) % 10 == 0:
            log("array on the wall (%s): step %d, %.1f iterations and %.1f ms per step over the last 10" %
                (prec, j + 1, np.mean(rec["iters"][-10:]), np.mean(rec["ms"][-10:])))
    Yf = sim.read_state()[0]
    sim.close()
    rec.update(workload="40 x 25 clamped filaments, N = 32 (S = 32000), spacing %ga, bases 2.2a above a no-slip "
                        "wall, travelling curvature wave from straight, dt = period/%d, %s, tol 1e-6" % (spacing, spb, prec),
               steps=len(rec["iters"]), mean_iters=float(np.mean(rec["iters"])),
               mean_applies=float(np.mean(rec["applies"])), mean_applies_f64=float(np.mean(rec["applies_f64"])),
               mean_ms=float(np.mean(rec["ms"][1:] or rec["ms"])), min_height=float(Yf[:, 2].min()))
    return rec


def traffic_per_launch():
    """HBM bytes per launch of the FP32-tile pair kernel from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        with open(os.path.join(ROOT, "paper_1903_12609_amd", "csrc", "rpy.hip"), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
        if t.get("rpy_hip_sha256") != sha:
            return None
        return float(t["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inputs, gpu):
    """The FP64 oracle on a bounded sample of the headline apply: all S targets against all
    S sources on every host core, and 1000 targets on one core (both in pairs/s), and the
    GPU results' relative L2 error against the oracle's on those targets."""
    import numpy as np
    import oracle
    Y, F, T = inputs
    S = Y.shape[0]
    nthreads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    V0, W0 = oracle.rpy_apply(Y, F, T, 1.0, 1.0, nthreads=nthreads)
    t_all = time.perf_counter() - t0
    idx = np.sort(np.random.default_rng(5).choice(S, 1000, replace=False))
    t0 = time.perf_counter()
    oracle.rpy_apply_targets(Y, F, T, 1.0, 1.0, idx, nthreads=1)
    t_one = time.perf_counter() - t0
    err = lambda x, r: float(np.linalg.norm(x - r) / np.linalg.norm(r))
    errors = {prec: {"V_rel_l2": err(gpu[prec]["V"], V0), "Omega_rel_l2": err(gpu[prec]["W"], W0)}
              for prec in gpu}
    log("cpu baseline: all cores %.2f s, one core %.2f s; errors %s" % (t_all, t_one, errors))
    return dict(value=float(S) ** 2 / t_all, unit="pairs/s", cores=nthreads, kind="oracle", cpu_model=_cpu_model(),
                sample="one FP64 apply of the headline workload (all %d targets x %d sources), %.1f s on %d threads"
                       % (S, S, t_all, nthreads),
                one_core={"value": 1000.0 * S / t_one, "unit": "pairs/s", "cores": 1,
                          "sample": "1000 sampled targets x %d sources, %.1f s" % (S, t_one)},
                gpu_error_vs_oracle=errors)


def sediment_steps(steps, warmup, graph):
    """Implicit steps of the sedimenting suspension (100 x 20, S = 2000) in FP64 and with FP32
    tiles: ms per step, iterations, pair-kernel time inside the steps."""
    from paper_1903_12609_amd import synth
    w = synth.sediment_suspension(M=100, N=20, side=200.0, seed=1002, dt_over_T=1 / 30)
    S = w.S
    out = {"workload": "sedimenting suspension, 100 filaments x 20 segments (S=2000), B=1e3, dt=T/30, tol 1e-6, "
                       "steric on, unbounded RPY; Broyden iterations in graph blocks of %d" % graph}
    for prec in ("f64", "f32tile"):
        el, applies, iters, tm = run_steps(w, prec, steps, warmup, graph)
        ms, nl = tm[prec]
        kern_s = ms * 1e-3 / max(nl, 1)
        out[prec] = {"ms_per_step": el / steps * 1e3, "pairs_per_s": applies * float(S) ** 2 / el,
                     "iters_per_step": iters / steps, "mobility_applies_per_step": applies / steps,
                     "pair_kernel_avg_us": kern_s * 1e6, "pair_kernel_launches_timed": nl,
                     "pair_kernel_tflops": FLOP_PER_PAIR * float(S) ** 2 / kern_s / 1e12}
        log("sediment steps", prec, out[prec])
    return out, w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # a step is one headline apply; the untimed ones first bring the GPU's clocks up (the
    # pair kernel's duration falls by ~8% over the first dozen launches from idle)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--graph", type=int, default=GRAPH_ITERS, help="Broyden iterations per graph block (0: off)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-solvers", action="store_true", help="skip the Broyden vs Newton-Krylov comparison")
    ap.add_argument("--fcm-only", action="store_true", help="only the FCM applies (for profiling)")
    ap.add_argument("--wall-only", action="store_true", help="only the wall-bounded mobility (for profiling)")
    ap.add_argument("--rpy-only", action="store_true", help="only the stand-alone mobility applies (for profiling)")
    ap.add_argument("--headline-only", action="store_true", help="only the headline applies (for profiling)")
    ap.add_argument("--steps-only", action="store_true", help="only the implicit-step workloads")
    ap.add_argument("--sediment500-only", action="store_true",
                    help="only the 500 x 32 suspension's steps (for profiling)")
    ap.add_argument("--array-wall-sweep", action="store_true",
                    help="only the dt sweep of the 40 x 25 x 32 active array above a wall")
    ap.add_argument("--array-wall-steps", action="store_true",
                    help="only the 200 steps of the 40 x 25 x 32 active array above a wall (spacing 40a)")
    ap.add_argument("--learned-only", action="store_true", help="only the learned warm start comparison")
    ap.add_argument("--ensemble-only", action="store_true", help="only the 256-suspension ensemble's steps")
    ap.add_argument("--sediment2000-only", action="store_true",
                    help="only the 100 x 20 suspension's steps (for profiling)")
    ap.add_argument("--fcm-steps-only", action="store_true",
                    help="only the solver comparison on the periodic FCM monolayer (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: runs on several GPUs are not part of this implementation",
              file=sys.stderr)
        sys.exit(2)
    import paper_1903_12609_amd as fil  # noqa: F401  (fails loudly without the HIP library)
    from paper_1903_12609_amd import synth
    if args.fcm_only:
        print(json.dumps({"fcm_apply": fcm_apply_bench()}))
        return
    if args.rpy_only:
        print(json.dumps({"rpy_apply": rpy_sweep(), "rpy_apply_batched": rpy_batched()}))
        return
    if args.sediment500_only:
        print(json.dumps({"sediment500x32_steps": suspension_steps(graph=args.graph)}))
        return
    if args.steps_only:
        out = {"sediment2000_steps": sediment_steps(20, 5, args.graph)[0], "sediment500x32_steps": suspension_steps(),
               "ensemble256_steps": ensemble_steps()}
        print(json.dumps(out))
        return
    if args.wall_only:
        print(json.dumps({"wall_mobility": wall_mobility_bench()}))
        return
    if args.array_wall_sweep:
        print(json.dumps({"array_wall_sweep": array_wall_sweep()}, default=float))
        return
    if args.array_wall_steps:
        print(json.dumps({"array_wall_steps": {"f32tile": array_wall_steps(),
                                               "f64": array_wall_steps(steps=50, prec="f64")}}, default=float))
        return
    if args.ensemble_only:
        print(json.dumps({"ensemble256_steps": ensemble_steps()}))
        return
    if args.sediment2000_only:
        print(json.dumps({"sediment2000_steps": sediment_steps(20, 5, args.graph)[0]}))
        return
    if args.learned_only:
        print(json.dumps({"learned_warm_start": learned_gain(log)}))
        return
    if args.fcm_steps_only:
        print(json.dumps({"fcm_monolayer_solvers": fcm_monolayer_steps()}))
        return

    head, inputs = apply_headline(args.steps, args.warmup)
    h32, h64 = head["f32tile"], head["f64"]
    S = h32["S"]
    flop = FLOP_PER_PAIR * float(S) ** 2
    achieved = flop / (h32["kernel_avg_us"] * 1e-6) / 1e12
    res = {
        "metric": "RPY pair-interactions/s (fp64 vs fp32) + ms/step to tol, plain vs learned",
        "value": h32["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h32["ms_per_apply"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": HEADLINE_WORKLOAD, "segments": S, "pairs_per_apply": float(S) ** 2,
                   "precision": "f32tile", "step": "one mobility apply"},
        "roofline": {"bound": "alu", "kernel": "rpy_f32_kernel<2,1>", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic_per_launch(), "avg_kernel_us": h32["kernel_avg_us"], "launches": args.steps,
                     "flop_per_launch": flop, "flop_per_pair": FLOP_PER_PAIR},
        "f64_apply": {"ms_per_apply": h64["ms_per_apply"], "pairs_per_s": h64["pairs_per_s"],
                      "kernel_avg_us": h64["kernel_avg_us"],
                      "kernel_tflops": flop / (h64["kernel_avg_us"] * 1e-6) / 1e12,
                      "frac_of_fp64_peak": flop / (h64["kernel_avg_us"] * 1e-6) / 1e12 / PEAK_FP64_TFLOPS},
        "f32_over_f64_time": h64["ms_per_apply"] / h32["ms_per_apply"],
    }
    if not args.headline_only:
        res["sediment2000_steps"], w = sediment_steps(20, 5, args.graph)
        res["sediment500x32_steps"] = suspension_steps()
        res["ensemble256_steps"] = ensemble_steps()
        res["array_wall_steps"] = {"f32tile": array_wall_steps(), "f64": array_wall_steps(steps=50, prec="f64")}
        if not args.no_sweep:
            res["rpy_apply"] = rpy_sweep()
            res["rpy_apply_batched"] = rpy_batched()
            res["fcm_apply"] = fcm_apply_bench()
            res["wall_mobility"] = wall_mobility_bench()
        if not args.no_solvers:
            res["solver_comparison"] = solver_comparison(w)
            res["fcm_monolayer_solvers"] = fcm_monolayer_steps()
        if not args.no_learned:
            res["learned_warm_start"] = learned_gain(log)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(inputs, head)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
