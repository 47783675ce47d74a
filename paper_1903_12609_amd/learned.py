"""Learned warm start: training data from the method's own converged steps,
training on the GPU, and the plain-versus-learned comparison.

Every number is computed by the library's kernels (the implicit steps, the
feature/target kernels, the BF16 MFMA network and its Adam update); this
module only sequences the calls, draws seeded permutations and holds device
tensors.

What the network predicts: the converged unknowns of a step minus a base guess, the
extrapolated first iterate plus the last step's own correction (the step target of
`Sim.step_target`); the prediction is added back to that base.

Training data ("single filament" source): independent sedimenting filaments
of N segments, each its own suspension in one batched simulation, with the
gravity number B log-uniform in [1e2, 1e4], isotropic orientations and a
small random planar bend; dt = T/30 of each filament's settling time T.
After `warm` steps (the features need three committed steps of history) every
step contributes one (features, target) pair per filament.  The
"suspension" source draws the pairs from small sedimenting suspensions of
the same filaments instead (placed like the sedimenting suspension at its
density), so the features see hydrodynamic interactions, and the "dense"
source from one large suspension at that density.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import Sim
from . import synth


def _batch(workloads):
    fil_off, sfo = [0], [0]
    for w in workloads:
        fil_off += list(fil_off[-1] + w.fil_off[1:])
        sfo.append(sfo[-1] + w.M)
    Y = np.concatenate([w.Y for w in workloads])
    q = np.concatenate([w.q for w in workloads])
    return np.array(fil_off), np.array(sfo), Y, q


def _ensemble(source, n_fil, N, seed, dt_over_T, per=10):
    rng = np.random.default_rng(seed)
    ws = []
    if source == "single":
        for i in range(n_fil):
            B = 10.0 ** rng.uniform(2.0, 4.0)
            w = synth.single_filament(N=N, seed=int(rng.integers(1 << 31)), B=B, dt_over_T=dt_over_T,
                                      bend=rng.uniform(0.0, 0.05))
            ws.append(w)
    elif source == "dense":
        # one suspension of n_fil filaments at the sedimenting suspension's density
        side = 200.0 * (n_fil * N / 2000.0) ** (1.0 / 3.0)
        ws.append(synth.sediment_suspension(M=n_fil, N=N, side=side, seed=int(rng.integers(1 << 31)),
                                            dt_over_T=dt_over_T))
    elif source == "suspension":
        for i in range(max(1, n_fil // per)):
            side = 200.0 * (per * N / 2000.0) ** (1.0 / 3.0)
            ws.append(synth.sediment_suspension(M=per, N=N, side=side, seed=int(rng.integers(1 << 31)),
                                                dt_over_T=dt_over_T))
    else:
        raise ValueError(source)
    return ws


def generate(n_fil=500, N=32, steps=100, warm=3, seed=2024, source="single", dt_over_T=1 / 30, log=None, per=10):
    """(features [n, 19N], targets [n, 6N]) float32 device tensors, n = n_fil x steps
    (source "suspension": n_fil / per suspensions of `per` filaments each).
    A simulation whose step fails (Broyden diverging) is dropped from that step
    on and replaced by a freshly seeded one until n samples are collected."""
    import torch
    from ._native import FilError
    feats, targs = [], []
    have, attempt = 0, 0
    t0 = time.perf_counter()
    while have < n_fil * steps:
        if attempt >= 10:
            raise RuntimeError("training data: too many diverging simulations")
        ws = _ensemble(source, n_fil, N, seed + 7919 * attempt, dt_over_T, per)
        attempt += 1
        fil_off, sfo, Y, q = _batch(ws)
        sim = Sim(fil_off, Y, q, ws[0].params, susp_fil_off=sfo)
        sim.set_suspension_params(dt=[w.params["dt"] for w in ws], grav=[w.params["grav"] for w in ws],
                                  FS=[w.params["FS"] for w in ws])
        try:
            for j in range(warm + steps):
                f = sim.features() if j >= warm else None
                sim.step()
                if j >= warm:
                    feats.append(f)
                    targs.append(sim.step_target())
                    have += f.shape[0]
                    if have >= n_fil * steps:
                        break
                if log and (j + 1) % 25 == 0:
                    log("training data: step %d (%.1f s)" % (j + 1, time.perf_counter() - t0))
        except FilError as e:
            if log:
                log("training data: simulation %d stopped (%s); %d samples so far" % (attempt, e, have))
        finally:
            sim.close()
    torch.cuda.synchronize()
    return torch.cat(feats)[:n_fil * steps], torch.cat(targs)[:n_fil * steps]


def train(mlp, feat, targ, epochs=60, batch=1024, lr=1e-3, val_frac=0.1, seed=7, log=None):
    """Fits the standardisation to the samples, then Adam with a cosine
    learning-rate schedule on the training split.  Returns the per-epoch
    (last minibatch, validation) losses."""
    import torch
    n = feat.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nval = int(round(val_frac * n))
    tr_idx, va_idx = np.sort(perm[nval:]), np.sort(perm[:nval])
    mlp.fit_norm(feat, targ)
    xb, t = mlp.standardize(feat, targ)
    batch = min(batch, mlp.max_batch)
    steps_per_epoch = max(1, len(tr_idx) // batch)
    total = epochs * steps_per_epoch
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    k = 0
    for ep in range(epochs):
        order = tr_idx[rng.permutation(len(tr_idx))]
        acc = 0.0
        for b in range(steps_per_epoch):
            rows = torch.from_numpy(order[b * batch:(b + 1) * batch].astype(np.int32)).cuda()
            lr_k = 0.5 * lr * (1.0 + math.cos(math.pi * k / total))
            mlp.train_step(xb, t, rows, lr_k, loss)
            acc += float(loss.item()) if b == steps_per_epoch - 1 else 0.0
            k += 1
        vl = validation_loss(mlp, xb, t, va_idx)
        hist.append((acc, vl))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log("epoch %d: train loss %.4f  validation loss %.4f" % (ep, acc, vl))
    return hist


def validation_loss(mlp, xb, t, idx):
    import torch
    if len(idx) == 0:
        return float("nan")
    tot, cnt = 0.0, 0
    for s in range(0, len(idx), mlp.max_batch):
        rows = torch.from_numpy(idx[s:s + mlp.max_batch].astype(np.int32)).cuda()
        loss, _ = mlp.backward(xb, t, rows=rows)
        tot += float(loss.item()) * rows.shape[0]
        cnt += rows.shape[0]
    return tot / cnt


def compare(w, mlp, steps=30, skip=5, prec="f64", log=None):
    """Plain and learned runs of the same suspension from the same initial
    state: mean Broyden iterations, mobility applies and wall ms per step over
    the steps after `skip` (the learned start needs three steps of history)."""
    import torch
    out = {}
    for mode in ("plain", "learned"):
        sim = Sim(w.fil_off, w.Y, w.q, w.params, prec=prec)
        if mode == "learned":
            sim.set_mlp(mlp)
        its, apps, ms, used = [], [], [], 0
        for j in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sim.step()[0]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
            if j >= skip:
                its.append(r["iters"])
                apps.append(r["applies"])
                ms.append(dt)
                used += r["used_learned"]
        out[mode] = dict(iters_per_step=float(np.mean(its)), applies_per_step=float(np.mean(apps)),
                         ms_per_step=float(np.mean(ms)), steps=len(its), learned_steps=used,
                         fallbacks=sim.fallbacks())
        if log:
            log("%s: %s" % (mode, out[mode]))
        sim.close()
    out["iteration_ratio"] = out["plain"]["iters_per_step"] / out["learned"]["iters_per_step"]
    out["time_ratio"] = out["plain"]["ms_per_step"] / out["learned"]["ms_per_step"]
    return out
