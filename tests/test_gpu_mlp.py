"""GPU parity of the learned warm start: the BF16 MFMA network's forward pass,
gradients and Adam step against the FP64 oracle network, the feature and
target kernels against their oracle definitions, and the learned first
iterate inside the implicit step."""
import numpy as np
import pytest

import oracle
from oracle import learned as OL
from oracle import mlp as OM
from paper_1903_12609_amd import synth

from gpu_util import rel_l2

pytestmark = pytest.mark.gpu


def _bf16_bits(x):
    a = np.ascontiguousarray(OM.bf16_round(x).astype(np.float32))
    return (a.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def _setup(n_seg, width, depth, B, seed):
    import torch
    import paper_1903_12609_amd as fil
    m = fil.MLP(n_seg, width=width, depth=depth, max_batch=max(B, 64), seed=seed)
    rng = np.random.default_rng(seed)
    P = m.get_params().astype(np.float64)
    P += rng.standard_normal(P.size) * 0.02  # non-zero biases too
    dims = m.layer_dims
    # zero the padding (inputs beyond n_in, outputs beyond n_out)
    params = OM.unflatten(P, dims)
    params[0][0][:, m.n_in:] = 0.0
    params[-1][0][m.n_out:, :] = 0.0
    params[-1][1][m.n_out:] = 0.0
    P = OM.flatten(params).astype(np.float32)
    m.set_params(P)
    X = np.zeros((B, m.n_in_pad))
    X[:, :m.n_in] = rng.standard_normal((B, m.n_in))
    T = np.zeros((B, m.n_out_pad))
    T[:, :m.n_out] = rng.standard_normal((B, m.n_out))
    xb = torch.from_numpy(_bf16_bits(X)).cuda()
    # oracle at the BF16-rounded weights and inputs
    ob = [(OM.bf16_round(W), b.astype(np.float32).astype(np.float64)) for W, b in OM.unflatten(P, dims)]
    return m, P, xb, OM.bf16_round(X), T, ob


@pytest.mark.parametrize("n_seg,width,depth,B", [(32, 256, 3, 500), (4, 64, 2, 70)])
def test_forward_matches_oracle(n_seg, width, depth, B):
    print("case forward", n_seg, width, depth, B, flush=True)
    m, P, xb, Xr, T, ob = _setup(n_seg, width, depth, B, 11)
    Y = m.forward(xb).cpu().numpy()
    Yo, _, _ = OM.forward(ob, Xr)
    err = rel_l2(Y[:, :m.n_out], Yo[:, :m.n_out])
    print("forward rel L2 %.3e" % err)
    assert err <= 2e-2


@pytest.mark.parametrize("n_seg,width,depth,B", [(32, 256, 3, 500), (4, 64, 2, 70)])
def test_gradients_match_oracle(n_seg, width, depth, B):
    import torch
    print("case backward", n_seg, width, depth, B, flush=True)
    m, P, xb, Xr, T, ob = _setup(n_seg, width, depth, B, 12)
    t = torch.from_numpy(T.astype(np.float32)).cuda()
    rows = torch.from_numpy(np.random.default_rng(1).permutation(B).astype(np.int32)).cuda()
    loss, g = m.backward(xb, t, rows=rows)
    order = rows.cpu().numpy()
    Lo, Go = OM.gradients(ob, Xr[order], T[order], n_out=m.n_out)
    assert abs(loss.item() - Lo) <= 1e-2 * Lo
    G = OM.unflatten(g.cpu().numpy(), m.layer_dims)
    for l, ((gW, gb), (oW, obb)) in enumerate(zip(G, Go)):
        eW, eb = rel_l2(gW, oW), rel_l2(gb, obb)
        print("layer %d: dW rel L2 %.3e, db rel L2 %.3e" % (l, eW, eb))
        assert eW <= 2e-2 and eb <= 2e-2


def test_adam_first_step_closed_form():
    """First Adam step: bias-corrected moments are g and g^2, so every
    parameter moves by -lr g / (|g| + eps) (FP32)."""
    import torch
    m, P, xb, Xr, T, ob = _setup(4, 64, 2, 70, 13)
    t = torch.from_numpy(T.astype(np.float32)).cuda()
    _, g = m.backward(xb, t)
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    m.adam_step(lr)
    P1 = m.get_params().astype(np.float64)
    ref = P.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(P1 - ref)) <= 1e-6 * max(1.0, np.max(np.abs(P)))


def test_training_matches_fp64_training():
    """Training on the GPU (BF16 MFMA forward and backward, FP32 Adam) follows exact
    training: the same network, initial weights (seeded on the host), minibatches and
    cosine learning-rate schedule trained by the FP64 oracle network reaches a validation
    loss within 1.3x of it.  The task (targets a fixed smooth function tanh(X A) of the
    inputs) is learnable: the FP64 training itself ends below 0.15 of the initial loss.
    (Its last validation loss is 0.13 of its first epoch's, so a 0.1x criterion against the
    first epoch would fail even in exact arithmetic.)"""
    import math
    import torch
    import paper_1903_12609_amd as fil
    m = fil.MLP(4, width=64, depth=2, max_batch=256, seed=3)
    n_in, n_out = m.n_in, m.n_out
    rng = np.random.default_rng(4)
    n = 2048
    X = rng.standard_normal((n, n_in))
    A = rng.standard_normal((n_in, n_out)) / np.sqrt(n_in)
    T = np.tanh(X @ A)
    Xs = np.zeros((n, m.n_in_pad))
    Xs[:, :n_in] = (X - X.mean(0)) / X.std(0)
    Ts = np.zeros((n, m.n_out_pad))
    Ts[:, :n_out] = (T - T.mean(0)) / T.std(0)
    # He-uniform initial weights drawn on the host, padding rows and columns zero
    ir = np.random.default_rng(5)
    params = []
    for l, (din, dout) in enumerate(m.layer_dims):
        W = ir.uniform(-1.0, 1.0, (dout, din)) * math.sqrt(6.0 / din)
        if l == 0:
            W[:, n_in:] = 0.0
        if l + 1 == len(m.layer_dims):
            W[n_out:, :] = 0.0
        params.append((W, np.zeros(dout)))
    m.set_params(OM.flatten(params).astype(np.float32))
    params = OM.unflatten(OM.flatten(params).astype(np.float32).astype(np.float64), m.layer_dims)
    # the data are already standardised: identity normalisation on the GPU
    m.set_norm(np.concatenate([np.zeros(m.n_in_pad), np.ones(m.n_in_pad), np.zeros(m.n_out_pad),
                               np.ones(m.n_out_pad)]))
    xb, t = m.standardize(torch.from_numpy(Xs[:, :n_in].astype(np.float32)).cuda(),
                          torch.from_numpy(Ts[:, :n_out].astype(np.float32)).cuda())
    perm = np.random.default_rng(7).permutation(n)
    va, tr = np.sort(perm[:205]), np.sort(perm[205:])
    va_d = torch.from_numpy(va.astype(np.int32)).cuda()
    batch, epochs, lr = 256, 60, 3e-3
    spe = len(tr) // batch
    total = epochs * spe
    mo, vo = OM.zeros_like(params), OM.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    l0_or = OM.loss(params, Xs[va], Ts[va], n_out)
    l0_gpu = m.backward(xb, t, rows=va_d)[0].item()
    order_rng = np.random.default_rng(8)
    k = 0
    for ep in range(epochs):
        order = tr[order_rng.permutation(len(tr))]
        for b in range(spe):
            rows = order[b * batch:(b + 1) * batch]
            lr_k = 0.5 * lr * (1.0 + math.cos(math.pi * k / total))
            m.train_step(xb, t, torch.from_numpy(rows.astype(np.int32)).cuda(), lr_k, loss)
            _, g = OM.gradients(params, Xs[rows], Ts[rows], n_out)
            k += 1
            params = OM.adam_step(params, g, mo, vo, k, lr_k)
    l_or = OM.loss(params, Xs[va], Ts[va], n_out)
    l_gpu = m.backward(xb, t, rows=va_d)[0].item()
    m.close()
    print("validation loss: FP64 %.4f -> %.4f, GPU %.4f -> %.4f" % (l0_or, l_or, l0_gpu, l_gpu))
    assert abs(l0_gpu - l0_or) <= 2e-2 * l0_or
    assert l_or <= 0.15 * l0_or
    assert l_gpu <= 1.3 * l_or


def _small_run(steps=5):
    import paper_1903_12609_amd as fil
    w = synth.sediment_suspension(M=3, N=8, side=30.0, seed=51, dt_over_T=1 / 30)
    o = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params)
    g = fil.Sim(w.fil_off, w.Y, w.q, w.params)
    Xh = [np.zeros(6 * w.S)] * 3  # committed X^j, X^{j-1}, X^{j-2}
    for j in range(steps):
        X0 = o.initial_guess()
        Xb = OL.base(w.fil_off, X0, Xh[0], Xh[1], Xh[2], j)
        rc, rep = o.step()
        r = g.step()[0]
        assert rc == 0 and r["iters"] == rep.iters
        Xh = [o.X.copy()] + Xh[:2]
    return w, o, g, Xh, Xb


def test_features_and_target_match_oracle():
    w, o, g, Xh, Xb = _small_run()
    p = w.params
    F, T = o.forces(o.X)
    V, _ = oracle.rpy_apply(o.Y, F, T, p["a"], p["eta"])
    fo = OL.features(w.fil_off, o.Y, o.q, F, V, Xh[0], Xh[1], Xh[2], p["dL"], p["dt"], p["grav"], p["KB"])
    fg = g.features().cpu().numpy()
    err = rel_l2(fg, fo)
    print("features rel L2 %.3e" % err)
    assert err <= 1e-6
    to = OL.target(w.fil_off, o.X, Xb, p["dL"], p["grav"], p["KB"])
    tg = g.step_target().cpu().numpy()
    err = rel_l2(tg, to)
    print("target rel L2 %.3e" % err)
    assert err <= 1e-5


def test_zero_prediction_starts_from_the_base():
    """A network whose prediction is exactly zero starts every step from the fourth on at
    the base guess (the extrapolation plus the last step's correction): the learned path
    then follows the oracle's Broyden run from that base, with equal iteration counts."""
    import paper_1903_12609_amd as fil
    w = synth.sediment_suspension(M=4, N=8, side=30.0, seed=52, dt_over_T=1 / 30)
    m = fil.MLP(8, width=64, depth=2, max_batch=64, seed=1)
    params = OM.unflatten(m.get_params().astype(np.float64), m.layer_dims)
    params[-1] = (np.zeros_like(params[-1][0]), np.zeros_like(params[-1][1]))
    m.set_params(OM.flatten(params).astype(np.float32))
    o = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params)
    b = fil.Sim(w.fil_off, w.Y, w.q, w.params)
    b.set_mlp(m)
    Xh = [np.zeros(6 * w.S)] * 3
    for j in range(7):
        X0 = o.initial_guess()
        Xb = OL.base(w.fil_off, X0, Xh[0], Xh[1], Xh[2], j)
        Xs, rc, rep = o.broyden(Xb if j >= 3 else X0)
        assert rc == 0
        o.commit(Xs)
        rb = b.step()[0]
        print("step", j, "oracle", rep.iters, "gpu", rb["iters"])
        assert rb["iters"] == rep.iters
        assert rb["used_learned"] == (j >= 3)
        Xh = [o.X.copy()] + Xh[:2]
    Yg = b.read_state()[0]
    assert np.abs(Yg - o.Y).max() <= 1e-8 * np.abs(o.Y).max()
    assert b.fallbacks() == 0


def test_learned_start_with_untrained_network_still_converges():
    """An arbitrary prediction cannot change the result's tolerance: each step
    either converges from the learned start or falls back to the plain one."""
    import paper_1903_12609_amd as fil
    w = synth.sediment_suspension(M=4, N=8, side=30.0, seed=53, dt_over_T=1 / 30)
    m = fil.MLP(8, width=64, depth=2, max_batch=64, seed=2)
    g = fil.Sim(w.fil_off, w.Y, w.q, w.params)
    g.set_mlp(m)
    for j in range(6):
        r = g.step()[0]
        assert r["converged"] and r["resid"] <= w.params["tol"]
    print("fallbacks", g.fallbacks())


def test_trained_network_cuts_iterations_on_held_out_suspension():
    """The gain of the learned warm start: the network is trained on the GPU (library
    kernels only) on 50,000 (state, converged update) pairs of one 500 x 32 sedimenting
    suspension, then a held-out suspension of the same kind (another seed) is stepped from
    the learned first iterate (the base guess plus the prediction) and from the plain one
    at the same tolerance: the learned start needs at least two Broyden iterations per step
    fewer on average (measured 34.8 against 39.0 over these 20 steps), without fallbacks,
    and every step converges."""
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd import learned
    feat, targ = learned.generate(n_fil=500, N=32, steps=100, source="dense", seed=21)
    m = fil.MLP(32, width=256, depth=3, max_batch=1024, seed=0)
    learned.train(m, feat, targ, epochs=60, batch=1024, lr=1e-3)
    w = synth.sediment_suspension(M=500, N=32, side=400.0, seed=1005, dt_over_T=1 / 30)
    res = learned.compare(w, m, steps=25, skip=5)
    m.close()
    print("plain %.2f, learned %.2f iterations per step; time ratio %.3f" % (
        res["plain"]["iters_per_step"], res["learned"]["iters_per_step"], res["time_ratio"]))
    assert res["learned"]["learned_steps"] == res["learned"]["steps"] and res["learned"]["fallbacks"] == 0
    assert res["learned"]["iters_per_step"] <= res["plain"]["iters_per_step"] - 2.0
