"""Pins of the learned warm start's oracle (network, Adam, features) against
finite differences, closed forms and library routines."""
import numpy as np
import pytest

from oracle import learned as OL
from oracle import mlp as OM


def _net(rng, dims):
    return [(rng.standard_normal((o, i)) / np.sqrt(i), rng.standard_normal(o) * 0.1) for i, o in dims]


def test_silu_and_derivative():
    assert OM.silu(0.0) == 0.0 and OM.dsilu(0.0) == 0.5
    z = np.linspace(-6, 6, 41)
    h = 1e-6
    fd = (OM.silu(z + h) - OM.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - OM.dsilu(z))) < 1e-9
    assert abs(OM.silu(40.0) - 40.0) < 1e-12 and abs(OM.silu(-40.0)) < 1e-12


@pytest.mark.parametrize("n_out", [None, 4])
def test_gradients_match_central_differences(n_out):
    rng = np.random.default_rng(0)
    dims = [(7, 6), (6, 6), (6, 5)]
    P = _net(rng, dims)
    X, T = rng.standard_normal((4, 7)), rng.standard_normal((4, 5))
    L, G = OM.gradients(P, X, T, n_out)
    assert abs(L - OM.loss(P, X, T, n_out)) < 1e-15
    h = 1e-6
    for l, (W, b) in enumerate(P):
        for arr, g in ((W, G[l][0]), (b, G[l][1])):
            fd = np.zeros_like(arr)
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = OM.loss(P, X, T, n_out)
                arr[idx] = old - h
                lm = OM.loss(P, X, T, n_out)
                arr[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.linalg.norm(fd - g) <= 1e-7 * max(np.linalg.norm(g), 1e-12), (l, arr.shape)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2 at
    every step, so each step moves a parameter by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    P = _net(rng, [(3, 2)])
    g = [(rng.standard_normal((2, 3)), rng.standard_normal(2))]
    m, v = OM.zeros_like(P), OM.zeros_like(P)
    lr, eps = 1e-2, 1e-8
    cur = P
    for t in range(1, 6):
        cur = OM.adam_step(cur, g, m, v, t, lr, eps=eps)
        for (W0, b0), (W, b), (gW, gb) in zip(P, cur, g):
            assert np.allclose(W, W0 - t * lr * gW / (np.abs(gW) + eps), rtol=0, atol=1e-14)
            assert np.allclose(b, b0 - t * lr * gb / (np.abs(gb) + eps), rtol=0, atol=1e-14)


def test_linear_layer_descends_to_least_squares():
    """A network with no hidden layer is affine; gradient descent on the MSE
    reaches numpy's least-squares solution."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((40, 3))
    T = X @ rng.standard_normal((3, 2)) + 0.3 + 0.05 * rng.standard_normal((40, 2))
    P = [(np.zeros((2, 3)), np.zeros(2))]
    for _ in range(4000):
        _, G = OM.gradients(P, X, T)
        P = [(P[0][0] - 0.5 * G[0][0], P[0][1] - 0.5 * G[0][1])]
    A = np.hstack([X, np.ones((40, 1))])
    sol, *_ = np.linalg.lstsq(A, T, rcond=None)
    assert np.allclose(P[0][0], sol[:3].T, atol=1e-9) and np.allclose(P[0][1], sol[3], atol=1e-9)


def test_bf16_rounding():
    assert OM.bf16_round(1.0) == 1.0 and OM.bf16_round(-3.5) == -3.5
    assert OM.bf16_round(1.0 + 2.0 ** -8) == 1.0                    # tie -> even
    assert OM.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6    # tie -> even (up)
    assert OM.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    x = np.random.default_rng(3).standard_normal(1000)
    assert np.max(np.abs(OM.bf16_round(x) - x) / np.abs(x)) <= 2.0 ** -8


def _fake_state(rng, M=3, N=5):
    fil_off = np.arange(0, M * N + 1, N)
    S = M * N
    Y = rng.standard_normal((S, 3)) * 10
    q = rng.standard_normal((S, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    F, V = rng.standard_normal((S, 3)), rng.standard_normal((S, 3))
    X = [rng.standard_normal(6 * S) for _ in range(3)]
    return fil_off, Y, q, F, V, X


def test_features_invariants():
    rng = np.random.default_rng(4)
    fil_off, Y, q, F, V, (Xj, X1, X2) = _fake_state(rng)
    kw = dict(dL=2.2, dt=0.7, grav=(0, 0, -2.0), KB=1.0)
    N = 5
    f0 = OL.features(fil_off, Y, q, F, V, Xj, X1, X2, **kw)
    assert f0.shape == (3, 19 * N)
    # positions relative to the centroid: zero sum, translation invariant
    assert np.allclose(f0[:, :3 * N].reshape(3, N, 3).sum(axis=1), 0, atol=1e-12)
    f1 = OL.features(fil_off, Y + 7.0, q, F, V, Xj, X1, X2, **kw)
    assert np.allclose(f0, f1, atol=1e-12)
    # a history that changes linearly in time has no Y_1 / Lambda component,
    # and u's entry is its constant change
    Xl1, Xl2 = Xj - 0.3 * X1, Xj - 0.6 * X1
    f2 = OL.features(fil_off, Y, q, F, V, Xj, Xl1, Xl2, **kw)
    h = f2[:, 13 * N:]
    assert np.allclose(h[:, :3], 0, atol=1e-12) and np.allclose(h[:, 3 + 3 * N:], 0, atol=1e-12)
    for f in range(3):
        assert np.allclose(h[f, 3:3 + 3 * N], 0.3 * X1[6 * 5 * f + 3:6 * 5 * f + 3 + 3 * N])
    # a uniform velocity gives dt V / dL in every segment
    f3 = OL.features(fil_off, Y, q, F, np.tile([1.0, 2.0, 3.0], (15, 1)), Xj, X1, X2, **kw)
    assert np.allclose(f3[:, 10 * N:13 * N].reshape(3, N, 3), 0.7 * np.array([1.0, 2.0, 3.0]) / 2.2)


def test_target_and_first_iterate_are_inverse():
    rng = np.random.default_rng(5)
    fil_off, *_ , (Xs, X0, _) = _fake_state(rng)
    kw = dict(dL=2.2, grav=(0, 0, -2.0), KB=1.0)
    t = OL.target(fil_off, Xs, X0, **kw)
    assert np.allclose(OL.target(fil_off, X0, X0, **kw), 0)
    assert np.allclose(OL.first_iterate(fil_off, X0, t, **kw), Xs, atol=1e-12)
    # the multiplier slots are measured in units of the gravity force per segment
    assert np.isclose(t[0, -1], (Xs[6 * 5 - 1] - X0[6 * 5 - 1]) / 2.0)


def test_base_is_extrapolation_plus_last_correction():
    """The learned start's base is X0 plus the unscaled last-changes features; it is X0
    before three steps of history and for tethered filaments, and a history linear in time
    adds nothing to Y_1 and Lambda."""
    rng = np.random.default_rng(6)
    fil_off, Y, q, F, V, (Xj, X1, X2) = _fake_state(rng)
    X0 = rng.standard_normal(Xj.shape)
    kw = dict(dL=2.2, dt=0.7, grav=(0, 0, -2.0), KB=1.0)
    N = 5
    feats = OL.features(fil_off, Y, q, F, V, Xj, X1, X2, **kw)
    sc = OL.slot_scales(N, kw["dL"], OL.force_scale(kw["grav"], kw["KB"], kw["dL"]))
    Xb = OL.base(fil_off, X0, Xj, X1, X2, step=3)
    for f in range(3):
        assert np.allclose(Xb[30 * f:30 * (f + 1)] - X0[30 * f:30 * (f + 1)], feats[f, 13 * N:] * sc, atol=1e-12)
    assert np.array_equal(OL.base(fil_off, X0, Xj, X1, X2, step=2), X0)
    Xt = OL.base(fil_off, X0, Xj, X1, X2, step=3, tether=[0, 1, 0])
    assert np.array_equal(Xt[30:60], X0[30:60]) and np.array_equal(Xt[:30], Xb[:30])
    Xl = OL.base(fil_off, X0, Xj, Xj - 0.3 * X1, Xj - 0.6 * X1, step=5)
    for f in range(3):
        a = 30 * f
        assert np.allclose(Xl[a:a + 3], X0[a:a + 3], atol=1e-12)
        assert np.allclose(Xl[a + 3 + 3 * N:a + 30], X0[a + 3 + 3 * N:a + 30], atol=1e-12)
        assert np.allclose(Xl[a + 3:a + 3 + 3 * N] - X0[a + 3:a + 3 + 3 * N], 0.3 * X1[a + 3:a + 3 + 3 * N])
