"""GPU parity of the RPY mobility apply against the FP64 oracle (Sec. 2.7.1)."""
import numpy as np
import pytest

import oracle
from paper_1903_12609_amd import synth

from gpu_util import dev, host, rel_l2

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12      # relative L2, FP64 pair math
F32_TOL = 1e-5       # relative L2 bound for the FP32-tile path (error is reported, not tuned)


def _apply(Y, F, T, prec, a=1.0, eta=1.0):
    import paper_1903_12609_amd as fil
    V, W = fil.rpy_mobility_apply(dev(Y), dev(F), dev(T), a, eta, prec)
    return host(V), host(W)


def _cases():
    rng = np.random.default_rng(0)
    yield "single", np.zeros((1, 3)), rng.standard_normal((1, 3)), rng.standard_normal((1, 3)), 1.0, 1.0
    Y = np.array([[0, 0, 0], [2.2, 0, 0.0]])
    yield "pair", Y, rng.standard_normal((2, 3)), rng.standard_normal((2, 3)), 1.0, 1.0
    for S in (37, 300, 1037):
        Y, F, T = synth.rpy_throughput_inputs(S, seed=S)
        yield "structured%d" % S, Y, F, T, 1.0, 1.0
    Y = rng.uniform(0, 9.0, (257, 3))                 # dense cloud: many overlapping pairs
    yield "overlapping257", Y, rng.standard_normal((257, 3)), rng.standard_normal((257, 3)), 1.0, 1.0
    Y = rng.uniform(0, 60.0, (777, 3))
    yield "cloud777_a0.7_eta2.5", Y, rng.standard_normal((777, 3)), rng.standard_normal((777, 3)), 0.7, 2.5
    w = synth.sediment_suspension()
    rng2 = np.random.default_rng(3)
    yield "sediment2000", w.Y, rng2.standard_normal((w.S, 3)), rng2.standard_normal((w.S, 3)), 1.0, 1.0


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_rpy_f64_parity(case):
    name, Y, F, T, a, eta = case
    print("case", name, Y.shape[0], flush=True)
    V0, W0 = oracle.rpy_apply(Y, F, T, a, eta, nthreads=8)
    V, W = _apply(Y, F, T, "f64", a, eta)
    assert rel_l2(V, V0) <= F64_TOL and rel_l2(W, W0) <= F64_TOL, (rel_l2(V, V0), rel_l2(W, W0))


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_rpy_f32tile_error_bound(case):
    name, Y, F, T, a, eta = case
    print("case", name, Y.shape[0], flush=True)
    V0, W0 = oracle.rpy_apply(Y, F, T, a, eta, nthreads=8)
    V, W = _apply(Y, F, T, "f32tile", a, eta)
    ev, ew = rel_l2(V, V0), rel_l2(W, W0)
    print("f32tile rel L2 V %.3e W %.3e" % (ev, ew))
    assert np.isfinite(V).all() and np.isfinite(W).all()
    assert ev <= F32_TOL and ew <= F32_TOL


@pytest.mark.parametrize("S", [16000, 32000])
def test_rpy_full_size_sampled(S):
    """Full-size applies (the launch configuration the benchmark times) checked
    on sampled targets the oracle computes one by one."""
    print("full size", S, flush=True)
    Y, F, T = synth.rpy_throughput_inputs(S, seed=7)
    idx = np.unique(np.concatenate([[0, 1, S // 2, S - 2, S - 1], np.random.default_rng(1).integers(0, S, 59)]))
    v0, w0 = oracle.rpy_apply_targets(Y, F, T, 1.0, 1.0, idx, nthreads=8)
    V, W = _apply(Y, F, T, "f64")
    assert rel_l2(V[idx], v0) <= F64_TOL and rel_l2(W[idx], w0) <= F64_TOL
    V, W = _apply(Y, F, T, "f32tile")
    print("f32tile sampled rel L2 V %.3e W %.3e" % (rel_l2(V[idx], v0), rel_l2(W[idx], w0)))
    assert rel_l2(V[idx], v0) <= F32_TOL and rel_l2(W[idx], w0) <= F32_TOL


@pytest.mark.parametrize("prec", ["f64", "f32tile"])
def test_rpy_large_path_overlaps(prec):
    """The large-size kernels (S >= 12,000: two targets per lane) and the batched items on a
    dense cloud where many pairs overlap (mean spacing ~1.7a < 2a): sampled targets against
    the oracle, so the overlap branch of those kernel forms is exercised."""
    import paper_1903_12609_amd as fil
    S = 12288
    rng = np.random.default_rng(31)
    Y = rng.uniform(0.0, 40.0, (S, 3))
    F, T = rng.standard_normal((S, 3)), rng.standard_normal((S, 3))
    idx = np.unique(np.concatenate([[0, 1, S // 2, S - 1], rng.integers(0, S, 60)]))
    v0, w0 = oracle.rpy_apply_targets(Y, F, T, 1.0, 1.0, idx, nthreads=8)
    tol = F64_TOL if prec == "f64" else F32_TOL
    V, W = _apply(Y, F, T, prec)
    ev, ew = rel_l2(V[idx], v0), rel_l2(W[idx], w0)
    print("%s stand-alone sampled rel L2 V %.3e W %.3e" % (prec, ev, ew))
    assert ev <= tol and ew <= tol
    off = np.array([0, S], dtype=np.int64)
    plan = fil.RpyBatch(off, prec)
    Vb, Wb = plan.apply(dev(Y), dev(F), dev(T), 1.0, 1.0)
    Vb, Wb = host(Vb), host(Wb)
    plan.close()
    ev, ew = rel_l2(Vb[idx], v0), rel_l2(Wb[idx], w0)
    print("%s batched sampled rel L2 V %.3e W %.3e" % (prec, ev, ew))
    assert ev <= tol and ew <= tol


def test_rpy_deterministic_and_empty():
    import torch
    import paper_1903_12609_amd as fil
    Y, F, T = synth.rpy_throughput_inputs(5000, seed=9)
    Yd, Fd, Td = dev(Y), dev(F), dev(T)
    for prec in ("f64", "f32tile"):
        V1, W1 = fil.rpy_mobility_apply(Yd, Fd, Td, 1.0, 1.0, prec)
        V2, W2 = fil.rpy_mobility_apply(Yd, Fd, Td, 1.0, 1.0, prec)
        torch.cuda.synchronize()
        assert torch.equal(V1, V2) and torch.equal(W1, W2)
    z = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    V, W = fil.rpy_mobility_apply(z, z, z)
    assert V.shape == (3, 0)


@pytest.mark.parametrize("prec", ["f64", "f32tile"])
def test_rpy_batched_wave_and_item_boundaries(prec):
    """Suspension sizes around the batched work item's boundaries (a wave owns 128
    consecutive targets, an item 512): every target of every suspension, the last ones
    included, equals its own oracle apply, whether its wave is full, partly filled, or
    (past the suspension's end) skips the item."""
    import paper_1903_12609_amd as fil
    rng = np.random.default_rng(23)
    sizes = [127, 128, 129, 255, 383, 384, 385, 511, 512, 513, 640, 2]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    Y = np.concatenate([synth.rpy_throughput_inputs(n, seed=40 + i)[0] for i, n in enumerate(sizes)])
    F, T = rng.standard_normal((off[-1], 3)), rng.standard_normal((off[-1], 3))
    plan = fil.RpyBatch(off, prec)
    V, W = plan.apply(dev(Y), dev(F), dev(T), 1.0, 1.0)
    V, W = host(V), host(W)
    plan.close()
    tol = F64_TOL if prec == "f64" else F32_TOL
    for i in range(len(sizes)):
        a, b = off[i], off[i + 1]
        V0, W0 = oracle.rpy_apply(Y[a:b], F[a:b], T[a:b], 1.0, 1.0, nthreads=8)
        ev, ew = rel_l2(V[a:b], V0), rel_l2(W[a:b], W0)
        # the last target alone (the end of the suspension's last wave)
        el = max(rel_l2(V[b - 1:b], V0[-1:]), rel_l2(W[b - 1:b], W0[-1:]))
        print("suspension %d (S=%d): rel L2 V %.3e W %.3e, last target %.3e" % (i, b - a, ev, ew, el))
        assert ev <= tol and ew <= tol and el <= 10 * tol


@pytest.mark.parametrize("prec", ["f64", "f32tile"])
def test_rpy_batched_matches_separate_applies(prec):
    """Ragged suspensions in one persistent launch (a plan built once, applied twice): each
    suspension's velocities equal its own oracle apply (FP64 to 1e-12, FP32 tiles within the
    FP32 bound), and the two applies are bitwise equal."""
    import torch
    import paper_1903_12609_amd as fil
    rng = np.random.default_rng(17)
    sizes = [1, 37, 600, 0, 129, 2500, 16]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    Ys = [synth.rpy_throughput_inputs(n, seed=20 + i)[0] if n else np.zeros((0, 3)) for i, n in enumerate(sizes)]
    Y = np.concatenate(Ys)
    F, T = rng.standard_normal((off[-1], 3)), rng.standard_normal((off[-1], 3))
    plan = fil.RpyBatch(off, prec)
    V1, W1 = plan.apply(dev(Y), dev(F), dev(T), 0.9, 1.3)
    V2, W2 = plan.apply(dev(Y), dev(F), dev(T), 0.9, 1.3)
    torch.cuda.synchronize()
    assert torch.equal(V1, V2) and torch.equal(W1, W2)
    V, W = host(V1), host(W1)
    tol = F64_TOL if prec == "f64" else F32_TOL
    for i in range(len(sizes)):
        a, b = off[i], off[i + 1]
        if a == b:
            continue
        V0, W0 = oracle.rpy_apply(Y[a:b], F[a:b], T[a:b], 0.9, 1.3, nthreads=8)
        ev, ew = rel_l2(V[a:b], V0), rel_l2(W[a:b], W0)
        print("suspension %d (S=%d): rel L2 V %.3e W %.3e" % (i, b - a, ev, ew))
        assert ev <= tol and ew <= tol
    plan.close()
