"""GPU parity of the periodic-box steps (the force-coupling-method mobility of
Sec. 2.7.2 in place of the RPY apply; the steric barrier of Sec. 2.6 between nearest
periodic images) against the oracle's, through fil_set_periodic_fcm: residuals at
perturbed iterates, whole trajectories, the invariance under moving filaments by box
vectors, and the argument checks."""
import numpy as np
import pytest

import oracle

import periodic_cases as pc
from gpu_util import rel_l2

pytestmark = pytest.mark.gpu


def _cases():
    fo, Y, q, params = pc.contact_pair(False)
    w = pc.small_monolayer()
    return {"contact_pair": (fo, Y, q, params), "monolayer6x8": (w.fil_off, w.Y, w.q, w.params)}


CASES = _cases()


def _pair(name, graph=8):
    import paper_1903_12609_amd as fil
    fo, Y, q, params = CASES[name]
    o = oracle.Sim(fo, Y, q, periodic=pc.periodic(), **params)
    g = fil.Sim(fo, Y, q, params, graph=graph)
    g.set_periodic_fcm(pc.BOX, pc.GRID, 7.5)
    return o, g


def _to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("name", list(CASES))
def test_periodic_residual_parity(name):
    print("case", name, flush=True)
    o, g = _pair(name)
    fo = CASES[name][0]
    rng = np.random.default_rng(8)
    X0 = o.initial_guess()
    for trial in range(3):
        X = X0.copy()
        for f in range(len(fo) - 1):
            s0, N = fo[f], fo[f + 1] - fo[f]
            X[6 * s0 + 3:6 * s0 + 3 + 3 * N] += rng.standard_normal(3 * N) * 0.05
            X[6 * s0 + 3 + 3 * N:6 * (s0 + N)] += rng.standard_normal(3 * (N - 1)) * 0.02
        f_or, _ = o.residual(X)
        f_gpu = g.residual(_to_dev(X)).cpu().numpy()
        # hipFFT against numpy's FFT, and atomics in the spreading: rounding only
        assert rel_l2(f_gpu, f_or) <= 1e-11, rel_l2(f_gpu, f_or)


@pytest.mark.parametrize("name", list(CASES))
def test_periodic_trajectory_parity(name, steps=5):
    """Both sides at tol 1e-8; equal iteration counts every step, positions to 1e-8."""
    print("case", name, steps, flush=True)
    o, g = _pair(name)
    for j in range(steps):
        rc, rep = o.step()
        assert rc == 0
        r = g.step()[0]
        assert r["converged"], (j, r)
        assert r["iters"] == rep.iters, (j, r["iters"], rep.iters)
    Y, q, X = g.read_state()
    assert rel_l2(Y, o.Y) <= 1e-8 and rel_l2(q, o.q) <= 1e-8, (rel_l2(Y, o.Y), rel_l2(q, o.q))


def test_periodic_box_shift_invariance():
    """The contact between nearest images only (filaments moved by -Lx and -Ly) gives the
    same motion as the contact side by side."""
    import paper_1903_12609_amd as fil
    out = []
    for shifted in (False, True):
        fo, Y, q, params = pc.contact_pair(shifted)
        g = fil.Sim(fo, Y, q, params, graph=8)
        g.set_periodic_fcm(pc.BOX, pc.GRID, 7.5)
        its = [g.step()[0]["iters"] for _ in range(3)]
        out.append((g.read_state()[0], g.read_state()[1], its, Y))
    (Y0, q0, it0, Yinit), (Y1, q1, it1, _) = out
    assert it0 == it1, (it0, it1)
    scale = np.abs(Y0 - Yinit).max()
    assert scale > 1e-3
    assert np.abs(Y1 - pc.shift_of() - Y0).max() <= 1e-9 * scale
    assert np.abs(q1 - q0).max() <= 1e-9


def test_periodic_refusals():
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd._native import FilError
    fo, Y, q, params = CASES["contact_pair"]
    g = fil.Sim(fo, Y, q, params)
    with pytest.raises(FilError):
        g.set_periodic_fcm((4.0, 40.0, 40.0), (32, 32, 32))  # a length below 4 chi a
    with pytest.raises(FilError):
        g.set_periodic_fcm(pc.BOX, (512, 512, 256))  # the Gaussian support spans over 65 points
    g.set_periodic_fcm(pc.BOX, pc.GRID)
    with pytest.raises(FilError):
        g.set_periodic_fcm(pc.BOX, pc.GRID)  # already set
    g.step()
    g2 = fil.Sim(fo, Y, q, params)
    g2.step()
    with pytest.raises(FilError):
        g2.set_periodic_fcm(pc.BOX, pc.GRID)  # after the first step
    g3 = fil.Sim(fo, Y, q, params, prec="f32tile")
    with pytest.raises(FilError):
        g3.set_periodic_fcm(pc.BOX, pc.GRID)
    g4 = fil.Sim(fo, Y, q, params, susp_fil_off=np.array([0, 2, 3]))
    with pytest.raises(FilError):
        g4.set_periodic_fcm(pc.BOX, pc.GRID)
