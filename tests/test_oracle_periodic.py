"""The oracle's periodic-box steps (the force-coupling-method mobility of Sec. 2.7.2 in
place of the RPY apply, the steric barrier of Sec. 2.6 between nearest periodic
images) pinned to what fixes them independently:

* the nearest-image steric force of two segments across a boundary is the unbounded
  force of the same two segments brought side by side, and the periodic forces do
  not change when any segment moves by a box vector;
* the mobility hook is pure plumbing: handing it the RPY apply reproduces the built-in
  residual to the last bit;
* a whole periodic step is invariant under moving filaments by box vectors, on a
  configuration whose only steric contact is between nearest images;
* with a zero force and torque field the FCM mobility returns zero velocities, so a
  straight filament with no load stays put (the drift-free special case).
"""
import numpy as np

import oracle
from oracle import fcm
from paper_1903_12609_amd import synth

import periodic_cases as pc


def test_steric_between_nearest_images():
    L = np.array([20.0, 18.0, 16.0])
    a, chi, FS = 1.0, 1.1, 3.0
    seg_fil = np.array([0, 1])
    Yp = np.array([[0.3, 5.0, 5.0], [L[0] - 0.7, 5.2, L[2] + 4.4]])  # nearest images 1.0, -0.2, 0.6 apart
    Yu = np.array([[0.3, 5.0, 5.0], [-0.7, 5.2, 4.4]])                # the same pair side by side
    Fp = oracle.steric(Yp, seg_fil, a, chi, FS, L=L)
    Fu = oracle.steric(Yu, seg_fil, a, chi, FS)
    assert np.abs(Fu).max() > 0.1
    np.testing.assert_allclose(Fp, Fu, rtol=1e-13, atol=0)
    assert np.abs(oracle.steric(Yp, seg_fil, a, chi, FS)).max() == 0.0  # unbounded: far apart
    # a dense cloud: moving segments by box vectors changes nothing
    rng = np.random.default_rng(4)
    Y = rng.uniform(0, L, (60, 3))
    sf = np.arange(60) // 6
    F0 = oracle.steric(Y, sf, a, chi, FS, L=L)
    assert np.count_nonzero(np.abs(F0).sum(1)) > 10
    Y2 = Y + rng.integers(-2, 3, (60, 3)) * L
    np.testing.assert_allclose(oracle.steric(Y2, sf, a, chi, FS, L=L), F0, rtol=1e-10, atol=1e-12 * np.abs(F0).max())
    assert abs(F0.sum(0)).max() <= 1e-12 * np.abs(F0).max()  # pairwise equal and opposite


def test_mobility_hook_is_plumbing():
    w = synth.sediment_suspension(M=4, N=10, side=30.0, seed=31, dt_over_T=1 / 30)
    p = dict(w.params)
    o1 = oracle.Sim(w.fil_off, w.Y, w.q, **p)
    o2 = oracle.Sim(w.fil_off, w.Y, w.q,
                    mobility=lambda Y, F, T: oracle.rpy_apply(Y, F, T, p["a"], p["eta"]), **p)
    X = o1.initial_guess()
    X[3:] += np.random.default_rng(2).standard_normal(X.size - 3) * 0.01
    f1, r1 = o1.residual(X)
    f2, r2 = o2.residual(X)
    assert np.array_equal(f1, f2) and r1 == r2


def _run(shifted, steps=3):
    fo, Y, q, params = pc.contact_pair(shifted)
    o = oracle.Sim(fo, Y, q, periodic=pc.periodic(), **params)
    its = []
    for _ in range(steps):
        rc, rep = o.step()
        assert rc == 0
        its.append(rep.iters)
    return o, its


def test_periodic_step_invariant_under_box_shifts():
    fo, Y, q, params = pc.contact_pair(True)
    seg_fil = np.repeat(np.arange(3), 8)
    # the contact exists only between nearest images
    assert np.abs(oracle.steric(Y, seg_fil, params["a"], params["chi"], params["FS"], L=pc.BOX)).max() > 0
    assert np.abs(oracle.steric(Y, seg_fil, params["a"], params["chi"], params["FS"])).max() == 0
    o0, it0 = _run(False)
    o1, it1 = _run(True)
    assert it0 == it1, (it0, it1)
    scale = np.abs(o0.Y - pc.contact_pair(False)[1]).max()  # displacement over the steps
    assert scale > 1e-3
    assert np.abs(o1.Y - pc.shift_of() - o0.Y).max() <= 1e-9 * scale
    assert np.abs(o1.q - o0.q).max() <= 1e-9


def test_unloaded_filament_stays_put():
    Y = np.array([[1.0, 2.0, 3.0], [3.2, 2.0, 3.0]])
    V, W = fcm.fcm_apply(Y, np.zeros((2, 3)), np.zeros((2, 3)), 1.0, 1.0, pc.BOX, pc.GRID)
    assert np.abs(V).max() == 0.0 and np.abs(W).max() == 0.0
    fo, Y, q, params = pc.contact_pair(False)
    params = dict(params, grav=(0.0, 0.0, 0.0))
    fo, Y, q = fo[:2], Y[16:24], q[16:24]  # the third filament alone, straight, no load
    o = oracle.Sim(fo, Y, q, periodic=pc.periodic(), **params)
    rc, rep = o.step()
    assert rc == 0
    assert np.abs(o.Y - Y).max() <= 1e-12
