"""The oracle's geometric switch (Sec. 5.2.2) pinned to its definition and to the beat it
must produce: the logistic transition between the old and the new torque, the reversal
when the base tangent reaches the extreme it is driven towards, and a pinned filament in
free space that beats between the two extremes with alternating drive."""
import math

import numpy as np

import oracle
from oracle import cilia

import cilia_cases as cc


def test_switch_logic():
    sw = cilia.GeometricSwitch([0, 1], [2], cc.AXIS, cc.NORMAL, 0.5, 3.0, 1.0, 4)
    t = np.zeros((1, 3))
    upright = np.array([[math.cos(-math.pi / 4), 0.0, math.sin(-math.pi / 4), 0.0]])  # tangent along z
    sw.update(upright, t)
    assert sw.dir[0] == 1 and np.allclose(t[0], [0.0, 3.0, 0.0])  # full tau_pos from the start
    assert abs(sw.theta(upright[0])) <= 1e-15
    # tilt the tangent to +0.6 rad about y: past theta_max, the drive reverses
    a = -math.pi / 4 + 0.3
    tilted = np.array([[math.cos(a), 0.0, math.sin(a), 0.0]])
    assert abs(sw.theta(tilted[0]) - 0.6) <= 1e-12
    sw.update(tilted, t)
    assert sw.dir[0] == -1 and sw.age[0] == 0
    lg = lambda k: 1.0 / (1.0 + math.exp(-12.0 * (k / 4 - 0.5)))
    assert abs(t[0, 1] - (3.0 + (-1.0 - 3.0) * lg(0))) <= 1e-15
    for k in range(1, 6):
        sw.update(tilted, t)
        want = -1.0 if k >= 4 else 3.0 + (-1.0 - 3.0) * lg(k)
        assert abs(t[0, 1] - want) <= 1e-15, (k, t[0, 1], want)


def test_pinned_cilia_beat_in_free_space():
    fo, Y, q, p = cc.pair()
    text = np.zeros((Y.shape[0], 3))
    o = oracle.Sim(fo, Y, q, text=text, **p)
    sw = cilia.GeometricSwitch(fo, p["tether"], cc.AXIS, cc.NORMAL, cc.THETA_MAX, cc.TAU_POS, cc.TAU_NEG, cc.N_TR)
    dirs, thetas = [], []
    for _ in range(30):
        sw.update(o.q, text)
        rc, rep = o.step()
        assert rc == 0
        dirs.append(sw.dir.copy())
        thetas.append(sw.theta(o.q[0]))
    d = np.array(dirs)[:, 0]
    assert (np.diff(d) != 0).sum() >= 2  # reversed at least twice
    assert max(thetas) >= cc.THETA_MAX and min(thetas) <= -cc.THETA_MAX
    assert np.abs(o.Y[0] - Y[0]).max() == 0.0 and np.abs(o.Y[cc.N] - Y[cc.N]).max() == 0.0  # pinned
