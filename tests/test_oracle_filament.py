"""Pins of the oracle's filament mechanics: discrete quaternion moment
(Sec. 2.9.2), internal forces and torques (Sec. 2.5), robot-arm reconstruction
(Sec. 2.9.3)."""
import math

import numpy as np
import pytest

import oracle
from paper_1903_12609_amd import synth


def zrot(th):
    return np.array([math.cos(th / 2), 0, 0, math.sin(th / 2)])


def xrot(th):
    return np.array([math.cos(th / 2), math.sin(th / 2), 0, 0])


@pytest.mark.parametrize("dth", [0.0, 0.01, 0.3, -1.1, 2.5])
def test_planar_bend_closed_form(dth):
    """q_n = rotation by theta_n about e_z: M = (4 K_B / dL) sin(dtheta / 4) e_z."""
    KB, KT, dL = 1.7, 0.6, 2.2
    th0 = 0.4
    M = oracle.moment(zrot(th0), zrot(th0 + dth), [0, 0, 0], dL, KB, KT)
    assert np.allclose(M, [0, 0, 4 * KB / dL * math.sin(dth / 4)], atol=1e-15)
    # consistent with the planar model K_B t_n x t_{n+1} / dL to third order
    if abs(dth) <= 0.3:
        tn = np.array([math.cos(th0), math.sin(th0), 0])
        tn1 = np.array([math.cos(th0 + dth), math.sin(th0 + dth), 0])
        assert np.allclose(M, KB * np.cross(tn, tn1) / dL, atol=KB / dL * abs(dth) ** 3)


@pytest.mark.parametrize("dphi", [0.05, -0.7, 1.9])
def test_pure_twist_closed_form(dphi):
    KB, KT, dL = 1.7, 0.6, 2.2
    M = oracle.moment(xrot(0.3), xrot(0.3 + dphi), [0, 0, 0], dL, KB, KT)
    assert np.allclose(M, [4 * KT / dL * math.sin(dphi / 4), 0, 0], atol=1e-15)


def test_preferred_curvature_arc_is_stress_free():
    dL, dth = 2.2, 0.2
    knu = 4 / dL * math.sin(dth / 4)
    M = oracle.moment(zrot(0.1), zrot(0.1 + dth), [0, 0, knu], dL, 1.0, 1.0)
    assert np.allclose(M, 0, atol=1e-16)


def test_moment_matches_frame_vector_form_to_second_order():
    """The frame-vector moment of Appendix B.2 (K_B t_m x t_{m+1}/dL + K_T beta (t_m+t_{m+1})/2,
    beta = (mu_{m+1}.nu_m - mu_m.nu_{m+1})/(2 dL)) agrees with the quaternion moment
    up to O(delta^2) relative for a small general rotation delta between segments."""
    rng = np.random.default_rng(30)
    KB, KT, dL = 1.3, 0.55, 2.2
    for _ in range(10):
        g = rng.standard_normal(4)
        q0 = g / np.linalg.norm(g)
        w = rng.standard_normal(3)
        w /= np.linalg.norm(w)
        delta = 1e-3
        q1 = oracle.qmul(oracle.qexp(delta * w), q0)
        R0, R1 = oracle.qrot(q0), oracle.qrot(q1)
        t0, m0, n0 = R0.T
        t1, m1, n1 = R1.T
        beta = (m1 @ n0 - m0 @ n1) / (2 * dL)
        Mfv = KB * np.cross(t0, t1) / dL + 0.5 * KT * beta * (t0 + t1)
        M = oracle.moment(q0, q1, [0, 0, 0], dL, KB, KT)
        assert np.linalg.norm(M - Mfv) <= 5 * delta ** 2 * np.linalg.norm(M)


def _random_filament(N, seed, bend=0.3):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(4)
    q = [g / np.linalg.norm(g)]
    for _ in range(N - 1):
        w = rng.standard_normal(3) * bend
        q.append(oracle.qmul(oracle.qexp(w), q[-1]))
    q = np.array(q)
    return q, synth.chain(rng.standard_normal(3), q)


def test_internal_force_balances():
    """Sum of F^C vanishes and sum of T^E vanishes (free ends, Sec. 2.5); with the
    constraints met, sum of (T^C + T^E + Y x F^C) vanishes too."""
    KB, KT, dL = 1.0, 0.8, 2.2
    for seed in range(5):
        N = 12
        q, Y = _random_filament(N, seed)
        rng = np.random.default_rng(seed + 50)
        Lam = rng.standard_normal((N - 1, 3))
        kap = rng.standard_normal((N - 1, 3)) * 0.1
        F, T = oracle.internal_forces(q, Lam, kap, dL, KB, KT)
        assert np.allclose(F.sum(0), 0, atol=1e-14)
        Fz, Tz = oracle.internal_forces(q, np.zeros((N - 1, 3)), kap, dL, KB, KT)
        assert np.allclose(Fz, 0) and np.allclose(Tz.sum(0), 0, atol=1e-14)   # sum of T^E
        assert np.allclose((T + np.cross(Y, F)).sum(0), 0, atol=1e-12)
        assert np.allclose(F[0], Lam[0]) and np.allclose(F[-1], -Lam[-1])       # free ends


def test_internal_forces_straight_filament_has_no_elastic_torque():
    q = np.tile(synth.random_unit_quaternion(np.random.default_rng(3)), (8, 1))
    F, T = oracle.internal_forces(q, np.zeros((7, 3)), np.zeros((7, 3)), 2.2, 1.0, 1.0)
    assert np.allclose(T, 0, atol=1e-16) and np.allclose(F, 0)


def test_reconstruction_robot_arm_and_unit_quaternions():
    """Y_n = Y_1 + dL/2 sum (t_{m-1} + t_m) satisfies every inextensibility
    constraint g_{n+1/2} = 0, and q = exp(u) . q^j stays unit."""
    w = synth.sediment_suspension(M=6, N=9, side=60.0, seed=5)
    sim = oracle.Sim(w.fil_off, w.Y, w.q, **w.params)
    rng = np.random.default_rng(1)
    X = rng.standard_normal(6 * w.S) * 0.5
    Y, q = sim.reconstruct(X)
    assert np.abs(np.linalg.norm(q, axis=1) - 1).max() < 1e-15
    for f in range(w.M):
        s0, s1 = w.fil_off[f], w.fil_off[f + 1]
        t = np.array([oracle.qrot(qq)[:, 0] for qq in q[s0:s1]])
        g = Y[s0 + 1:s1] - Y[s0:s1 - 1] - 0.5 * w.params["dL"] * (t[:-1] + t[1:])
        assert np.abs(g).max() < 1e-13 * w.params["dL"]
        assert np.allclose(Y[s0], X[6 * s0:6 * s0 + 3])
    # X = (Y_1, 0, ...) reproduces the generator's own chain
    X0 = np.zeros(6 * w.S)
    for f in range(w.M):
        X0[6 * w.fil_off[f]:6 * w.fil_off[f] + 3] = w.Y[w.fil_off[f]]
    Y0, q0 = sim.reconstruct(X0)
    assert np.allclose(Y0, w.Y, atol=1e-12) and np.allclose(q0, w.q, atol=1e-15)
