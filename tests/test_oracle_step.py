"""Pins of the oracle's implicit step: residual of the reduced system
(Sec. 2.9.3), explicit approximate Jacobian J0 (Appendix B.2), bad Broyden
(Alg. 2) and the BDF2 / Lie-group update."""
import math

import numpy as np
import pytest

import oracle
from paper_1903_12609_amd import synth


def fd_jacobian(fun, X, h_rel=1e-6):
    f0 = fun(X)
    J = np.zeros((len(f0), len(X)))
    for i in range(len(X)):
        h = h_rel * max(1.0, abs(X[i]))
        e = np.zeros_like(X)
        e[i] = h
        J[:, i] = (fun(X + e) - fun(X - e)) / (2 * h)
    return J


def _small_sim(M=1, N=6, seed=9, **over):
    w = synth.sediment_suspension(M=M, N=N, side=15.0 * M, seed=seed, dt_over_T=0.05)
    p = dict(w.params)
    p.update(over)
    return w, oracle.Sim(w.fil_off, w.Y, w.q, **p)


@pytest.mark.parametrize("step_index", [0, 3])
def test_j0_equals_drag_jacobian_at_straight_untwisted_state(step_index):
    """At u = 0 on a straight, untwisted filament every approximation of
    Appendix B.2 (Taylor dexpinv, frame-vector moment, d t/d u = [x t]) is exact
    to first order, so J0 must equal the Jacobian of the drag-only residual f0."""
    q0 = synth.random_unit_quaternion(np.random.default_rng(4))
    N = 6
    q = np.tile(q0, (N, 1))
    Y = synth.chain(np.zeros(3), q)
    sim = oracle.Sim([0, N], Y, q, dt=3.7, drag_only=1, KB=1.3, KT=0.7)
    sim.St.step = step_index
    rng = np.random.default_rng(5)
    X = np.zeros(6 * N)
    X[:3] = Y[0] + rng.standard_normal(3)
    X[3 + 3 * N:] = rng.standard_normal(3 * (N - 1))       # arbitrary multipliers
    J0 = sim.j0_filament(0, X)
    Jfd = fd_jacobian(lambda x: sim.residual(x)[0], X)
    assert np.allclose(J0, Jfd, rtol=0, atol=1e-7 * np.abs(Jfd).max())


def test_j0_tethered_equals_drag_jacobian_at_straight_state():
    """Reading R11: clamped base, multipliers lambda_1, lambda_2 in the Y_1, u_1 slots."""
    N = 5
    q0 = np.array([math.cos(-math.pi / 4), 0, math.sin(-math.pi / 4), 0])
    q = np.tile(q0, (N, 1))
    Y = synth.chain(np.array([1.0, 2.0, 0.0]), q)
    sim = oracle.Sim([0, N], Y, q, dt=2.0, drag_only=1, tether=[1], base=Y[:1])
    sim.St.step = 2
    rng = np.random.default_rng(6)
    X = np.zeros(6 * N)
    X[:6] = rng.standard_normal(6)
    X[3 + 3 * N:] = rng.standard_normal(3 * (N - 1))
    J0 = sim.j0_filament(0, X)
    Jfd = fd_jacobian(lambda x: sim.residual(x)[0], X)
    assert np.allclose(J0, Jfd, rtol=0, atol=1e-7 * np.abs(Jfd).max())


def test_j0_multiplier_columns_at_rotated_state():
    """Columns of J0 for the multipliers Lambda involve no frame-vector
    approximation: only the three-term Taylor dexpinv (Appendix B.2), whose error
    is O(|u|^4).  At |u| ~ 0.1 they must match the drag-only Jacobian to ~1e-6."""
    q0 = synth.random_unit_quaternion(np.random.default_rng(8))
    N = 6
    q = synth.bent_quaternions(q0, N, 0.2)
    Y = synth.chain(np.zeros(3), q)
    sim = oracle.Sim([0, N], Y, q, dt=2.5, drag_only=1, KB=1.1, KT=0.9)
    sim.St.step = 4
    rng = np.random.default_rng(9)
    X = np.zeros(6 * N)
    X[:3] = Y[0]
    X[3:3 + 3 * N] = rng.standard_normal(3 * N) * 0.06
    X[3 + 3 * N:] = rng.standard_normal(3 * (N - 1))
    J0 = sim.j0_filament(0, X)
    Jfd = fd_jacobian(lambda x: sim.residual(x)[0], X)
    cols = slice(3 + 3 * N, 6 * N)
    assert np.allclose(J0[:, cols], Jfd[:, cols], rtol=0, atol=2e-6 * np.abs(Jfd[:, cols]).max())


def test_j0_close_to_drag_jacobian_when_bent():
    """Away from the straight state J0 stays a first-order approximation of the
    drag-only Jacobian: the relative mismatch shrinks with the bend."""
    errs = []
    for bend in (0.04, 0.02):
        q0 = synth.random_unit_quaternion(np.random.default_rng(7))
        N = 6
        q = synth.bent_quaternions(q0, N, bend)
        Y = synth.chain(np.zeros(3), q)
        sim = oracle.Sim([0, N], Y, q, dt=3.0, drag_only=1)
        sim.St.step = 3
        X = np.zeros(6 * N)
        X[:3] = Y[0]
        J0 = sim.j0_filament(0, X)
        Jfd = fd_jacobian(lambda x: sim.residual(x)[0], X)
        errs.append(np.abs(J0 - Jfd).max() / np.abs(Jfd).max())
    assert errs[0] < 1e-2 and errs[1] < 0.6 * errs[0]


@pytest.mark.parametrize("M", [1, 2])
def test_broyden_root_equals_newton_root(M):
    """Alg. 2 converges to the same root as Newton's method (Sec. 3) with a
    central finite-difference Jacobian."""
    w, sim = _small_sim(M=M, N=5, seed=11 + M, tol=1e-12, kmax=200)
    X0 = sim.initial_guess()
    Xb, rc, rep = sim.broyden(X0)
    assert rc == 0 and rep.resid <= 1e-12
    X = X0.copy()
    for _ in range(30):
        f, r = sim.residual(X)
        if r <= 1e-13:
            break
        J = fd_jacobian(lambda x: sim.residual(x)[0], X, h_rel=1e-7)
        X = X - np.linalg.solve(J, f)
    assert sim.residual(X)[1] <= 1e-12
    assert np.abs(Xb - X).max() <= 1e-9 * max(1.0, np.abs(X).max())


def test_single_filament_100_steps_invariants():
    """Each step meets the tolerance; quaternions stay unit to round-off
    (Sec. 2.9.3, multiplicative update); constraints hold (robot arm)."""
    w = synth.single_filament(N=15)
    sim = oracle.Sim(w.fil_off, w.Y, w.q, **w.params)
    for j in range(100):
        rc, rep = sim.step()
        assert rc == 0 and rep.resid <= w.params["tol"]
    assert np.abs(np.linalg.norm(sim.q, axis=1) - 1).max() <= 1e-14
    t = np.array([oracle.qrot(q)[:, 0] for q in sim.q])
    g = sim.Y[1:] - sim.Y[:-1] - 0.5 * w.params["dL"] * (t[:-1] + t[1:])
    assert np.abs(g).max() <= 1e-13 * w.params["dL"]
    # it sedimented (gravity along -z) and bent
    assert sim.Y[:, 2].mean() < -10 * w.params["dL"]


def test_single_segment_moves_on_exact_straight_line():
    """N = 1 under gravity: V = F / (6 pi eta a) is constant, so BDF1 then BDF2
    reproduce Y^j = Y^0 + j dt V exactly (to round-off)."""
    q = np.array([[1.0, 0, 0, 0]])
    Y = np.array([[0.5, -1.0, 2.0]])
    g = (0.1, -0.2, -0.3)
    sim = oracle.Sim([0, 1], Y, q, dt=2.0, grav=g, tol=1e-14)
    V = np.array(g) / (6 * math.pi)
    for j in range(1, 6):
        rc, rep = sim.step()
        assert rc == 0
        assert np.allclose(sim.Y[0], Y[0] + j * 2.0 * V, rtol=0, atol=1e-13)
    assert np.allclose(sim.q[0], q[0], atol=1e-15)


def test_tethered_active_filaments():
    """Clamped bases stay fixed, the base quaternion never changes, every step converges."""
    w = synth.active_array(nx=2, ny=1, N=8, spacing=20.0)
    sim = oracle.Sim(w.fil_off, w.Y, w.q, **w.params)
    base_q = sim.q[w.fil_off[:-1]].copy()
    for j in range(5):
        rc, rep = sim.step()
        assert rc == 0
    assert np.array_equal(sim.Y[w.fil_off[:-1]], w.params["base"])
    assert np.array_equal(sim.q[w.fil_off[:-1]], base_q)
    assert np.abs(sim.Y - w.Y).max() > 1e-3          # the drive bent them


@pytest.mark.slow
def test_second_order_in_time():
    """BDF2 is second order (Sec. 4.2): halving dt divides the error by ~4."""
    def run(dt_over_T, tol):
        w = synth.single_filament(N=10, dt_over_T=dt_over_T, tol=tol, kmax=200)
        sim = oracle.Sim(w.fil_off, w.Y, w.q, **w.params)
        n = int(round(2.0 / dt_over_T))
        for _ in range(n):
            rc, rep = sim.step()
            assert rc == 0
        return sim.Y.copy()
    ref = run(1 / 128, 1e-12)
    errs = [np.abs(run(h, 1e-11) - ref).max() for h in (1 / 8, 1 / 16, 1 / 32)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def test_j0_pinned_equals_drag_jacobian_at_straight_state():
    """Pinned base (position held, rotation free, as the cilia bases of Sec. 5.2.2):
    lambda_1 in the Y_1 slot, u_1 an ordinary unknown."""
    N = 5
    q0 = np.array([math.cos(-math.pi / 4), 0, math.sin(-math.pi / 4), 0])
    q = np.tile(q0, (N, 1))
    Y = synth.chain(np.array([1.0, 2.0, 0.0]), q)
    sim = oracle.Sim([0, N], Y, q, dt=2.0, drag_only=1, tether=[2], base=Y[:1])
    sim.St.step = 2
    rng = np.random.default_rng(7)
    X = np.zeros(6 * N)
    X[:3] = rng.standard_normal(3)
    X[3 + 3 * N:] = rng.standard_normal(3 * (N - 1))
    J0 = sim.j0_filament(0, X)
    Jfd = fd_jacobian(lambda x: sim.residual(x)[0], X)
    assert np.allclose(J0, Jfd, rtol=0, atol=1e-7 * np.abs(Jfd).max())


def test_pinned_filament_hangs_below_its_pin():
    """A pinned filament started 60 degrees from the vertical swings down under gravity
    and comes to rest hanging straight below the pin (the base never moves)."""
    N = 8
    th = math.radians(60.0)
    # tangent e_x rotated to (sin th, 0, -cos th): about y by -(pi/2 - th)
    q0 = np.array([math.cos(-(math.pi / 2 - th) / 2), 0, math.sin(-(math.pi / 2 - th) / 2), 0])
    q = np.tile(q0, (N, 1))
    Y = synth.chain(np.array([0.0, 0.0, 50.0]), q)
    params, T = synth.sedimentation_params(N, 10.0, 1.0, 1e-10, 200, steric=False)
    sim = oracle.Sim([0, N], Y, q, tether=[2], base=Y[:1], **params)
    for _ in range(60):
        rc, rep = sim.step()
        assert rc == 0
    t = np.array([oracle.qrot(qq)[:, 0] for qq in sim.q])
    assert np.abs(sim.Y[0] - Y[0]).max() == 0.0
    assert np.abs(t - np.array([0.0, 0.0, -1.0])).max() <= 1e-3
    assert abs(sim.Y[-1, 2] - (50.0 - (N - 1) * params["dL"])) <= 1e-2


def _motor_filament(Sp, N=10, d0=4.5977, tilt_deg=15.0):
    """A filament on a rotating motor (Sec. 5.2.1): base d0 from the z axis, tilted 15 degrees
    away from it; omega from the Sperm number Sp = zeta_perp omega L^4 / K_B, 0.05 rad per
    step."""
    tilt = math.radians(tilt_deg)
    phi = -(math.pi / 2 - tilt)
    q = np.tile([math.cos(phi / 2), 0, math.sin(phi / 2), 0], (N, 1))
    Y = synth.chain(np.array([d0, 0.0, 0.0]), q)
    L = N * synth.DL
    w = Sp / (4 * math.pi / (math.log(L) + 0.5) * L ** 4)
    sim = oracle.Sim([0, N], Y, q, dt=0.05 / w, tol=1e-10, kmax=100, tether=[3], base=Y[:1], motor_d0=d0,
                     motor_w=w)
    return sim, Y, (d0 + (N - 1) * synth.DL * math.sin(tilt))


def test_motor_filament_limits():
    """Low Sp: nearly rigid rotation, the free end at d0 + L sin(15 deg) from the axis; high
    Sp: the filament collapses towards the axis.  The base follows the motor's circle."""
    sim, Y, d_rigid = _motor_filament(0.1)
    for _ in range(20):
        rc, rep = sim.step()
        assert rc == 0
    assert abs(math.hypot(*sim.Y[-1, :2]) / d_rigid - 1.0) <= 1e-3
    assert abs(math.hypot(*sim.Y[0, :2]) - 4.5977) <= 1e-12
    assert abs(math.atan2(sim.Y[0, 1], sim.Y[0, 0]) - 20 * 0.05) <= 1e-12
    sim, Y, d_rigid = _motor_filament(300.0)
    ds = []
    for _ in range(40):
        rc, rep = sim.step()
        assert rc == 0
        ds.append(math.hypot(*sim.Y[-1, :2]) / d_rigid)
    assert ds[-1] < 0.9 and ds[-1] < ds[19]


@pytest.mark.parametrize("tether", [0, 1])
def test_j0_with_preferred_curvature_equals_drag_jacobian_at_straight_state(tether):
    """Appendix B.2 with a preferred curvature: the moment carries -R(q_{n+1/2}) D kappa,
    whose derivative in u is taken from the rotation of the frame vectors.  At u = 0 on a
    straight, untwisted filament the midpoint frame turns by exactly half of each
    neighbour's rotation to first order, so J0 (its kappa_nu entries included) must equal
    the drag-only Jacobian there, free and clamped, with the drive of Sec. 5.3 at a set
    phase and time (reading R5: kappa_nu only)."""
    N = 6
    L = N * synth.DL
    q0 = np.array([math.cos(-math.pi / 4), 0, math.sin(-math.pi / 4), 0]) if tether else \
        synth.random_unit_quaternion(np.random.default_rng(14))
    q = np.tile(q0, (N, 1))
    Y = synth.chain(np.array([0.5, -1.0, 2.0]), q)
    extra = dict(tether=[1], base=Y[:1]) if tether else {}
    sim = oracle.Sim([0, N], Y, q, dt=1.7, drag_only=1, KB=1.2, KT=0.8, K0=10.61 / L, kw=2 * math.pi / L,
                     omega=0.37, phase=[1.1], **extra)
    sim.St.step = 3
    sim.St.t = 2.9
    rng = np.random.default_rng(15 + tether)
    X = np.zeros(6 * N)
    X[:3] = rng.standard_normal(3) if tether else Y[0] + rng.standard_normal(3)
    if tether:
        X[3:6] = rng.standard_normal(3)
    X[3 + 3 * N:] = rng.standard_normal(3 * (N - 1))
    J0 = sim.j0_filament(0, X)
    Jfd = fd_jacobian(lambda x: sim.residual(x)[0], X)
    # the drive is large: without the kappa terms of dM/du this test must fail
    sim0 = oracle.Sim([0, N], Y, q, dt=1.7, drag_only=1, KB=1.2, KT=0.8, **extra)
    sim0.St.step, sim0.St.t = 3, 2.9
    assert np.abs(sim0.j0_filament(0, X) - Jfd).max() > 1e-3 * np.abs(Jfd).max()
    assert np.allclose(J0, Jfd, rtol=0, atol=1e-7 * np.abs(Jfd).max())
