"""Seeded synthetic workloads for the filament solver.

This module builds inputs only: initial filament placements, orientations and
random force/torque fields with the shapes, sizes and parameter values of the
paper's workloads.  It contains none of the method's arithmetic (no mobility,
no moments, no time stepping); both the GPU library's tests and the CPU oracle
take their inputs from here.  Geometry used for placement (rotating the
x-axis by a quaternion, a straight or gently bent chain of segments) is written
out here independently with axis-angle (Rodrigues) rotation.

Parameter recipes (units a = eta = 1, K_B = K_T = 1, segment spacing 2.2a):
  * gravity number B = L^3 W / K_B, W the force per unit length, L = N dL;
    every segment carries W dL along -z; settling time T = eta L / W.
  * steric barrier strength F^S = 1e3 K_B / L^2, range chi = 1.1.
  * the time step of the sedimenting workloads is a fraction of T, the active
    array's a fraction of its beat period 2 pi / omega.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

A = 1.0
ETA = 1.0
KB = 1.0
KT = 1.0
DL = 2.2 * A
CHI = 1.1


def _rotate_ex(q):
    """Image of e_x under the rotation encoded by unit quaternion(s) q [...,4],
    computed through axis-angle form (Rodrigues)."""
    q = np.asarray(q, dtype=np.float64)
    w, v = q[..., 0], q[..., 1:]
    s = np.linalg.norm(v, axis=-1)
    ang = 2.0 * np.arctan2(s, w)
    k = np.where(s[..., None] > 0, v / np.where(s > 0, s, 1.0)[..., None], 0.0)
    ex = np.zeros_like(k)
    ex[..., 0] = 1.0
    kx = np.cross(k, ex)
    kd = k[..., 0]
    c, sn = np.cos(ang)[..., None], np.sin(ang)[..., None]
    return ex * c + kx * sn + k * kd[..., None] * (1.0 - c)


def _rotate(q, vec):
    """Rotate a 3-vector by unit quaternion q via axis-angle (Rodrigues)."""
    w, v = q[0], np.asarray(q[1:])
    s = np.linalg.norm(v)
    if s == 0:
        return np.array(vec, dtype=np.float64)
    ang = 2.0 * math.atan2(s, w)
    k = v / s
    vec = np.asarray(vec, dtype=np.float64)
    return vec * math.cos(ang) + np.cross(k, vec) * math.sin(ang) + k * np.dot(k, vec) * (1 - math.cos(ang))


def _axis_angle_quat(axis, ang):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    return np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis])


def _hamilton(p, q):
    p0, pv, q0, qv = p[0], p[1:], q[0], q[1:]
    return np.concatenate([[p0 * q0 - pv @ qv], p0 * qv + q0 * pv + np.cross(pv, qv)])


def random_unit_quaternion(rng):
    """Normalised 4-D standard-normal draw: uniform orientation (Appendix A.5)."""
    g = rng.standard_normal(4)
    return g / np.linalg.norm(g)


def chain(base, quats, dL=DL):
    """Positions of a chain whose consecutive segments satisfy the discrete
    inextensibility constraint: Y_{n+1} = Y_n + dL/2 (t_n + t_{n+1})."""
    t = _rotate_ex(quats)
    Y = np.empty((len(quats), 3))
    Y[0] = base
    for n in range(1, len(quats)):
        Y[n] = Y[n - 1] + 0.5 * dL * (t[n - 1] + t[n])
    return Y


def bent_quaternions(q0, N, delta, axis_body=(0.0, 1.0, 0.0)):
    """q_n = rot(n delta about the frame axis R(q0) axis_body) . q0: a planar arc."""
    ax = _rotate(q0, axis_body)
    return np.stack([_hamilton(_axis_angle_quat(ax, n * delta), q0) if delta != 0 else np.array(q0)
                     for n in range(N)])


@dataclasses.dataclass
class Workload:
    """A suspension: filament offsets, initial positions/quaternions and parameters."""
    name: str
    fil_off: np.ndarray      # [M+1] int64
    Y: np.ndarray            # [S,3]
    q: np.ndarray            # [S,4]
    params: dict             # a, eta, dL, KB, KT, chi, FS, grav, dt, tol, kmax, ...
    steps: int = 1
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def M(self):
        return len(self.fil_off) - 1

    @property
    def S(self):
        return int(self.fil_off[-1])


def sedimentation_params(N, B=1e3, dt_over_T=1.0, tol=1e-6, kmax=100, steric=True):
    L = N * DL
    W = B * KB / L ** 3
    T = ETA * L / W
    return dict(a=A, eta=ETA, dL=DL, KB=KB, KT=KT, chi=CHI, FS=(1e3 * KB / L ** 2 if steric else 0.0),
                grav=(0.0, 0.0, -W * DL), dt=dt_over_T * T, tol=tol, kmax=kmax), T


def single_filament(N=15, seed=1001, B=1e3, dt_over_T=1.0, tol=1e-6, kmax=100, bend=0.0):
    """One straight filament along a seed-random direction, centred at the origin."""
    rng = np.random.default_rng(seed)
    q0 = random_unit_quaternion(rng)
    q = bent_quaternions(q0, N, bend)
    Y = chain(np.zeros(3), q)
    Y -= Y.mean(axis=0)
    params, T = sedimentation_params(N, B, dt_over_T, tol, kmax, steric=True)
    return Workload("single_filament", np.array([0, N], dtype=np.int64), Y, q, params,
                    extra=dict(T=T))


def _place(rng, M_fil, Ns, side, max_bend, min_sep=DL, max_tries=100000):
    """Random sequential placement with rejection when any segment comes closer than
    min_sep to a placed one.  Placed segments are hashed into cubic cells of side min_sep,
    so a candidate is compared only with the segments of its own and the neighbouring
    cells (every segment within min_sep of it lies there)."""
    Ys, qs = [], []
    cells = {}
    pts = []
    tries = 0
    for m in range(M_fil):
        N = Ns[m]
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("placement failed: suspension too dense")
            q0 = random_unit_quaternion(rng)
            delta = rng.uniform(0.0, max_bend) if max_bend > 0 else 0.0
            q = bent_quaternions(q0, N, delta)
            centre = rng.uniform(0.0, side, 3)
            Y = chain(np.zeros(3), q)
            Y += centre - Y.mean(axis=0)
            near = set()
            for c in np.floor(Y / min_sep).astype(np.int64):
                for dx in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dz in (-1, 0, 1):
                            near.update(cells.get((c[0] + dx, c[1] + dy, c[2] + dz), ()))
            if near:
                P = np.asarray([pts[i] for i in sorted(near)])
                d2 = ((Y[:, None, :] - P[None, :, :]) ** 2).sum(-1)
                if d2.min() < min_sep ** 2:
                    continue
            break
        for y in Y:
            cells.setdefault(tuple(np.floor(y / min_sep).astype(np.int64)), []).append(len(pts))
            pts.append(y)
        Ys.append(Y)
        qs.append(q)
    fil_off = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int64)
    return fil_off, np.concatenate(Ys), np.concatenate(qs)


def sediment_suspension(M=100, N=20, side=200.0, seed=1002, B=1e3, dt_over_T=1.0, tol=1e-6, kmax=100,
                        max_bend=0.02):
    """Filaments with centres uniform in a cube, isotropic orientations, a small
    seed-random planar bend, overlaps below 2.2a rejected (Appendix A.5 style)."""
    rng = np.random.default_rng(seed)
    fil_off, Y, q = _place(rng, M, [N] * M, side, max_bend)
    params, T = sedimentation_params(N, B, dt_over_T, tol, kmax, steric=True)
    return Workload("sediment_suspension", fil_off, Y, q, params, extra=dict(T=T, side=side))


# the paper's periodic monolayer: a 141 dL x 141 dL x 8.8 dL box on a 1024 x 1024 x 64 grid
MONOLAYER_BOX = (141.0 * DL, 141.0 * DL, 8.8 * DL)
MONOLAYER_GRID = (1024, 1024, 64)


def periodic_monolayer(M=256, N=15, box=MONOLAYER_BOX, grid=MONOLAYER_GRID, seed=1005, B=1e3, dt_over_T=1 / 300,
                       tol=1e-4, kmax=100, min_sep=DL, max_tries=200000):
    """Straight filaments in the centre plane z = Lz / 2 of a periodic box: centres uniform
    over the plane, orientations uniform in the plane, placements closer than min_sep to
    a placed segment (nearest periodic image) rejected.  The force per unit length W
    acts in the plane, along -y.  Positions are not wrapped into the box."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    Ys, qs = [], []
    placed = np.zeros((0, 3))
    tries = 0
    for m in range(M):
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("placement failed: monolayer too dense")
            th = rng.uniform(0.0, 2 * math.pi)
            q = np.tile(np.array([math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]), (N, 1))
            Y = chain(np.zeros(3), q)
            Y += np.array([rng.uniform(0, box[0]), rng.uniform(0, box[1]), box[2] / 2]) - Y.mean(axis=0)
            if len(placed):
                d = Y[:, None, :] - placed[None, :, :]
                d -= box * np.round(d / box)
                if (d ** 2).sum(-1).min() < min_sep ** 2:
                    continue
            break
        Ys.append(Y)
        qs.append(q)
        placed = np.concatenate([placed, Y])
    params, T = sedimentation_params(N, B, dt_over_T, tol, kmax, steric=True)
    params["grav"] = (0.0, params["grav"][2], 0.0)
    return Workload("periodic_monolayer", np.arange(0, M * N + 1, N, dtype=np.int64), np.concatenate(Ys),
                    np.concatenate(qs), params, extra=dict(T=T, box=tuple(box), grid=tuple(grid)))


def active_array(nx=40, ny=25, N=32, spacing=20.0, seed=1003, tol=1e-6, kmax=100, steps_per_beat=100, base_z=0.0):
    """Base-clamped filaments on a square lattice, initially straight along +z,
    driven by kappa_nu(s,t) = K0 sin(k s - omega t + phi) with K0 = 10.61/L,
    k = 2 pi / L and (4 pi omega eta / K_B)^(1/4) L = 10 (Sec. 5.3 parameters).
    The base segments sit at height base_z (above a wall at z = 0: base_z >= a)."""
    rng = np.random.default_rng(seed)
    L = N * DL
    M = nx * ny
    qz = _axis_angle_quat((0.0, 1.0, 0.0), -math.pi / 2)   # e_x -> e_z
    base = np.array([[i * spacing, j * spacing, base_z] for i in range(nx) for j in range(ny)])
    Y = np.concatenate([b + np.outer(np.arange(N) * DL, [0, 0, 1.0]) for b in base])
    q = np.tile(qz, (M * N, 1))
    omega = 1e4 * KB / (4 * math.pi * ETA * L ** 4)
    phase = rng.uniform(0.0, 2 * math.pi, M)
    params = dict(a=A, eta=ETA, dL=DL, KB=KB, KT=KT, chi=CHI, FS=1e3 * KB / L ** 2, grav=(0.0, 0.0, 0.0),
                  dt=(2 * math.pi / omega) / steps_per_beat, tol=tol, kmax=kmax, K0=10.61 / L,
                  kw=2 * math.pi / L, omega=omega, phase=phase, tether=np.ones(M, dtype=np.int32), base=base)
    return Workload("active_array", np.arange(0, M * N + 1, N, dtype=np.int64), Y, q, params,
                    extra=dict(L=L))


def batched_ensemble(n_susp=256, seed=1004, tol=1e-6, kmax=100, dt_over_T=1.0, B=1e3):
    """Independent suspensions of uneven sizes: M_i ~ U{1..64}, N_i ~ U{10..50},
    placed like the sedimenting suspension in a cube scaled to its density."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_susp):
        M = int(rng.integers(1, 65))
        N = int(rng.integers(10, 51))
        side = 200.0 * (M * N / 2000.0) ** (1.0 / 3.0)
        fil_off, Y, q = _place(rng, M, [N] * M, side, 0.02)
        params, T = sedimentation_params(N, B, dt_over_T, tol, kmax, steric=True)
        out.append(Workload("suspension_%d" % i, fil_off, Y, q, params, extra=dict(T=T, side=side)))
    return out


def rpy_throughput_inputs(S, seed=7, structured=True):
    """Positions, forces and torques for throughput runs of the mobility apply:
    filament-major chains (32 segments, lattice of bent filaments) and
    F, T ~ N(0, 1) per component."""
    rng = np.random.default_rng(seed)
    if structured:
        N = 32
        M = (S + N - 1) // N
        nx = int(math.ceil(math.sqrt(M)))
        Ys = []
        for m in range(M):
            q0 = _axis_angle_quat((0.0, 1.0, 0.0), -math.pi / 2)
            q = bent_quaternions(q0, N, 0.05 * rng.uniform(-1, 1))
            b = np.array([(m % nx) * 20.0, (m // nx) * 20.0, 0.0])
            Ys.append(chain(b, q))
        Y = np.concatenate(Ys)[:S]
    else:
        Y = rng.uniform(0, 10.0 * S ** (1.0 / 3.0), (S, 3))
    F = rng.standard_normal((S, 3))
    T = rng.standard_normal((S, 3))
    return Y, F, T


def active_array_mobility_inputs(nx=40, ny=25, N=32, spacing=20.0, seed=7, bend=0.05, base_z=0.0):
    """Mobility inputs at the active array's size and layout: nx x ny filaments of N segments
    (S = 32000 by default) standing on a square lattice of spacing 20a, each a planar arc
    bent by a seed-random angle in [-bend, bend] per segment (the shape of a beating
    filament), with F, T ~ N(0, 1) per component.  Filament-major order, row by row."""
    rng = np.random.default_rng(seed)
    qz = _axis_angle_quat((0.0, 1.0, 0.0), -math.pi / 2)   # e_x -> e_z
    Ys = []
    for i in range(nx):
        for j in range(ny):
            q = bent_quaternions(qz, N, bend * rng.uniform(-1, 1))
            Ys.append(chain(np.array([i * spacing, j * spacing, base_z]), q))
    Y = np.concatenate(Ys)
    S = Y.shape[0]
    return Y, rng.standard_normal((S, 3)), rng.standard_normal((S, 3))


def random_cloud(S, seed, side, min_sep=None):
    """Uniform random points in a cube (optionally with a minimum separation)."""
    rng = np.random.default_rng(seed)
    if min_sep is None:
        return rng.uniform(0, side, (S, 3))
    pts = []
    while len(pts) < S:
        p = rng.uniform(0, side, 3)
        if all(np.sum((p - x) ** 2) >= min_sep ** 2 for x in pts):
            pts.append(p)
    return np.array(pts)
