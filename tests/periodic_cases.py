"""Periodic-box cases shared by the oracle and GPU tests of the force-coupling-method
steps (Sec. 2.7.2 mobility, Sec. 2.6 steric barrier between nearest periodic images).

* ``contact_pair(shifted)``: two parallel straight filaments 1.7a apart, staggered by
  half a segment (nearest segments 2.02a apart, inside the steric range 2.2a), one of
  them across the x boundary, plus a third filament elsewhere.  With ``shifted`` the
  first filament is moved by -Lx along x and the second by -Ly along y: the same
  periodic configuration, with the contact now only between nearest images.
* ``small_monolayer()``: a seeded monolayer of 6 filaments of 8 segments in a
  16 dL x 16 dL x 8 dL box on a 32 x 32 x 16 grid, placed down to 1.9a apart.
"""
import math

import numpy as np

from paper_1903_12609_amd import synth

BOX = (16 * synth.DL, 16 * synth.DL, 8 * synth.DL)
GRID = (32, 32, 16)


def _straight(N, centre, th):
    q = np.tile(np.array([math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]), (N, 1))
    Y = synth.chain(np.zeros(3), q)
    return Y - Y.mean(axis=0) + np.asarray(centre, dtype=np.float64), q


def contact_pair(shifted=False, N=8, dt_over_T=1 / 30, tol=1e-8):
    Lx, Ly, Lz = BOX
    centres = [np.array([Lx - 3.0, 10.0, Lz / 2]), np.array([Lx - 3.0 + 1.1, 11.7, Lz / 2]),
               np.array([12.0, 27.0, Lz / 2])]
    if shifted:
        centres[0] = centres[0] - np.array([Lx, 0.0, 0.0])
        centres[1] = centres[1] - np.array([0.0, Ly, 0.0])
    Ys, qs = [], []
    for c, th in zip(centres, (0.0, 0.0, 0.7)):
        Y, q = _straight(N, c, th)
        Ys.append(Y)
        qs.append(q)
    params, T = synth.sedimentation_params(N, 1e3, dt_over_T, tol, 100, steric=True)
    params["grav"] = (0.0, params["grav"][2], 0.0)
    fil_off = np.arange(0, 3 * N + 1, N, dtype=np.int64)
    return fil_off, np.concatenate(Ys), np.concatenate(qs), params


def shift_of(N=8):
    """Per-segment displacement of the shifted contact pair from the unshifted one."""
    Lx, Ly, _ = BOX
    d = np.zeros((3 * N, 3))
    d[:N, 0] = -Lx
    d[N:2 * N, 1] = -Ly
    return d


def small_monolayer(dt_over_T=1 / 30, tol=1e-8):
    return synth.periodic_monolayer(M=6, N=8, box=BOX, grid=GRID, seed=5, dt_over_T=dt_over_T, tol=tol,
                                    min_sep=1.9)


def periodic(cut=7.5):
    """The oracle's periodic set-up; the rotation averaged by parts, as on the GPU."""
    return dict(box=BOX, grid=GRID, cut=cut, omega="by_parts")
