"""Oracle of the learned warm start's data (test infrastructure only).

Plain numpy statements of the per-filament features, the training target and
the way a prediction becomes the first Broyden iterate.  These are not part of
the paper's method: they choose what the network sees and predicts around the
paper's extrapolated first iterate (Sec. 3.3.3).  For a filament of N segments
(arrays in the caller's [S, 3] / [S, 4] layouts, X in the solver's per-filament
order [Y_1 | u_1..u_N | Lambda_{3/2}..Lambda_{N-1/2}]):

  features (19N, group-major)
    (Y_n - centroid) / L, L = N dL                      3N
    q_n                                                  4N
    F_n / F_s                                            3N
    dt * mean(V_{n-1}, V_n, V_{n+1}) / dL (in-filament)  3N
    last changes of the unknowns:                        6N
       Y_1 and Lambda: X^j - 2 X^{j-1} + X^{j-2}, u: X^j - X^{j-1},
       scaled by 1/dL (Y_1), 1 (u), 1/F_s (Lambda)
  base (6N): X0 plus the last step's correction X^j - X0^j, which is the unscaled
     last-changes group (from the fourth step on, free filaments only),
  target (6N): (X* - base) with the same slot scales,
  first iterate: base + prediction * scales,
with F_s the magnitude of the gravity force per segment, or K_B / dL^2 when
there is none.
"""
from __future__ import annotations

import numpy as np


def force_scale(grav, KB, dL):
    g = float(np.linalg.norm(grav))
    return g if g > 0 else KB / dL ** 2


def slot_scales(N, dL, Fs):
    s = np.ones(6 * N)
    s[:3] = dL
    s[3 + 3 * N:] = Fs
    return s


def features(fil_off, Y, q, F, V, Xj, Xjm1, Xjm2, dL, dt, grav, KB):
    fil_off = np.asarray(fil_off)
    M = len(fil_off) - 1
    N = int(fil_off[1] - fil_off[0])
    Fs = force_scale(grav, KB, dL)
    L = N * dL
    out = np.zeros((M, 19 * N))
    sc = slot_scales(N, dL, Fs)
    for f in range(M):
        s0, s1 = fil_off[f], fil_off[f + 1]
        assert s1 - s0 == N
        y = Y[s0:s1]
        out[f, :3 * N] = ((y - y.mean(axis=0)) / L).ravel()
        out[f, 3 * N:7 * N] = q[s0:s1].ravel()
        out[f, 7 * N:10 * N] = (F[s0:s1] / Fs).ravel()
        v = V[s0:s1]
        avg = np.array([v[max(n - 1, 0):min(n + 2, N)].mean(axis=0) for n in range(N)])
        out[f, 10 * N:13 * N] = (dt * avg / dL).ravel()
        xj, x1, x2 = (A[6 * s0:6 * s1] for A in (Xj, Xjm1, Xjm2))
        h = xj - 2.0 * x1 + x2
        h[3:3 + 3 * N] = xj[3:3 + 3 * N] - x1[3:3 + 3 * N]
        out[f, 13 * N:] = h / sc
    return out


def base(fil_off, X0, Xj, Xjm1, Xjm2, step, tether=None):
    """X0 plus the last step's correction for every free filament when three committed
    steps of history exist (step >= 3), else X0.  The correction of step j is its
    converged X^j minus its extrapolated first iterate: X^j - 2 X^{j-1} + X^{j-2} for
    Y_1 and Lambda, u^j - u^{j-1} for u."""
    fil_off = np.asarray(fil_off)
    Xb = np.array(X0, dtype=np.float64)
    if step < 3:
        return Xb
    for f in range(len(fil_off) - 1):
        if tether is not None and tether[f]:
            continue
        a, b = 6 * fil_off[f], 6 * fil_off[f + 1]
        N = int(fil_off[f + 1] - fil_off[f])
        d = Xj[a:b] - 2.0 * Xjm1[a:b] + Xjm2[a:b]
        d[3:3 + 3 * N] = Xj[a + 3:a + 3 + 3 * N] - Xjm1[a + 3:a + 3 + 3 * N]
        Xb[a:b] += d
    return Xb


def target(fil_off, Xstar, Xb, dL, grav, KB):
    """(X* - Xb) / slot scales per filament, Xb the base (see base())."""
    fil_off = np.asarray(fil_off)
    M = len(fil_off) - 1
    N = int(fil_off[1] - fil_off[0])
    sc = slot_scales(N, dL, force_scale(grav, KB, dL))
    return np.stack([(Xstar[6 * fil_off[f]:6 * fil_off[f + 1]] - Xb[6 * fil_off[f]:6 * fil_off[f + 1]]) / sc
                     for f in range(M)])


def first_iterate(fil_off, Xb, pred, dL, grav, KB):
    """Xb + pred * scales for every filament (pred [M, 6N], de-standardised)."""
    fil_off = np.asarray(fil_off)
    N = int(fil_off[1] - fil_off[0])
    sc = slot_scales(N, dL, force_scale(grav, KB, dL))
    X = np.array(Xb, dtype=np.float64)
    for f in range(len(fil_off) - 1):
        X[6 * fil_off[f]:6 * fil_off[f + 1]] += pred[f] * sc
    return X
