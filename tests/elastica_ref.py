"""Clamped filament under an end load (the spatial-convergence problem of Sec. 4.1):
the analytic elastica and the discrete set-up shared by the oracle and GPU tests.

The continuum problem: a filament clamped horizontally at s = 0 and loaded by a force
F along -z at s = l.  With theta(s) the angle of the tangent to the load line, the
first integral of the moment balance gives (Landau & Lifshitz's elastica)

    s = sqrt(K_B / (2F)) * integral_{theta(s)}^{pi/2} dphi / sqrt(cos theta_L - cos phi),

with theta_L = theta(l) fixed by s = l.  Only F l^2 / K_B matters for theta(s / l).

Discrete reading: the clamp holds segment 1 (its centre and orientation), the load acts
on segment N, so the loaded arc is l = (N - 1) dL and segment n sits at s_n = (n - 1) dL.
"""
import math

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq


def elastica_theta(fl2):
    """theta as a function of s / l for F l^2 / K_B = fl2, and theta_L."""
    c = math.sqrt(1.0 / (2.0 * fl2))  # sqrt(K_B / (2F)) / l

    def integral(th, thL):
        # phi = thL + w^2 removes the endpoint singularity; cos thL - cos phi is
        # evaluated as 2 sin(thL + w^2/2) sin(w^2/2), without cancellation
        def f(w):
            if w == 0.0:
                return 2.0 / math.sqrt(math.sin(thL))
            return 2.0 * w / math.sqrt(2.0 * math.sin(thL + 0.5 * w * w) * math.sin(0.5 * w * w))

        w0, w1 = math.sqrt(max(th - thL, 0.0)), math.sqrt(math.pi / 2 - thL)
        return quad(f, w0, w1, epsabs=1e-14, epsrel=1e-13, limit=200)[0]

    thL = brentq(lambda t: c * integral(t, t) - 1.0, 1e-3, math.pi / 2 - 1e-9, xtol=1e-15)

    def theta(sl):
        if sl <= 0.0:
            return math.pi / 2
        if sl >= 1.0:
            return thL
        return brentq(lambda t: c * integral(t, thL) - sl, thL, math.pi / 2, xtol=1e-15)

    return theta, thL


def tangent_angles(q):
    """Angle of each segment's tangent t = R(q) e_x to the load line (-z)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    tz = 2.0 * (x * z - w * y)
    return np.arccos(np.clip(-tz, -1.0, 1.0))


def clamped_filament(N, ell=40.0, KB=1.0, fl2=1.93, steps_per_tau=20, tol=1e-10):
    """Straight filament along x, clamped at segment 1, end load F = fl2 K_B / l^2 on
    segment N; dt is a fraction of the slowest bending relaxation time
    (6 pi eta a / dL) l^4 / (12.36 K_B).  Returns fil_off, Y, q, params, fext [N, 3]."""
    dL = ell / (N - 1)
    a = dL / 2.2
    q = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (N, 1))
    Y = np.zeros((N, 3))
    Y[:, 0] = dL * np.arange(N)
    tau = 6.0 * math.pi * a / dL * ell ** 4 / KB / 12.36
    params = dict(a=a, eta=1.0, dL=dL, KB=KB, KT=KB, chi=1.1, FS=0.0, grav=(0.0, 0.0, 0.0), dt=tau / steps_per_tau,
                  tol=tol, kmax=100, tether=np.array([1], dtype=np.int32), base=Y[:1].copy())
    fext = np.zeros((N, 3))
    fext[-1, 2] = -fl2 * KB / ell ** 2
    return np.array([0, N], dtype=np.int64), Y, q, params, fext


def l2_angle_error(q, dL, ell, theta):
    """E_2 = sqrt(dL sum_n (theta^n - theta(s_n))^2), s_n = (n - 1) dL."""
    th = tangent_angles(q)
    s = dL * np.arange(len(q)) / ell
    ex = np.array([theta(v) for v in s])
    return math.sqrt(dL * float(np.sum((th - ex) ** 2)))
