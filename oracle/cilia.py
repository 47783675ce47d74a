"""Test infrastructure (not the product path): the geometric switch of model cilia
(Sec. 5.2.2) for the oracle's steps.

Every pinned filament (tether 2) is driven by a torque about a fixed unit axis applied to
its base segment.  Let theta be the angle from the unit wall normal n to the base tangent
t, signed about the axis: theta = atan2((n x t) . axis, n . t).  The drive points towards
+theta_max (magnitude tau_pos) or -theta_max (magnitude tau_neg); once theta reaches the
extreme it drives towards, it reverses.  The torque then passes from its value at the
switch to the new one along the logistic curve 1 / (1 + exp(-12 (k / n_tr - 1/2))) over
the next n_tr steps (k the steps since the switch).  All filaments start driving towards
+theta_max at full tau_pos.  The switch is decided from the committed configuration
before each step.
"""
import math

import numpy as np


class GeometricSwitch:
    def __init__(self, fil_off, tether, axis, normal, theta_max, tau_pos, tau_neg, n_tr):
        self.fil_off = np.asarray(fil_off)
        self.tether = np.asarray(tether)
        self.axis = np.asarray(axis, dtype=np.float64)
        self.normal = np.asarray(normal, dtype=np.float64)
        self.theta_max, self.tau_pos, self.tau_neg, self.n_tr = theta_max, tau_pos, tau_neg, n_tr
        M = len(self.fil_off) - 1
        self.dir = np.ones(M, dtype=np.int64)
        self.age = np.full(M, n_tr, dtype=np.int64)
        self.tau0 = np.full(M, float(tau_pos))

    def _torque(self, f):
        tau1 = self.tau_pos if self.dir[f] > 0 else -self.tau_neg
        if self.age[f] >= self.n_tr:
            return tau1
        x = self.age[f] / self.n_tr - 0.5
        return self.tau0[f] + (tau1 - self.tau0[f]) / (1.0 + math.exp(-12.0 * x))

    @staticmethod
    def tangent(q):
        """t = R(q) e_x of a unit quaternion (w, x, y, z)."""
        w, x, y, z = q
        return np.array([1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)])

    def theta(self, q_base):
        t = self.tangent(q_base)
        return math.atan2(float(np.dot(np.cross(self.normal, t), self.axis)), float(np.dot(self.normal, t)))

    def update(self, q, text):
        """Decide the switch from the committed quaternions q [S, 4]; write the base
        torques into text [S, 3] in place."""
        text[:] = 0.0
        for f in range(len(self.fil_off) - 1):
            if self.tether[f] != 2:
                continue
            s0 = self.fil_off[f]
            th = self.theta(q[s0])
            if self.dir[f] * th >= self.theta_max:
                self.tau0[f] = self._torque(f)
                self.dir[f] = -self.dir[f]
                self.age[f] = 0
            elif self.age[f] < self.n_tr:
                self.age[f] += 1
            text[s0] = self._torque(f) * self.axis
