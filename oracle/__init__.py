"""Plain FP64 CPU oracle for the quaternion filament method (arXiv:1903.12609).

TEST INFRASTRUCTURE ONLY.  This package is the checker the GPU library is
compared against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
does.  It shares no code with the GPU path.

The numerics live in ``fil_oracle.c`` (plain C, double precision); this module
only builds it with gcc and marshals numpy arrays (array-of-structures layout:
vectors ``[S, 3]``, quaternions ``[S, 4]``, unknowns ``[6S]``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fil_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class Params(C.Structure):
    _fields_ = [
        ("M", C.c_int64), ("fil_off", _i64p),
        ("a", C.c_double), ("eta", C.c_double), ("dL", C.c_double), ("KB", C.c_double), ("KT", C.c_double),
        ("chi", C.c_double), ("FS", C.c_double), ("grav", C.c_double * 3),
        ("dt", C.c_double), ("tol", C.c_double), ("kmax", C.c_int64),
        ("K0", C.c_double), ("kw", C.c_double), ("omega", C.c_double), ("phase", _dp),
        ("tether", _i32p), ("motor_d0", C.c_double), ("motor_w", C.c_double), ("base", _dp),
        ("nthreads", C.c_int64), ("drag_only", C.c_int64),
        ("fext", _dp), ("text", _dp), ("Lper", _dp), ("mobility", C.c_void_p), ("mob_ctx", C.c_void_p),
    ]


# (V, W) = M(Y) (F, T) over [S][3] arrays, in place of the unbounded RPY apply
MOBILITY_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int64, _dp, _dp, _dp, _dp, _dp)


class State(C.Structure):
    _fields_ = [("Y", _dp), ("Yprev", _dp), ("q", _dp), ("X", _dp), ("Xprev", _dp),
                ("t", C.c_double), ("step", C.c_int64)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int64), ("applies", C.c_int64), ("resid", C.c_double), ("converged", C.c_int64)]


def _declare(L):
    L.or_qmul.argtypes = [_dp, _dp, _dp]
    L.or_qrot.argtypes = [_dp, _dp]
    L.or_qsqrt.argtypes = [_dp, _dp]
    L.or_qmid.argtypes = [_dp, _dp, _dp]
    L.or_qexp.argtypes = [_dp, _dp]
    L.or_dexpinv.argtypes = [_dp, _dp, _dp]
    L.or_rpy_blocks.argtypes = [_dp, C.c_int, C.c_double, C.c_double, _dp, _dp, _dp, _dp]
    L.or_rpy_apply.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, _dp, _dp, C.c_int64]
    L.or_rpy_matrix.argtypes = [C.c_int64, _dp, C.c_double, C.c_double, _dp]
    L.or_rpy_apply_targets.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int64, _i64p, _dp,
                                       _dp, C.c_int64]
    L.or_steric.argtypes = [C.c_int64, _dp, _i64p, C.c_double, C.c_double, C.c_double, _dp, _dp]
    L.or_moment.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
    L.or_internal_forces.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp, _dp]
    L.or_reconstruct.argtypes = [C.POINTER(Params), _dp, _dp, C.c_double, _dp, _dp]
    L.or_forces.argtypes = [C.POINTER(Params), _dp, _dp, _dp, C.c_double, _dp, _dp]
    L.or_residual.argtypes = [C.POINTER(Params), C.POINTER(State), _dp, _dp, _dp, _dp]
    L.or_residual.restype = C.c_double
    L.or_j0_filament.argtypes = [C.POINTER(Params), C.c_int64, C.c_int64, _dp, _dp, C.c_double, _dp]
    L.or_lu.argtypes = [C.c_int64, _dp, _i64p]
    L.or_lu.restype = C.c_int
    L.or_lu_solve.argtypes = [C.c_int64, _dp, _i64p, _dp]
    L.or_initial_guess.argtypes = [C.POINTER(Params), C.POINTER(State), _dp]
    L.or_broyden.argtypes = [C.POINTER(Params), C.POINTER(State), _dp, C.POINTER(Report)]
    L.or_broyden.restype = C.c_int
    L.or_bdf2_step.argtypes = [C.POINTER(Params), C.POINTER(State), C.POINTER(Report)]
    L.or_bdf2_step.restype = C.c_int


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


# --------------------------------------------------------------------------- quaternions
def qmul(p, q):
    p, q, r = _f64(p), _f64(q), np.zeros(4)
    lib().or_qmul(_p(p), _p(q), _p(r))
    return r


def qrot(q):
    q, R = _f64(q), np.zeros(9)
    lib().or_qrot(_p(q), _p(R))
    return R.reshape(3, 3)


def qsqrt(p):
    p, r = _f64(p), np.zeros(4)
    lib().or_qsqrt(_p(p), _p(r))
    return r


def qmid(qn, qn1):
    qn, qn1, r = _f64(qn), _f64(qn1), np.zeros(4)
    lib().or_qmid(_p(qn), _p(qn1), _p(r))
    return r


def qexp(u):
    u, r = _f64(u), np.zeros(4)
    lib().or_qexp(_p(u), _p(r))
    return r


def dexpinv(u, w):
    u, w, r = _f64(u), _f64(w), np.zeros(3)
    lib().or_dexpinv(_p(u), _p(w), _p(r))
    return r


# --------------------------------------------------------------------------- mobility
def rpy_blocks(r, self_pair, a, eta):
    r = _f64(r)
    out = [np.zeros(9) for _ in range(4)]
    lib().or_rpy_blocks(_p(r), int(bool(self_pair)), a, eta, *[_p(o) for o in out])
    return [o.reshape(3, 3) for o in out]


def rpy_apply(Y, F, T, a, eta, nthreads=0):
    """(V, Omega) = RPY mobility applied to (F, T); arrays [S, 3]."""
    Y, F, T = _f64(Y), _f64(F), _f64(T)
    S = Y.shape[0]
    V, W = np.zeros((S, 3)), np.zeros((S, 3))
    lib().or_rpy_apply(S, _p(Y), _p(F), _p(T), a, eta, _p(V), _p(W), int(nthreads))
    return V, W


def rpy_apply_targets(Y, F, T, a, eta, idx, nthreads=0):
    """(V, Omega) at the targets idx only; arrays [S, 3], result [len(idx), 3]."""
    Y, F, T = _f64(Y), _f64(F), _f64(T)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    V, W = np.zeros((len(idx), 3)), np.zeros((len(idx), 3))
    lib().or_rpy_apply_targets(Y.shape[0], _p(Y), _p(F), _p(T), a, eta, len(idx), idx.ctypes.data_as(_i64p),
                               _p(V), _p(W), int(nthreads))
    return V, W


def rpy_matrix(Y, a, eta):
    Y = _f64(Y)
    S = Y.shape[0]
    Mg = np.zeros((6 * S, 6 * S))
    lib().or_rpy_matrix(S, _p(Y), a, eta, _p(Mg))
    return Mg


def steric(Y, seg_fil, a, chi, FS, L=None):
    """Steric barrier forces [S, 3]; L [3]: the lengths of a periodic box (None: unbounded)."""
    Y = _f64(Y)
    seg_fil = np.ascontiguousarray(seg_fil, dtype=np.int64)
    FB = np.zeros_like(Y)
    Lp = None if L is None else _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    lib().or_steric(Y.shape[0], _p(Y), seg_fil.ctypes.data_as(_i64p), a, chi, FS, None if Lp is None else _p(Lp),
                    _p(FB))
    return FB


# --------------------------------------------------------------------------- filament mechanics
def moment(qn, qn1, kap, dL, KB, KT):
    qn, qn1, kap, M = _f64(qn), _f64(qn1), _f64(kap), np.zeros(3)
    lib().or_moment(_p(qn), _p(qn1), _p(kap), dL, KB, KT, _p(M))
    return M


def internal_forces(q, Lam, kap, dL, KB, KT):
    """Internal F^C and T^C + T^E of one filament; q [N,4], Lam, kap [N-1,3]."""
    q = _f64(q)
    N = q.shape[0]
    Lam = _f64(Lam if N > 1 else np.zeros((1, 3)))
    kap = _f64(kap if N > 1 else np.zeros((1, 3)))
    F, T = np.zeros((N, 3)), np.zeros((N, 3))
    lib().or_internal_forces(N, _p(q), _p(Lam), _p(kap), dL, KB, KT, _p(F), _p(T))
    return F, T


# --------------------------------------------------------------------------- the implicit step
class Sim:
    """Oracle simulation: parameters + state for one suspension.

    ``fil_off`` [M+1] segment offsets; ``Y0`` [S,3] and ``q0`` [S,4] the initial
    configuration (from the shared synthetic generators).  Keyword parameters
    mirror the method's: a, eta, dL, KB, KT, chi, FS, grav, dt, tol, kmax, K0,
    kw, omega, phase [M], tether [M] (0 free, 1 clamped, 2 pinned: base position held,
    rotation free, 3 on a rotating motor: motor_d0, motor_w), base [M,3], fext [S,3] and text [S,3] (further external forces and
    torques on each segment), nthreads; periodic = dict(box [3], grid [3], cut, omega) puts the
    suspension in a periodic box with the force-coupling-method mobility (Sec. 2.7.2) and
    nearest-image steric forces; mobility = callable (Y, F, T) -> (V, W) over [S, 3] arrays
    replaces the RPY apply otherwise.
    """

    def __init__(self, fil_off, Y0, q0, **kw):
        self.fil_off = np.ascontiguousarray(fil_off, dtype=np.int64)
        M = len(self.fil_off) - 1
        S = int(self.fil_off[-1])
        self.M, self.S = M, S
        self._keep = []
        P = Params()
        P.M = M
        P.fil_off = self.fil_off.ctypes.data_as(_i64p)
        P.a = kw.get("a", 1.0)
        P.eta = kw.get("eta", 1.0)
        P.dL = kw.get("dL", 2.2 * P.a)
        P.KB = kw.get("KB", 1.0)
        P.KT = kw.get("KT", P.KB)
        P.chi = kw.get("chi", 1.1)
        P.FS = kw.get("FS", 0.0)
        g = kw.get("grav", (0.0, 0.0, 0.0))
        P.grav[0], P.grav[1], P.grav[2] = g
        P.dt = kw["dt"]
        P.tol = kw.get("tol", 1e-6)
        P.kmax = kw.get("kmax", 100)
        P.K0 = kw.get("K0", 0.0)
        P.kw = kw.get("kw", 0.0)
        P.omega = kw.get("omega", 0.0)
        ph = kw.get("phase")
        if ph is not None:
            ph = _f64(ph)
            self._keep.append(ph)
            P.phase = _p(ph)
        th = kw.get("tether")
        if th is not None:
            th = np.ascontiguousarray(th, dtype=np.int32)
            base = _f64(kw["base"], (M, 3))
            self._keep += [th, base]
            P.tether = th.ctypes.data_as(_i32p)
            P.base = _p(base)
        P.motor_d0 = kw.get("motor_d0", 0.0)
        P.motor_w = kw.get("motor_w", 0.0)
        fx = kw.get("fext")
        if fx is not None:
            fx = _f64(fx, (S, 3))
            self._keep.append(fx)
            P.fext = _p(fx)
        tx = kw.get("text")
        if tx is not None:
            tx = _f64(tx, (S, 3))
            self._keep.append(tx)
            P.text = _p(tx)
        P.nthreads = kw.get("nthreads", 0)
        P.drag_only = int(kw.get("drag_only", 0))
        per = kw.get("periodic")
        mob = kw.get("mobility")
        if per is not None:
            # periodic box with the force-coupling-method mobility
            from .fcm import fcm_apply
            Lp = _f64(np.broadcast_to(np.asarray(per["box"], dtype=np.float64), (3,)))
            self._keep.append(Lp)
            P.Lper = _p(Lp)
            box, grid, cut, a_, eta_ = per["box"], per["grid"], per.get("cut", 7.5), P.a, P.eta
            om = per.get("omega", "curl")
            mob = lambda Y, F, T: fcm_apply(Y, F, T, a_, eta_, box, grid, cut=cut, omega=om)
        if mob is not None:
            def _cb(ctx, n, Yp, Fp, Tp, Vp, Wp, _mob=mob):
                V = np.ctypeslib.as_array(Vp, shape=(n, 3))
                W = np.ctypeslib.as_array(Wp, shape=(n, 3))
                try:
                    Vn, Wn = _mob(*(np.ctypeslib.as_array(p, shape=(n, 3)).copy() for p in (Yp, Fp, Tp)))
                    V[:] = Vn
                    W[:] = Wn
                except Exception:  # an error inside the callback reaches C as NaN velocities
                    V[:] = np.nan
                    W[:] = np.nan
                    raise
            cb = MOBILITY_FN(_cb)
            self._keep.append(cb)
            P.mobility = C.cast(cb, C.c_void_p)
        self.P = P
        self.Y = _f64(Y0, (S, 3)).copy()
        self.Yprev = self.Y.copy()
        self.q = _f64(q0, (S, 4)).copy()
        self.X = np.zeros(6 * S)
        self.Xprev = np.zeros(6 * S)
        self.St = State()
        self._bind_state()
        self.St.t = 0.0
        self.St.step = 0

    def _bind_state(self):
        self.St.Y, self.St.Yprev, self.St.q = _p(self.Y), _p(self.Yprev), _p(self.q)
        self.St.X, self.St.Xprev = _p(self.X), _p(self.Xprev)

    @property
    def step_index(self):
        return int(self.St.step)

    @property
    def time(self):
        return float(self.St.t)

    def initial_guess(self):
        X0 = np.zeros(6 * self.S)
        lib().or_initial_guess(C.byref(self.P), C.byref(self.St), _p(X0))
        return X0

    def residual(self, X, want_config=False):
        X = _f64(X).copy()
        f = np.zeros(6 * self.S)
        Y, q = np.zeros((self.S, 3)), np.zeros((self.S, 4))
        r = lib().or_residual(C.byref(self.P), C.byref(self.St), _p(X), _p(f), _p(Y), _p(q))
        return (f, r, Y, q) if want_config else (f, r)

    def reconstruct(self, X):
        X = _f64(X).copy()
        Y, q = np.zeros((self.S, 3)), np.zeros((self.S, 4))
        lib().or_reconstruct(C.byref(self.P), _p(self.q), _p(X), self.St.t + self.P.dt, _p(Y), _p(q))
        return Y, q

    def forces(self, X, Y=None, q=None, tt=None):
        """Total force and torque (internal + tether + gravity + steric) on every
        segment at configuration (Y, q) (default: the committed state) with the
        multipliers of X."""
        Y = self.Y if Y is None else _f64(Y, (self.S, 3))
        q = self.q if q is None else _f64(q, (self.S, 4))
        tt = self.St.t if tt is None else tt
        F, T = np.zeros((self.S, 3)), np.zeros((self.S, 3))
        lib().or_forces(C.byref(self.P), _p(Y), _p(q), _p(_f64(X).copy()), tt, _p(F), _p(T))
        return F, T

    def j0_filament(self, f, X):
        N = int(self.fil_off[f + 1] - self.fil_off[f])
        X = _f64(X).copy()
        _, q = self.reconstruct(X)
        J = np.zeros((6 * N, 6 * N))
        lib().or_j0_filament(C.byref(self.P), f, self.St.step, _p(q), _p(X), self.St.t + self.P.dt, _p(J))
        return J

    def broyden(self, X0):
        X = _f64(X0).copy()
        rep = Report()
        rc = lib().or_broyden(C.byref(self.P), C.byref(self.St), _p(X), C.byref(rep))
        return X, rc, rep

    def commit(self, X):
        """Accept X as the converged unknowns of the step: q^{j+1} = exp(u) . q^j, the
        robot-arm positions, the history shift and t += dt (as or_bdf2_step does)."""
        X = _f64(X).copy()
        Yn, qn = self.reconstruct(X)
        self.Yprev[:] = self.Y
        self.Y[:] = Yn
        self.q[:] = qn
        self.Xprev[:] = self.X
        self.X[:] = X
        self.St.t += self.P.dt
        self.St.step += 1

    def step(self):
        rep = Report()
        rc = lib().or_bdf2_step(C.byref(self.P), C.byref(self.St), C.byref(rep))
        return rc, rep
