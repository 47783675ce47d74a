"""MI355X filament library: Python binding of libfil.so.

The hot path of the implicit quaternion filament method (arXiv:1903.12609)
runs in hand-written HIP kernels; this module only hands torch device
tensors (float64, component-major ``[3, S]``) and the current HIP stream to
the C ABI declared in ``include/fil.h``.
"""
from __future__ import annotations

import os

from ._native import FilError, PREC, check, lib  # noqa: F401

__all__ = ["FilError", "MLP", "Sim", "rpy_mobility_apply", "rpy_mobility_apply_batched", "rpy_workspace_bytes",
           "rpy_wall_apply",
           "filament_internal_forces"]


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_soa(name, t, rows, S):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (rows, S):
        raise ValueError("%s must be a contiguous float64 CUDA tensor of shape (%d, %d)" % (name, rows, S))


def rpy_workspace_bytes(S, prec="f64"):
    return int(lib().fil_rpy_workspace_bytes(int(S), PREC[prec]))


def rpy_mobility_apply(Y, F, T, a=1.0, eta=1.0, prec="f64", V=None, W=None, work=None, events=None):
    """(V, Omega) = RPY mobility (Sec. 2.7.1) applied to forces F and torques T at
    positions Y; all float64 CUDA tensors of shape (3, S).  events: optional pair of
    torch.cuda.Event (enable_timing) stamped at the start and end of the pair kernel."""
    import torch
    S = Y.shape[1]
    for n, t in (("Y", Y), ("F", F), ("T", T)):
        _check_soa(n, t, 3, S)
    V = torch.empty_like(Y) if V is None else V
    W = torch.empty_like(Y) if W is None else W
    nb = rpy_workspace_bytes(S, prec)
    if work is None or work.numel() < nb:
        work = torch.empty(max(nb, 1), dtype=torch.uint8, device=Y.device)
    evs = (None, None)
    if events is not None:
        for e in events:
            if not e.cuda_event:  # torch creates the event at its first record
                e.record()
        evs = (events[0].cuda_event, events[1].cuda_event)
    check(lib().fil_rpy_mobility_apply_timed(S, _ptr(Y), _ptr(F), _ptr(T), float(a), float(eta), PREC[prec],
                                             _ptr(V), _ptr(W), _ptr(work), work.numel(), evs[0], evs[1], _stream()))
    return V, W


def rpy_wall_apply(Y, F, T, a=1.0, eta=1.0, prec="f64", V=None, W=None, work=None):
    """(V, Omega) = RPY mobility above the no-slip wall z = 0 applied to forces F and
    torques T at positions Y; float64 CUDA tensors of shape (3, S).  prec: "f64" or
    "f32tile"."""
    import torch
    S = Y.shape[1]
    for n, t in (("Y", Y), ("F", F), ("T", T)):
        _check_soa(n, t, 3, S)
    V = torch.empty_like(Y) if V is None else V
    W = torch.empty_like(Y) if W is None else W
    nb = int(lib().fil_rpy_wall_workspace_bytes(S))
    if work is None or work.numel() < nb:
        work = torch.empty(max(nb, 1), dtype=torch.uint8, device=Y.device)
    check(lib().fil_rpy_wall_apply(S, _ptr(Y), _ptr(F), _ptr(T), float(a), float(eta), PREC[prec], _ptr(V), _ptr(W),
                                   _ptr(work), work.numel(), _stream()))
    return V, W


def filament_internal_forces(fil_off, q, Lam, kappa, dL, KB, KT, F, T):
    """F += F^C, T += T^C + T^E for every filament (Sec. 2.5, 2.9.2).
    fil_off: int64 CUDA tensor [M+1]; q: (4, S); Lam, kappa: (3, S-M) (kappa may be None);
    F, T: (3, S), accumulated in place."""
    import torch
    M = fil_off.numel() - 1
    S = q.shape[1]
    if fil_off.dtype != torch.int64 or not fil_off.is_cuda:
        raise ValueError("fil_off must be an int64 CUDA tensor")
    _check_soa("q", q, 4, S)
    _check_soa("Lam", Lam, 3, S - M)
    if kappa is not None:
        _check_soa("kappa", kappa, 3, S - M)
    _check_soa("F", F, 3, S)
    _check_soa("T", T, 3, S)
    check(lib().fil_filament_internal_forces(M, S, _ptr(fil_off), _ptr(q), _ptr(Lam), _ptr(kappa), float(dL),
                                             float(KB), float(KT), _ptr(F), _ptr(T), _stream()))
    return F, T


class RpyBatch:
    """Plan of the batched mobility apply for suspensions at the host offsets susp_off
    [nsusp+1] in one precision; its applies only enqueue work."""

    def __init__(self, susp_off, prec="f64"):
        import ctypes
        import numpy as np
        off = np.ascontiguousarray(susp_off, dtype=np.int64)
        self.S = int(off[-1])
        h = ctypes.c_void_p()
        check(lib().fil_rpy_batch_create(len(off) - 1, off.ctypes.data_as(ctypes.c_void_p), PREC[prec],
                                         ctypes.byref(h)))
        self._h = h
        self.work_bytes = int(lib().fil_rpy_batch_workspace_bytes(h))

    def apply(self, Y, F, T, a=1.0, eta=1.0, V=None, W=None, work=None):
        import torch
        for n, t in (("Y", Y), ("F", F), ("T", T)):
            _check_soa(n, t, 3, self.S)
        V = torch.empty_like(Y) if V is None else V
        W = torch.empty_like(Y) if W is None else W
        if work is None:
            work = torch.empty(max(self.work_bytes, 1), dtype=torch.uint8, device=Y.device)
        check(lib().fil_rpy_mobility_apply_batched(self._h, _ptr(Y), _ptr(F), _ptr(T), float(a), float(eta), _ptr(V),
                                                   _ptr(W), _ptr(work), work.numel(), _stream()))
        return V, W

    def close(self):
        if getattr(self, "_h", None):
            lib().fil_rpy_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rpy_mobility_apply_batched(susp_off, Y, F, T, a=1.0, eta=1.0, prec="f64", V=None, W=None):
    """Independent suspensions in one persistent launch; susp_off: host int sequence [nsusp+1]
    (builds a plan for this one call)."""
    plan = RpyBatch(susp_off, prec)
    try:
        return plan.apply(Y, F, T, a, eta, V, W)
    finally:
        import torch
        torch.cuda.current_stream().synchronize()  # the plan is freed after the apply has run
        plan.close()


class _DevView:
    """Zero-copy torch view of a library-owned device array."""

    def __init__(self, ptr, shape):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<f8", "data": (int(ptr), False),
                                         "version": 2, "strides": None}


class FCM:
    """Force-coupling-method mobility in a periodic box (Sec. 2.7.2): box lengths [3],
    grid points [3], radius a, viscosity eta, Gaussian truncation in widths."""

    def __init__(self, box, grid, a=1.0, eta=1.0, cut=7.5):
        import ctypes
        import numpy as np
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
        g = np.ascontiguousarray(np.broadcast_to(np.asarray(grid, dtype=np.int32), (3,)))
        h = ctypes.c_void_p()
        check(lib().fil_fcm_create(b.ctypes.data_as(ctypes.c_void_p), g.ctypes.data_as(ctypes.c_void_p), float(a),
                                   float(eta), float(cut), ctypes.byref(h)))
        self._h = h

    def apply(self, Y, F, T, V=None, Omega=None):
        """(V, Omega) for device float64 tensors Y, F, T of shape [3, S]."""
        import torch
        S = Y.shape[1]
        V = torch.empty_like(Y) if V is None else V
        Omega = torch.empty_like(Y) if Omega is None else Omega
        check(lib().fil_fcm_apply(self._h, S, _ptr(Y), _ptr(F), _ptr(T), _ptr(V), _ptr(Omega), _stream()))
        return V, Omega

    def close(self):
        if getattr(self, "_h", None):
            lib().fil_fcm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sim:
    """A simulation of one or more independent suspensions on the GPU.

    fil_off [M+1] segment offsets; Y0 [S,3], q0 [S,4] the initial configuration;
    params: a, eta, dL, KB, KT, chi, FS, grav, dt, tol, kmax, K0, kw, omega and
    optional phase [M], tether [M]; susp_fil_off [nsusp+1] groups filaments
    into suspensions (default: one suspension).  prec: "f64" or "f32tile".
    j0_mode: "auto", "banded" or "dense"; j0_factor: "auto" or "unstaged" (the band LU
    kernel without LDS staging, the form large ensembles take).
    """

    def __init__(self, fil_off, Y0, q0, params, susp_fil_off=None, prec="f64", j0_mode="auto", graph=0,
                 j0_factor="auto"):
        import ctypes
        import numpy as np
        from ._native import Params
        self.fil_off = np.ascontiguousarray(fil_off, dtype=np.int64)
        M = len(self.fil_off) - 1
        self.M, self.S = M, int(self.fil_off[-1])
        sfo = np.ascontiguousarray([0, M] if susp_fil_off is None else susp_fil_off, dtype=np.int64)
        self.susp_fil_off = sfo
        self.nsusp = len(sfo) - 1
        P = Params()
        P.a, P.eta, P.dL = params.get("a", 1.0), params.get("eta", 1.0), params.get("dL", 2.2)
        P.KB, P.KT = params.get("KB", 1.0), params.get("KT", params.get("KB", 1.0))
        P.chi, P.FS = params.get("chi", 1.1), params.get("FS", 0.0)
        g = params.get("grav", (0.0, 0.0, 0.0))
        P.grav[0], P.grav[1], P.grav[2] = g
        P.dt, P.tol, P.kmax = params["dt"], params.get("tol", 1e-6), int(params.get("kmax", 100))
        P.prec = PREC[prec]
        P.j0_mode = {"auto": 0, "banded": 1, "dense": 2}[j0_mode]
        P.j0_factor = {"auto": 0, "unstaged": 1}[j0_factor]
        P.K0, P.kw, P.omega = params.get("K0", 0.0), params.get("kw", 0.0), params.get("omega", 0.0)
        self.params = P
        Y0 = np.ascontiguousarray(Y0, dtype=np.float64).reshape(self.S, 3)
        q0 = np.ascontiguousarray(q0, dtype=np.float64).reshape(self.S, 4)
        ph = params.get("phase")
        ph = None if ph is None else np.ascontiguousarray(ph, dtype=np.float64)
        th = params.get("tether")
        th = None if th is None else np.ascontiguousarray(th, dtype=np.int32)
        vp = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        check(lib().fil_create(ctypes.byref(P), self.nsusp, vp(sfo), vp(self.fil_off), vp(Y0), vp(q0), vp(ph),
                               vp(th), ctypes.byref(h)))
        self._h = h
        check(lib().fil_set_stream(h, _stream()))
        if graph:
            self.set_graph(graph)

    def set_graph(self, iters_per_launch=4):
        """Run Broyden iterations in captured HIP-graph blocks of this many iterations (0: off)."""
        check(lib().fil_set_graph(self._h, int(iters_per_launch)))

    def set_suspension_params(self, dt=None, grav=None, FS=None):
        """Per-suspension dt [nsusp], gravity force [nsusp,3] and F^S [nsusp] (before the first step)."""
        import ctypes
        import numpy as np
        ns = self.nsusp
        arrs = []
        for a, shape in ((dt, (ns,)), (grav, (ns, 3)), (FS, (ns,))):
            arrs.append(None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape)))
        vp = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        check(lib().fil_set_suspension_params(self._h, *[vp(a) for a in arrs]))

    def set_external_forces(self, F):
        """Further external force on every segment, [S, 3] (None removes it; before the first step)."""
        import ctypes
        import numpy as np
        if F is None:
            check(lib().fil_set_external_forces(self._h, None))
            return
        a = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(self.S, 3))
        check(lib().fil_set_external_forces(self._h, a.ctypes.data_as(ctypes.c_void_p)))

    def set_geometric_switch(self, axis, normal, theta_max, tau_pos, tau_neg, n_transition=10):
        """Geometric-switch base torques of the pinned filaments (Sec. 5.2.2); before the first step."""
        import ctypes
        import numpy as np
        ax = np.ascontiguousarray(np.asarray(axis, dtype=np.float64).reshape(3))
        nm = np.ascontiguousarray(np.asarray(normal, dtype=np.float64).reshape(3))
        check(lib().fil_set_geometric_switch(self._h, ax.ctypes.data_as(ctypes.c_void_p),
                                             nm.ctypes.data_as(ctypes.c_void_p), float(theta_max), float(tau_pos),
                                             float(tau_neg), int(n_transition)))

    def read_switch(self):
        """Switch direction (+1 / -1) of every filament, int32 [M] (synchronising)."""
        import ctypes
        import numpy as np
        out = np.zeros(self.M, dtype=np.int32)
        check(lib().fil_read_switch(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_motor(self, d0, omega):
        """Rotating motor of the tether-3 bases (Sec. 5.2.1); before the first step."""
        check(lib().fil_set_motor(self._h, float(d0), float(omega)))

    def set_wall(self):
        """No-slip plane wall at z = 0 (wall-bounded RPY mobility); before the first step."""
        check(lib().fil_set_wall(self._h))

    def set_periodic_fcm(self, box, grid, cut=7.5):
        """Periodic box of lengths box [3] with the force-coupling-method mobility on a grid
        of grid [3] points (Gaussians truncated at cut widths); before the first step."""
        import ctypes
        import numpy as np
        b = np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
        g = np.ascontiguousarray(np.broadcast_to(np.asarray(grid, dtype=np.int32), (3,)))
        check(lib().fil_set_periodic_fcm(self._h, b.ctypes.data_as(ctypes.c_void_p), g.ctypes.data_as(ctypes.c_void_p),
                                         float(cut)))

    def features(self):
        """Raw per-filament features [M, 19N] (float32, device) at the committed state."""
        import torch
        N = int(self.fil_off[1] - self.fil_off[0])
        out = torch.empty((self.M, 19 * N), dtype=torch.float32, device="cuda")
        check(lib().fil_sim_features(self._h, _ptr(out)))
        return out

    def step_target(self):
        """Scaled converged-minus-extrapolated unknowns of the last step [M, 6N] (float32, device)."""
        import torch
        N = int(self.fil_off[1] - self.fil_off[0])
        out = torch.empty((self.M, 6 * N), dtype=torch.float32, device="cuda")
        check(lib().fil_sim_step_target(self._h, _ptr(out)))
        return out

    def set_mlp(self, mlp, enable=True):
        """Use (or stop using) a trained MLP for the first iterate of each step."""
        self._mlp = mlp if enable else None
        check(lib().fil_sim_set_mlp(self._h, mlp._h if mlp is not None else None, int(enable)))

    def fallbacks(self):
        import ctypes
        n = ctypes.c_int64()
        check(lib().fil_sim_fallbacks(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().fil_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, raise_on_fail=True):
        """One implicit step; returns per-suspension reports (dicts)."""
        import ctypes
        from ._native import StepReport
        reps = (StepReport * self.nsusp)()
        rc = lib().fil_bdf2_step(self._h, reps)
        out = [dict(iters=r.iters, applies=r.mobility_applies, applies_f64=r.applies_f64,
                    converged=bool(r.converged), resid=r.resid, used_learned=bool(r.used_learned))
               for r in reps]
        if rc != 0 and raise_on_fail:
            check(rc)
        return out if rc == 0 else (rc, out)

    def jfnk_step(self, precond="j0", krylov_tol=1e-4, fd_delta=1e-7, krylov_max=1000, raise_on_fail=True):
        """One step by Jacobian-free Newton-Krylov (precond: "none", "pdt" or "j0");
        returns a dict of Newton and GMRES iterations and mobility applies."""
        return self._krylov_step(lib().fil_jfnk_step, precond, krylov_tol, fd_delta, krylov_max, raise_on_fail)

    def jfb_step(self, precond="j0", krylov_tol=1e-4, fd_delta=1e-7, krylov_max=1000, raise_on_fail=True):
        """One step by the Jacobian-free good Broyden method JFB-g ("newton" holds the
        Broyden iterations)."""
        return self._krylov_step(lib().fil_jfb_step, precond, krylov_tol, fd_delta, krylov_max, raise_on_fail)

    def _krylov_step(self, fn, precond, krylov_tol, fd_delta, krylov_max, raise_on_fail):
        import ctypes
        from ._native import JfnkReport
        rep = JfnkReport()
        rc = fn(self._h, {"none": 0, "pdt": 1, "j0": 2}[precond], float(krylov_tol), float(fd_delta),
                int(krylov_max), ctypes.byref(rep))
        out = dict(newton=rep.newton_iters, krylov=rep.krylov_iters, applies=rep.mobility_applies,
                   converged=bool(rep.converged), resid=rep.resid)
        if rc != 0 and raise_on_fail:
            check(rc)
        return out if rc == 0 else (rc, out)

    def read_state(self):
        """(Y [S,3], q [S,4], X^j [6S]) as numpy arrays (synchronising)."""
        import ctypes
        import numpy as np
        Y, q, X = np.zeros((self.S, 3)), np.zeros((self.S, 4)), np.zeros(6 * self.S)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        check(lib().fil_read_state(self._h, vp(Y), vp(q), vp(X)))
        return Y, q, X

    def checkpoint(self, path):
        """Committed state and per-suspension parameters to a file (synchronising)."""
        check(lib().fil_checkpoint(self._h, os.fsencode(path)))

    def restore(self, path):
        """State from a checkpoint of a simulation with the same layout."""
        check(lib().fil_restore(self._h, os.fsencode(path)))

    def time_step(self):
        import ctypes
        t, st = ctypes.c_double(), ctypes.c_int64()
        check(lib().fil_get_state(self._h, None, None, None, None, None, ctypes.byref(t), ctypes.byref(st)))
        return t.value, st.value

    def iterate(self):
        """Zero-copy view (torch, [6S]) of the current Broyden iterate X."""
        import ctypes
        import torch
        x = ctypes.c_void_p()
        check(lib().fil_get_state(self._h, None, None, None, ctypes.byref(x), None, None, None))
        return torch.as_tensor(_DevView(x.value, (6 * self.S,)), device="cuda")

    def set_timing(self, enable=True):
        check(lib().fil_set_timing(self._h, int(enable)))

    def timing(self):
        """{"f64": (ms, launches), "f32tile": (ms, launches)} of the mobility pair
        kernels since set_timing (summed durations, HIP events on the sim's stream)."""
        import ctypes
        ms, n = (ctypes.c_double * 2)(), (ctypes.c_int64 * 2)()
        check(lib().fil_get_timing(self._h, ms, n))
        return {"f64": (ms[0], n[0]), "f32tile": (ms[1], n[1])}

    def residual(self, X):
        import torch
        f = torch.empty(6 * self.S, dtype=torch.float64, device="cuda")
        check(lib().fil_residual(self._h, _ptr(X), _ptr(f)))
        return f

    def broyden_begin(self, X0):
        import torch
        f0 = torch.empty(6 * self.S, dtype=torch.float64, device="cuda")
        check(lib().fil_broyden_begin(self._h, _ptr(X0), _ptr(f0)))
        return f0

    def broyden_update(self, f_new):
        import torch
        dX = torch.empty(6 * self.S, dtype=torch.float64, device="cuda")
        check(lib().fil_broyden_update(self._h, _ptr(f_new), _ptr(dX)))
        return dX


class MLP:
    """The learned warm start's network for filaments of n_seg segments
    (19 n_seg inputs, `depth` SiLU layers of `width`, 6 n_seg outputs)."""

    def __init__(self, n_seg, width=256, depth=3, max_batch=1024, seed=0):
        import ctypes
        h = ctypes.c_void_p()
        check(lib().fil_mlp_create(n_seg, width, depth, max_batch, seed, ctypes.byref(h)))
        self._h = h
        dims = (ctypes.c_int32 * 8)()
        n = ctypes.c_int64()
        check(lib().fil_mlp_dims(h, dims, ctypes.byref(n)))
        (self.n_in, self.n_in_pad, self.n_out, self.n_out_pad, self.width, self.depth, self.max_batch,
         self.n_seg) = list(dims)
        self.n_params = n.value
        self.layer_dims = [(self.n_in_pad if l == 0 else width, width if l < depth else self.n_out_pad)
                           for l in range(depth + 1)]

    def close(self):
        if getattr(self, "_h", None):
            lib().fil_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        P = np.zeros(self.n_params, dtype=np.float32)
        check(lib().fil_mlp_get_params(self._h, P.ctypes.data))
        return P

    def set_params(self, P):
        import numpy as np
        P = np.ascontiguousarray(P, dtype=np.float32)
        assert P.size == self.n_params
        check(lib().fil_mlp_set_params(self._h, P.ctypes.data))

    def save(self, path):
        """Parameters and normalisation to a file."""
        check(lib().fil_mlp_save(self._h, os.fsencode(path)))

    def load(self, path):
        """Parameters and normalisation from a file of a network of the same architecture."""
        check(lib().fil_mlp_load(self._h, os.fsencode(path)))

    def get_norm(self):
        import numpy as np
        a = np.zeros(2 * (self.n_in_pad + self.n_out_pad), dtype=np.float32)
        check(lib().fil_mlp_get_norm(self._h, a.ctypes.data))
        return a

    def set_norm(self, a):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        check(lib().fil_mlp_set_norm(self._h, a.ctypes.data))

    def fit_norm(self, feat, targ):
        check(lib().fil_mlp_fit_norm(self._h, feat.shape[0], _ptr(feat), _ptr(targ), _stream()))

    def standardize(self, feat=None, targ=None):
        """(bf16 features as int16 [n, n_in_pad], standardised targets [n, n_out_pad]) on the device."""
        import torch
        n = (feat if feat is not None else targ).shape[0]
        xb = None if feat is None else torch.empty((n, self.n_in_pad), dtype=torch.int16, device="cuda")
        t = None if targ is None else torch.empty((n, self.n_out_pad), dtype=torch.float32, device="cuda")
        p = lambda a: None if a is None else _ptr(a)
        check(lib().fil_mlp_standardize(self._h, n, p(feat), p(targ), p(xb), p(t), _stream()))
        return xb, t

    def forward(self, xb):
        import torch
        Y = torch.empty((xb.shape[0], self.n_out_pad), dtype=torch.float32, device="cuda")
        check(lib().fil_mlp_forward(self._h, xb.shape[0], _ptr(xb), _ptr(Y), _stream()))
        return Y

    def backward(self, xb, t, rows=None, B=None):
        """(loss, flat gradient) of a minibatch (device tensors)."""
        import torch
        B = (rows.shape[0] if rows is not None else xb.shape[0]) if B is None else B
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        check(lib().fil_mlp_backward(self._h, B, None if rows is None else _ptr(rows), _ptr(xb), _ptr(t), _ptr(g),
                                     _ptr(loss), _stream()))
        return loss, g

    def adam_step(self, lr):
        check(lib().fil_mlp_adam_step(self._h, float(lr), _stream()))

    def train_step(self, xb, t, rows, lr, loss):
        check(lib().fil_mlp_train_step(self._h, rows.shape[0], _ptr(rows), _ptr(xb), _ptr(t), float(lr), _ptr(loss),
                                       _stream()))
