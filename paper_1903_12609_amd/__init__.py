"""MI355X filament library: Python binding of libfil.so.

The hot path of the implicit quaternion filament method (arXiv:1903.12609)
runs in hand-written HIP kernels; this module only hands torch device
tensors (float64, component-major ``[3, S]``) and the current HIP stream to
the C ABI declared in ``include/fil.h``.
"""
from __future__ import annotations

from ._native import FilError, PREC, check, lib  # noqa: F401

__all__ = ["FilError", "rpy_mobility_apply", "rpy_workspace_bytes", "filament_internal_forces"]


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


def rpy_mobility_apply(Y, F, T, a=1.0, eta=1.0, prec="f64", V=None, W=None, work=None):
    """(V, Omega) = RPY mobility (Sec. 2.7.1) applied to forces F and torques T at
    positions Y; all float64 CUDA tensors of shape (3, S)."""
    import torch
    S = Y.shape[1]
    for n, t in (("Y", Y), ("F", F), ("T", T)):
        _check_soa(n, t, 3, S)
    V = torch.empty_like(Y) if V is None else V
    W = torch.empty_like(Y) if W is None else W
    nb = rpy_workspace_bytes(S, prec)
    if work is None or work.numel() < nb:
        work = torch.empty(max(nb, 1), dtype=torch.uint8, device=Y.device)
    check(lib().fil_rpy_mobility_apply(S, _ptr(Y), _ptr(F), _ptr(T), float(a), float(eta), PREC[prec], _ptr(V),
                                       _ptr(W), _ptr(work), work.numel(), _stream()))
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
