"""Helpers for GPU parity tests: device transfers and error norms."""
import numpy as np


def dev(a, rows_first=True):
    """numpy [S, k] (AoS) -> contiguous float64 CUDA tensor [k, S] (SoA)."""
    import torch
    a = np.asarray(a, dtype=np.float64)
    if rows_first:
        a = a.T
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    """CUDA tensor [k, S] (SoA) -> numpy [S, k] (AoS)."""
    return t.detach().cpu().numpy().T.copy()


def rel_l2(x, ref):
    x, ref = np.asarray(x), np.asarray(ref)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))
