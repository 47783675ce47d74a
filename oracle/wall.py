"""Test infrastructure (not the product path): the Rotne-Prager-Yamakawa mobility of
equal spheres above a no-slip plane wall z = 0, the wall-bounded RPY tensor that the paper
cites for its cilia (Sec. 2.7.1, Sec. 5.2.2; Swan & Brady 2007), built here from its
definition.

Blake's solution for a unit point force at y above the wall (velocity at x, times 8 pi eta):
    G_ij(x, y) = S_ij(x - y) - S_ij(x - y*) + 2 y_3 s_j d/dx_j [y_3 r*_i / |r*|^3 - S_i3(r*)],
with S_ij(v) = delta_ij / |v| + v_i v_j / |v|^3, y* = (y_1, y_2, -y_3) the mirror point,
r* = x - y*, s = (1, 1, -1) (no sum over j).  The mobility of spheres of radius a at x
(target) and y (source) is the free-space RPY tensor (the oracle's, with its overlap
forms) plus the image part G^im = G - S(x - y) under the Faxen operators of both spheres:
    tt = (1 + a^2/6 lap_x)(1 + a^2/6 lap_y) G^im / (8 pi eta)
    tr = 1/2 curl_y (1 + a^2/6 lap_x) G^im / (8 pi eta)   (translation at x, torque at y)
    rt = 1/2 curl_x (1 + a^2/6 lap_y) G^im / (8 pi eta)   (rotation at x, force at y)
    rr = 1/4 curl_x curl_y G^im / (8 pi eta)
The self terms are the free ones, 1/(6 pi eta a) and 1/(8 pi eta a^3), plus the image part
at x = y.  The derivatives are taken symbolically (sympy) from these formulas and
evaluated with numpy over all pairs at once, in float64.
"""
import functools

import numpy as np
import sympy as sp

_x = sp.symbols("x1 x2 x3", real=True)
_y = sp.symbols("y1 y2 y3", real=True)
_a = sp.Symbol("a", positive=True)


def _S(v, i, j):
    n = sp.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    return (1 if i == j else 0) / n + v[i] * v[j] / n ** 3


def blake_symbolic(image_only=False):
    """G_ij(x, y) (times 8 pi eta) as a 3 x 3 sympy matrix in x1..x3, y1..y3."""
    r = [_x[k] - _y[k] for k in range(3)]
    rs = [_x[0] - _y[0], _x[1] - _y[1], _x[2] + _y[2]]
    ns = sp.sqrt(rs[0] ** 2 + rs[1] ** 2 + rs[2] ** 2)
    G = sp.zeros(3, 3)
    for i in range(3):
        for j in range(3):
            inner = _y[2] * rs[i] / ns ** 3 - _S(rs, i, 2)
            s = 1 if j < 2 else -1
            g = -_S(rs, i, j) + 2 * _y[2] * s * sp.diff(inner, _x[j])
            G[i, j] = g if image_only else g + _S(r, i, j)
    return G


def _lap(e, v):
    return sum(sp.diff(e, vk, 2) for vk in v)


def _eps(i, j, k):
    return int(sp.LeviCivita(i, j, k))


@functools.lru_cache(maxsize=None)
def _image_functions():
    """numpy functions of (x1, x2, x3, y1, y2, y3, a) for the 36 image entries (times 8 pi eta)."""
    G = blake_symbolic(image_only=True)
    Ly = [[G[i, j] + _a ** 2 / 6 * _lap(G[i, j], _y) for j in range(3)] for i in range(3)]
    Lx = [[G[i, j] + _a ** 2 / 6 * _lap(G[i, j], _x) for j in range(3)] for i in range(3)]
    tt = [[Ly[i][j] + _a ** 2 / 6 * _lap(Ly[i][j], _x) for j in range(3)] for i in range(3)]
    tr = [[sum(_eps(j, m, n) * sp.diff(Lx[i][n], _y[m]) for m in range(3) for n in range(3)) / 2
           for j in range(3)] for i in range(3)]
    rt = [[sum(_eps(i, k, l) * sp.diff(Ly[l][j], _x[k]) for k in range(3) for l in range(3)) / 2
           for j in range(3)] for i in range(3)]
    rr = [[sum(_eps(i, k, l) * _eps(j, m, n) * sp.diff(G[l, n], _x[k], _y[m])
               for k in range(3) for l in range(3) for m in range(3) for n in range(3)) / 4
           for j in range(3)] for i in range(3)]
    args = list(_x) + list(_y) + [_a]
    out = {}
    for name, M in (("tt", tt), ("tr", tr), ("rt", rt), ("rr", rr)):
        flat = [M[i][j] for i in range(3) for j in range(3)]
        out[name] = sp.lambdify(args, flat, modules="numpy", cse=True)
    return out


def wall_matrix(Y, a, eta):
    """The 6S x 6S mobility [V; Omega] = M [F; T] (rows and columns ordered like the
    oracle's free-space rpy_matrix: all V, then all Omega, each [S][3]) of spheres at
    Y [S, 3] above the wall z = 0."""
    from . import rpy_matrix
    Y = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(-1, 3))
    S = Y.shape[0]
    M = rpy_matrix(Y, a, eta).copy()
    fn = _image_functions()
    xi = [np.repeat(Y[:, k], S) for k in range(3)]   # target of pair (i, j) at i * S + j
    yj = [np.tile(Y[:, k], S) for k in range(3)]     # source
    c = 1.0 / (8.0 * np.pi * eta)
    for name, (ro, co) in (("tt", (0, 0)), ("tr", (0, 3 * S)), ("rt", (3 * S, 0)), ("rr", (3 * S, 3 * S))):
        vals = fn[name](*xi, *yj, a)
        for e in range(9):
            i, j = divmod(e, 3)
            v = np.broadcast_to(np.asarray(vals[e], dtype=np.float64), (S * S,)).reshape(S, S)
            M[ro + i:ro + 3 * S:3, co + j:co + 3 * S:3] += c * v
    return M


def wall_rpy_apply(Y, F, T, a, eta, targets=None):
    """(V, Omega) [S, 3] of spheres at Y above the wall with forces F and torques T [S, 3];
    with targets (indices) only those rows, [len(targets), 3]."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    F = np.asarray(F, dtype=np.float64).reshape(-1, 3)
    T = np.asarray(T, dtype=np.float64).reshape(-1, 3)
    S = Y.shape[0]
    if targets is None:
        M = wall_matrix(Y, a, eta)
        u = M @ np.concatenate([F.ravel(), T.ravel()])
        return u[:3 * S].reshape(S, 3), u[3 * S:].reshape(S, 3)
    from . import rpy_apply_targets
    idx = np.asarray(targets, dtype=np.int64)
    V, W = rpy_apply_targets(Y, F, T, a, eta, idx)
    fn = _image_functions()
    n = len(idx)
    xi = [np.repeat(Y[idx, k], S) for k in range(3)]
    yj = [np.tile(Y[:, k], n) for k in range(3)]
    c = 1.0 / (8.0 * np.pi * eta)
    for name, out, src in (("tt", V, F), ("tr", V, T), ("rt", W, F), ("rr", W, T)):
        vals = fn[name](*xi, *yj, a)
        for e in range(9):
            i, j = divmod(e, 3)
            v = np.broadcast_to(np.asarray(vals[e], dtype=np.float64), (n * S,)).reshape(n, S)
            out[:, i] += c * (v @ src[:, j])
    return V, W
