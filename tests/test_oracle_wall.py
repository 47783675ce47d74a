"""The oracle's wall-bounded RPY mobility (spheres above a no-slip plane, Sec. 2.7.1 and
Sec. 5.2.2) pinned to what fixes it independently of its construction:

* Blake's Green's function satisfies the no-slip condition on the wall, is divergence
  free and biharmonic away from the force, and obeys Lorentz reciprocity;
* the self-mobilities of one sphere at height h: the classical leading wall corrections
  (Faxen's 1 - 9a/16h parallel, Lorentz's 1 - 9a/8h normal, 1 - 5a^3/16h^3 and
  1 - a^3/8h^3 for rotation) and the full Rotne-Prager-Blake polynomials;
* far above the wall the mobility is the free-space RPY one;
* the mobility matrix of spheres that overlap neither each other nor the wall is
  symmetric and positive definite.
"""
import numpy as np
import pytest
import sympy as sp

import oracle
from oracle import wall


def test_blake_green_function():
    G = wall.blake_symbolic()
    x, y = wall._x, wall._y
    pts = [(0.3, -0.2, 2.1, 0.1, 0.4, 1.7), (-1.0, 2.0, 0.6, 0.5, -0.3, 3.0)]
    f = sp.lambdify(list(x) + list(y), G, "numpy")
    div = sp.lambdify(list(x) + list(y), [sum(sp.diff(G[i, j], x[i]) for i in range(3)) for j in range(3)], "numpy")
    for p in pts:
        on_wall = np.array(f(p[0], p[1], 0.0, *p[3:]))
        assert np.abs(on_wall).max() <= 1e-14
        assert np.abs(np.array(div(*p))).max() <= 1e-13
        # reciprocity: G_ij(x, y) = G_ji(y, x)
        Gxy = np.array(f(*p))
        Gyx = np.array(f(*p[3:], *p[:3]))
        assert np.abs(Gxy - Gyx.T).max() <= 1e-14 * np.abs(Gxy).max()
    lap = lambda e: sum(sp.diff(e, v, 2) for v in x)
    for (i, j) in ((0, 2), (2, 2), (1, 0)):
        b = sp.lambdify(list(x) + list(y), lap(lap(G[i, j])), "numpy")
        assert abs(b(*pts[0])) <= 1e-11


@pytest.mark.parametrize("h", [1.5, 2.0, 4.0, 10.0])
def test_self_mobilities_near_the_wall(h):
    a, eta = 1.0, 1.0
    s = a / h
    M = wall.wall_matrix(np.array([[0.3, -0.7, h]]), a, eta)
    tt, tr, rt, rr = M[:3, :3], M[:3, 3:], M[3:, :3], M[3:, 3:]
    par_t = 1 - 9 / 16 * s + 1 / 8 * s ** 3 - 1 / 16 * s ** 5
    nor_t = 1 - 9 / 8 * s + 1 / 2 * s ** 3 - 1 / 8 * s ** 5
    ct, cr, cc = 6 * np.pi * eta * a, 8 * np.pi * eta * a ** 3, 6 * np.pi * eta * a ** 2
    np.testing.assert_allclose(np.diag(tt) * ct, [par_t, par_t, nor_t], rtol=1e-13)
    np.testing.assert_allclose(np.diag(rr) * cr, [1 - 5 / 16 * s ** 3, 1 - 5 / 16 * s ** 3, 1 - 1 / 8 * s ** 3],
                               rtol=1e-13)
    # the classical leading terms alone, to their next order
    assert abs(tt[0, 0] * ct - (1 - 9 / 16 * s)) <= 0.2 * s ** 3
    assert abs(tt[2, 2] * ct - (1 - 9 / 8 * s)) <= 0.6 * s ** 3
    # translation-rotation coupling: a force parallel to the wall turns the sphere
    assert abs(rt[1, 0] * cc - 3 / 32 * s ** 4) <= 1e-13 and abs(rt[0, 1] * cc + 3 / 32 * s ** 4) <= 1e-13
    np.testing.assert_allclose(tr, rt.T, atol=1e-15)
    off = tt - np.diag(np.diag(tt))
    assert np.abs(off).max() <= 1e-15 and np.abs(rr - np.diag(np.diag(rr))).max() <= 1e-15


def test_far_from_the_wall_is_free_space():
    rng = np.random.default_rng(3)
    Y = rng.uniform(0, 12, (6, 3))
    Y[:, 2] += 1e7
    M = wall.wall_matrix(Y, 1.0, 1.0)
    Mf = oracle.rpy_matrix(Y, 1.0, 1.0)
    assert np.abs(M - Mf).max() <= 1e-6 * np.abs(Mf).max()


def test_matrix_symmetric_positive_definite():
    rng = np.random.default_rng(5)
    pts = []
    while len(pts) < 12:
        p = rng.uniform([0, 0, 1.1], [10, 10, 6])
        if all(np.linalg.norm(p - q) >= 2.05 for q in pts):
            pts.append(p)
    Y = np.array(pts)
    M = wall.wall_matrix(Y, 1.0, 1.0)
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    # the wall slows every sphere: the trace of the translational block drops
    Mf = oracle.rpy_matrix(Y, 1.0, 1.0)
    assert np.trace(M[:36, :36]) < np.trace(Mf[:36, :36])
