"""Pins of the oracle's quaternion algebra (Sec. 2.9.1, 2.9.3, Appendix A.1)
against textbook values, scipy's rotation routines and finite differences."""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")


def _rand_unit(rng, n=None):
    g = rng.standard_normal((n, 4) if n else 4)
    return g / np.linalg.norm(g, axis=-1, keepdims=True)


def _scipy_quat(q):
    # scipy stores (x, y, z, w)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]])


def test_basis_products():
    one, i, j, k = np.eye(4)
    assert np.allclose(oracle.qmul(i, j), k)
    assert np.allclose(oracle.qmul(j, k), i)
    assert np.allclose(oracle.qmul(k, i), j)
    assert np.allclose(oracle.qmul(j, i), -k)
    for e in (i, j, k):
        assert np.allclose(oracle.qmul(e, e), -one)
    assert np.allclose(oracle.qmul(one, i), i)


def test_product_associative_and_norm_multiplicative():
    rng = np.random.default_rng(1)
    for _ in range(20):
        p, q, r = rng.standard_normal((3, 4))
        lhs = oracle.qmul(oracle.qmul(p, q), r)
        rhs = oracle.qmul(p, oracle.qmul(q, r))
        assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-13)
        assert math.isclose(np.linalg.norm(oracle.qmul(p, q)), np.linalg.norm(p) * np.linalg.norm(q), rel_tol=1e-13)


def test_rotation_matrix_matches_scipy_and_composition():
    rng = np.random.default_rng(2)
    for _ in range(20):
        p, q = _rand_unit(rng), _rand_unit(rng)
        R = oracle.qrot(q)
        assert np.allclose(R, _scipy_quat(q).as_matrix(), atol=1e-14)
        assert np.allclose(oracle.qrot(oracle.qmul(p, q)), oracle.qrot(p) @ R, atol=1e-13)
        # w' = q . (0, w) . q^*
        w = rng.standard_normal(3)
        qc = q * np.array([1, -1, -1, -1])
        wq = oracle.qmul(oracle.qmul(q, np.concatenate([[0], w])), qc)
        assert np.allclose(wq[1:], R @ w, atol=1e-13)
        assert abs(wq[0]) < 1e-14


def test_rotation_about_z_textbook():
    th = 0.7
    q = np.array([math.cos(th / 2), 0, 0, math.sin(th / 2)])
    assert np.allclose(oracle.qrot(q) @ [1, 0, 0], [math.cos(th), math.sin(th), 0], atol=1e-15)


def test_sqrt_properties():
    rng = np.random.default_rng(3)
    for _ in range(50):
        p = _rand_unit(rng)
        h = oracle.qsqrt(p)
        assert math.isclose(np.linalg.norm(h), 1.0, rel_tol=1e-14)          # (a) unit
        assert np.allclose(oracle.qmul(h, h), p, atol=1e-14)               # (b) h.h = p
        assert h[0] >= 0
    assert np.array_equal(oracle.qsqrt([-1.0, 0, 0, 0]), [0, 0, 0, 1.0])


def test_sqrt_maps_a_to_b():
    """Appendix A.1: (a.b, a x b)^{1/2} rotates a onto b."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        a, b = rng.standard_normal((2, 3))
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        h = oracle.qsqrt(np.concatenate([[a @ b], np.cross(a, b)]))
        assert np.allclose(oracle.qrot(h) @ a, b, atol=1e-13)


def test_midpoint_is_half_rotation():
    rng = np.random.default_rng(5)
    for _ in range(20):
        qn = _rand_unit(rng)
        axis = rng.standard_normal(3)
        axis /= np.linalg.norm(axis)
        th = rng.uniform(-2.5, 2.5)
        qn1 = oracle.qmul(oracle.qexp(th * axis), qn)
        mid = oracle.qmid(qn, qn1)
        assert np.allclose(mid, oracle.qmul(oracle.qexp(0.5 * th * axis), qn), atol=1e-13)


def test_exp_matches_scipy_rotvec():
    rng = np.random.default_rng(6)
    for _ in range(30):
        u = rng.standard_normal(3) * rng.uniform(0, 3)
        q = oracle.qexp(u)
        r = Rotation.from_rotvec(u).as_quat()
        assert np.allclose(q, [r[3], r[0], r[1], r[2]], atol=1e-14)
    assert np.array_equal(oracle.qexp([0, 0, 0]), [1, 0, 0, 0])


def test_fixed_axis_example():
    """Sec. 2.9.3 worked example: Omega = alpha e_z from q(0) = I gives
    u(t) = alpha t e_z and q(t) = (cos(alpha t/2), 0, 0, sin(alpha t/2))."""
    ex = json.load(open(GOLD))["fixed_axis_rotation"]
    for alpha, t in ex["cases"]:
        u = np.array([0, 0, alpha * t])
        q = oracle.qexp(u)
        assert np.allclose(q, [math.cos(alpha * t / 2), 0, 0, math.sin(alpha * t / 2)], atol=1e-15)
        # u' = dexpinv_u(Omega) = Omega along a fixed axis
        assert np.allclose(oracle.dexpinv(u, [0, 0, alpha]), [0, 0, alpha], atol=1e-14)


def _angvel_of_exp(u, v, h=1e-6):
    """Omega with d/ds exp(u + s v) = 1/2 (0, Omega) . exp(u), by central differences."""
    qp, qm, q = oracle.qexp(u + h * v), oracle.qexp(u - h * v), oracle.qexp(u)
    dq = (qp - qm) / (2 * h)
    w = 2 * oracle.qmul(dq, q * np.array([1, -1, -1, -1]))
    return w[1:]


@pytest.mark.parametrize("scale", [1e-5, 1e-3, 0.02, 0.5, 1.5, 3.0])
def test_dexpinv_inverts_the_differential_of_exp(scale):
    """dexpinv_u(Omega) is the u-rate that produces angular velocity Omega."""
    rng = np.random.default_rng(int(scale * 1e6) % 2**31)
    for _ in range(10):
        u = rng.standard_normal(3)
        u *= scale / np.linalg.norm(u)
        v = rng.standard_normal(3)
        om = _angvel_of_exp(u, v)
        assert np.allclose(oracle.dexpinv(u, om), v, atol=2e-8 * max(1, np.linalg.norm(v)))


def test_dexpinv_taylor_branch_is_continuous():
    """The small-|u| branch (reading R10) meets the closed form at the switch."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        w = rng.standard_normal(3)
        lo = oracle.dexpinv(d * (1e-3 * (1 - 1e-9)), w)
        hi = oracle.dexpinv(d * (1e-3 * (1 + 1e-9)), w)
        # u itself moves by 2e-12 across the switch (a ~1e-12 change); a wrong
        # x^2/720 term would jump by ~1e-9
        assert np.allclose(lo, hi, rtol=0, atol=2e-11 * np.linalg.norm(w))


def test_dexpinv_three_term_taylor_limit():
    """Appendix B.2: dexpinv_u(v) ~ v - u x v/2 + u x (u x v)/12 for small u."""
    rng = np.random.default_rng(8)
    for _ in range(10):
        u = rng.standard_normal(3) * 1e-2
        v = rng.standard_normal(3)
        tay = v - 0.5 * np.cross(u, v) + np.cross(u, np.cross(u, v)) / 12
        assert np.allclose(oracle.dexpinv(u, v), tay, atol=1e-8 * np.linalg.norm(v))
