"""Pins of the oracle's RPY mobility (Sec. 2.7.1) and steric barrier (Sec. 2.6).

The far-field blocks are checked against Stokes-flow singularities evaluated
by finite differences (Stokeslet, its Laplacian and curl, the rotlet), the
overlap branch against the self limit and value/slope continuity at r = 2a,
and the assembled matrix against symmetry and positive-definiteness."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1903_12609_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def oseen(x, eta=1.0):
    """Stokeslet G(x) = (I/|x| + x x^T/|x|^3) / (8 pi eta)."""
    r = np.linalg.norm(x)
    return (np.eye(3) / r + np.outer(x, x) / r ** 3) / (8 * math.pi * eta)


def curl_of_field(fun, x, h=1e-4):
    """Curl of a vector field by central differences."""
    J = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, j] = (fun(x + e) - fun(x - e)) / (2 * h)
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])


def laplacian_of_tensor(fun, x, h=1e-3):
    L = -6 * fun(x)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        L = L + fun(x + e) + fun(x - e)
    return L / h ** 2


@pytest.mark.parametrize("case", GOLD["single_sphere_mobility"]["cases"])
def test_single_sphere(case):
    a, eta = case["a"], case["eta"]
    rng = np.random.default_rng(11)
    F, T = rng.standard_normal((2, 1, 3))
    V, W = oracle.rpy_apply(np.zeros((1, 3)), F, T, a, eta)
    assert np.allclose(V, F / (6 * math.pi * eta * a), rtol=1e-15, atol=0)
    assert np.allclose(W, T / (8 * math.pi * eta * a ** 3), rtol=1e-15, atol=0)


@pytest.mark.parametrize("d", [2.2, 5.0, 100.0])
def test_far_field_tt_is_stokeslet_plus_laplacian(d):
    """Non-overlapping M^tt = (1 + a^2/3 Laplacian) Stokeslet."""
    rng = np.random.default_rng(12)
    a, eta = 1.0, 1.0
    for _ in range(3):
        x = rng.standard_normal(3)
        x *= d / np.linalg.norm(x)
        Mtt, Mtr, Mrt, Mrr = oracle.rpy_blocks(x, False, a, eta)
        ref = oseen(x) + a * a / 3 * laplacian_of_tensor(oseen, x, h=1e-3 * d)
        assert np.allclose(Mtt, ref, rtol=1e-6, atol=1e-8 / d)


@pytest.mark.parametrize("d", [2.2, 5.0, 40.0])
def test_rotation_translation_coupling_is_half_curl_of_stokeslet(d):
    """Omega of a sphere in the Stokeslet flow: Mrt F = 1/2 curl(G F); by symmetry
    Mtr T = T x r / (8 pi eta r^3), the point-torque (rotlet) flow.  Pins reading R1."""
    rng = np.random.default_rng(13)
    for _ in range(3):
        x = rng.standard_normal(3)
        x *= d / np.linalg.norm(x)
        F = rng.standard_normal(3)
        Mtt, Mtr, Mrt, Mrr = oracle.rpy_blocks(x, False, 1.0, 1.0)
        w = 0.5 * curl_of_field(lambda y: oseen(y) @ F, x, h=1e-4 * d)
        assert np.allclose(Mrt @ F, w, rtol=1e-7, atol=1e-12)
        T = rng.standard_normal(3)
        ref = np.cross(T, x) / (8 * math.pi * d ** 3)
        assert np.allclose(Mtr @ T, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("d", [2.2, 5.0, 40.0])
def test_rotation_rotation_is_half_curl_of_rotlet(d):
    rng = np.random.default_rng(14)
    for _ in range(3):
        x = rng.standard_normal(3)
        x *= d / np.linalg.norm(x)
        T = rng.standard_normal(3)
        Mrr = oracle.rpy_blocks(x, False, 1.0, 1.0)[3]
        rotlet = lambda y: np.cross(T, y) / (8 * math.pi * np.linalg.norm(y) ** 3)
        w = 0.5 * curl_of_field(rotlet, x, h=1e-4 * d)
        assert np.allclose(Mrr @ T, w, rtol=1e-7, atol=1e-12)


def test_far_field_tends_to_oseen():
    x = np.array([1.0, 2.0, -2.0]) * 1e4
    Mtt, Mtr, Mrt, Mrr = oracle.rpy_blocks(x, False, 1.0, 1.0)
    assert np.allclose(Mtt, oseen(x), rtol=1e-8)


def _blocks_at(rvec, a=1.0):
    return np.stack(oracle.rpy_blocks(rvec, False, a, 1.0))


@pytest.mark.parametrize("a", [1.0, 0.7])
def test_overlap_continuity_value_and_slope_at_contact(a):
    """Reading R2: the overlap forms (polynomials in r) meet the far-field tensors
    at r = 2a in value and first derivative; together with the self limit this
    fixes every coefficient."""
    rh = np.array([2.0, -1.0, 0.5])
    rh /= np.linalg.norm(rh)
    c = 2 * a
    lo, hi = _blocks_at(rh * c * (1 - 1e-12), a), _blocks_at(rh * c * (1 + 1e-12), a)
    assert np.allclose(lo, hi, rtol=0, atol=1e-12 / a ** 3)
    h = 1e-5 * a
    slope_in = (_blocks_at(rh * (c - h), a) - _blocks_at(rh * (c - 3 * h), a)) / (2 * h)
    slope_out = (_blocks_at(rh * (c + 3 * h), a) - _blocks_at(rh * (c + h), a)) / (2 * h)
    # one-sided second-order-free estimates at c -+ 2h; curvature error O(h)
    assert np.allclose(slope_in, slope_out, rtol=0, atol=5e-5 / a ** 4)


def test_overlap_tends_to_self_terms():
    a, eta = 1.3, 0.8
    for d in (1e-9, 1e-6):
        blocks = oracle.rpy_blocks(np.array([d, 0, 0]), False, a, eta)
        selfb = oracle.rpy_blocks(np.zeros(3), True, a, eta)
        for b, s in zip(blocks, selfb):
            assert np.allclose(b, s, rtol=0, atol=0.1 * d)     # every correction is O(r)
    # coincident distinct spheres: exactly the self mobility
    blocks = oracle.rpy_blocks(np.zeros(3), False, a, eta)
    selfb = oracle.rpy_blocks(np.zeros(3), True, a, eta)
    for b, s in zip(blocks, selfb):
        assert np.allclose(b, s, atol=0)


@pytest.mark.parametrize("overlap", [False, True])
def test_assembled_matrix_symmetric_positive_definite(overlap):
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        S = 40
        if overlap:
            Y = rng.uniform(0, 6.0, (S, 3))       # dense: many r < 2a
        else:
            Y = synth.random_cloud(S, seed, 30.0, min_sep=2.05)
        Mg = oracle.rpy_matrix(Y, 1.0, 1.0)
        assert np.allclose(Mg, Mg.T, rtol=0, atol=1e-15)
        np.linalg.cholesky(Mg)                    # raises unless SPD
        F, T = rng.standard_normal((2, S, 3))
        V, W = oracle.rpy_apply(Y, F, T, 1.0, 1.0)
        assert (F * V).sum() + (T * W).sum() > 0
        # apply equals the assembled matrix
        x = np.concatenate([F.ravel(), T.ravel()])
        y = Mg @ x
        assert np.allclose(np.concatenate([V.ravel(), W.ravel()]), y, rtol=1e-13, atol=1e-15)


def test_linearity_translation_rotation_covariance():
    rng = np.random.default_rng(20)
    S = 30
    Y = rng.uniform(0, 12.0, (S, 3))
    F, T, F2, T2 = rng.standard_normal((4, S, 3))
    V, W = oracle.rpy_apply(Y, F, T, 1.0, 1.0)
    V2, W2 = oracle.rpy_apply(Y, F2, T2, 1.0, 1.0)
    Vs, Ws = oracle.rpy_apply(Y, 2 * F - F2, 2 * T - T2, 1.0, 1.0)
    assert np.allclose(Vs, 2 * V - V2, atol=1e-13)
    assert np.allclose(Ws, 2 * W - W2, atol=1e-13)
    Vt, Wt = oracle.rpy_apply(Y + np.array([3.0, -7.0, 11.0]), F, T, 1.0, 1.0)
    assert np.allclose(Vt, V, atol=1e-13) and np.allclose(Wt, W, atol=1e-13)
    from scipy.spatial.transform import Rotation
    R = Rotation.random(random_state=3).as_matrix()
    Vr, Wr = oracle.rpy_apply(Y @ R.T, F @ R.T, T @ R.T, 1.0, 1.0)
    assert np.allclose(Vr, V @ R.T, atol=1e-13)
    # torque and angular velocity are axial vectors; proper rotations keep them covariant
    assert np.allclose(Wr, W @ R.T, atol=1e-13)


def test_parallel_targets_same_result():
    Y, F, T = synth.rpy_throughput_inputs(300, seed=2)
    V1, W1 = oracle.rpy_apply(Y, F, T, 1.0, 1.0, nthreads=1)
    V4, W4 = oracle.rpy_apply(Y, F, T, 1.0, 1.0, nthreads=4)
    assert np.array_equal(V1, V4) and np.array_equal(W1, W4)


# ------------------------------------------------------------------ steric barrier, Sec. 2.6
def test_steric_contact_strength_range_and_direction():
    chi = GOLD["steric_contact_strength"]["chi"]
    a, FS = 1.0, 3.5
    e = np.array([0.6, 0.0, 0.8])
    Y = np.stack([np.zeros(3), 2 * a * e])
    FB = oracle.steric(Y, [0, 1], a, chi, FS)
    assert np.allclose(FB[0], -FS * e, rtol=1e-14)     # F^S at contact, pushing 0 away from 1
    assert np.allclose(FB[1], FS * e, rtol=1e-14)
    Y = np.stack([np.zeros(3), 2 * chi * a * e * (1 + 1e-12)])
    assert np.all(oracle.steric(Y, [0, 1], a, chi, FS) == 0)
    Y = np.stack([np.zeros(3), 2 * chi * a * e * (1 - 1e-6)])
    f = oracle.steric(Y, [0, 1], a, chi, FS)
    assert 0 < np.linalg.norm(f[0]) < 1e-15 * FS * 1e6


def test_steric_quartic_profile_and_neighbour_exclusion():
    a, chi, FS = 1.0, 1.1, 2.0
    d = 2.1
    Y = np.stack([np.zeros(3), [d, 0, 0], [2 * d, 0, 0]])
    # same filament: 0-1 and 1-2 are neighbours (excluded), 0-2 too far
    assert np.all(oracle.steric(Y, [0, 0, 0], a, chi, FS) == 0)
    FB = oracle.steric(Y, [0, 1, 2], a, chi, FS)
    b = (4 * a * a * chi * chi - d * d) / (4 * a * a * (chi * chi - 1))
    assert b > 0
    # profile is (1 - x)^4 in x = (r^2 - 4a^2) / (4a^2 (chi^2 - 1)): check ratio at two distances
    Y2 = np.stack([np.zeros(3), [2.15, 0, 0]])
    f1 = np.linalg.norm(oracle.steric(np.stack([np.zeros(3), [d, 0, 0]]), [0, 1], a, chi, FS)[0])
    f2 = np.linalg.norm(oracle.steric(Y2, [0, 1], a, chi, FS)[0])
    x = lambda r: (r * r - 4 * a * a) / (4 * a * a * (chi * chi - 1))
    assert math.isclose(f1 / f2, ((1 - x(d)) ** 4 * d) / ((1 - x(2.15)) ** 4 * 2.15), rel_tol=1e-13)
    assert np.allclose(FB.sum(axis=0), 0, atol=1e-14)   # pairwise equal and opposite


def test_sampled_targets_match_full_apply():
    Y, F, T = synth.rpy_throughput_inputs(400, seed=5)
    V, W = oracle.rpy_apply(Y, F, T, 1.0, 1.0)
    idx = np.array([0, 3, 17, 399, 200])
    v, w = oracle.rpy_apply_targets(Y, F, T, 1.0, 1.0, idx)
    assert np.array_equal(v, V[idx]) and np.array_equal(w, W[idx])
