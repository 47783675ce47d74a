"""The oracle's force-coupling-method mobility (Sec. 2.7.2) pinned to what is known
independently of it: the self-mobilities of a particle in a periodic box (Hasimoto's
expansion; the rotational one of a sphere), the symmetry and positive definiteness of
the mobility matrix that spreading and averaging with the same Gaussians produce, and
the far field of a pair against the free-space RPY tensors."""
import numpy as np

import oracle
from oracle import fcm

HASIMOTO = 2.837297  # periodic correction of the drag of a sphere in a cubic lattice


def _single(L, n, F, T):
    Y = np.array([[L / 2 + 0.13, L / 2 - 0.21, L / 2 + 0.05]])  # off the grid nodes
    return fcm.fcm_apply(Y, np.array([F]), np.array([T]), 1.0, 1.0, L, n)


def test_self_mobilities_in_a_periodic_box():
    d = []
    for L, n in ((16.0, 48), (32.0, 96)):
        V, _ = _single(L, n, [1.0, 0.0, 0.0], [0.0, 0.0, 0.0])
        mu = V[0, 0] * 6.0 * np.pi
        ref = 1.0 - HASIMOTO / L + 4.0 * np.pi / 3.0 / L ** 3
        d.append(mu - ref)
        # the translational mobility of the Gaussian is 1 / (6 pi eta a) with the lattice
        # correction up to a third-order term (Gaussian vs sphere)
        assert abs(mu - ref) <= 0.25 / L ** 3, (L, mu, ref)
        _, W = _single(L, n, [0.0, 0.0, 0.0], [0.0, 0.0, 1.0])
        om = W[0, 2] * 8.0 * np.pi
        assert abs(om - (1.0 - 4.0 * np.pi / 3.0 / L ** 3)) <= 1e-7, (L, om)
    assert 6.0 < d[0] / d[1] < 10.0  # third order in a / L


def test_mobility_matrix_symmetric_positive_definite():
    rng = np.random.default_rng(9)
    L, n, S = 12.0, 32, 3
    Y = rng.uniform(0, L, (S, 3))
    M = np.zeros((6 * S, 6 * S))
    for j in range(6 * S):
        e = np.zeros(6 * S)
        e[j] = 1.0
        V, W = fcm.fcm_apply(Y, e[:3 * S].reshape(S, 3), e[3 * S:].reshape(S, 3), 1.0, 1.0, L, n)
        M[:, j] = np.concatenate([V.ravel(), W.ravel()])
    # translation-translation: spreading and averaging with the same Gaussian are adjoint
    # on the grid, so that block is symmetric to rounding
    tt = M[:3 * S, :3 * S]
    assert np.abs(tt - tt.T).max() <= 1e-13 * np.abs(M).max()
    # the rotlet is spread with the analytic grad Theta and Omega averaged from the
    # spectral curl: adjoint in the continuum, here up to the discretisation (3e-8)
    assert np.abs(M - M.T).max() <= 1e-7 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0


def test_pair_far_field_matches_rpy():
    """Two particles 8a apart in a 48a box: the pair block of the FCM mobility is the
    free-space RPY one shifted by the lattice term -2.837 / (6 pi eta L) (the same shift
    as the self term at leading order)."""
    L, n = 48.0, 144
    Y = np.array([[L / 2 - 4.0 + 0.1, L / 2 + 0.07, L / 2 - 0.03], [L / 2 + 4.0 + 0.1, L / 2 + 0.07, L / 2 - 0.03]])
    F = np.array([[0.3, 1.0, -0.5], [0.0, 0.0, 0.0]])
    T = np.zeros((2, 3))
    V, _ = fcm.fcm_apply(Y, F, T, 1.0, 1.0, L, n)
    Vr, _ = oracle.rpy_apply(Y, F, T, 1.0, 1.0)
    ref = Vr[1] - HASIMOTO / (6.0 * np.pi * L) * F[0]
    assert np.linalg.norm(V[1] - ref) <= 0.02 * np.linalg.norm(Vr[1]), (V[1], ref)


def _matrix(Y, L, n, omega):
    S = Y.shape[0]
    M = np.zeros((6 * S, 6 * S))
    for j in range(6 * S):
        e = np.zeros(6 * S)
        e[j] = 1.0
        V, W = fcm.fcm_apply(Y, e[:3 * S].reshape(S, 3), e[3 * S:].reshape(S, 3), 1.0, 1.0, L, n, omega=omega)
        M[:, j] = np.concatenate([V.ravel(), W.ravel()])
    return M


def test_rotation_average_by_parts():
    """Omega as the average of u x grad Theta (integration by parts over the periodic box)
    against the average of the spectral vorticity: the same rotation up to the grid's
    discretisation, the same rotational self-mobility, and a mobility matrix that is now
    symmetric to rounding (the averaging is the exact adjoint of the rotlet spreading)."""
    rng = np.random.default_rng(9)
    L, S = 12.0, 3
    Y = rng.uniform(0, L, (S, 3))
    Mb = _matrix(Y, L, 32, "by_parts")
    Mc = _matrix(Y, L, 32, "curl")
    assert np.array_equal(Mb[:3 * S], Mc[:3 * S])  # the translational rows are unchanged
    assert np.abs(Mb - Mb.T).max() <= 1e-13 * np.abs(Mb).max()
    assert np.linalg.eigvalsh(0.5 * (Mb + Mb.T)).min() > 0.0
    # the difference is the grid's: it falls spectrally with the spacing (measured 2.6e-6,
    # 5.8e-10 and 1.6e-12 of max|Omega| at h = 0.375a, 0.3a, 0.25a)
    d32 = np.abs(Mb - Mc).max() / np.abs(Mc).max()
    Mb48, Mc48 = _matrix(Y, L, 48, "by_parts"), _matrix(Y, L, 48, "curl")
    d48 = np.abs(Mb48 - Mc48).max() / np.abs(Mc48).max()
    assert d32 <= 1e-5 and d48 <= 1e-11 and d48 <= 1e-4 * d32, (d32, d48)
    Ls, ns = 16.0, 48
    Y1 = np.array([[Ls / 2 + 0.13, Ls / 2 - 0.21, Ls / 2 + 0.05]])
    _, W = fcm.fcm_apply(Y1, np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]), 1.0, 1.0, Ls, ns, omega="by_parts")
    assert abs(W[0, 2] * 8.0 * np.pi - (1.0 - 4.0 * np.pi / 3.0 / Ls ** 3)) <= 1e-7
