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
