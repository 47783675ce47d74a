"""GPU force-coupling-method mobility (Sec. 2.7.2) against the oracle's, on the same
grids: forces and torques of several segments in a rectangular periodic box.  The GPU
averages the rotation by parts (the oracle's omega="by_parts"); on a fine grid it also
matches the oracle's average of the spectral vorticity."""
import numpy as np
import pytest

from oracle import fcm as ofcm

from gpu_util import dev, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("box,grid,cut", [((12.0, 12.0, 12.0), (32, 32, 32), 7.5),
                                          ((16.0, 10.0, 12.0), (48, 30, 36), 7.5),
                                          ((12.0, 12.0, 12.0), (32, 32, 32), 4.0)])
def test_fcm_apply_matches_oracle(box, grid, cut):
    import paper_1903_12609_amd as fil
    print("case fcm", box, grid, cut, flush=True)
    rng = np.random.default_rng(11)
    S = 7
    Y = rng.uniform(-2.0, 1.2 * min(box), (S, 3))  # some outside the box: wrapped
    F = rng.standard_normal((S, 3))
    T = rng.standard_normal((S, 3))
    Vo, Wo = ofcm.fcm_apply(Y, F, T, 1.0, 1.0, box, grid, cut=cut, omega="by_parts")
    m = fil.FCM(box, grid, a=1.0, eta=1.0, cut=cut)
    V, W = m.apply(dev(Y), dev(F), dev(T))
    V, W = host(V), host(W)
    assert rel_l2(V, Vo) <= 1e-11 and rel_l2(W, Wo) <= 1e-11, (rel_l2(V, Vo), rel_l2(W, Wo))
    m.close()


def test_fcm_rotation_matches_vorticity_average_on_a_fine_grid():
    """h = 0.25a: the by-parts rotation equals the spectral-vorticity average to the
    grid's (spectrally small) discretisation error, 1.6e-12 of max|Omega| in the oracle."""
    import paper_1903_12609_amd as fil
    rng = np.random.default_rng(12)
    box, grid, S = (12.0, 12.0, 12.0), (48, 48, 48), 5
    Y = rng.uniform(0.0, 12.0, (S, 3))
    F = rng.standard_normal((S, 3))
    T = rng.standard_normal((S, 3))
    Vo, Wo = ofcm.fcm_apply(Y, F, T, 1.0, 1.0, box, grid, omega="curl")
    m = fil.FCM(box, grid, a=1.0, eta=1.0)
    V, W = m.apply(dev(Y), dev(F), dev(T))
    V, W = host(V), host(W)
    assert rel_l2(V, Vo) <= 1e-11 and rel_l2(W, Wo) <= 1e-10, (rel_l2(V, Vo), rel_l2(W, Wo))
    m.close()


def test_fcm_refusals():
    import paper_1903_12609_amd as fil
    from paper_1903_12609_amd._native import FilError
    with pytest.raises(FilError):
        fil.FCM((4.0, 4.0, 4.0), (8, 8, 8), cut=7.5)  # support larger than the grid
    with pytest.raises(FilError):
        fil.FCM((10.0, 10.0, 10.0), (32, 32, 32), cut=1.0)
