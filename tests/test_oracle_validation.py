"""The oracle's external-force term against the analytic elastica (Sec. 4.1): the steady
shape of a clamped filament under an end load converges at second order in dL."""
import numpy as np

import elastica_ref as er
import oracle


def test_oracle_clamped_elastica():
    theta, thL = er.elastica_theta(1.93)
    # the analytic solution itself: clamp horizontal, and s(theta_L) = l
    assert abs(theta(0.0) - np.pi / 2) < 1e-15 and 0.80 < thL < 0.81
    errs = []
    for N in (11, 21):
        fo, Y, q, params, fext = er.clamped_filament(N)
        o = oracle.Sim(fo, Y, q, nthreads=4, fext=fext, **params)
        for _ in range(300):
            rc, _ = o.step()
            assert rc == 0
        errs.append(er.l2_angle_error(o.q, params["dL"], 40.0, theta))
    # observed on the GPU path: 9.89e-4 and 2.38e-4
    assert errs[0] < 2e-3 and 3.6 < errs[0] / errs[1] < 4.6, errs
