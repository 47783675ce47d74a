"""GPU parity of the per-filament internal forces (Sec. 2.5, 2.9.2)."""
import numpy as np
import pytest

import oracle
from paper_1903_12609_amd import synth

from gpu_util import dev, host, rel_l2

pytestmark = pytest.mark.gpu


def test_internal_forces_parity():
    import torch
    import paper_1903_12609_amd as fil
    rng = np.random.default_rng(2)
    Ns = [1, 2, 5, 20, 64, 70, 33]
    fil_off = np.concatenate([[0], np.cumsum(Ns)]).astype(np.int64)
    S, M = int(fil_off[-1]), len(Ns)
    qs, Lams, kaps = [], [], []
    for N in Ns:
        q0 = synth.random_unit_quaternion(rng)
        qf = [q0]
        for _ in range(N - 1):
            qf.append(oracle.qmul(oracle.qexp(rng.standard_normal(3) * 0.3), qf[-1]))
        qs.append(np.array(qf))
        Lams.append(rng.standard_normal((N - 1, 3)))
        kaps.append(rng.standard_normal((N - 1, 3)) * 0.2)
    q = np.concatenate(qs)
    F0 = rng.standard_normal((S, 3))
    T0 = rng.standard_normal((S, 3))
    Fr, Tr = F0.copy(), T0.copy()
    for f, N in enumerate(Ns):
        s0 = fil_off[f]
        dF, dT = oracle.internal_forces(qs[f], Lams[f], kaps[f], 2.2, 1.3, 0.7)
        Fr[s0:s0 + N] += dF
        Tr[s0:s0 + N] += dT
    Fd, Td = dev(F0), dev(T0)
    fil.filament_internal_forces(torch.from_numpy(fil_off).cuda(), dev(q), dev(np.concatenate(Lams)),
                                 dev(np.concatenate(kaps)), 2.2, 1.3, 0.7, Fd, Td)
    assert rel_l2(host(Fd), Fr) <= 1e-14 and rel_l2(host(Td), Tr) <= 1e-13
