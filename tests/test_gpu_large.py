"""GPU parity of the kernel forms that large suspensions and ensembles take: more than 256
filaments (256-thread residual and update kernels), the band LU without LDS staging, and a
batched simulation whose suspensions hold more than 256 filaments together.  Same protocol
as the step tests: equal Broyden iteration counts per step (Alg. 2 at tol 1e-6), positions
and quaternions to 1e-8 relative L2 after the steps."""
import numpy as np
import pytest

import oracle
from paper_1903_12609_amd import synth

from gpu_util import rel_l2

pytestmark = pytest.mark.gpu


def _many():
    # 300 filaments of 5 segments (1500 segments) in a cube of side 90a, dt = T/15
    return synth.sediment_suspension(M=300, N=5, side=90.0, seed=71, dt_over_T=1 / 15)


def _to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("j0_mode,graph,j0_factor", [("dense", 0, "auto"), ("banded", 0, "auto"),
                                                     ("dense", 8, "auto"), ("banded", 8, "unstaged")])
def test_many_filaments_trajectory(j0_mode, graph, j0_factor):
    """M = 300 > 256: the residual and Broyden-update kernels run 256 threads per filament."""
    import paper_1903_12609_amd as fil
    print("case many-filaments", j0_mode, graph, j0_factor, flush=True)
    w = _many()
    assert w.M > 256
    o = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params)
    g = fil.Sim(w.fil_off, w.Y, w.q, w.params, j0_mode=j0_mode, graph=graph, j0_factor=j0_factor)
    for j in range(5):
        rc, rep = o.step()
        assert rc == 0
        r = g.step()[0]
        assert r["converged"] and r["resid"] <= w.params["tol"]
        assert r["iters"] == rep.iters, (j, r["iters"], rep.iters)
    Y, q, _ = g.read_state()
    g.close()
    assert rel_l2(Y, o.Y) <= 1e-8 and rel_l2(q, o.q) <= 1e-8, (rel_l2(Y, o.Y), rel_l2(q, o.q))


def _first_step_cases():
    return {"single15": synth.single_filament(N=15),
            "susp8x20": synth.sediment_suspension(M=8, N=20, side=60.0, seed=21, dt_over_T=1 / 30),
            "tethered3x2x16": synth.active_array(nx=3, ny=2, N=16, spacing=20.0, seed=22),
            "many300x5": _many()}


FIRST = _first_step_cases()


@pytest.mark.parametrize("j0_mode", ["banded", "dense"])
@pytest.mark.parametrize("name", list(FIRST))
def test_unstaged_factor_first_quasi_newton_step(name, j0_mode):
    """X1 = X0 - J0^{-1} f(X0) with the band LU kernel that keeps no rows in LDS (the form
    ensembles too large for four rounds of resident workgroups take), against the oracle's
    dense LU of Appendix B.2's J0; and bitwise equal to the staged kernel's X1."""
    import paper_1903_12609_amd as fil
    print("case", name, j0_mode, flush=True)
    w = FIRST[name]
    o = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params)
    X0 = o.initial_guess()
    f0, _ = o.residual(X0)
    X1 = X0.copy()
    for f in range(w.M):
        a, b = 6 * w.fil_off[f], 6 * w.fil_off[f + 1]
        X1[a:b] -= np.linalg.solve(o.j0_filament(f, X0), f0[a:b])
    out = {}
    for form in ("unstaged", "auto"):
        g = fil.Sim(w.fil_off, w.Y, w.q, w.params, j0_mode=j0_mode, j0_factor=form)
        g.broyden_begin(_to_dev(X0))
        out[form] = g.iterate().cpu().numpy()
        g.close()
    assert rel_l2(out["unstaged"], X1) <= 1e-11, rel_l2(out["unstaged"], X1)
    assert np.array_equal(out["unstaged"], out["auto"])


@pytest.mark.parametrize("j0_mode", ["dense", "banded"])
def test_batched_suspensions_over_256_filaments(j0_mode):
    """Three suspensions of 120, 100 and 90 filaments (310 together) in one simulation: the
    ragged mobility work list, the 256-thread per-filament kernels and per-suspension
    convergence; each matches its own oracle run.  Banded: J0^{-1} f by the band solve
    kernel, whose waves then hold filaments of different lengths and of suspensions that
    have already converged."""
    import paper_1903_12609_amd as fil
    print("case batched-310", j0_mode, flush=True)
    ws = [synth.sediment_suspension(M=m, N=n, side=s, seed=80 + m, dt_over_T=1 / 15)
          for m, n, s in ((120, 5, 70.0), (100, 6, 70.0), (90, 4, 60.0))]
    fil_off = [0]
    for w in ws:
        fil_off += list(fil_off[-1] + w.fil_off[1:])
    sfo = np.concatenate([[0], np.cumsum([w.M for w in ws])])
    assert sfo[-1] > 256
    g = fil.Sim(fil_off, np.concatenate([w.Y for w in ws]), np.concatenate([w.q for w in ws]), ws[0].params,
                susp_fil_off=sfo, graph=8, j0_mode=j0_mode)
    g.set_suspension_params(dt=[w.params["dt"] for w in ws], grav=[w.params["grav"] for w in ws],
                            FS=[w.params["FS"] for w in ws])
    os_ = [oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params) for w in ws]
    for j in range(4):
        reps = g.step()
        for i, o in enumerate(os_):
            rc, rep = o.step()
            assert rc == 0 and reps[i]["converged"] and reps[i]["iters"] == rep.iters, (j, i, reps[i], rep.iters)
    Yg, qg, _ = g.read_state()
    g.close()
    assert rel_l2(Yg, np.concatenate([o.Y for o in os_])) <= 1e-8
    assert rel_l2(qg, np.concatenate([o.q for o in os_])) <= 1e-8


def test_band_solve_kernel_mixed_lengths():
    """Band path with 300 filaments of 2 to 50 segments: J0^{-1} f is formed by the band
    solve kernel of its own (four filaments of different lengths per wave) before the
    update, and
    X1 = X0 - J0^{-1} f(X0) matches the oracle's dense LU solve."""
    import paper_1903_12609_amd as fil
    print("case band solve kernel", flush=True)
    rng = np.random.default_rng(91)
    Ns = [int(n) for n in rng.integers(2, 51, 300)]
    base = synth.sediment_suspension(M=2, N=10, seed=91)
    fil_off, Y, q = synth._place(rng, 300, Ns, 260.0, 0.02)
    o = oracle.Sim(fil_off, Y, q, nthreads=8, **base.params)
    X0 = o.initial_guess()
    f0, _ = o.residual(X0)
    X1 = X0.copy()
    for f in range(300):
        a, b = 6 * fil_off[f], 6 * fil_off[f + 1]
        X1[a:b] -= np.linalg.solve(o.j0_filament(f, X0), f0[a:b])
    g = fil.Sim(fil_off, Y, q, base.params, j0_mode="banded")
    g.broyden_begin(_to_dev(X0))
    X1g = g.iterate().cpu().numpy()
    g.close()
    assert rel_l2(X1g, X1) <= 1e-11, rel_l2(X1g, X1)
