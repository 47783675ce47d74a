"""GPU parity of the implicit step against the oracle: residual of the reduced
system (Sec. 2.9.3), the first quasi-Newton step with the explicit J0
(Appendix B.2), every bad-Broyden iterate (Alg. 2) and whole trajectories."""
import numpy as np
import pytest

import oracle
from paper_1903_12609_amd import synth

from gpu_util import rel_l2

pytestmark = pytest.mark.gpu


def _workloads():
    w1 = synth.single_filament(N=15)
    w2 = synth.sediment_suspension(M=8, N=20, side=60.0, seed=21, dt_over_T=1 / 30)
    w3 = synth.active_array(nx=3, ny=2, N=16, spacing=20.0, seed=22)
    return {"single15": w1, "susp8x20": w2, "tethered3x2x16": w3}


WL = _workloads()


def _pair(w, j0_mode="auto", **over):
    import paper_1903_12609_amd as fil
    p = dict(w.params)
    p.update(over)
    o = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **p)
    g = fil.Sim(w.fil_off, w.Y, w.q, p, j0_mode=j0_mode)
    return o, g


def _to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("name", list(WL))
def test_residual_parity(name):
    print("case", name, flush=True)
    w = WL[name]
    o, g = _pair(w)
    rng = np.random.default_rng(3)
    X0 = o.initial_guess()
    for trial in range(3):
        X = X0.copy()
        for f in range(w.M):
            s0, N = w.fil_off[f], w.fil_off[f + 1] - w.fil_off[f]
            X[6 * s0 + 3:6 * s0 + 3 + 3 * N] += rng.standard_normal(3 * N) * 0.05
            X[6 * s0 + 3 + 3 * N:6 * (s0 + N)] += rng.standard_normal(3 * (N - 1)) * 0.02
        f_or, _ = o.residual(X)
        f_gpu = g.residual(_to_dev(X)).cpu().numpy()
        assert rel_l2(f_gpu, f_or) <= 1e-12, rel_l2(f_gpu, f_or)


@pytest.mark.parametrize("j0_mode", ["banded", "dense"])
@pytest.mark.parametrize("name", list(WL))
def test_first_quasi_newton_step(name, j0_mode):
    """X1 = X0 - J0^{-1} f(X0) with J0 assembled, row-differenced into a band and
    factorised on the GPU (applied by banded sweeps or as an explicit inverse)."""
    print("case", name, j0_mode, flush=True)
    w = WL[name]
    o, g = _pair(w, j0_mode)
    X0 = o.initial_guess()
    f0, _ = o.residual(X0)
    X1 = X0.copy()
    for f in range(w.M):
        a, b = 6 * w.fil_off[f], 6 * w.fil_off[f + 1]
        X1[a:b] -= np.linalg.solve(o.j0_filament(f, X0), f0[a:b])
    f0_gpu = g.broyden_begin(_to_dev(X0)).cpu().numpy()
    assert rel_l2(f0_gpu, f0) <= 1e-12
    assert rel_l2(g.iterate().cpu().numpy(), X1) <= 1e-11


@pytest.mark.parametrize("N", [32, 48, 64])
def test_first_quasi_newton_step_long_filaments(N):
    """The explicit inverse of long filaments' blocks: 192, 288 and 384 unknowns take the
    inverse kernel's 64-, 32- and 16-column forms (the widest whose LDS fits a CU)."""
    print("case N", N, flush=True)
    w = synth.sediment_suspension(M=3, N=N, side=40.0 + 3.0 * N, seed=23 + N, dt_over_T=1 / 30)
    o, g = _pair(w, "dense")
    X0 = o.initial_guess()
    f0, _ = o.residual(X0)
    X1 = X0.copy()
    for f in range(w.M):
        a, b = 6 * w.fil_off[f], 6 * w.fil_off[f + 1]
        X1[a:b] -= np.linalg.solve(o.j0_filament(f, X0), f0[a:b])
    f0_gpu = g.broyden_begin(_to_dev(X0)).cpu().numpy()
    assert rel_l2(f0_gpu, f0) <= 1e-12
    assert rel_l2(g.iterate().cpu().numpy(), X1) <= 1e-11


@pytest.mark.parametrize("j0_mode", ["banded", "dense"])
@pytest.mark.parametrize("name", list(WL))
def test_every_broyden_iterate(name, j0_mode):
    """The GPU reuses H_k f_{k+1} for c_{k+1} and the next step; the oracle applies
    Alg. 2 literally.  Iterates X_1..X_6 agree."""
    print("case", name, j0_mode, flush=True)
    w = WL[name]
    o, g = _pair(w, j0_mode)
    X0 = o.initial_guess()
    g.broyden_begin(_to_dev(X0))
    for n in range(1, 7):
        o.P.kmax, o.P.tol = n, 0.0
        Xn, rc, rep = o.broyden(X0)
        assert rep.iters == n
        Xg = g.iterate().cpu().numpy()
        assert rel_l2(Xg, Xn) <= 1e-10 * n, (n, rel_l2(Xg, Xn))
        fn = g.residual(g.iterate().clone())
        g.broyden_update(fn)


@pytest.mark.parametrize("name,steps,j0_mode", [("single15", 100, "auto"), ("susp8x20", 10, "auto"),
                                                ("tethered3x2x16", 5, "auto"), ("susp8x20", 10, "banded")])
def test_trajectory_parity(name, steps, j0_mode):
    """Protocol: both sides at tol 1e-6; where the per-step iteration counts agree,
    positions match to 1e-8 relative L2 at the end."""
    print("case", name, steps, j0_mode, flush=True)
    w = WL[name]
    o, g = _pair(w, j0_mode)
    for j in range(steps):
        rc, rep = o.step()
        assert rc == 0
        r = g.step()[0]
        assert r["converged"] and r["resid"] <= w.params["tol"]
        assert r["iters"] == rep.iters, (j, r["iters"], rep.iters)
    Y, q, X = g.read_state()
    assert rel_l2(Y, o.Y) <= 1e-8 and rel_l2(q, o.q) <= 1e-8, (rel_l2(Y, o.Y), rel_l2(q, o.q))
    assert np.abs(np.linalg.norm(q, axis=1) - 1).max() <= 1e-14
    t = np.array([oracle.qrot(qq)[:, 0] for qq in q])
    for f in range(w.M):
        a, b = w.fil_off[f], w.fil_off[f + 1]
        gap = Y[a + 1:b] - Y[a:b - 1] - 0.5 * w.params["dL"] * (t[a:b - 1] + t[a + 1:b])
        # met to rounding: a few ulps of the positions, which grow as the filament settles
        assert np.abs(gap).max() <= 1e-13 * w.params["dL"] + 8 * np.finfo(float).eps * np.abs(Y).max()


def _ragged():
    """Filaments of 1, 2, 7, 20, 33 and 64 segments in one suspension: the smallest and
    largest sizes of the per-filament kernels beside ordinary ones."""
    rng = np.random.default_rng(23)
    Ns = [1, 2, 64, 7, 20, 33]
    fil_off, Y, q = synth._place(rng, len(Ns), Ns, 80.0, 0.02)
    params, _ = synth.sedimentation_params(20, 1e3, 1 / 30, 1e-6, 100, steric=True)
    return synth.Workload("ragged", fil_off, Y, q, params)


@pytest.mark.parametrize("j0_mode,graph", [("dense", 0), ("banded", 0), ("dense", 3)])
def test_ragged_filament_sizes(j0_mode, graph):
    """Protocol as test_trajectory_parity, 6 steps, for filaments of 1 to 64 segments."""
    import paper_1903_12609_amd as fil
    print("case ragged", j0_mode, graph, flush=True)
    w = _ragged()
    o = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params)
    g = fil.Sim(w.fil_off, w.Y, w.q, w.params, j0_mode=j0_mode, graph=graph)
    for j in range(6):
        rc, rep = o.step()
        assert rc == 0
        r = g.step()[0]
        assert r["converged"] and r["resid"] <= w.params["tol"]
        assert r["iters"] == rep.iters, (j, r["iters"], rep.iters)
    Y, q, X = g.read_state()
    assert rel_l2(Y, o.Y) <= 1e-8 and rel_l2(q, o.q) <= 1e-8, (rel_l2(Y, o.Y), rel_l2(q, o.q))


def test_trajectory_tight_tolerance():
    """At tol 1e-11 the converged roots agree independently of iteration counts."""
    w = WL["single15"]
    o, g = _pair(w, tol=1e-11, kmax=200)
    for j in range(20):
        assert o.step()[0] == 0
        g.step()
    Y, q, _ = g.read_state()
    assert rel_l2(Y, o.Y) <= 1e-9


def test_batched_suspensions_match_separate_runs():
    """Uneven suspensions in one simulation (one persistent mobility launch)
    reproduce their separate oracle runs."""
    import paper_1903_12609_amd as fil
    ws = [synth.sediment_suspension(M=m, N=n, side=40.0 * m ** (1 / 3), seed=30 + m, dt_over_T=1 / 30)
          for m, n in ((1, 12), (3, 20), (5, 10), (2, 33))]
    params = dict(ws[0].params)
    fil_off = [0]
    for w in ws:
        fil_off += list(fil_off[-1] + w.fil_off[1:])
    sfo = np.concatenate([[0], np.cumsum([w.M for w in ws])])
    Y = np.concatenate([w.Y for w in ws])
    q = np.concatenate([w.q for w in ws])
    g = fil.Sim(fil_off, Y, q, params, susp_fil_off=sfo)
    os_ = [oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **params) for w in ws]
    for j in range(4):
        reps = g.step()
        for i, o in enumerate(os_):
            rc, rep = o.step()
            assert rc == 0 and reps[i]["iters"] == rep.iters
    Yg, _, _ = g.read_state()
    Yo = np.concatenate([o.Y for o in os_])
    assert rel_l2(Yg, Yo) <= 1e-8


def test_batched_suspensions_with_their_own_parameters():
    """Suspensions of different N carry their own dt, gravity W dL and F^S
    (each from its own length L); each matches its own oracle run."""
    import paper_1903_12609_amd as fil
    ws = [synth.sediment_suspension(M=m, N=n, side=40.0 * m ** (1 / 3), seed=40 + m, dt_over_T=1 / 30)
          for m, n in ((2, 12), (4, 20), (1, 33))]
    fil_off = [0]
    for w in ws:
        fil_off += list(fil_off[-1] + w.fil_off[1:])
    sfo = np.concatenate([[0], np.cumsum([w.M for w in ws])])
    g = fil.Sim(fil_off, np.concatenate([w.Y for w in ws]), np.concatenate([w.q for w in ws]), ws[0].params,
                susp_fil_off=sfo)
    g.set_suspension_params(dt=[w.params["dt"] for w in ws], grav=[w.params["grav"] for w in ws],
                            FS=[w.params["FS"] for w in ws])
    os_ = [oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params) for w in ws]
    for j in range(4):
        reps = g.step()
        for i, o in enumerate(os_):
            rc, rep = o.step()
            assert rc == 0 and reps[i]["iters"] == rep.iters
    Yg, _, _ = g.read_state()
    Yo = np.concatenate([o.Y for o in os_])
    assert rel_l2(Yg, Yo) <= 1e-8


def test_f32tile_steps_finish_in_fp64():
    """FP32-tile mode: every step starts with FP32 pair tiles and ends on an FP64
    residual within tol, so the trajectory stays within the tolerance of the
    FP64 oracle's."""
    import paper_1903_12609_amd as fil
    w = WL["susp8x20"]
    o = oracle.Sim(w.fil_off, w.Y, w.q, nthreads=8, **w.params)
    g = fil.Sim(w.fil_off, w.Y, w.q, w.params, prec="f32tile")
    for j in range(8):
        r = g.step()[0]
        rc, rep = o.step()
        assert rc == 0 and r["converged"] and r["resid"] <= w.params["tol"]
        assert 1 <= r["applies_f64"] < r["applies"], r
    Yg, _, _ = g.read_state()
    err = rel_l2(Yg, o.Y)
    print("f32tile trajectory vs FP64 oracle after 8 steps: rel L2 %.3e" % err)
    assert err <= 1e-6


@pytest.mark.parametrize("case", ["susp8x20-dense-U4", "tethered-banded-U3", "batched-U1", "f32tile-U5"])
def test_graph_blocks_reproduce_host_loop(case):
    """Broyden iterations replayed from captured HIP graphs (device-side
    convergence test) give the same iteration counts and bitwise the same
    trajectory as the host-driven loop, over several steps (every block graph
    is replayed many times with eager work in between)."""
    import paper_1903_12609_amd as fil
    print("case", case, flush=True)
    prec = "f32tile" if case.startswith("f32tile") else "f64"
    U = int(case.rsplit("U", 1)[1])
    if case.startswith("batched"):
        ws = [synth.sediment_suspension(M=m, N=n, side=40.0 * m ** (1 / 3), seed=60 + m, dt_over_T=1 / 30)
              for m, n in ((2, 12), (3, 20), (1, 9))]
        fil_off = [0]
        for w in ws:
            fil_off += list(fil_off[-1] + w.fil_off[1:])
        sfo = np.concatenate([[0], np.cumsum([w.M for w in ws])])
        args = (fil_off, np.concatenate([w.Y for w in ws]), np.concatenate([w.q for w in ws]), ws[0].params)
        kw = dict(susp_fil_off=sfo)
    else:
        w = WL["tethered3x2x16"] if case.startswith("tethered") else WL["susp8x20"]
        args = (w.fil_off, w.Y, w.q, w.params)
        kw = dict(j0_mode="banded" if "banded" in case else "dense")
    a = fil.Sim(*args, prec=prec, **kw)
    b = fil.Sim(*args, prec=prec, graph=U, **kw)
    b.set_timing(True)
    for j in range(6):
        ra, rb = a.step(), b.step()
        assert [r["iters"] for r in ra] == [r["iters"] for r in rb], (j, ra, rb)
        assert [r["applies_f64"] for r in ra] == [r["applies_f64"] for r in rb]
        assert [r["resid"] for r in ra] == [r["resid"] for r in rb]
    assert np.array_equal(a.read_state()[0], b.read_state()[0])
    assert np.array_equal(a.read_state()[2], b.read_state()[2])
    tm = b.timing()
    assert tm["f64"][1] + tm["f32tile"][1] > 0
