"""The oracle's Jacobian-free Newton-Krylov solver (Sec. 3.1) pinned to independent
results: its GMRES against a direct dense solve, and its Newton step against the
root that the oracle's bad Broyden (Alg. 2, a different method) finds."""
import numpy as np

import oracle
from oracle import jfnk
from paper_1903_12609_amd import synth


def test_gmres_matches_a_direct_solve():
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * 4.0 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x_ref = np.linalg.solve(A, b)
    for restart in (40, 7):  # without and with restarts
        x, its = jfnk.gmres(lambda v: A @ v, b, 1e-12, restart, 10000)
        assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref), (restart, its)
    x, its = jfnk.gmres(lambda v: A @ v, b, 1e-12, 40, 10000)
    assert its <= n  # full GMRES terminates within n steps


def test_newton_krylov_root_equals_broyden_root():
    w = synth.single_filament(N=15)
    p = dict(w.params, tol=1e-11, kmax=200)
    a = oracle.Sim(w.fil_off, w.Y, w.q, **p)
    X_b, rc, rep = a.broyden(a.initial_guess())
    assert rc == 0
    for pc in ("j0", "none"):
        b = oracle.Sim(w.fil_off, w.Y, w.q, **p)
        rc, r = jfnk.jfnk_step(b, precond=pc, krylov_tol=1e-10)
        assert rc == 0 and r["resid"] <= 1e-11
        assert np.abs(b.X - X_b).max() <= 1e-9 * max(1.0, np.abs(X_b).max()), (pc, np.abs(b.X - X_b).max())


def test_jfb_root_equals_broyden_root():
    """JFB-g (good Broyden with J0 = grad f0 by finite differences) reaches the root of
    the oracle's bad Broyden."""
    w = synth.single_filament(N=15)
    p = dict(w.params, tol=1e-11, kmax=200)
    a = oracle.Sim(w.fil_off, w.Y, w.q, **p)
    X_b, rc, rep = a.broyden(a.initial_guess())
    assert rc == 0
    b = oracle.Sim(w.fil_off, w.Y, w.q, **p)
    rc, r = jfnk.jfb_step(b, precond="j0", krylov_tol=1e-10)
    assert rc == 0 and r["resid"] <= 1e-11
    assert np.abs(b.X - X_b).max() <= 1e-9 * max(1.0, np.abs(X_b).max())
