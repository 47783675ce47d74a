"""Test infrastructure (not the product path): plain Jacobian-free Newton-Krylov (Sec. 3.1)
and Jacobian-free good Broyden (JFB-g, Sec. 3.2.1 with Alg. 1) steps on top of the
oracle's residual and J0 blocks, to check the GPU solvers against.  Linear systems are
solved by restarted GMRES (Arnoldi with modified Gram-Schmidt, Givens rotations).  JFNK
takes each J v by the finite difference (f(X + delta v) - f(X)) / delta; JFB-g takes
J0 v the same way from f0, the residual with the drag-only mobility and without steric
or external forces, at the initial guess.  Preconditioners (Sec. 3.3.1): none; right,
P_dt applied as its inverse (multiplier unknowns scaled by 6 pi eta a / dt, undoing the
dt / (6 pi eta a) of their Jacobian columns); left, J0^{-1} with the block-diagonal J0 of
the initial guess (Sec. 3.2.2).
"""
import numpy as np
import scipy.linalg as sla


def gmres(apply, b, rtol, restart, maxit):
    """x with |b - A x| <= rtol |b| (x0 = 0); returns x and the iterations taken."""
    n = b.shape[0]
    x = np.zeros(n)
    nb = np.linalg.norm(b)
    its = 0
    if nb == 0.0:
        return x, 0
    while True:
        r = b - apply(x) if its > 0 else b.copy()
        beta = np.linalg.norm(r)
        if beta <= rtol * nb or its >= maxit:
            return x, its
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        g = np.zeros(restart + 1)
        g[0] = beta
        cs, sn = np.zeros(restart), np.zeros(restart)
        k = 0
        while k < restart and its < maxit:
            w = apply(V[k])
            its += 1
            for j in range(k + 1):
                H[j, k] = np.dot(V[j], w)
                w = w - H[j, k] * V[j]
            hn = np.linalg.norm(w)
            V.append(w / hn if hn > 0 else w)
            col = H[:k + 1, k].copy()
            for j in range(k):
                t = cs[j] * col[j] + sn[j] * col[j + 1]
                col[j + 1] = -sn[j] * col[j] + cs[j] * col[j + 1]
                col[j] = t
            rr = np.hypot(col[k], hn)
            cs[k], sn[k] = (col[k] / rr, hn / rr) if rr > 0 else (1.0, 0.0)
            col[k] = rr
            H[:k + 1, k] = col
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k += 1
            if abs(g[k]) <= rtol * nb or hn == 0.0:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k])
        x = x + np.array(V[:k]).T @ y
        if abs(g[k]) <= rtol * nb:
            return x, its


def jfnk_step(sim, precond="j0", krylov_tol=1e-4, fd_delta=1e-7, krylov_max=1000, restart=100):
    """One step of `sim` (an oracle Sim) by Newton-Krylov; commits it when converged.
    Returns (rc, dict(newton, krylov, applies, resid))."""
    P = sim.P
    X = sim.initial_guess()
    f, r = sim.residual(X)
    applies = 1
    lu = []
    if precond == "j0":
        for fi in range(sim.M):
            lu.append(sla.lu_factor(sim.j0_filament(fi, X)))
    pinv = np.ones(6 * sim.S)
    if precond == "pdt":
        for fi in range(sim.M):
            s0, N = int(sim.fil_off[fi]), int(sim.fil_off[fi + 1] - sim.fil_off[fi])
            pinv[6 * s0 + 3 + 3 * N:6 * (s0 + N)] = 6.0 * np.pi * P.eta * P.a / P.dt

    def j0_solve(v):
        out = np.empty_like(v)
        for fi in range(sim.M):
            a, b = 6 * int(sim.fil_off[fi]), 6 * int(sim.fil_off[fi + 1])
            out[a:b] = sla.lu_solve(lu[fi], v[a:b])
        return out

    newton = kry = 0
    while not r <= P.tol:
        if not np.isfinite(r) or newton >= P.kmax:
            return (-4 if not np.isfinite(r) else -3), dict(newton=newton, krylov=kry, applies=applies, resid=r)
        f0 = f
        n_apply = [0]

        def apply(v):
            u = pinv * v if precond == "pdt" else v
            fp, _ = sim.residual(X + fd_delta * u)
            n_apply[0] += 1
            Jv = (fp - f0) / fd_delta
            return j0_solve(Jv) if precond == "j0" else Jv

        b = -j0_solve(f0) if precond == "j0" else -f0
        x, its = gmres(apply, b, krylov_tol, restart, krylov_max)
        kry += its
        applies += n_apply[0]
        dX = pinv * x if precond == "pdt" else x
        X = X + dX
        f, r = sim.residual(X)
        applies += 1
        newton += 1
    sim.commit(X)
    return 0, dict(newton=newton, krylov=kry, applies=applies, resid=r)


def jfb_step(sim, precond="j0", krylov_tol=1e-4, fd_delta=1e-7, krylov_max=1000, restart=100):
    """One step of `sim` by the Jacobian-free good Broyden method JFB-g (Sec. 3.2.1,
    Alg. 1): dX = -[J0 + sum_i c_i d_i^T]^{-1} f(X_k) by GMRES, J0 v taken by finite
    differences of f0 (drag-only mobility, no steric or external forces) at the
    initial guess, then c = f(X_{k+1}) / |dX|, d = dX / |dX|.  Commits when converged.
    Returns (rc, dict(newton=Broyden iterations, krylov, applies, resid))."""
    P = sim.P
    X = sim.initial_guess()
    X0 = X.copy()
    f, r = sim.residual(X)
    applies = 1
    lu = []
    if precond == "j0":
        for fi in range(sim.M):
            lu.append(sla.lu_factor(sim.j0_filament(fi, X)))
    pinv = np.ones(6 * sim.S)
    if precond == "pdt":
        for fi in range(sim.M):
            s0, N = int(sim.fil_off[fi]), int(sim.fil_off[fi + 1] - sim.fil_off[fi])
            pinv[6 * s0 + 3 + 3 * N:6 * (s0 + N)] = 6.0 * np.pi * P.eta * P.a / P.dt

    def j0_solve(v):
        out = np.empty_like(v)
        for fi in range(sim.M):
            a, b = 6 * int(sim.fil_off[fi]), 6 * int(sim.fil_off[fi + 1])
            out[a:b] = sla.lu_solve(lu[fi], v[a:b])
        return out

    def f0(Xv):
        P.drag_only = 1
        try:
            return sim.residual(Xv)[0]
        finally:
            P.drag_only = 0

    f00 = f0(X0)
    C, D = [], []
    it = kry = 0
    while not r <= P.tol:
        if not np.isfinite(r) or it >= P.kmax:
            return (-4 if not np.isfinite(r) else -3), dict(newton=it, krylov=kry, applies=applies, resid=r)

        def apply(v):
            u = pinv * v if precond == "pdt" else v
            Jv = (f0(X0 + fd_delta * u) - f00) / fd_delta
            for c, d in zip(C, D):
                Jv = Jv + c * np.dot(d, u)
            return j0_solve(Jv) if precond == "j0" else Jv

        b = -j0_solve(f) if precond == "j0" else -f
        x, its = gmres(apply, b, krylov_tol, restart, krylov_max)
        kry += its
        dX = pinv * x if precond == "pdt" else x
        X = X + dX
        f, r = sim.residual(X)
        applies += 1
        it += 1
        nx = np.linalg.norm(dX)
        C.append(f / nx)
        D.append(dX / nx)
    sim.commit(X)
    return 0, dict(newton=it, krylov=kry, applies=applies, resid=r)
