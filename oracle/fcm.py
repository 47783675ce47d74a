"""Test infrastructure (not the product path): a plain force-coupling-method mobility
(Sec. 2.7.2) to check the GPU apply against.

In a periodic box [0, Lx) x [0, Ly) x [0, Lz) on an nx x ny x nz grid (spacings h_i = L_i / n_i):
  * the body force  f(x) = sum_m F_m Delta_m(x) - 1/2 sum_m T_m x grad Theta_m(x),  with
    Delta_m, Theta_m Gaussians of widths sigma_D = a / sqrt(pi) and
    sigma_T = a / (6 sqrt(pi))^(1/3) about Y_m (periodic images by minimum distance),
    each truncated at distance cut * sigma;
  * the Stokes equations solved spectrally: u_k = (I - k k^T / k^2) f_k / (eta k^2),
    u_0 = 0, and the vorticity w_k = i k x u_k; modes on a Nyquist plane (wave number
    index n_i / 2 on an even axis) are dropped, since the spectral curl of a real field is
    not defined there;
  * V_n = sum over the grid of u Delta_n hx hy hz and Omega_n = 1/2 sum of w Theta_n hx hy hz
    (the trapezoidal rule).
With omega="by_parts" the rotation is the same average after integrating by parts over
the periodic box, Omega_n = 1/2 int u x grad Theta_n dV = 1/2 int (r x u) Theta_n / sigma_T^2
dV (r = x - Y_n), summed by the same rule: no vorticity field is formed, and the averaging
is then the exact adjoint of the rotlet spreading.  The two forms agree up to the grid's
discretisation error.
Everything is evaluated on the whole grid with numpy, in float64.
"""
import numpy as np


def widths(a):
    return a / np.sqrt(np.pi), a / (6.0 * np.sqrt(np.pi)) ** (1.0 / 3.0)


def _axes(L, n):
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy()
    n = np.broadcast_to(np.asarray(n, dtype=np.int64), (3,)).copy()
    return L, n, L / n


def _gauss(Y, L, n, sigma, cut):
    """Gaussian of width sigma about Y on the grid, minimum-image distances, truncated at
    cut * sigma; also the offsets r = x - Y (minimum image), shape [3, nx, ny, nz]."""
    L, n, h = _axes(L, n)
    d = []
    for c in range(3):
        x = np.arange(n[c]) * h[c] - Y[c]
        d.append(x - L[c] * np.round(x / L[c]))
    rx, ry, rz = np.meshgrid(d[0], d[1], d[2], indexing="ij")
    r2 = rx * rx + ry * ry + rz * rz
    g = (2.0 * np.pi * sigma * sigma) ** -1.5 * np.exp(-r2 / (2.0 * sigma * sigma))
    g[r2 >= (cut * sigma) ** 2] = 0.0
    return g, np.stack([rx, ry, rz])


def fcm_apply(Y, F, T, a, eta, L, n, cut=7.5, omega="curl"):
    """(V, Omega) [S, 3] of S segments at Y [S, 3] with forces F and torques T [S, 3];
    L and n are the box lengths and grid sizes (scalars for a cube); omega: "curl" (the
    average of the spectral vorticity) or "by_parts"."""
    if omega not in ("curl", "by_parts"):
        raise ValueError("omega must be 'curl' or 'by_parts'")
    Y, F, T = (np.asarray(v, dtype=np.float64).reshape(-1, 3) for v in (Y, F, T))
    L, n, h = _axes(L, n)
    sD, sT = widths(a)
    f = np.zeros((3, n[0], n[1], n[2]))
    for m in range(Y.shape[0]):
        gD, _ = _gauss(Y[m], L, n, sD, cut)
        gT, r = _gauss(Y[m], L, n, sT, cut)
        for c in range(3):
            f[c] += F[m, c] * gD
        # -1/2 T x grad Theta, grad Theta = -r / sigma_T^2 Theta
        gradT = -r * gT / (sT * sT)
        f[0] -= 0.5 * (T[m, 1] * gradT[2] - T[m, 2] * gradT[1])
        f[1] -= 0.5 * (T[m, 2] * gradT[0] - T[m, 0] * gradT[2])
        f[2] -= 0.5 * (T[m, 0] * gradT[1] - T[m, 1] * gradT[0])
    fk = np.fft.fftn(f, axes=(1, 2, 3))
    k1 = [2.0 * np.pi * np.fft.fftfreq(int(n[c]), d=h[c]) for c in range(3)]
    kx, ky, kz = np.meshgrid(k1[0], k1[1], k1[2], indexing="ij")
    k = np.stack([kx, ky, kz])
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    kf = (k * fk).sum(axis=0)
    uk = (fk - k * kf / k2) / (eta * k2)
    uk[:, 0, 0, 0] = 0.0
    for c in range(3):
        if n[c] % 2 == 0:
            idx = [slice(None)] * 4
            idx[1 + c] = int(n[c]) // 2
            uk[tuple(idx)] = 0.0
    u = np.real(np.fft.ifftn(uk, axes=(1, 2, 3)))
    if omega == "curl":
        wk = 1j * np.stack([k[1] * uk[2] - k[2] * uk[1], k[2] * uk[0] - k[0] * uk[2], k[0] * uk[1] - k[1] * uk[0]])
        w = np.real(np.fft.ifftn(wk, axes=(1, 2, 3)))
    V, W = np.zeros_like(Y), np.zeros_like(Y)
    dv = float(np.prod(h))
    for m in range(Y.shape[0]):
        gD, _ = _gauss(Y[m], L, n, sD, cut)
        gT, r = _gauss(Y[m], L, n, sT, cut)
        V[m] = (u * gD).sum(axis=(1, 2, 3)) * dv
        if omega == "curl":
            W[m] = 0.5 * (w * gT).sum(axis=(1, 2, 3)) * dv
        else:
            rxu = np.stack([r[1] * u[2] - r[2] * u[1], r[2] * u[0] - r[0] * u[2], r[0] * u[1] - r[1] * u[0]])
            W[m] = 0.5 * (rxu * gT).sum(axis=(1, 2, 3)) * dv / (sT * sT)
    return V, W
