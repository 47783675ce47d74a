"""Writes wall_image.h: the wall (image) part of the Rotne-Prager-Blake mobility of two
spheres of radius a above a no-slip plane z = 0 (the wall-bounded RPY tensor cited in
Sec. 2.7.1), as straight-line C for the GPU kernel.

Construction.  Blake's solution for a point force at y = (y1, y2, h) above the wall is
the free Stokeslet at y plus an image system at y* = (y1, y2, -h):
    G_ij = S_ij(x - y) - S_ij(R) + 2 h s_j d/dR_j [h R_i / R^3 - S_i3(R)],
    S_ij(v) = delta_ij / |v| + v_i v_j / |v|^3,  R = x - y*,  s = (1, 1, -1)
(no sum over j in s_j d/dR_j).  The mobility adds to the free-space RPY tensor the image
part G^im = G - S(x - y) under the Faxen operators of both spheres:
    tt = (1 + a^2/6 lap_x)(1 + a^2/6 lap_y) G^im / (8 pi eta)
    rt = 1/2 curl_x (1 + a^2/6 lap_y) G^im / (8 pi eta)     (rotation at x, force at y)
    tr = 1/2 curl_y (1 + a^2/6 lap_x) G^im / (8 pi eta)     (translation at x, torque at y)
    rr = 1/4 curl_x curl_y G^im / (8 pi eta)
Here the image part is written in the variables R = x - y* and h = y_3 (x_3 = R_3 - h),
d/dx = d/dR at fixed h, d/dy_1,2 = -d/dR_1,2 and d/dy_3 = d/dh + d/dR_3 (R_3 = x_3 + y_3).

Output form.  The image system is symmetric about the wall normal e, so each block is a
combination of a few tensors built from R, e and c = R x e whose scalar coefficients depend
on |R|, R_3, h and a only (see coefficients()).  The header evaluates those 18 coefficients
(common subexpressions shared) and applies the blocks to F and T through the dot products
R.F, c.F, R.T, c.T: a few hundred flops per pair instead of the 36 explicit entries.

Run:  python gen_wall_image.py   (writes wall_image.h beside it; needs sympy and mpmath)
"""
import os
import time

import sympy as sp
from sympy.printing.c import C99CodePrinter

R1, R2, R3, h, a = sp.symbols("R1 R2 R3 h a", real=True)
ir = sp.Symbol("ir", positive=True)  # 1 / |R|
Rv = [R1, R2, R3]
Rn = sp.sqrt(R1 ** 2 + R2 ** 2 + R3 ** 2)


def S(i, j):
    return (1 if i == j else 0) / Rn + Rv[i] * Rv[j] / Rn ** 3


def Gim(i, j):
    s = 1 if j < 2 else -1
    inner = h * Rv[i] / Rn ** 3 - S(i, 2)
    return -S(i, j) + 2 * h * s * sp.diff(inner, Rv[j])


# derivatives: x_k -> d/dR_k ; y_1, y_2 -> -d/dR_1, -d/dR_2 ; y_3 -> d/dh + d/dR_3
def dx(e, k):
    return sp.diff(e, Rv[k])


def dy(e, k):
    if k < 2:
        return -sp.diff(e, Rv[k])
    return sp.diff(e, h) + sp.diff(e, R3)


def lapx(e):
    return sum(dx(dx(e, k), k) for k in range(3))


def lapy(e):
    return sum(dy(dy(e, k), k) for k in range(3))


EPS = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}


class _Printer(C99CodePrinter):
    """Integer powers as products, half-integer powers through sqrt."""

    def _print_Pow(self, e):
        b, n = e.base, e.exp
        if n.is_Integer:
            k = int(n)
            base = "(" + self._print(b) + ")"
            prod = "*".join([base] * abs(k)) if k != 0 else "1.0"
            return "(" + prod + ")" if k > 0 else "(1.0/(" + prod + "))"
        if n.is_Rational and n.q == 2:
            k = int(n.p)
            sq = "sqrt(" + self._print(b) + ")"
            if k == 1:
                return sq
            if k == -1:
                return "(1.0/" + sq + ")"
            return self._print_Pow(sp.Pow(b, sp.Rational(k - 1, 2))) + "*" + sq if k > 0 else \
                "(1.0/(" + sq + "*" + self._print(sp.Pow(b, sp.Rational(-k - 1, 2))) + "))"
        return super()._print_Pow(e)


class _PrinterF32(_Printer):
    """As _Printer, with single-precision literals (no promotion to double)."""

    def _print_Rational(self, e):
        return "(%d.0f/%d.0f)" % (e.p, e.q)

    def _print_Float(self, e):
        return repr(float(e)) + "f"

    def _print_Pow(self, e):
        return super()._print_Pow(e).replace("1.0/", "1.0f/").replace('"1.0"', '"1.0f"')


def blocks():
    """The four image blocks (times 8 pi eta) as 3 x 3 lists of sympy expressions."""
    G = [[Gim(i, j) for j in range(3)] for i in range(3)]
    Ly = [[G[i][j] + a ** 2 / 6 * lapy(G[i][j]) for j in range(3)] for i in range(3)]
    tt = [[Ly[i][j] + a ** 2 / 6 * lapx(Ly[i][j]) for j in range(3)] for i in range(3)]
    rt = [[sum(c * dx(Ly[l][j], k) for (ii, k, l), c in EPS.items() if ii == i) / 2 for j in range(3)]
          for i in range(3)]
    Lx = [[G[i][j] + a ** 2 / 6 * lapx(G[i][j]) for j in range(3)] for i in range(3)]
    # tr_ij: translation i at x from torque j at y = 1/2 eps_jmn d/dy_m Lx_in
    tr = [[sum(c * dy(Lx[i][n], m) for (jj, m, n), c in EPS.items() if jj == j) / 2 for j in range(3)]
          for i in range(3)]
    rr = [[sum(c1 * c2 * dx(dy(G[l][n], m), k)
               for (ii, k, l), c1 in EPS.items() if ii == i
               for (jj, m, n), c2 in EPS.items() if jj == j) / 4 for j in range(3)] for i in range(3)]
    return {"tt": tt, "tr": tr, "rt": rt, "rr": rr}


def _div(e, d):
    q, r = sp.div(sp.Poly(sp.expand(e), R1), sp.Poly(d, R1))
    assert r.is_zero, "a basis coefficient is not polynomial"
    return q.as_expr()


def _even_r1(e):
    """R1 enters a coefficient only through R1^2 = 1/ir^2 - R3^2 (the coefficients are
    functions of |R|, R3, h and a alone: the image system is symmetric about the wall normal)."""
    out = 0
    for (k,), c in sp.Poly(sp.expand(e), R1).terms():
        assert k % 2 == 0, "odd power of R1 in a coefficient"
        out += c * (1 / ir ** 2 - R3 ** 2) ** (k // 2)
    return sp.expand(out)


def coefficients(B):
    """Each block on a basis of tensors built from R, the wall normal e = (0, 0, 1) and
    c = R x e = (R2, -R1, 0), with scalar coefficients in ir, R3, h and a:
        true tensors (tt, rr):   A I + B R R^T + C R e^T + D e R^T + E e e^T
        pseudo-tensors (tr, rt): beta [e]x + gamma (c R^T + R c^T) + eps c e^T + zeta e c^T
    ([e]x v = e x v).  Read off in the plane R2 = 0, where the basis is independent."""
    rho2 = R1 ** 2 + R2 ** 2 + R3 ** 2
    E = {b: [[sp.expand(M[i][j].subs(rho2, 1 / ir ** 2).subs(R2, 0)) for j in range(3)] for i in range(3)]
         for b, M in B.items()}
    co = {}
    for b in ("tt", "rr"):
        M = E[b]
        assert all(sp.expand(M[i][j]) == 0 for i, j in ((0, 1), (1, 0), (1, 2), (2, 1)))
        A = M[1][1]
        Bc = _div(M[0][0] - M[1][1], R1 ** 2)
        C = _div(M[0][2], R1) - Bc * R3
        D = _div(M[2][0], R1) - Bc * R3
        Ec = M[2][2] - A - Bc * R3 ** 2 - (C + D) * R3
        co[b] = [_even_r1(x) for x in (A, Bc, C, D, Ec)]
    for b in ("tr", "rt"):
        P = E[b]
        assert all(sp.expand(P[i][j]) == 0 for i, j in ((0, 0), (0, 2), (1, 1), (2, 0), (2, 2)))
        beta = -(P[0][1] - P[1][0]) / 2
        gam = _div(-(P[0][1] + P[1][0]) / 2, R1 ** 2)
        eps = _div(-P[1][2], R1) - gam * R3
        zet = _div(-P[2][1], R1) - gam * R3
        co[b] = [_even_r1(x) for x in (beta, gam, eps, zet)]
    return co


def check(B, co, trials=20):
    """The basis form against the full blocks at random points, in 30-digit arithmetic."""
    import random
    import mpmath
    mpmath.mp.dps = 30
    full = {b: sp.lambdify((R1, R2, R3, h, a), sp.Matrix(M), "mpmath") for b, M in B.items()}
    cf = {b: sp.lambdify((ir, R3, h, a), co[b], "mpmath") for b in co}
    rng = random.Random(1)
    worst = 0
    for _ in range(trials):
        r = [mpmath.mpf(rng.uniform(-20, 20)), mpmath.mpf(rng.uniform(-20, 20)), mpmath.mpf(rng.uniform(2.5, 40))]
        hh, aa = mpmath.mpf(rng.uniform(1.2, float(r[2]) - 1.0)), mpmath.mpf(rng.choice([1.0, 0.7]))
        irr = 1 / mpmath.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
        e, c = [0, 0, 1], [r[1], -r[0], 0]
        ex = [[0, -1, 0], [1, 0, 0], [0, 0, 0]]
        for b in B:
            M, k = full[b](r[0], r[1], r[2], hh, aa), cf[b](irr, r[2], hh, aa)
            sc = max(abs(M[i, j]) for i in range(3) for j in range(3))
            for i in range(3):
                for j in range(3):
                    if b in ("tt", "rr"):
                        rec = (k[0] * (i == j) + k[1] * r[i] * r[j] + k[2] * r[i] * e[j] + k[3] * e[i] * r[j] +
                               k[4] * e[i] * e[j])
                    else:
                        rec = k[0] * ex[i][j] + k[1] * (c[i] * r[j] + r[i] * c[j]) + k[2] * c[i] * e[j] + k[3] * e[i] * c[j]
                    worst = max(worst, abs(rec - M[i, j]) / sc)
    assert worst < 1e-25, worst
    return worst


HEADER = """// Generated by gen_wall_image.py: the image part of the Rotne-Prager-Blake mobility
// (Blake's image system under the Faxen operators of both spheres) applied to one source's
// force and torque.  Variables: R = x - y* (y* the mirror image of the source), ir = 1/|R|,
// h = source height, a the radius; e = (0, 0, 1) the wall normal and c = R x e.  Each block
// (times 8 pi eta) is written on a basis of tensors built from R, e and c:
//   tt, rr = A I + B R R^T + C R e^T + D e R^T + E e e^T
//   tr, rt = beta [e]x + gamma (c R^T + R c^T) + eps c e^T + zeta e c^T
// with coefficients that depend on ir, R3, h and a only.  Two forms: double, and float
// (single-precision literals throughout).  Do not edit.
#pragma once

namespace fil {
"""

TEMPLATE = """
// vi += (tt F + tr T), wi += (rt F + rr T), all times 8 pi eta
__device__ __host__ inline void %(name)s(%(T)s R1, %(T)s R2, %(T)s R3, %(T)s ir, %(T)s h, %(T)s a,
                                         const %(T)s F[3], const %(T)s T[3], %(T)s vi[3], %(T)s wi[3]) {
%(body)s
    const %(T)s c1 = R2, c2 = -R1;
    const %(T)s rF = R1 * F[0] + R2 * F[1] + R3 * F[2], rT = R1 * T[0] + R2 * T[1] + R3 * T[2];
    const %(T)s cF = c1 * F[0] + c2 * F[1], cT = c1 * T[0] + c2 * T[1];
    // tt F
    %(T)s k = tt_B * rF + tt_C * F[2];
    vi[0] += tt_A * F[0] + k * R1;
    vi[1] += tt_A * F[1] + k * R2;
    vi[2] += tt_A * F[2] + k * R3 + tt_D * rF + tt_E * F[2];
    // tr T
    k = tr_gamma * rT + tr_eps * T[2];
    vi[0] += -tr_beta * T[1] + k * c1 + tr_gamma * cT * R1;
    vi[1] += tr_beta * T[0] + k * c2 + tr_gamma * cT * R2;
    vi[2] += tr_gamma * cT * R3 + tr_zeta * cT;
    // rt F
    k = rt_gamma * rF + rt_eps * F[2];
    wi[0] += -rt_beta * F[1] + k * c1 + rt_gamma * cF * R1;
    wi[1] += rt_beta * F[0] + k * c2 + rt_gamma * cF * R2;
    wi[2] += rt_gamma * cF * R3 + rt_zeta * cF;
    // rr T
    k = rr_B * rT + rr_C * T[2];
    wi[0] += rr_A * T[0] + k * R1;
    wi[1] += rr_A * T[1] + k * R2;
    wi[2] += rr_A * T[2] + k * R3 + rr_D * rT + rr_E * T[2];
}
"""


def main():
    t0 = time.time()
    B = blocks()
    co = coefficients(B)
    print("basis coefficients in %.1f s; reconstruction error %.1e" % (time.time() - t0, check(B, co)), flush=True)
    names = {"tt": ["A", "B", "C", "D", "E"], "rr": ["A", "B", "C", "D", "E"],
             "tr": ["beta", "gamma", "eps", "zeta"], "rt": ["beta", "gamma", "eps", "zeta"]}
    outs, exprs = [], []
    for b in ("tt", "tr", "rt", "rr"):
        for n, e in zip(names[b], co[b]):
            outs.append("%s_%s" % (b, n))
            exprs.append(e)
    reps, red = sp.cse(exprs, symbols=sp.numbered_symbols("t"), optimizations="basic")
    text = HEADER
    for name, T, pr in (("wall_image_apply", "double", _Printer()), ("wall_image_apply_f32", "float", _PrinterF32())):
        lines = ["    const %s %s = %s;" % (T, s_, pr.doprint(e)) for s_, e in reps]
        lines += ["    const %s %s = %s;" % (T, n, pr.doprint(e)) for n, e in zip(outs, red)]
        text += TEMPLATE % {"name": name, "T": T, "body": "\n".join(lines)}
    text += "\n}  // namespace fil\n"
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wall_image.h")
    with open(out, "w") as f:
        f.write(text)
    print("wrote", out, "(%d temporaries)" % len(reps))


if __name__ == "__main__":
    main()
