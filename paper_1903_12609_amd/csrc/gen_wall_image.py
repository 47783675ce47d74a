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

Run:  python gen_wall_image.py   (writes wall_image.h beside it; needs sympy)
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


def main():
    t0 = time.time()
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
    blocks = {"tt": tt, "tr": tr, "rt": rt, "rr": rr}
    names, exprs = [], []
    rho2 = R1 ** 2 + R2 ** 2 + R3 ** 2
    for b, M in blocks.items():
        for i in range(3):
            for j in range(3):
                names.append("%s[%d][%d]" % (b, i, j))
                # every power of |R| in terms of ir = 1/|R|: products instead of divisions
                e = M[i][j].subs(rho2, 1 / ir ** 2)
                left = [q for q in e.atoms(sp.Pow) if q.base.is_Add and q.base.has(R1) and q.exp.is_negative]
                assert not left, "a negative power of |R| was left"
                exprs.append(e)
    print("derived in %.1f s" % (time.time() - t0), flush=True)
    reps, red = sp.cse(exprs, symbols=sp.numbered_symbols("t"), optimizations="basic")
    print("cse in %.1f s: %d temporaries" % (time.time() - t0, len(reps)), flush=True)
    lines = []
    pr = _Printer()
    for s_, e in reps:
        lines.append("    const double %s = %s;" % (s_, pr.doprint(e)))
    for n, e in zip(names, red):
        lines.append("    %s = %s;" % (n, pr.doprint(e)))
    body = "\n".join(lines)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wall_image.h")
    with open(out, "w") as f:
        f.write("// Generated by gen_wall_image.py: the image part of the Rotne-Prager-Blake mobility\n"
                "// blocks times 8 pi eta, in the variables R = x - y* (y* the mirror image of the\n"
                "// source), ir = 1/|R| and h = source height; a the radius.  Do not edit.\n"
                "#pragma once\n\n"
                "namespace fil {\n\n"
                "__device__ __host__ inline void wall_image_blocks(double R1, double R2, double R3, double ir, "
                "double h, double a,\n"
                "                                                  double tt[3][3], double tr[3][3], "
                "double rt[3][3], double rr[3][3]) {\n"
                + body + "\n}\n\n}  // namespace fil\n")
    print("wrote", out, "(%d lines)" % len(lines))


if __name__ == "__main__":
    main()
