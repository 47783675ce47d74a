/*
 * fil_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, double-precision CPU statement of the implicit quaternion
 * filament method of Schoeller, Townsend, Westwood & Keaveny, "Methods for
 * suspensions of passive and active filaments" (arXiv:1903.12609).  It is the
 * checker the GPU library is compared against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark load it; it shares no code,
 * header or table with the GPU path, and the GPU path never calls it.
 *
 * Layout here is array-of-structures: a vector field over S segments is
 * double[S][3], quaternions are double[S][4] stored (q0, q1, q2, q3).
 * Segments are filament-major; fil_off[M+1] gives each filament's range.
 * The unknown vector of one filament (Sec. 2.9.3, reduced system) is
 *   X_f = [ Y_1 (3) | u_1 .. u_N (3N) | Lambda_{3/2} .. Lambda_{N-1/2} (3(N-1)) ]
 * and the global X concatenates filaments, filament f starting at 6*fil_off[f].
 * A clamped (tethered) filament stores the tether multipliers lambda_1,
 * lambda_2 in the Y_1 and u_1 slots (Sec. 5.2.1, tethering constraints).  A pinned
 * filament (base position held, its rotation free, as the cilia bases of Sec. 5.2.2)
 * stores lambda_1 in the Y_1 slot and keeps u_1 as an unknown.
 *
 * Parity: every function below is pinned by a CPU test (tests/test_oracle_*.py)
 * except where its comment says "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3]) {
    double c0 = a[1] * b[2] - a[2] * b[1];
    double c1 = a[2] * b[0] - a[0] * b[2];
    double c2 = a[0] * b[1] - a[1] * b[0];
    c[0] = c0; c[1] = c1; c[2] = c2;
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
/* 3x3 matrices are row-major double[9] */
static void mat_vec(const double A[9], const double x[3], double y[3]) {
    for (int i = 0; i < 3; i++) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}
static void mat_mul(const double A[9], const double B[9], double C[9]) {
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}
/* [v x]: the matrix with [v x] w = v x w */
static void skew(const double v[3], double A[9]) {
    A[0] = 0;     A[1] = -v[2]; A[2] = v[1];
    A[3] = v[2];  A[4] = 0;     A[5] = -v[0];
    A[6] = -v[1]; A[7] = v[0];  A[8] = 0;
}
/* [x v] = -[v x]: the matrix with [x v] w = w x v */
static void rskew(const double v[3], double A[9]) {
    skew(v, A);
    for (int i = 0; i < 9; i++) A[i] = -A[i];
}
static void eye3(double A[9], double s) {
    memset(A, 0, 9 * sizeof(double));
    A[0] = A[4] = A[8] = s;
}

/* ------------------------------------------------------------------------ */
/* Quaternions, Sec. 2.9.1 and Appendix A.1                                  */
/* ------------------------------------------------------------------------ */
/* product p.q = (p0 q0 - p.q, p0 q + q0 p + p x q)  (Sec. 2.9.1) */
void or_qmul(const double p[4], const double q[4], double r[4]) {
    double pv[3] = {p[1], p[2], p[3]}, qv[3] = {q[1], q[2], q[3]}, c[3];
    cross3(pv, qv, c);
    double r0 = p[0] * q[0] - dot3(pv, qv);
    double r1 = p[0] * qv[0] + q[0] * pv[0] + c[0];
    double r2 = p[0] * qv[1] + q[0] * pv[1] + c[1];
    double r3 = p[0] * qv[2] + q[0] * pv[2] + c[2];
    r[0] = r0; r[1] = r1; r[2] = r2; r[3] = r3;
}
static void qconj(const double q[4], double r[4]) { r[0] = q[0]; r[1] = -q[1]; r[2] = -q[2]; r[3] = -q[3]; }

/* rotation matrix R(q), Sec. 2.9.1 (row-major); its columns are the frame (t, mu, nu) */
void or_qrot(const double q[4], double R[9]) {
    double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    R[0] = 1 - 2 * q2 * q2 - 2 * q3 * q3; R[1] = 2 * (q1 * q2 - q3 * q0);     R[2] = 2 * (q1 * q3 + q2 * q0);
    R[3] = 2 * (q1 * q2 + q3 * q0);     R[4] = 1 - 2 * q1 * q1 - 2 * q3 * q3; R[5] = 2 * (q3 * q2 - q1 * q0);
    R[6] = 2 * (q1 * q3 - q2 * q0);     R[7] = 2 * (q3 * q2 + q1 * q0);     R[8] = 1 - 2 * q2 * q2 - 2 * q1 * q1;
}
/* frame vectors t = R e_x, mu = R e_y, nu = R e_z */
static void frame(const double q[4], double t[3], double mu[3], double nu[3]) {
    double R[9];
    or_qrot(q, R);
    if (t) { t[0] = R[0]; t[1] = R[3]; t[2] = R[6]; }
    if (mu) { mu[0] = R[1]; mu[1] = R[4]; mu[2] = R[7]; }
    if (nu) { nu[0] = R[2]; nu[1] = R[5]; nu[2] = R[8]; }
}

/* square root, Appendix A.1: (p0, p) -> (sqrt((p0+1)/2), p / sqrt(2(p0+1))), and
 * (0,0,0,1) when p0 = -1 (taken literally, reading R3) */
void or_qsqrt(const double p[4], double r[4]) {
    if (p[0] == -1.0) { r[0] = 0; r[1] = 0; r[2] = 0; r[3] = 1; return; }
    double d = sqrt(2.0 * (p[0] + 1.0));
    r[0] = sqrt((p[0] + 1.0) / 2.0);
    r[1] = p[1] / d; r[2] = p[2] / d; r[3] = p[3] / d;
}

/* interpolated quaternion q_{n+1/2} = (q_{n+1} . q_n^*)^{1/2} . q_n  (Sec. 2.9.2) */
void or_qmid(const double qn[4], const double qn1[4], double r[4]) {
    double c[4], p[4], h[4];
    qconj(qn, c);
    or_qmul(qn1, c, p);
    or_qsqrt(p, h);
    or_qmul(h, qn, r);
}

/* exponential map exp(u) = (cos(|u|/2), sin(|u|/2) u/|u|), Sec. 2.9.3; exp(0) = identity */
void or_qexp(const double u[3], double r[4]) {
    double x = norm3(u);
    if (x == 0.0) { r[0] = 1; r[1] = r[2] = r[3] = 0; return; }
    double s = sin(0.5 * x) / x;
    r[0] = cos(0.5 * x); r[1] = s * u[0]; r[2] = s * u[1]; r[3] = s * u[2];
}

/* dexp^{-1}_u(w) = w - 1/2 u x w - (|u| cot(|u|/2) - 2)/(2|u|^2) u x (u x w), Sec. 2.9.3.
 * For |u| < 1e-3 the coefficient is its Taylor series 1/12 + x^2/720 + x^4/30240
 * (reading R10); at |u| = 0 it is 1/12, which gives the three-term Taylor form of
 * Appendix B.2. */
void or_dexpinv(const double u[3], const double w[3], double r[3]) {
    double x = norm3(u), uw[3], uuw[3], coef;
    cross3(u, w, uw);
    cross3(u, uw, uuw);
    if (x < 1e-3) {
        double x2 = x * x;
        coef = 1.0 / 12.0 + x2 / 720.0 + x2 * x2 / 30240.0;
    } else {
        coef = -(x / tan(0.5 * x) - 2.0) / (2.0 * x * x);
    }
    for (int i = 0; i < 3; i++) r[i] = w[i] - 0.5 * uw[i] + coef * uuw[i];
}

/* ------------------------------------------------------------------------ */
/* RPY mobility, Sec. 2.7.1                                                  */
/* ------------------------------------------------------------------------ */
/* The four 3x3 blocks coupling target n to source m for displacement
 * r = Y_n - Y_m.  self != 0 selects the n = m entries.  For r >= 2a the blocks
 * are the printed unbounded tensors; (eps . rhat)_{ij} = eps_{ijk} rhat_k
 * (reading R1).  For r < 2a the paper only cites the overlapping-sphere
 * correction; the equal-radius regularised forms are used (reading R2):
 *   Mtt = 1/(6 pi eta a) [(1 - 9r/(32a)) I + 3r/(32a) rhat rhat]
 *   Mrr = 1/(8 pi eta a^3) [(1 - 27r/(32a) + 5r^3/(64a^3)) I + (9r/(32a) - 3r^3/(64a^3)) rhat rhat]
 *   Mtr = Mrt = 1/(16 pi eta a^2) (r/a - 3r^2/(8a^2)) eps . rhat
 * with rhat rhat r-weighted terms taken as 0 at r = 0. */
void or_rpy_blocks(const double r[3], int self, double a, double eta,
                   double Mtt[9], double Mtr[9], double Mrt[9], double Mrr[9]) {
    double d = norm3(r);
    double rh[3] = {0, 0, 0};
    if (d > 0) { rh[0] = r[0] / d; rh[1] = r[1] / d; rh[2] = r[2] / d; }
    double RR[9], E[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) RR[3 * i + j] = rh[i] * rh[j];
    /* E_ij = eps_ijk rhat_k */
    E[0] = 0;      E[1] = rh[2];  E[2] = -rh[1];
    E[3] = -rh[2]; E[4] = 0;      E[5] = rh[0];
    E[6] = rh[1];  E[7] = -rh[0]; E[8] = 0;
    double ctt_i, ctt_r, crr_i, crr_r, ctr;
    if (self) {
        ctt_i = 1.0 / (6.0 * PI * eta * a); ctt_r = 0;
        crr_i = 1.0 / (8.0 * PI * eta * a * a * a); crr_r = 0;
        ctr = 0;
    } else if (d >= 2.0 * a) {
        ctt_i = (1.0 + 2.0 * a * a / (3.0 * d * d)) / (8.0 * PI * eta * d);
        ctt_r = (1.0 - 2.0 * a * a / (d * d)) / (8.0 * PI * eta * d);
        crr_i = -1.0 / (16.0 * PI * eta * d * d * d);
        crr_r = 3.0 / (16.0 * PI * eta * d * d * d);
        ctr = 1.0 / (8.0 * PI * eta * d * d);
    } else {
        double x = d / a;
        ctt_i = (1.0 - 9.0 * x / 32.0) / (6.0 * PI * eta * a);
        ctt_r = (3.0 * x / 32.0) / (6.0 * PI * eta * a);
        crr_i = (1.0 - 27.0 * x / 32.0 + 5.0 * x * x * x / 64.0) / (8.0 * PI * eta * a * a * a);
        crr_r = (9.0 * x / 32.0 - 3.0 * x * x * x / 64.0) / (8.0 * PI * eta * a * a * a);
        ctr = (x - 3.0 * x * x / 8.0) / (16.0 * PI * eta * a * a);
    }
    for (int k = 0; k < 9; k++) {
        double I = (k == 0 || k == 4 || k == 8) ? 1.0 : 0.0;
        Mtt[k] = ctt_i * I + ctt_r * RR[k];
        Mrr[k] = crr_i * I + crr_r * RR[k];
        Mtr[k] = ctr * E[k];
        Mrt[k] = ctr * E[k];
    }
}

/* (V_n, Omega_n) = sum_m [[Mtt, Mtr],[Mrt, Mrr]]_{nm} (F_m, T_m): the direct pairwise
 * sum of Sec. 2.7.1.  OpenMP only splits the target loop. */
void or_rpy_apply(int64_t S, const double* Y, const double* F, const double* T, double a, double eta,
                  double* V, double* W, int64_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads((int)nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t n = 0; n < S; n++) {
        double v[3] = {0, 0, 0}, w[3] = {0, 0, 0};
        for (int64_t m = 0; m < S; m++) {
            double r[3] = {Y[3 * n] - Y[3 * m], Y[3 * n + 1] - Y[3 * m + 1], Y[3 * n + 2] - Y[3 * m + 2]};
            double Mtt[9], Mtr[9], Mrt[9], Mrr[9], y1[3], y2[3], y3[3], y4[3];
            or_rpy_blocks(r, n == m, a, eta, Mtt, Mtr, Mrt, Mrr);
            mat_vec(Mtt, F + 3 * m, y1);
            mat_vec(Mtr, T + 3 * m, y2);
            mat_vec(Mrt, F + 3 * m, y3);
            mat_vec(Mrr, T + 3 * m, y4);
            for (int i = 0; i < 3; i++) { v[i] += y1[i] + y2[i]; w[i] += y3[i] + y4[i]; }
        }
        for (int i = 0; i < 3; i++) { V[3 * n + i] = v[i]; W[3 * n + i] = w[i]; }
    }
}

/* The same sum for a subset of targets idx[0..ntgt) only (sampled checks at full size);
 * V, W are [ntgt][3]. */
void or_rpy_apply_targets(int64_t S, const double* Y, const double* F, const double* T, double a, double eta,
                          int64_t ntgt, const int64_t* idx, double* V, double* W, int64_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads((int)nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < ntgt; i++) {
        int64_t n = idx[i];
        double v[3] = {0, 0, 0}, w[3] = {0, 0, 0};
        for (int64_t m = 0; m < S; m++) {
            double r[3] = {Y[3 * n] - Y[3 * m], Y[3 * n + 1] - Y[3 * m + 1], Y[3 * n + 2] - Y[3 * m + 2]};
            double Mtt[9], Mtr[9], Mrt[9], Mrr[9], y1[3], y2[3], y3[3], y4[3];
            or_rpy_blocks(r, n == m, a, eta, Mtt, Mtr, Mrt, Mrr);
            mat_vec(Mtt, F + 3 * m, y1);
            mat_vec(Mtr, T + 3 * m, y2);
            mat_vec(Mrt, F + 3 * m, y3);
            mat_vec(Mrr, T + 3 * m, y4);
            for (int k = 0; k < 3; k++) { v[k] += y1[k] + y2[k]; w[k] += y3[k] + y4[k]; }
        }
        for (int k = 0; k < 3; k++) { V[3 * i + k] = v[k]; W[3 * i + k] = w[k]; }
    }
}

/* Assembled 6S x 6S grand mobility (row-major), unknowns ordered (F_1..F_S, T_1..T_S). */
void or_rpy_matrix(int64_t S, const double* Y, double a, double eta, double* Mg) {
    int64_t n6 = 6 * S;
    for (int64_t n = 0; n < S; n++)
        for (int64_t m = 0; m < S; m++) {
            double r[3] = {Y[3 * n] - Y[3 * m], Y[3 * n + 1] - Y[3 * m + 1], Y[3 * n + 2] - Y[3 * m + 2]};
            double Mtt[9], Mtr[9], Mrt[9], Mrr[9];
            or_rpy_blocks(r, n == m, a, eta, Mtt, Mtr, Mrt, Mrr);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    Mg[(3 * n + i) * n6 + 3 * m + j] = Mtt[3 * i + j];
                    Mg[(3 * n + i) * n6 + 3 * S + 3 * m + j] = Mtr[3 * i + j];
                    Mg[(3 * S + 3 * n + i) * n6 + 3 * m + j] = Mrt[3 * i + j];
                    Mg[(3 * S + 3 * n + i) * n6 + 3 * S + 3 * m + j] = Mrr[3 * i + j];
                }
        }
}

/* ------------------------------------------------------------------------ */
/* Steric barrier, Sec. 2.6                                                   */
/* ------------------------------------------------------------------------ */
/* F^B_n = sum_m F^S ((4a^2 chi^2 - r^2) / (4a^2 (chi^2 - 1)))^4 r_nm / (2a) for r < 2 chi a,
 * skipping m = n and the neighbours m = n +- 1 of the same filament.  seg_fil[S]
 * gives each segment's filament.  Lper[3] (or NULL: unbounded) are the lengths of a
 * periodic box, where r_nm is the nearest periodic image of Y_n - Y_m (the cutoff is
 * below half of every length).  Adds into FB. */
void or_steric(int64_t S, const double* Y, const int64_t* seg_fil, double a, double chi, double FS,
               const double* Lper, double* FB) {
    double rc = 2.0 * chi * a;
    for (int64_t n = 0; n < S; n++)
        for (int64_t m = 0; m < S; m++) {
            if (m == n) continue;
            if (seg_fil[m] == seg_fil[n] && (m == n + 1 || m + 1 == n)) continue;
            double r[3] = {Y[3 * n] - Y[3 * m], Y[3 * n + 1] - Y[3 * m + 1], Y[3 * n + 2] - Y[3 * m + 2]};
            if (Lper)
                for (int i = 0; i < 3; i++) r[i] -= Lper[i] * nearbyint(r[i] / Lper[i]);
            double d2 = dot3(r, r);
            if (d2 >= rc * rc) continue;
            double b = (4.0 * a * a * chi * chi - d2) / (4.0 * a * a * (chi * chi - 1.0));
            double f = FS * b * b * b * b / (2.0 * a);
            for (int i = 0; i < 3; i++) FB[3 * n + i] += f * r[i];
        }
}

/* ------------------------------------------------------------------------ */
/* Internal moments and forces, Sec. 2.5 and Sec. 2.9.2                       */
/* ------------------------------------------------------------------------ */
/* M_{n+1/2} = R(q_{n+1/2}) D (2 [q_{n+1/2}^* . (q_{n+1} - q_n)/dL]_{R3} - (gamma0, kmu, knu)),
 * D = diag(KT, KB, KB)  (eq. for the discrete quaternion moment, Sec. 2.9.2). */
void or_moment(const double qn[4], const double qn1[4], const double kap[3], double dL, double KB, double KT,
               double M[3]) {
    double h[4], hc[4], dq[4], p[4], R[9], z[3];
    or_qmid(qn, qn1, h);
    qconj(h, hc);
    for (int i = 0; i < 4; i++) dq[i] = (qn1[i] - qn[i]) / dL;
    or_qmul(hc, dq, p);
    double D[3] = {KT, KB, KB};
    for (int i = 0; i < 3; i++) z[i] = D[i] * (2.0 * p[i + 1] - kap[i]);
    or_qrot(h, R);
    mat_vec(R, z, M);
}

/* One filament of N segments: adds F^C_n = Lambda_{n+1/2} - Lambda_{n-1/2} into F and
 * T^C_n + T^E_n into T, where T^C_n = dL/2 t_n x (Lambda_{n+1/2} + Lambda_{n-1/2}) and
 * T^E_n = M_{n+1/2} - M_{n-1/2}; Lambda_{1/2} = Lambda_{N+1/2} = M_{1/2} = M_{N+1/2} = 0
 * (Sec. 2.5).  Lam and kap are [N-1][3] (joint k between segments k and k+1); kap holds
 * (gamma0, kappa_mu, kappa_nu). */
void or_internal_forces(int64_t N, const double* q, const double* Lam, const double* kap, double dL, double KB,
                        double KT, double* F, double* T) {
    for (int64_t n = 0; n < N; n++) {
        double lp[3] = {0, 0, 0}, lm[3] = {0, 0, 0}, mp[3] = {0, 0, 0}, mm[3] = {0, 0, 0};
        if (n + 1 < N) {
            memcpy(lp, Lam + 3 * n, sizeof lp);
            or_moment(q + 4 * n, q + 4 * (n + 1), kap + 3 * n, dL, KB, KT, mp);
        }
        if (n > 0) {
            memcpy(lm, Lam + 3 * (n - 1), sizeof lm);
            or_moment(q + 4 * (n - 1), q + 4 * n, kap + 3 * (n - 1), dL, KB, KT, mm);
        }
        double t[3], ls[3], tc[3];
        frame(q + 4 * n, t, NULL, NULL);
        for (int i = 0; i < 3; i++) ls[i] = lp[i] + lm[i];
        cross3(t, ls, tc);
        for (int i = 0; i < 3; i++) {
            F[3 * n + i] += lp[i] - lm[i];
            T[3 * n + i] += 0.5 * dL * tc[i] + mp[i] - mm[i];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The implicit step: Sec. 2.9.3 (system), Sec. 3.2 (Alg. 2), Appendix B.2 (J0) */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t M;               /* filaments */
    const int64_t* fil_off;  /* [M+1] segment offsets, filament-major */
    double a, eta, dL, KB, KT;
    double chi, FS;          /* steric barrier, Sec. 2.6; FS == 0 switches it off */
    double grav[3];          /* external (gravity) force on every segment */
    double dt, tol;          /* time step; Broyden stops at max|f| / a <= tol */
    int64_t kmax;            /* Broyden iteration cap */
    /* preferred curvature kappa_nu(s,t) = K0 sin(kw s - omega t + phase[f]) (Sec. 5.3) */
    double K0, kw, omega;
    const double* phase;     /* [M] or NULL for no preferred curvature */
    const int32_t* tether;   /* [M], 1 = base clamped (Sec. 5.2.1), 2 = base pinned, 3 = base on a
                              * rotating motor (Sec. 5.2.1); NULL: all free */
    double motor_d0, motor_w; /* the motor: base distance from its z axis and rotation rate */
    const double* base;      /* [M][3] clamped base positions */
    int64_t nthreads;        /* OpenMP threads for the RPY target loop (0: default) */
    int64_t drag_only;       /* 1: diagonal drag mobility, no steric, no gravity: the f0 of Sec. 3.2.1 */
    const double* fext;      /* [S][3] further external force on each segment (Sec. 2.5), or NULL */
    const double* text;      /* [S][3] further external torque on each segment (Sec. 2.5), or NULL */
    /* periodic box (Sec. 2.7.2): its lengths [3] for the steric barrier's nearest images
     * (NULL: unbounded), and a mobility (V, W) = M(Y) (F, T) over [S][3] arrays that takes
     * the place of the unbounded RPY apply (NULL: RPY) */
    const double* Lper;
    void (*mobility)(void* ctx, int64_t S, const double* Y, const double* F, const double* T, double* V, double* W);
    void* mob_ctx;
} or_params;

typedef struct {
    double* Y;      /* [S][3]  Y^j */
    double* Yprev;  /* [S][3]  Y^{j-1} */
    double* q;      /* [S][4]  q^j */
    double* X;      /* [6S]    converged unknowns of step j (holds u^j, Lambda^j, ...) */
    double* Xprev;  /* [6S]    converged unknowns of step j-1 */
    double t;
    int64_t step;   /* number of completed steps */
} or_state;

typedef struct {
    int64_t iters;      /* Broyden updates taken */
    int64_t applies;    /* residual (mobility) evaluations */
    double resid;       /* final max|f| / a */
    int64_t converged;
} or_report;

static int64_t total_segments(const or_params* P) { return P->fil_off[P->M]; }
static int is_tethered(const or_params* P, int64_t f) { return P->tether && P->tether[f]; }
/* the base orientation is prescribed too (lambda_2 in the u_1 slot): held (1) or turned by the motor (3) */
static int is_clamped(const or_params* P, int64_t f) { return P->tether && (P->tether[f] == 1 || P->tether[f] == 3); }
static int is_motor(const or_params* P, int64_t f) { return P->tether && P->tether[f] == 3; }
/* the motor's prescribed base rotation per step, u_1 = (0, 0, omega dt) */
static void motor_u(const or_params* P, double u[3]) { u[0] = 0; u[1] = 0; u[2] = P->motor_w * P->dt; }
/* the motor's base position at time tt: on the circle of radius d0 about the z axis through
 * base - (d0, 0, 0) (base = the initial Y_1), at angle omega tt */
static void motor_base(const or_params* P, int64_t f, double tt, double y[3]) {
    y[0] = P->base[3 * f] - P->motor_d0 + P->motor_d0 * cos(P->motor_w * tt);
    y[1] = P->base[3 * f + 1] + P->motor_d0 * sin(P->motor_w * tt);
    y[2] = P->base[3 * f + 2];
}

/* BDF coefficients: y - a1 y^j - a2 y^{j-1} - b dt v = 0,  u - g u^j - b dt dexpinv(Omega) = 0.
 * The first step is BDF1 (reading R7), every later one BDF2 (Sec. 2.9.3). */
static void bdf_coeffs(int64_t step, double* a1, double* a2, double* b, double* g) {
    if (step == 0) { *a1 = 1.0; *a2 = 0.0; *b = 1.0; *g = 0.0; }
    else { *a1 = 4.0 / 3.0; *a2 = -1.0 / 3.0; *b = 2.0 / 3.0; *g = 1.0 / 3.0; }
}

/* preferred curvature at joint k (between segments k and k+1, 0-based k), evaluated at
 * s = (k+1) dL and time tt (reading R4: the joint n+1/2 uses s_{n+1}) */
static void joint_kappa(const or_params* P, int64_t f, int64_t k, double tt, double kap[3]) {
    kap[0] = 0; kap[1] = 0; kap[2] = 0;
    if (P->phase) kap[2] = P->K0 * sin(P->kw * (double)(k + 1) * P->dL - P->omega * tt + P->phase[f]);
}

/* Rebuild the configuration from X: q_n = exp(u_n) . q_n^j, t_n = R(q_n) e_x and the
 * robot-arm positions Y_n = Y_1 + dL/2 sum_{m=2}^{n} (t_{m-1} + t_m) (Sec. 2.9.3).
 * A clamped filament keeps Y_1 = base and u_1 = 0. */
void or_reconstruct(const or_params* P, const double* qj, const double* X, double tt, double* Yo, double* qo) {
    for (int64_t f = 0; f < P->M; f++) {
        int64_t s0 = P->fil_off[f], N = P->fil_off[f + 1] - s0;
        const double* Xf = X + 6 * s0;
        for (int64_t n = 0; n < N; n++) {
            double u[3] = {Xf[3 + 3 * n], Xf[4 + 3 * n], Xf[5 + 3 * n]}, e[4];
            if (n == 0 && is_clamped(P, f)) { u[0] = u[1] = u[2] = 0; }
            if (n == 0 && is_motor(P, f)) motor_u(P, u);
            or_qexp(u, e);
            or_qmul(e, qj + 4 * (s0 + n), qo + 4 * (s0 + n));
        }
        double y[3];
        if (is_motor(P, f)) motor_base(P, f, tt, y);
        else if (is_tethered(P, f)) memcpy(y, P->base + 3 * f, sizeof y);
        else memcpy(y, Xf, sizeof y);
        memcpy(Yo + 3 * s0, y, sizeof y);
        double tprev[3];
        frame(qo + 4 * s0, tprev, NULL, NULL);
        for (int64_t n = 1; n < N; n++) {
            double tn[3];
            frame(qo + 4 * (s0 + n), tn, NULL, NULL);
            for (int i = 0; i < 3; i++) {
                y[i] += 0.5 * P->dL * (tprev[i] + tn[i]);
                Yo[3 * (s0 + n) + i] = y[i];
            }
            memcpy(tprev, tn, sizeof tn);
        }
    }
}

/* Forces and torques the segments exert on the fluid for configuration (Y, q) and
 * multipliers in X: F^H = F^C + F^B + gravity (+ further external forces),
 * T^H = T^C + T^E (Sec. 2.5 and the
 * mobility problem of Sec. 2.7), plus tether multipliers on clamped bases. */
void or_forces(const or_params* P, const double* Y, const double* q, const double* X, double tt, double* F,
               double* T) {
    int64_t S = total_segments(P);
    memset(F, 0, 3 * S * sizeof(double));
    memset(T, 0, 3 * S * sizeof(double));
    for (int64_t f = 0; f < P->M; f++) {
        int64_t s0 = P->fil_off[f], N = P->fil_off[f + 1] - s0;
        double* Lam = (double*)calloc(3 * (N > 1 ? N - 1 : 1), sizeof(double));
        double* kap = (double*)calloc(3 * (N > 1 ? N - 1 : 1), sizeof(double));
        for (int64_t k = 0; k + 1 < N; k++) {
            memcpy(Lam + 3 * k, X + 6 * s0 + 3 + 3 * N + 3 * k, 3 * sizeof(double));
            joint_kappa(P, f, k, tt, kap + 3 * k);
        }
        or_internal_forces(N, q + 4 * s0, Lam, kap, P->dL, P->KB, P->KT, F + 3 * s0, T + 3 * s0);
        if (is_tethered(P, f)) {
            /* tethered base, Y_1 held: F^C_1 += lambda_1; clamped (u_1^j = 0) also
             * T^C_1 += lambda_2 (Sec. 5.2.1) */
            for (int i = 0; i < 3; i++) {
                F[3 * s0 + i] += X[6 * s0 + i];
                if (is_clamped(P, f) && !is_motor(P, f)) T[3 * s0 + i] += X[6 * s0 + 3 + i];
            }
            if (is_motor(P, f)) {
                /* T^C_1 += D^T lambda_2 with D v = dexpinv_{u_1}(v) = v - 1/2 u x v + c u x (u x v)
                 * (Sec. 5.2.1), so D^T v = v + 1/2 u x v + c u x (u x v), c as in or_dexpinv */
                double u[3], l[3] = {X[6 * s0 + 3], X[6 * s0 + 4], X[6 * s0 + 5]}, ul[3], uul[3];
                motor_u(P, u);
                cross3(u, l, ul);
                cross3(u, ul, uul);
                double x = norm3(u);
                double c = x < 1e-3 ? 1.0 / 12.0 + x * x / 720.0 + x * x * x * x / 30240.0
                                    : -(x / tan(0.5 * x) - 2.0) / (2.0 * x * x);
                for (int i = 0; i < 3; i++) T[3 * s0 + i] += l[i] + 0.5 * ul[i] + c * uul[i];
            }
        }
        free(Lam);
        free(kap);
    }
    for (int64_t n = 0; n < S; n++)
        for (int i = 0; i < 3; i++) F[3 * n + i] += P->grav[i] + (P->fext ? P->fext[3 * n + i] : 0.0);
    if (P->text)
        for (int64_t n = 0; n < 3 * S; n++) T[n] += P->text[n];
    if (P->FS != 0.0) {
        int64_t* seg_fil = (int64_t*)malloc(S * sizeof(int64_t));
        for (int64_t f = 0; f < P->M; f++)
            for (int64_t n = P->fil_off[f]; n < P->fil_off[f + 1]; n++) seg_fil[n] = f;
        or_steric(S, Y, seg_fil, P->a, P->chi, P->FS, P->Lper, F);
        free(seg_fil);
    }
}

/* Residual f(X) of the reduced system (Sec. 2.9.3), rows ordered like X:
 *   f^1   = Y_1 - a1 Y_1^j - a2 Y_1^{j-1} - b dt V_1
 *   f^2_n = u_n - g u_n^j - b dt dexpinv_{u_n}(Omega_n)          n = 1..N
 *   f^3_n = Y_n(X) - a1 Y_n^j - a2 Y_n^{j-1} - b dt V_n             n = 2..N
 * Returns max|f| / a.  Yout, qout (may be NULL) receive the configuration. */
double or_residual(const or_params* P, const or_state* St, const double* X, double* fout, double* Yout,
                   double* qout) {
    int64_t S = total_segments(P);
    double a1, a2, b, g;
    bdf_coeffs(St->step, &a1, &a2, &b, &g);
    double tt = St->t + P->dt;
    double* Y = (double*)malloc(3 * S * sizeof(double));
    double* q = (double*)malloc(4 * S * sizeof(double));
    double* F = (double*)malloc(3 * S * sizeof(double));
    double* T = (double*)malloc(3 * S * sizeof(double));
    double* V = (double*)malloc(3 * S * sizeof(double));
    double* W = (double*)malloc(3 * S * sizeof(double));
    or_reconstruct(P, St->q, X, St->t + P->dt, Y, q);
    if (P->drag_only) {
        /* f0: M replaced by diag(M) and no steric or external forces (Sec. 3.2.1) */
        or_params P0 = *P;
        P0.FS = 0; P0.grav[0] = P0.grav[1] = P0.grav[2] = 0; P0.fext = NULL; P0.text = NULL;
        or_forces(&P0, Y, q, X, tt, F, T);
        for (int64_t i = 0; i < 3 * S; i++) {
            V[i] = F[i] / (6.0 * PI * P->eta * P->a);
            W[i] = T[i] / (8.0 * PI * P->eta * P->a * P->a * P->a);
        }
    } else {
        or_forces(P, Y, q, X, tt, F, T);
        if (P->mobility)
            P->mobility(P->mob_ctx, S, Y, F, T, V, W);
        else
            or_rpy_apply(S, Y, F, T, P->a, P->eta, V, W, P->nthreads);
    }
    double fmax = 0.0;
    for (int64_t f = 0; f < P->M; f++) {
        int64_t s0 = P->fil_off[f], N = P->fil_off[f + 1] - s0;
        const double* Xf = X + 6 * s0;
        const double* Xj = St->X + 6 * s0;
        double* ff = fout + 6 * s0;
        for (int i = 0; i < 3; i++)
            ff[i] = Y[3 * s0 + i] - a1 * St->Y[3 * s0 + i] - a2 * St->Yprev[3 * s0 + i] - b * P->dt * V[3 * s0 + i];
        for (int64_t n = 0; n < N; n++) {
            double u[3] = {Xf[3 + 3 * n], Xf[4 + 3 * n], Xf[5 + 3 * n]};
            double uj[3] = {Xj[3 + 3 * n], Xj[4 + 3 * n], Xj[5 + 3 * n]}, d[3];
            if (n == 0 && is_clamped(P, f)) { u[0] = u[1] = u[2] = 0; uj[0] = uj[1] = uj[2] = 0; }
            if (n == 0 && is_motor(P, f)) { motor_u(P, u); motor_u(P, uj); }
            or_dexpinv(u, W + 3 * (s0 + n), d);
            for (int i = 0; i < 3; i++) ff[3 + 3 * n + i] = u[i] - g * uj[i] - b * P->dt * d[i];
        }
        for (int64_t n = 1; n < N; n++)
            for (int i = 0; i < 3; i++) {
                int64_t s = s0 + n;
                ff[3 + 3 * N + 3 * (n - 1) + i] =
                    Y[3 * s + i] - a1 * St->Y[3 * s + i] - a2 * St->Yprev[3 * s + i] - b * P->dt * V[3 * s + i];
            }
    }
    for (int64_t i = 0; i < 6 * S; i++) fmax = fmax > fabs(fout[i]) ? fmax : fabs(fout[i]);
    if (Yout) memcpy(Yout, Y, 3 * S * sizeof(double));
    if (qout) memcpy(qout, q, 4 * S * sizeof(double));
    free(Y); free(q); free(F); free(T); free(V); free(W);
    return fmax / P->a;
}

/* Frame-vector approximation of dM_{k+1/2}/du_k (which = 0) or /du_{k+1} (which = 1),
 * Appendix B.2.  Frames of segments k and k+1 are (t0,m0,n0), (t1,m1,n1). */
static void dM_du(const double t0[3], const double m0[3], const double n0[3], const double t1[3],
                  const double m1[3], const double n1[3], const double kap[3], double dL, double KB, double KT,
                  int which, double out[9]) {
    double beta = (dot3(m1, n0) - dot3(m0, n1)) / (2.0 * dL) - kap[0];
    double c1[3], c2[3], gvec[3], ts[3], A[9], B[9], C[9];
    cross3(n0, m1, c1);
    cross3(m0, n1, c2);
    for (int i = 0; i < 3; i++) { gvec[i] = c1[i] - c2[i]; ts[i] = t0[i] + t1[i]; }
    double sgn = which == 0 ? 1.0 : -1.0;
    if (which == 0) { rskew(t1, A); rskew(t0, B); mat_mul(A, B, C); }       /* [x t_{m+1}][x t_m] */
    else { skew(t0, A); rskew(t1, B); mat_mul(A, B, C); }                  /* [t_m x][x t_{m+1}] */
    const double* mu = which == 0 ? m0 : m1;
    const double* nu = which == 0 ? n0 : n1;
    const double* tt = which == 0 ? t0 : t1;
    double Rm[9], Rn[9], Rt[9];
    rskew(mu, Rm); rskew(nu, Rn); rskew(tt, Rt);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            int k = 3 * i + j;
            out[k] = KB * (C[k] / dL - 0.5 * kap[1] * Rm[k] - 0.5 * kap[2] * Rn[k]) +
                     0.5 * KT * (beta * Rt[k] + sgn * ts[i] * gvec[j] / (2.0 * dL));
        }
}

/* Explicit block-diagonal approximate Jacobian J0 of one filament (Sec. 3.2.2,
 * Appendix B.2), evaluated at the configuration (q, Lambda, u) of X.  J is
 * (6N) x (6N) row-major.  cT = b dt/(6 pi eta a), cR = b dt/(8 pi eta a^3).
 * Clamped filaments replace the Y_1, u_1 columns by lambda_1, lambda_2 (reading R11);
 * pinned ones only the Y_1 column, by lambda_1.
 * Reading R12: the torque T_m in the J22 diagonal is the internal torque T^C + T^E. */
void or_j0_filament(const or_params* P, int64_t f, int64_t step, const double* q, const double* X, double tt,
                    double* J) {
    int64_t s0 = P->fil_off[f], N = P->fil_off[f + 1] - s0, n6 = 6 * N;
    int teth = is_tethered(P, f), clamp = is_clamped(P, f);
    double a1, a2, b, g;
    bdf_coeffs(step, &a1, &a2, &b, &g);
    double cT = b * P->dt / (6.0 * PI * P->eta * P->a);
    double cR = b * P->dt / (8.0 * PI * P->eta * P->a * P->a * P->a);
    memset(J, 0, n6 * n6 * sizeof(double));
    const double* Xf = X + 6 * s0;
#define IDX_U(n) (3 + 3 * (n))                 /* u_n, 0-based n */
#define IDX_L(k) (3 + 3 * N + 3 * (k))         /* Lambda_{k+3/2}: joint k between segments k, k+1 */
#define ROW_F3(n) (3 + 3 * N + 3 * ((n) - 1))  /* f^3_n, 0-based n >= 1 */
#define SET(r, c, Mat, s)                                                     \
    for (int _i = 0; _i < 3; _i++)                                            \
        for (int _j = 0; _j < 3; _j++) J[((r) + _i) * n6 + (c) + _j] += (s) * (Mat)[3 * _i + _j];
    double I3[9];
    eye3(I3, 1.0);
    double *t = (double*)malloc(3 * N * sizeof(double)), *mu = (double*)malloc(3 * N * sizeof(double)),
           *nu = (double*)malloc(3 * N * sizeof(double)), *Tm = (double*)calloc(3 * N, sizeof(double)),
           *Fd = (double*)calloc(3 * N, sizeof(double));
    for (int64_t n = 0; n < N; n++) frame(q + 4 * (s0 + n), t + 3 * n, mu + 3 * n, nu + 3 * n);
    double* Lam = (double*)calloc(3 * (N > 1 ? N - 1 : 1), sizeof(double));
    double* kap = (double*)calloc(3 * (N > 1 ? N - 1 : 1), sizeof(double));
    for (int64_t k = 0; k + 1 < N; k++) {
        memcpy(Lam + 3 * k, Xf + IDX_L(k), 3 * sizeof(double));
        joint_kappa(P, f, k, tt, kap + 3 * k);
    }
    or_internal_forces(N, q + 4 * s0, Lam, kap, P->dL, P->KB, P->KT, Fd, Tm);

    /* f^1 row */
    if (teth) { SET(0, 0, I3, -cT); }
    else { SET(0, 0, I3, 1.0); }
    if (N > 1) { SET(0, IDX_L(0), I3, -cT); }
    /* f^3 rows */
    for (int64_t m = 1; m < N; m++) {
        if (!teth) { SET(ROW_F3(m), 0, I3, 1.0); }
        SET(ROW_F3(m), IDX_L(m - 1), I3, cT);
        if (m + 1 < N) { SET(ROW_F3(m), IDX_L(m), I3, -cT); }
        for (int64_t n = 0; n <= m; n++) {
            if (n == 0 && clamp) continue;
            double w = (n == 0 || n == m) ? 1.0 : 2.0;
            double A[9];
            rskew(t + 3 * n, A);
            SET(ROW_F3(m), IDX_U(n), A, 0.5 * P->dL * w);
        }
    }
    /* f^2 rows */
    for (int64_t m = 0; m < N; m++) {
        double um[3] = {Xf[IDX_U(m)], Xf[IDX_U(m) + 1], Xf[IDX_U(m) + 2]};
        if (m == 0 && clamp) { um[0] = um[1] = um[2] = 0; }
        double U[9], U2[9], Tay[9];
        skew(um, U);
        mat_mul(U, U, U2);
        for (int k = 0; k < 9; k++) Tay[k] = I3[k] - 0.5 * U[k] + U2[k] / 12.0;
        int r = IDX_U(m);
        /* Lambda columns: dT_m/dLambda = dL/2 [t_m x] for joints m-1 and m */
        double Tx[9], A[9];
        skew(t + 3 * m, Tx);
        mat_mul(Tay, Tx, A);
        if (m >= 1) { SET(r, IDX_L(m - 1), A, -cR * 0.5 * P->dL); }
        if (m + 1 < N) { SET(r, IDX_L(m), A, -cR * 0.5 * P->dL); }
        /* elastic moment derivatives */
        double dMp_um[9] = {0}, dMp_up[9] = {0}, dMm_um[9] = {0}, dMm_uprev[9] = {0};
        if (m + 1 < N) {
            dM_du(t + 3 * m, mu + 3 * m, nu + 3 * m, t + 3 * (m + 1), mu + 3 * (m + 1), nu + 3 * (m + 1),
                  kap + 3 * m, P->dL, P->KB, P->KT, 0, dMp_um);
            dM_du(t + 3 * m, mu + 3 * m, nu + 3 * m, t + 3 * (m + 1), mu + 3 * (m + 1), nu + 3 * (m + 1),
                  kap + 3 * m, P->dL, P->KB, P->KT, 1, dMp_up);
        }
        if (m >= 1) {
            dM_du(t + 3 * (m - 1), mu + 3 * (m - 1), nu + 3 * (m - 1), t + 3 * m, mu + 3 * m, nu + 3 * m,
                  kap + 3 * (m - 1), P->dL, P->KB, P->KT, 1, dMm_um);
            dM_du(t + 3 * (m - 1), mu + 3 * (m - 1), nu + 3 * (m - 1), t + 3 * m, mu + 3 * m, nu + 3 * m,
                  kap + 3 * (m - 1), P->dL, P->KB, P->KT, 0, dMm_uprev);
        }
        /* off-diagonal u columns */
        if (m + 1 < N) { mat_mul(Tay, dMp_up, A); SET(r, IDX_U(m + 1), A, -cR); }
        if (m >= 1 && !(m == 1 && clamp)) { mat_mul(Tay, dMm_uprev, A); SET(r, IDX_U(m - 1), A, cR); }
        /* diagonal block */
        if (m == 0 && clamp) {
            SET(r, IDX_U(0), I3, -cR); /* lambda_2 column */
        } else {
            double ls[3] = {0, 0, 0};
            if (m + 1 < N) for (int i = 0; i < 3; i++) ls[i] += Lam[3 * m + i];
            if (m >= 1) for (int i = 0; i < 3; i++) ls[i] += Lam[3 * (m - 1) + i];
            double Ls[9], Tt[9], dT[9];
            rskew(ls, Ls);
            rskew(t + 3 * m, Tt);
            mat_mul(Ls, Tt, dT);
            for (int k = 0; k < 9; k++) dT[k] = 0.5 * P->dL * dT[k] + dMp_um[k] - dMm_um[k];
            double Tv[3] = {Tm[3 * m], Tm[3 * m + 1], Tm[3 * m + 2]}, uT[3];
            cross3(um, Tv, uT);
            double XT[9], XuT[9], UdT[9], UXT[9], U2dT[9], B[9];
            rskew(Tv, XT);
            rskew(uT, XuT);
            mat_mul(U, dT, UdT);
            mat_mul(U, XT, UXT);
            mat_mul(U2, dT, U2dT);
            for (int k = 0; k < 9; k++)
                B[k] = I3[k] - cR * (dT[k] - 0.5 * (XT[k] + UdT[k]) + (XuT[k] + UXT[k] + U2dT[k]) / 12.0);
            SET(r, IDX_U(m), B, 1.0);
        }
    }
#undef SET
#undef IDX_U
#undef IDX_L
#undef ROW_F3
    free(t); free(mu); free(nu); free(Tm); free(Fd); free(Lam); free(kap);
}

/* Dense LU with partial pivoting, A = P L U in place (n x n row-major); returns 0 on success */
int or_lu(int64_t n, double* A, int64_t* piv) {
    for (int64_t k = 0; k < n; k++) {
        int64_t p = k;
        double best = fabs(A[k * n + k]);
        for (int64_t i = k + 1; i < n; i++)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return -1;
        if (p != k)
            for (int64_t j = 0; j < n; j++) { double tmp = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = tmp; }
        for (int64_t i = k + 1; i < n; i++) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int64_t j = k + 1; j < n; j++) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}
void or_lu_solve(int64_t n, const double* LU, const int64_t* piv, double* x) {
    for (int64_t k = 0; k < n; k++)
        if (piv[k] != k) { double tmp = x[k]; x[k] = x[piv[k]]; x[piv[k]] = tmp; }
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < i; j++) x[i] -= LU[i * n + j] * x[j];
    for (int64_t i = n - 1; i >= 0; i--) {
        for (int64_t j = i + 1; j < n; j++) x[i] -= LU[i * n + j] * x[j];
        x[i] /= LU[i * n + i];
    }
}

/* Warm start X0 (reading R8): step 0 -> (Y_1^0, 0, 0); step 1 -> (2Y_1^1 - Y_1^0, u^1, Lambda^1);
 * later steps extrapolate Y_1 and the multipliers linearly and reuse u^j. */
void or_initial_guess(const or_params* P, const or_state* St, double* X0) {
    int64_t S = total_segments(P);
    memset(X0, 0, 6 * S * sizeof(double));
    for (int64_t f = 0; f < P->M; f++) {
        int64_t s0 = P->fil_off[f], N = P->fil_off[f + 1] - s0;
        double* x = X0 + 6 * s0;
        const double* xj = St->X + 6 * s0;
        const double* xp = St->Xprev + 6 * s0;
        int teth = is_tethered(P, f);
        if (St->step == 0) {
            if (!teth) memcpy(x, St->Y + 3 * s0, 3 * sizeof(double));
            continue;
        }
        for (int64_t i = 0; i < 6 * N; i++) {
            int is_u = (i >= 3 && i < 3 + 3 * N) && !(is_clamped(P, f) && i < 6);
            if (is_u) x[i] = xj[i];
            else if (i < 3 && !teth) x[i] = 2.0 * St->Y[3 * s0 + i] - St->Yprev[3 * s0 + i];
            else x[i] = (St->step >= 2) ? 2.0 * xj[i] - xp[i] : xj[i];
        }
    }
}

/* Limited-memory bad Broyden with the explicit block-diagonal J0 (Alg. 2, Sec. 3.2.2),
 * solving f(X) = 0 for one step from X (in: warm start, out: solution).  Follows the
 * algorithm as stated: each iteration applies H_k = J0^{-1} + sum_i c_i d_i^T afresh. */
int or_broyden(const or_params* P, const or_state* St, double* X, or_report* rep) {
    int64_t S = total_segments(P), n = 6 * S, K = P->kmax;
    double tt = St->t + P->dt;
    /* J0 at X0, factorised per filament */
    double* Yc = (double*)malloc(3 * S * sizeof(double));
    double* qc = (double*)malloc(4 * S * sizeof(double));
    or_reconstruct(P, St->q, X, St->t + P->dt, Yc, qc);
    double** LU = (double**)malloc(P->M * sizeof(double*));
    int64_t** piv = (int64_t**)malloc(P->M * sizeof(int64_t*));
    int bad = 0;
    for (int64_t f = 0; f < P->M; f++) {
        int64_t N = P->fil_off[f + 1] - P->fil_off[f];
        LU[f] = (double*)malloc(36 * N * N * sizeof(double));
        piv[f] = (int64_t*)malloc(6 * N * sizeof(int64_t));
        or_j0_filament(P, f, St->step, qc, X, tt, LU[f]);
        if (or_lu(6 * N, LU[f], piv[f])) bad = 1;
    }
    double* c = (double*)calloc((K + 1) * n, sizeof(double));
    double* d = (double*)calloc((K + 1) * n, sizeof(double));
    double* fk = (double*)malloc(n * sizeof(double));
    double* fn = (double*)malloc(n * sizeof(double));
    double* dX = (double*)malloc(n * sizeof(double));
    double* h = (double*)malloc(n * sizeof(double));
    int64_t k = 0;
    rep->applies = 1;
    double res = or_residual(P, St, X, fk, NULL, NULL);
    /* h = H_k v */
#define APPLY_H(v, out)                                                                      \
    do {                                                                                     \
        memcpy(out, v, n * sizeof(double));                                                  \
        for (int64_t f_ = 0; f_ < P->M; f_++) {                                              \
            int64_t o_ = 6 * P->fil_off[f_], N_ = P->fil_off[f_ + 1] - P->fil_off[f_];       \
            or_lu_solve(6 * N_, LU[f_], piv[f_], out + o_);                                  \
        }                                                                                    \
        for (int64_t i_ = 0; i_ < k; i_++) {                                                 \
            double s_ = 0;                                                                   \
            for (int64_t j_ = 0; j_ < n; j_++) s_ += d[i_ * n + j_] * v[j_];                 \
            for (int64_t j_ = 0; j_ < n; j_++) out[j_] += c[i_ * n + j_] * s_;               \
        }                                                                                    \
    } while (0)
    while (!bad && res > P->tol && k < K && isfinite(res)) {
        APPLY_H(fk, h);
        for (int64_t j = 0; j < n; j++) { dX[j] = -h[j]; X[j] += dX[j]; }
        double resn = or_residual(P, St, X, fn, NULL, NULL);
        rep->applies++;
        double nrm = 0;
        for (int64_t j = 0; j < n; j++) { double df = fn[j] - fk[j]; nrm += df * df; }
        nrm = sqrt(nrm);
        APPLY_H(fn, h);
        for (int64_t j = 0; j < n; j++) {
            c[k * n + j] = -h[j] / nrm;
            d[k * n + j] = (fn[j] - fk[j]) / nrm;
        }
        k++;
        memcpy(fk, fn, n * sizeof(double));
        res = resn;
    }
#undef APPLY_H
    rep->iters = k;
    rep->resid = res;
    rep->converged = (!bad && res <= P->tol) ? 1 : 0;
    for (int64_t f = 0; f < P->M; f++) { free(LU[f]); free(piv[f]); }
    free(LU); free(piv); free(c); free(d); free(fk); free(fn); free(dX); free(h); free(Yc); free(qc);
    return rep->converged ? 0 : -3;
}

/* One implicit step (Sec. 2.9.3): warm start, Broyden solve, then the multiplicative
 * update q^{j+1} = exp(u^{j+1}) . q^j, robot-arm positions and the history shift. */
int or_bdf2_step(const or_params* P, or_state* St, or_report* rep) {
    int64_t S = total_segments(P);
    double* X = (double*)malloc(6 * S * sizeof(double));
    or_initial_guess(P, St, X);
    int rc = or_broyden(P, St, X, rep);
    if (rc == 0) {
        double* Yn = (double*)malloc(3 * S * sizeof(double));
        double* qn = (double*)malloc(4 * S * sizeof(double));
        or_reconstruct(P, St->q, X, St->t + P->dt, Yn, qn);
        memcpy(St->Yprev, St->Y, 3 * S * sizeof(double));
        memcpy(St->Y, Yn, 3 * S * sizeof(double));
        memcpy(St->q, qn, 4 * S * sizeof(double));
        memcpy(St->Xprev, St->X, 6 * S * sizeof(double));
        memcpy(St->X, X, 6 * S * sizeof(double));
        St->t += P->dt;
        St->step += 1;
        free(Yn); free(qn);
    }
    free(X);
    return rc;
}
