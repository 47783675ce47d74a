// Device kernels of the implicit step (Sec. 2.9.3 system, Alg. 2 bad Broyden,
// Sec. 3.2.2 / Appendix B.2 explicit J0) of arXiv:1903.12609.
//
// Vector layouts: positions, forces, velocities are component-major [3][S];
// quaternions [4][S]; the unknown / residual vectors are filament-major
// [6S] with filament f's block [Y_1 | u_1..u_N | Lambda_{3/2}..Lambda_{N-1/2}]
// at 6*seg_off[f].  Every segment owns exactly six residual rows:
// segment 0 of a filament owns f^1 and f^2_1, segment n >= 1 owns f^2_n, f^3_n.
#include "common.h"
#include "kernels.h"
#include "quat.h"
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "solver.h"

namespace fil {

__device__ __forceinline__ V3 ld3(const double* __restrict__ v, int64_t ld, int64_t i) {
    return v3(v[i], v[ld + i], v[2 * ld + i]);
}
__device__ __forceinline__ void st3(double* __restrict__ v, int64_t ld, int64_t i, V3 x) {
    v[i] = x.x;
    v[ld + i] = x.y;
    v[2 * ld + i] = x.z;
}
__device__ __forceinline__ V3 ldx(const double* __restrict__ X, int64_t i) { return v3(X[i], X[i + 1], X[i + 2]); }
__device__ __forceinline__ Q4 ldq(const double* __restrict__ q, int64_t S, int64_t s) {
    return Q4{q[s], q[S + s], q[2 * S + s], q[3 * S + s]};
}
__device__ __forceinline__ void stq(double* __restrict__ q, int64_t S, int64_t s, Q4 x) {
    q[s] = x.w;
    q[S + s] = x.x;
    q[2 * S + s] = x.y;
    q[3 * S + s] = x.z;
}

// lane l receives lane l+1's value, lane 63 zero: a DPP shift of the whole wave
// by one lane (VALU only, no LDS round trip)
__device__ __forceinline__ double wave_next_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// wave-uniform lane read of a double (the lane index must be uniform)
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int l) {
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

// DPP lane moves inside each row of 16 lanes (VALU only, no LDS round trip); a lane
// whose source falls outside its row receives zero.  Every lane of the wave must be
// active.
enum : int {
    kDppQuadSwap1 = 0xb1,  // quad permutation [1,0,3,2]
    kDppQuadSwap2 = 0x4e,  // quad permutation [2,3,0,1]
    kDppHalfMirror = 0x141,
    kDppRowMirror = 0x140,
    kDppRowShr = 0x110,  // + shift (1..15)
    kDppRowBcast = 0x150,  // + lane (0..15): every lane of a row receives that lane of its row
};
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
// one 64-bit DPP move (the row broadcast is the one control 64-bit DPP takes)
template <int CTRL>
__device__ __forceinline__ double dpp64_f64(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const unsigned lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xf, 0xf, true);
    const unsigned hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xf, 0xf, true);
    return ((unsigned long long)hi << 32) | lo;
}

// op over each row of 16 lanes, left in every lane of the row: pairs, quads, half rows,
// rows.  Each step combines a lane with its partner symmetrically, so for a commutative
// op every lane of a row holds the same bits.
template <typename Op>
__device__ __forceinline__ double row_allreduce_f64(double v, Op op) {
    v = op(v, dpp_f64<kDppQuadSwap1>(v));
    v = op(v, dpp_f64<kDppQuadSwap2>(v));
    v = op(v, dpp_f64<kDppHalfMirror>(v));
    return op(v, dpp_f64<kDppRowMirror>(v));
}
template <typename Op>
__device__ __forceinline__ unsigned long long row_allreduce_u64(unsigned long long v, Op op) {
    v = op(v, dpp_u64<kDppQuadSwap1>(v));
    v = op(v, dpp_u64<kDppQuadSwap2>(v));
    v = op(v, dpp_u64<kDppHalfMirror>(v));
    return op(v, dpp_u64<kDppRowMirror>(v));
}

// sum over the wave in a fixed order (rows, then (r0 + r1) + (r2 + r3)); uniform result
__device__ __forceinline__ double wave_sum(double v) {
    v = row_allreduce_f64(v, [](double a, double b) { return a + b; });
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// maximum over the wave of unsigned 64-bit values; uniform result
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    auto mx = [](unsigned long long a, unsigned long long b) { return a > b ? a : b; };
    v = row_allreduce_u64(v, mx);
    return mx(mx(readlane_u64(v, 0), readlane_u64(v, 16)), mx(readlane_u64(v, 32), readlane_u64(v, 48)));
}

// inclusive prefix sum over the wave: shifts by 1, 2, 4, 8 inside each row, then each
// row adds the totals of the rows before it
__device__ __forceinline__ double wave_inclusive_sum(double v, int lane) {
    v += dpp_f64<kDppRowShr + 1>(v);
    v += dpp_f64<kDppRowShr + 2>(v);
    v += dpp_f64<kDppRowShr + 4>(v);
    v += dpp_f64<kDppRowShr + 8>(v);
    const double t0 = readlane_f64(v, 15), t1 = readlane_f64(v, 31), t2 = readlane_f64(v, 47);
    const int row = lane >> 4;
    const double t01 = t0 + t1;
    const double carry = row == 0 ? 0.0 : row == 1 ? t0 : row == 2 ? t01 : t01 + t2;
    return row == 0 ? v : v + carry;
}

// preferred curvature of joint k (between local segments k and k+1) at time tt,
// evaluated at s = (k+1) dL
__device__ __forceinline__ V3 joint_kappa(const SimDev& d, int64_t f, int64_t k, double tt) {
    if (!d.phase) return v3(0, 0, 0);
    return v3(0, 0, d.K0 * sin(d.kw * (double)(k + 1) * d.dL - d.omega * tt + d.phase[f]));
}

// ---------------------------------------------------------------- state + forces
// Filament f's configuration from its unknowns Xf (global memory or LDS):
// q_n = exp(u_n) q^j_n, t_n, robot-arm positions Y_n = Y_1 + dL/2 sum_{m<n} (t_m + t_{m+1})
// and the filament's bounding box, then F = F^C + gravity (+ external) (+ lambda_1),
// T = T^C + T^E (+ lambda_2).  Every thread of the workgroup calls it (it holds a
// barrier); lane n of the first wave owns segment n (N <= 64) and passes q^j_n (read
// by the caller, possibly well before).  Nothing may follow it in the caller that
// needs a barrier.
// the rotating motor of a tether-3 base (Sec. 5.2.1): the prescribed rotation per step
// u_1 = (0, 0, omega dt) and the base on its circle at time tt
__device__ __forceinline__ V3 motor_u(const SimDev& d, int64_t f) {
    return v3(0.0, 0.0, d.motor_w * d.spar[kSpar * d.fil_susp[f]]);
}
__device__ __forceinline__ V3 motor_base(const SimDev& d, int64_t f, double tt) {
    double s, c;
    sincos(d.motor_w * tt, &s, &c);
    return v3(d.base[3 * f] - d.motor_d0 + d.motor_d0 * c, d.base[3 * f + 1] + d.motor_d0 * s, d.base[3 * f + 2]);
}

__device__ void filament_state(const SimDev& d, int64_t f, const double* Xf, Q4 qjn, double tt,
                               double* __restrict__ Yc, double* __restrict__ qc, double* __restrict__ F,
                               double* __restrict__ T, double* __restrict__ box) {
    const int64_t S = d.S;
    const int64_t s0 = d.seg_off[f];
    const int N = (int)(d.seg_off[f + 1] - s0);
    const int teth = d.tether[f];
    __shared__ double sq[kMaxSeg][4];
    __shared__ double st[kMaxSeg][3];
    const int n = threadIdx.x;
    const bool seg = n < N;
    if (seg) {
        V3 u = ldx(Xf, 3 + 3 * n);
        if (teth == 1 && n == 0) u = v3(0, 0, 0);  // clamped base: u_1 = 0
        if (teth == 3 && n == 0) u = motor_u(d, f);  // base turned by the motor
        const Q4 q = qmul(qexp(u), qjn);
        stq(qc, S, s0 + n, q);
        sq[n][0] = q.w; sq[n][1] = q.x; sq[n][2] = q.y; sq[n][3] = q.z;
        const V3 t = frame_t(q);
        st[n][0] = t.x; st[n][1] = t.y; st[n][2] = t.z;
    }
    __syncthreads();
    if (n >= 64) return;
    {
        // wave prefix sum of the half-segment steps, then the bounding box
        double e[3];
        if (n == 0) {
            const V3 y1 = teth == 3 ? motor_base(d, f, tt)
                          : teth ? v3(d.base[3 * f], d.base[3 * f + 1], d.base[3 * f + 2]) : ldx(Xf, 0);
            e[0] = y1.x;
            e[1] = y1.y;
            e[2] = y1.z;
        } else {
            for (int i = 0; i < 3; i++) e[i] = seg ? (0.5 * d.dL) * (st[n - 1][i] + st[n][i]) : 0.0;
        }
        for (int i = 0; i < 3; i++) e[i] = wave_inclusive_sum(e[i], n);
        if (seg) st3(Yc, S, s0 + n, v3(e[0], e[1], e[2]));
        double lo[3], hi[3];
        for (int i = 0; i < 3; i++) {
            const double y = seg ? e[i] : readlane_f64(e[i], 0);
            lo[i] = row_allreduce_f64(y, [](double a, double b) { return fmin(a, b); });
            hi[i] = row_allreduce_f64(y, [](double a, double b) { return fmax(a, b); });
            lo[i] = fmin(fmin(readlane_f64(lo[i], 0), readlane_f64(lo[i], 16)),
                         fmin(readlane_f64(lo[i], 32), readlane_f64(lo[i], 48)));
            hi[i] = fmax(fmax(readlane_f64(hi[i], 0), readlane_f64(hi[i], 16)),
                         fmax(readlane_f64(hi[i], 32), readlane_f64(hi[i], 48)));
        }
        if (n == 0) {
            double* b = box + 6 * f;
            for (int i = 0; i < 3; i++) {
                b[i] = lo[i];
                b[3 + i] = hi[i];
            }
        }
    }
    if (!seg) return;
    const Q4 qn{sq[n][0], sq[n][1], sq[n][2], sq[n][3]};
    V3 lp = v3(0, 0, 0), lm = v3(0, 0, 0), mp = v3(0, 0, 0), mm = v3(0, 0, 0);
    if (n + 1 < N) {
        lp = ldx(Xf, 3 + 3 * N + 3 * n);
        mp = joint_moment(qn, Q4{sq[n + 1][0], sq[n + 1][1], sq[n + 1][2], sq[n + 1][3]}, joint_kappa(d, f, n, tt),
                          d.dL, d.KB, d.KT);
    }
    if (n > 0) {
        lm = ldx(Xf, 3 + 3 * N + 3 * (n - 1));
        mm = joint_moment(Q4{sq[n - 1][0], sq[n - 1][1], sq[n - 1][2], sq[n - 1][3]}, qn,
                          joint_kappa(d, f, n - 1, tt), d.dL, d.KB, d.KT);
    }
    const double* sp = d.spar + kSpar * d.fil_susp[f];
    V3 fc = lp - lm + v3(sp[1], sp[2], sp[3]);
    if (d.fext) fc = fc + ld3(d.fext, S, s0 + n);
    V3 tc = (0.5 * d.dL) * cross(v3(st[n][0], st[n][1], st[n][2]), lp + lm) + (mp - mm);
    if (d.text) tc = tc + ld3(d.text, S, s0 + n);
    if (teth && n == 0) {
        fc = fc + ldx(Xf, 0);                   // lambda_1 of a held base
        if (teth == 1) tc = tc + ldx(Xf, 3);    // lambda_2 of a clamped one
        if (teth == 3) {                        // D^T lambda_2 on the motor's base, D = dexpinv_{u_1}
            const V3 um = motor_u(d, f), l2 = ldx(Xf, 3);
            tc = tc + dexpinv(um, l2) + cross(um, l2);
        }
    }
    st3(F, S, s0 + n, fc);
    st3(T, S, s0 + n, tc);
}

// one 64-lane workgroup per filament
__global__ void __launch_bounds__(64) state_forces_kernel(SimDev d, const double* __restrict__ X,
                                                        const double* __restrict__ qj, const double* __restrict__ ttp,
                                                        const int32_t* __restrict__ active,
                                                        double* __restrict__ Yc, double* __restrict__ qc,
                                                        double* __restrict__ F, double* __restrict__ T,
                                                        double* __restrict__ box) {
    const int64_t f = blockIdx.x;
    if (!active[d.fil_susp[f]]) return;
    const int64_t s0 = d.seg_off[f];
    const int N = (int)(d.seg_off[f + 1] - s0);
    const Q4 qjn = threadIdx.x < N ? ldq(qj, d.S, s0 + threadIdx.x) : Q4{1.0, 0.0, 0.0, 0.0};
    // t^{j+1} is read on the device so that captured launches stay valid
    filament_state(d, f, X + 6 * s0, qjn, *ttp, Yc, qc, F, T, box);
}

int state_forces_launch(const SimDev& d, const double* X, const double* qj, const double* tt, const int32_t* active,
                        double* Yc, double* qc, double* F, double* T, double* box, hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    state_forces_kernel<<<(unsigned)d.M, 64, 0, st>>>(d, X, qj, tt, active, Yc, qc, F, T, box);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// ---------------------------------------------------------------- steric barrier
// F^B_n = sum_m F^S ((4a^2 chi^2 - r^2)/(4a^2 (chi^2-1)))^4 r_nm/(2a) for r < 2 chi a,
// excluding m = n and same-filament neighbours (Sec. 2.6).  The block of target
// filament f tests the bounding boxes of its suspension's filaments 64 at a time
// (one per lane), then walks the segments of every filament within the cutoff
// with wave-uniform (scalar) loads.  It finishes the force F^H = F^C + F^B +
// gravity and writes the mobility source record of each of its segments.  In a
// periodic box r_nm is the nearest image (the cutoff is below half of every box
// length) and two filaments are near when their box centres, nearest image apart,
// are closer than the half-widths plus the cutoff along every axis; that never
// misses a pair of segments within the cutoff.
// r - L round(r / L): the nearest periodic image of a separation
__device__ __forceinline__ double nearest_image(double r, double L) { return r - L * rint(r / L); }

// gap along one axis between the intervals [lo_a, hi_a] and [lo_b, hi_b] of a periodic
// axis of length L: the nearest-image distance of the centres less both half-widths
__device__ __forceinline__ double box_gap_periodic(double lo_a, double hi_a, double lo_b, double hi_b, double L) {
    const double dc = nearest_image(0.5 * (lo_b + hi_b) - 0.5 * (lo_a + hi_a), L);
    return fmax(0.0, fabs(dc) - 0.5 * (hi_a - lo_a) - 0.5 * (hi_b - lo_b));
}

__global__ void __launch_bounds__(64 * kStericWaves) steric_pack_kernel(SimDev d, const double* __restrict__ Yc,
                                                       const double* __restrict__ box,
                                                       const int32_t* __restrict__ active, double* __restrict__ F,
                                                       const double* __restrict__ T, int prec, void* __restrict__ pk) {
    const int64_t f = blockIdx.x;
    const int32_t isus = d.fil_susp[f];
    if (!active[isus]) return;
    const int64_t S = d.S;
    const int64_t s0 = d.seg_off[f], N = d.seg_off[f + 1] - s0;
    const int lane = threadIdx.x & 63;  // N <= 64
    const int wave = threadIdx.x >> 6;   // the waves split each neighbour's segments
    const bool valid = lane < N;
    const int64_t sn = s0 + (valid ? lane : N - 1);
    const double y0 = Yc[sn], y1 = Yc[S + sn], y2 = Yc[2 * S + sn];
    // the forces and torques for the source record are read now, used at the end
    double Fp[3] = {0.0, 0.0, 0.0}, Tp[3] = {0.0, 0.0, 0.0};
    if (wave == 0)
        for (int i = 0; i < 3; i++) {
            Fp[i] = F[i * S + sn];
            Tp[i] = T[i * S + sn];
        }
    double fx = 0, fy = 0, fz = 0;
    const double FS = d.spar[kSpar * isus + 4];
    if (FS != 0.0) {
        const double rc = 2.0 * d.chi * d.a, rc2 = rc * rc;
        const double k4 = 4.0 * d.a * d.a * d.chi * d.chi, kden = 1.0 / (4.0 * d.a * d.a * (d.chi * d.chi - 1.0));
        const double fscale = FS / (2.0 * d.a);
        const double* bf = box + 6 * f;
        const double lo0 = bf[0], lo1 = bf[1], lo2 = bf[2], hi0 = bf[3], hi1 = bf[4], hi2 = bf[5];
        const int64_t g0 = d.susp_fil_off[isus], g1 = d.susp_fil_off[isus + 1];
        for (int64_t gb = g0; gb < g1; gb += 64) {
            bool near = false;
            const int64_t g = gb + lane;
            if (g < g1) {
                const double* bx = box + 6 * g;
                double gx, gy, gz;
                if (!d.periodic) {
                    gx = fmax(0.0, fmax(bx[0] - hi0, lo0 - bx[3]));
                    gy = fmax(0.0, fmax(bx[1] - hi1, lo1 - bx[4]));
                    gz = fmax(0.0, fmax(bx[2] - hi2, lo2 - bx[5]));
                } else {
                    gx = box_gap_periodic(lo0, hi0, bx[0], bx[3], d.per[0]);
                    gy = box_gap_periodic(lo1, hi1, bx[1], bx[4], d.per[1]);
                    gz = box_gap_periodic(lo2, hi2, bx[2], bx[5], d.per[2]);
                }
                near = gx * gx + gy * gy + gz * gz < rc2;
            }
            unsigned long long mask = __ballot(near);
            // one coalesced load of a near filament's positions, then lane broadcasts;
            // the next near filament's load is issued before the current one is used
            auto load_pos = [&](unsigned long long msk, double& q0, double& q1, double& q2) {
                const int64_t g2 = gb + (__ffsll((long long)msk) - 1);
                const int64_t a0 = d.seg_off[g2];
                const int nn = (int)(d.seg_off[g2 + 1] - a0);
                const int64_t ml = a0 + (lane < nn ? lane : 0);
                q0 = Yc[ml];
                q1 = Yc[S + ml];
                q2 = Yc[2 * S + ml];
            };
            double p0 = 0.0, p1 = 0.0, p2 = 0.0;
            if (mask) load_pos(mask, p0, p1, p2);
            while (mask) {
                const int l = __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                double n0 = 0.0, n1 = 0.0, n2 = 0.0;
                if (mask) load_pos(mask, n0, n1, n2);
                const int64_t gg = gb + l;
                const int64_t m0 = d.seg_off[gg];
                const int ng = (int)(d.seg_off[gg + 1] - m0);  // <= 64
                for (int q = wave; q < ng; q += kStericWaves) {
                    const int64_t m = m0 + q;
                    double rx = y0 - readlane_f64(p0, q), ry = y1 - readlane_f64(p1, q),
                           rz = y2 - readlane_f64(p2, q);
                    if (d.periodic) {
                        rx = nearest_image(rx, d.per[0]);
                        ry = nearest_image(ry, d.per[1]);
                        rz = nearest_image(rz, d.per[2]);
                    }
                    const double r2 = rx * rx + ry * ry + rz * rz;
                    const bool excluded = m == sn || (gg == f && (m == sn + 1 || m + 1 == sn));
                    if (r2 < rc2 && !excluded) {
                        const double bb = (k4 - r2) * kden;
                        const double b2 = bb * bb;
                        const double sc = fscale * b2 * b2;
                        fx += sc * rx;
                        fy += sc * ry;
                        fz += sc * rz;
                    }
                }
                p0 = n0;
                p1 = n1;
                p2 = n2;
            }
        }
    }
    // fixed-order combination of the waves' partial forces
    __shared__ double red[kStericWaves][3][64];
    red[wave][0][lane] = fx;
    red[wave][1][lane] = fy;
    red[wave][2][lane] = fz;
    __syncthreads();
    if (wave != 0 || !valid) return;
    fx = red[0][0][lane];
    fy = red[0][1][lane];
    fz = red[0][2][lane];
    for (int w = 1; w < kStericWaves; w++) {
        fx += red[w][0][lane];
        fy += red[w][1][lane];
        fz += red[w][2][lane];
    }
    fx += Fp[0];
    fy += Fp[1];
    fz += Fp[2];
    F[sn] = fx;
    F[S + sn] = fy;
    F[2 * S + sn] = fz;
    // FP64 source records here; the FP32-tile records need the tile origins and are written
    // by the mobility launch itself
    if (prec == FIL_PREC_F64) rpy_pack_record_f64(static_cast<double*>(pk), sn, y0, y1, y2, fx, fy, fz, Tp[0], Tp[1], Tp[2]);
}

int steric_pack_launch(const SimDev& d, const double* Yc, const double* box, const int32_t* active, double* F,
                       const double* T, int prec, void* pk, hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    steric_pack_kernel<<<(unsigned)d.M, 64 * kStericWaves, 0, st>>>(d, Yc, box, active, F, T, prec, pk);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// ---------------------------------------------------------------- geometric switch
// Geometric-switch driving torque of model cilia (Sec. 5.2.2): a torque about a fixed axis
// drives the base of every pinned filament until the angle theta between the wall normal
// and the base tangent (signed about the axis) reaches +theta_max or -theta_max, where
// the drive reverses, its magnitude switching between tau_pos (driving towards
// +theta_max) and tau_neg (towards -theta_max).  For the stability of the implicit
// steps the torque passes from the old value to the new one along a logistic curve over
// n_tr steps.  The switch is decided once per step from the committed configuration.
__device__ __forceinline__ double switch_torque(const SwitchArgs& a, int dir, int age, double tau0) {
    const double tau1 = dir > 0 ? a.tau_pos : -a.tau_neg;
    if (age >= a.n_tr) return tau1;
    const double x = (double)age / (double)a.n_tr - 0.5;
    const double sg = 1.0 / (1.0 + exp(-12.0 * x));
    return tau0 + (tau1 - tau0) * sg;
}

// one thread per filament
__global__ void __launch_bounds__(64) switch_torque_kernel(SimDev d, SwitchArgs a, const double* __restrict__ qj,
                                                           double* __restrict__ text) {
    const int64_t f = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (f >= d.M) return;
    const int64_t S = d.S, s0 = d.seg_off[f], N = d.seg_off[f + 1] - s0;
    for (int64_t n = 0; n < N; n++)
        for (int c = 0; c < 3; c++) text[c * S + s0 + n] = 0.0;
    if (d.tether[f] != 2) return;
    const Q4 q = ldq(qj, S, s0);
    const V3 t = frame_t(q);
    const V3 nrm = v3(a.normal[0], a.normal[1], a.normal[2]), ax = v3(a.axis[0], a.axis[1], a.axis[2]);
    const double theta = atan2(dot(cross(nrm, t), ax), dot(nrm, t));
    int dir = a.dir[f], age = a.age[f];
    double tau0 = a.tau0[f];
    if (dir * theta >= a.theta_max) {
        tau0 = switch_torque(a, dir, age, tau0);
        dir = -dir;
        age = 0;
    } else if (age < a.n_tr) {
        age++;
    }
    const double tau = switch_torque(a, dir, age, tau0);
    for (int c = 0; c < 3; c++) text[c * S + s0] = tau * a.axis[c];
    a.dir[f] = dir;
    a.age[f] = age;
    a.tau0[f] = tau0;
}

int switch_torque_launch(const SimDev& d, const SwitchArgs& a, const double* qj, double* text, hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    switch_torque_kernel<<<(unsigned)ceil_div(d.M, (int64_t)64), 64, 0, st>>>(d, a, qj, text);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}


// ---------------------------------------------------------------- residual
// f^1 = Y_1 - a1 Y_1^j - a2 Y_1^{j-1} - b dt V_1
// f^2_n = u_n - g u_n^j - b dt dexpinv_{u_n}(Omega_n)
// f^3_n = Y_n - a1 Y_n^j - a2 Y_n^{j-1} - b dt V_n
// One workgroup per filament.  Per suspension it also records max|f| and
// max|b dt (V, dexpinv Omega)| (the size of the mobility term, which sets the
// rounding floor of a reduced-precision apply), each as the bit pattern of a
// non-negative double so that an integer atomicMax orders it (a NaN compares above
// every finite value).  When the velocities come from the mobility partials they
// are also stored to V, W.  For a Broyden update it leaves the filament's share of
// the update's dot products.

// Filament f's share of the dot products of Broyden update k (Alg. 2), its rows of
// f in LDS: h < k: d_h . f;  h = k: |f - fprev|^2;  h = k+1: (f - fprev) . f.
// Dot h is reduced by wave h mod (NT / 64) in a fixed order, two dots per pass.
template <int NT>
__device__ void filament_dots(const SimDev& d, int64_t f, const DotArgs& da, const double* sf, int nrow) {
    constexpr int NW = NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t e0 = 6 * d.seg_off[f], n6 = 6 * d.S;
    const int nd = da.k + 2;
    auto term = [&](int h, int e, double fn) {
        if (h < da.k) return da.Dhist[(int64_t)h * n6 + e0 + e] * fn;
        const double df = fn - da.fprev[e0 + e];
        return df * (h == da.k ? df : fn);
    };
    for (int h0 = wave; h0 < nd; h0 += 2 * NW) {
        const int h1 = h0 + NW;
        double a0 = 0.0, a1 = 0.0;
        for (int e = lane; e < nrow; e += 64) {
            const double fn = sf[e];
            a0 += term(h0, e, fn);
            if (h1 < nd) a1 += term(h1, e, fn);
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        if (lane == 0) {
            da.dpart[f * d.max_dots + h0] = a0;
            if (h1 < nd) da.dpart[f * d.max_dots + h1] = a1;
        }
    }
}

// Up to kSplit threads share one sum (over mobility partials, inverse columns or
// history vectors) so that each has few loads in flight; partial sums are combined
// in a fixed order.
constexpr int kSplit = 8;
constexpr int lds_rows(int nt) { return nt > 6 * kMaxSeg ? nt : 6 * kMaxSeg; }

template <int NT>
__global__ void __launch_bounds__(NT) residual_kernel(SimDev d, BdfCoef bc, const double* __restrict__ X,
                                                    const double* __restrict__ Xj, const double* __restrict__ Yc,
                                                    const double* __restrict__ Yj, const double* __restrict__ Yjm1,
                                                    double* __restrict__ V, double* __restrict__ W,
                                                    const double* __restrict__ part, int K,
                                                    const int32_t* __restrict__ active, double* __restrict__ fout,
                                                    unsigned long long* __restrict__ resbits,
                                                    unsigned long long* __restrict__ resbits_next, DotArgs da) {
    const int64_t S = d.S;
    // the other buffer is zeroed for the next evaluation (its last reader has run)
    if (blockIdx.x == 0)
        for (int64_t i = threadIdx.x; i < 2 * d.nsusp; i += blockDim.x) resbits_next[i] = 0ull;
    const int64_t f = blockIdx.x;
    const int32_t isus = d.fil_susp[f];
    if (!active[isus]) return;
    const int64_t s0 = d.seg_off[f];
    const int N = (int)(d.seg_off[f + 1] - s0);
    const int ni = 6 * N;  // items (c, l): velocity component c of segment l
    __shared__ double sv[6][kMaxSeg];
    __shared__ double sf[6 * kMaxSeg];
    __shared__ double red[lds_rows(NT)];
    // read ahead: the residual inputs of the first wave's segment, and each wave's
    // terms of its first two dot products for the first 128 rows
    const int n = threadIdx.x;
    const bool seg = n < N;
    const int teth = d.tether[f];
    V3 ycur = v3(0, 0, 0), yold = v3(0, 0, 0), yold2 = v3(0, 0, 0), uu = v3(0, 0, 0), uj = v3(0, 0, 0);
    if (seg) {
        const int64_t s = s0 + n;
        ycur = ld3(Yc, S, s);
        yold = ld3(Yj, S, s);
        yold2 = ld3(Yjm1, S, s);
        uu = ldx(X + 6 * s0, 3 + 3 * n);
        uj = ldx(Xj + 6 * s0, 3 + 3 * n);
    }
    constexpr int NW = NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t e0 = 6 * s0, n6 = 6 * S;
    const int nd = da.k + 2;
    const int h0 = wave, h1 = wave + NW;
    const bool dpre = NT >= 1024 && da.k >= 0 && ni <= 128;  // uniform (1024-thread form only)
    double dt0[2] = {0.0, 0.0}, dt1[2] = {0.0, 0.0}, fpv[2] = {0.0, 0.0};
    if (dpre) {
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const int e = min(lane + 64 * r, ni - 1);  // clamped; rows past ni are not used
            fpv[r] = da.fprev[e0 + e];
            if (h0 < da.k) dt0[r] = da.Dhist[(int64_t)h0 * n6 + e0 + e];
            if (h1 < da.k) dt1[r] = da.Dhist[(int64_t)h1 * n6 + e0 + e];
        }
    }
    if (part) {
        // R threads per item, thread q summing partials q, q + R, ...
        const int R = max(1, min(kSplit, NT / ni));
        const int64_t stride = 6 * S;
        for (int e = threadIdx.x; e < R * ni; e += NT) {
            const int q = e / ni, item = e - q * ni;
            const int c = item / N, l = item - c * N;
            const double* pp = part + (int64_t)c * S + s0 + l;
            double a0 = 0.0, a1 = 0.0;
            int k = q;
            for (; k + R < K; k += 2 * R) {
                a0 += pp[(int64_t)k * stride];
                a1 += pp[(int64_t)(k + R) * stride];
            }
            if (k < K) a0 += pp[(int64_t)k * stride];
            red[e] = a0 + a1;
        }
        __syncthreads();
        for (int item = threadIdx.x; item < ni; item += NT) {
            double v = red[item];
            for (int q = 1; q < R; q++) v += red[q * ni + item];
            const int c = item / N, l = item - c * N;
            const int64_t s = s0 + l;
            if (c < 3) V[c * S + s] = v;
            else W[(c - 3) * S + s] = v;
            sv[c][l] = v;
        }
    } else {
        for (int item = threadIdx.x; item < ni; item += NT) {
            const int c = item / N, l = item - c * N;
            const int64_t s = s0 + l;
            sv[c][l] = c < 3 ? V[c * S + s] : W[(c - 3) * S + s];
        }
    }
    __syncthreads();
    if (n < 64) {
        double amax = 0.0, vmax = 0.0;
        if (seg) {
            const double bdt = bc.b * d.spar[kSpar * isus];
            double* ff = fout + 6 * s0;
            const V3 vel = v3(sv[0][n], sv[1][n], sv[2][n]);
            const V3 om = v3(sv[3][n], sv[4][n], sv[5][n]);
            const V3 yres = ycur - bc.a1 * yold - bc.a2 * yold2 - bdt * vel;
            V3 u = uu;
            if (teth == 1 && n == 0) u = uj = v3(0, 0, 0);
            if (teth == 3 && n == 0) u = uj = motor_u(d, f);
            const V3 dom = dexpinv(u, om);
            const V3 ures = u - bc.g * uj - bdt * dom;
            vmax = fabs(bdt) * fmax(fmax(fmax(fabs(vel.x), fabs(vel.y)), fmax(fabs(vel.z), fabs(dom.x))),
                                    fmax(fabs(dom.y), fabs(dom.z)));
            const int ry = n == 0 ? 0 : 3 + 3 * N + 3 * (n - 1);
            ff[ry] = sf[ry] = yres.x;
            ff[ry + 1] = sf[ry + 1] = yres.y;
            ff[ry + 2] = sf[ry + 2] = yres.z;
            ff[3 + 3 * n] = sf[3 + 3 * n] = ures.x;
            ff[4 + 3 * n] = sf[4 + 3 * n] = ures.y;
            ff[5 + 3 * n] = sf[5 + 3 * n] = ures.z;
            amax = fmax(fmax(fmax(fabs(yres.x), fabs(yres.y)), fmax(fabs(yres.z), fabs(ures.x))),
                        fmax(fabs(ures.y), fabs(ures.z)));
            if (!(yres.x == yres.x && yres.y == yres.y && yres.z == yres.z && ures.x == ures.x &&
                  ures.y == ures.y && ures.z == ures.z))
                amax = __longlong_as_double(0x7ff8000000000000ll);
        }
        // the workgroup belongs to one suspension: wave maxima, one atomic each (results
        // unused, so the workgroup does not wait for them)
        const unsigned long long ma = wave_max_u64((unsigned long long)__double_as_longlong(amax));
        const unsigned long long mv = wave_max_u64((unsigned long long)__double_as_longlong(vmax));
        if (n == 0) {
            atomicMax(&resbits[isus], ma);
            atomicMax(&resbits[d.nsusp + isus], mv);
        }
    }
    if (da.k < 0) return;
    __syncthreads();
    if (!dpre) {
        filament_dots<NT>(d, f, da, sf, ni);
        return;
    }
    // the first pass from the terms read ahead (ni <= 128: two rows per lane), then any
    // further dots as in filament_dots
    auto term = [&](int h, int r, double dterm) {
        const int e = lane + 64 * r;
        if (e >= ni) return 0.0;
        const double fn = sf[e];
        if (h < da.k) return dterm * fn;
        const double df = fn - fpv[r];
        return df * (h == da.k ? df : fn);
    };
    if (h0 < nd) {
        double a0 = term(h0, 0, dt0[0]) + term(h0, 1, dt0[1]);
        double a1 = h1 < nd ? term(h1, 0, dt1[0]) + term(h1, 1, dt1[1]) : 0.0;
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        if (lane == 0) {
            da.dpart[f * d.max_dots + h0] = a0;
            if (h1 < nd) da.dpart[f * d.max_dots + h1] = a1;
        }
    }
    for (int g0 = wave + 2 * NW; g0 < nd; g0 += 2 * NW) {
        const int g1 = g0 + NW;
        double a0 = 0.0, a1 = 0.0;
        for (int r = 0; r < 2; r++) {
            const int e = lane + 64 * r;
            if (e >= ni) continue;
            a0 += term(g0, r, g0 < da.k ? da.Dhist[(int64_t)g0 * n6 + e0 + e] : 0.0);
            if (g1 < nd) a1 += term(g1, r, g1 < da.k ? da.Dhist[(int64_t)g1 * n6 + e0 + e] : 0.0);
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        if (lane == 0) {
            da.dpart[f * d.max_dots + g0] = a0;
            if (g1 < nd) da.dpart[f * d.max_dots + g1] = a1;
        }
    }
}

// workgroup size of the per-filament kernels: 1024 threads (more loads in flight per
// filament) while one workgroup per CU covers all filaments, else 256
int fil_threads(const SimDev& d) { return d.M <= 256 ? 1024 : 256; }

int residual_launch(const SimDev& d, const BdfCoef& bc, const double* X, const double* Xj, const double* Yc,
                    const double* Yj, const double* Yjm1, double* V, double* W, const double* part, int K,
                    const int32_t* active, double* f, unsigned long long* resbits, unsigned long long* resbits_next,
                    const DotArgs& da, hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    if (fil_threads(d) == 1024)
        residual_kernel<1024><<<(unsigned)d.M, 1024, 0, st>>>(d, bc, X, Xj, Yc, Yj, Yjm1, V, W, part, K, active, f,
                                                              resbits, resbits_next, da);
    else
        residual_kernel<256><<<(unsigned)d.M, 256, 0, st>>>(d, bc, X, Xj, Yc, Yj, Yjm1, V, W, part, K, active, f,
                                                            resbits, resbits_next, da);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// ---------------------------------------------------------------- warm start
// step 0: (Y_1^0, 0, 0); step 1: (2Y_1^1 - Y_1^0, u^1, Lambda^1); later steps
// extrapolate Y_1 and the multipliers linearly and reuse u^j.
__global__ void __launch_bounds__(256) initial_guess_kernel(SimDev d, int64_t step, const double* __restrict__ Yj,
                                                          const double* __restrict__ Yjm1,
                                                          const double* __restrict__ Xj,
                                                          const double* __restrict__ Xjm1,
                                                          const double* __restrict__ Xjm2, double* __restrict__ X0,
                                                          double* __restrict__ X0c, double* __restrict__ Xb,
                                                          int32_t* __restrict__ active, SuspLog* __restrict__ log,
                                                          double* __restrict__ time_d, double tt) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0) {
        for (int64_t i = threadIdx.x; i < d.nsusp; i += blockDim.x) {
            active[i] = 1;
            log[i] = SuspLog{0, 0, 0, 0, 0.0};
        }
        if (threadIdx.x == 0) *time_d = tt;
    }
    if (s >= d.S) return;
    const int32_t f = d.seg_fil[s];
    const int64_t s0 = d.seg_off[f], N = d.seg_off[f + 1] - s0, n = s - s0;
    const int teth = d.tether[f];
    // the six slots this segment owns: Y_1 / lambda_1 (n == 0) or Lambda_{n-1/2}, then u_n / lambda_2
    const int64_t r0 = 6 * s0 + (n == 0 ? 0 : 3 + 3 * N + 3 * (n - 1));
    const int64_t r1 = 6 * s0 + 3 + 3 * n;
    for (int i = 0; i < 3; i++) {
        double x0, x1;
        if (step == 0) {
            x0 = (n == 0 && !teth) ? Yj[i * d.S + s] : 0.0;
            x1 = 0.0;
        } else {
            if (n == 0 && !teth) x0 = 2.0 * Yj[i * d.S + s] - Yjm1[i * d.S + s];
            else x0 = step >= 2 ? 2.0 * Xj[r0 + i] - Xjm1[r0 + i] : Xj[r0 + i];
            if (n == 0 && (teth == 1 || teth == 3)) x1 = step >= 2 ? 2.0 * Xj[r1 + i] - Xjm1[r1 + i] : Xj[r1 + i];
            else x1 = Xj[r1 + i];
        }
        X0[r0 + i] = X0c[r0 + i] = x0;
        X0[r1 + i] = X0c[r1 + i] = x1;
        // base of the learned first iterate: the extrapolation plus the last step's own
        // correction (its converged unknowns minus its extrapolation: the second difference
        // of Y_1 and Lambda, the first difference of u), for free filaments from step 3 on
        const bool hist = step >= 3 && !teth;
        Xb[r0 + i] = hist ? x0 + (Xj[r0 + i] - 2.0 * Xjm1[r0 + i] + Xjm2[r0 + i]) : x0;
        Xb[r1 + i] = hist ? x1 + (Xj[r1 + i] - Xjm1[r1 + i]) : x1;
    }
}

int initial_guess_launch(const SimDev& d, int64_t step, const double* Yj, const double* Yjm1, const double* Xj,
                         const double* Xjm1, const double* Xjm2, double* X0, double* X0c, double* Xb, int32_t* active,
                         SuspLog* log, double* time_d, double tt, hipStream_t st) {
    initial_guess_kernel<<<(unsigned)std::max<int64_t>(1, ceil_div(d.S, 256)), 256, 0, st>>>(
        d, step, Yj, Yjm1, Xj, Xjm1, Xjm2, X0, X0c, Xb, active, log, time_d, tt);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// One workgroup: the device log to the pinned slot `counter` mod 2 (the count of
// exports so far, advanced here in stream order, so a captured export needs no
// host argument per launch).
__global__ void __launch_bounds__(256) log_export_kernel(const SuspLog* __restrict__ log, int64_t ns,
                                                       SuspLog* __restrict__ slot0, SuspLog* __restrict__ slot1,
                                                       int64_t* __restrict__ counter) {
    const int64_t c = *counter;
    SuspLog* out = (c & 1) ? slot1 : slot0;
    for (int64_t i = threadIdx.x; i < ns; i += blockDim.x) out[i] = log[i];
    __threadfence_system();
    __syncthreads();  // every thread has read the count
    if (threadIdx.x == 0) *counter = c + 1;
}

int log_export_launch(const SuspLog* log, int64_t ns, SuspLog* slot0, SuspLog* slot1, int64_t* counter,
                      hipStream_t st) {
    log_export_kernel<<<1, 256, 0, st>>>(log, ns, slot0, slot1, counter);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// ---------------------------------------------------------------- J0 assembly
struct M33 {
    double m[9];
};
__device__ __forceinline__ M33 mzero() {
    M33 r;
    for (int i = 0; i < 9; i++) r.m[i] = 0.0;
    return r;
}
__device__ __forceinline__ M33 meye(double s) {
    M33 r = mzero();
    r.m[0] = r.m[4] = r.m[8] = s;
    return r;
}
// [v x] w = v x w
__device__ __forceinline__ M33 mskew(V3 v) {
    M33 r;
    r.m[0] = 0; r.m[1] = -v.z; r.m[2] = v.y;
    r.m[3] = v.z; r.m[4] = 0; r.m[5] = -v.x;
    r.m[6] = -v.y; r.m[7] = v.x; r.m[8] = 0;
    return r;
}
__device__ __forceinline__ M33 mscale(M33 a, double s) {
    for (int i = 0; i < 9; i++) a.m[i] *= s;
    return a;
}
__device__ __forceinline__ M33 madd(M33 a, M33 b) {
    for (int i = 0; i < 9; i++) a.m[i] += b.m[i];
    return a;
}
__device__ __forceinline__ M33 mmul(const M33& a, const M33& b) {
    M33 r;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            r.m[3 * i + j] = a.m[3 * i] * b.m[j] + a.m[3 * i + 1] * b.m[3 + j] + a.m[3 * i + 2] * b.m[6 + j];
    return r;
}
__device__ __forceinline__ M33 mouter(V3 a, V3 b) {
    M33 r;
    const double av[3] = {a.x, a.y, a.z}, bv[3] = {b.x, b.y, b.z};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r.m[3 * i + j] = av[i] * bv[j];
    return r;
}

struct SegFrame {
    V3 t, mu, nu;
};

// Frame-vector approximation of dM_{k+1/2}/du_k (second = false) or du_{k+1}
// (second = true), Appendix B.2; a = frame of segment k, b = frame of k+1.
__device__ M33 dmoment_du(const SegFrame& a, const SegFrame& b, V3 kap, double dL, double KB, double KT,
                          bool second) {
    const double beta = (dot(b.mu, a.nu) - dot(a.mu, b.nu)) / (2.0 * dL) - kap.x;
    const V3 gv = cross(a.nu, b.mu) - cross(a.mu, b.nu);
    const V3 ts = a.t + b.t;
    M33 bend;
    if (!second) bend = mmul(mskew(-1.0 * b.t), mskew(-1.0 * a.t));   // [x t_{k+1}][x t_k]
    else bend = mmul(mskew(a.t), mskew(-1.0 * b.t));                  // [t_k x][x t_{k+1}]
    const SegFrame& own = second ? b : a;
    M33 r = madd(mscale(bend, KB / dL),
                 madd(mscale(mskew(-1.0 * own.mu), -0.5 * KB * kap.y), mscale(mskew(-1.0 * own.nu), -0.5 * KB * kap.z)));
    r = madd(r, mscale(mskew(-1.0 * own.t), 0.5 * KT * beta));
    r = madd(r, mscale(mouter(ts, gv), (second ? -1.0 : 1.0) * 0.5 * KT / (2.0 * dL)));
    return r;
}

// ---------------------------------------------------------------- J0 blocks
// Per-filament data staged in LDS for the J0 blocks: frame (t, mu, nu), u, and the
// internal torque T^C + T^E of every segment.
struct J0Ctx {
    const double (*sh)[15];
    const double* Xf;
    int N, teth;
    int64_t f;
    double tt, cT, cR;
};

__device__ __forceinline__ SegFrame frame_at(const J0Ctx& c, int n) {
    const double* p = c.sh[n];
    return SegFrame{v3(p[0], p[1], p[2]), v3(p[3], p[4], p[5]), v3(p[6], p[7], p[8])};
}

// Block (I, J) of the explicit approximate Jacobian (Appendix B.2) in the
// original ordering.  Row blocks: 0 -> f^1, 1..N -> f^2_m (m = I-1), N+1..2N-1 ->
// f^3_m (m = I-N).  Column blocks: 0 -> Y_1 (lambda_1 when the base is held: tether 1
// clamped or 2 pinned), 1..N -> u_n (n = J-1; lambda_2 for n = 0 when clamped),
// N+1..2N-1 -> Lambda of joint J-N-1.
// cT = b dt/(6 pi eta a), cR = b dt/(8 pi eta a^3).
__device__ M33 j0_block(const SimDev& d, const J0Ctx& c, int I, int Jb) {
    const int N = c.N;
    const int teth = c.teth;
    // base orientation prescribed (held, or turned by the motor: the same drag-model rows)
    const bool clamped = teth == 1 || teth == 3;
    M33 B = mzero();
    if (I == 0) {  // f^1
        if (Jb == 0) B = meye(teth ? -c.cT : 1.0);
        else if (N > 1 && Jb == N + 1) B = meye(-c.cT);
    } else if (I > N) {  // f^3_m, m = 1..N-1
        const int m = I - N;
        if (Jb == 0) {
            if (!teth) B = meye(1.0);
        } else if (Jb <= N) {
            const int n = Jb - 1;
            if (n <= m && !(n == 0 && clamped)) {
                const double w = (n == 0 || n == m) ? 1.0 : 2.0;
                B = mscale(mskew(-1.0 * frame_at(c, n).t), 0.5 * d.dL * w);
            }
        } else {
            const int k = Jb - N - 1;
            if (k == m - 1) B = meye(c.cT);
            else if (k == m) B = meye(-c.cT);
        }
    } else {  // f^2_m
        const int m = I - 1;
        const double* pm = c.sh[m];
        const V3 um = v3(pm[9], pm[10], pm[11]);
        const M33 U = mskew(um), U2 = mmul(U, U);
        const M33 Tay = madd(madd(meye(1.0), mscale(U, -0.5)), mscale(U2, 1.0 / 12.0));
        const SegFrame fm = frame_at(c, m);
        if (Jb > N) {
            const int k = Jb - N - 1;
            if (k == m - 1 || k == m) B = mscale(mmul(Tay, mskew(fm.t)), -c.cR * 0.5 * d.dL);
        } else if (Jb >= 1) {
            const int n = Jb - 1;
            if (n == m + 1 && m + 1 < N) {
                const M33 dM = dmoment_du(fm, frame_at(c, m + 1), joint_kappa(d, c.f, m, c.tt), d.dL, d.KB, d.KT, true);
                B = mscale(mmul(Tay, dM), -c.cR);
            } else if (n == m - 1 && !(m == 1 && clamped)) {
                const M33 dM =
                    dmoment_du(frame_at(c, m - 1), fm, joint_kappa(d, c.f, m - 1, c.tt), d.dL, d.KB, d.KT, false);
                B = mscale(mmul(Tay, dM), c.cR);
            } else if (n == m) {
                if (clamped && m == 0) {
                    B = meye(-c.cR);
                } else {
                    V3 ls = v3(0, 0, 0);
                    if (m + 1 < N) ls = ls + ldx(c.Xf, 3 + 3 * N + 3 * m);
                    if (m >= 1) ls = ls + ldx(c.Xf, 3 + 3 * N + 3 * (m - 1));
                    M33 dT = mscale(mmul(mskew(-1.0 * ls), mskew(-1.0 * fm.t)), 0.5 * d.dL);
                    if (m + 1 < N)
                        dT = madd(dT, dmoment_du(fm, frame_at(c, m + 1), joint_kappa(d, c.f, m, c.tt), d.dL, d.KB, d.KT,
                                                 false));
                    if (m >= 1)
                        dT = madd(dT, mscale(dmoment_du(frame_at(c, m - 1), fm, joint_kappa(d, c.f, m - 1, c.tt), d.dL,
                                                        d.KB, d.KT, true),
                                             -1.0));
                    const V3 Tv = v3(pm[12], pm[13], pm[14]);
                    const M33 XT = mskew(-1.0 * Tv), XuT = mskew(-1.0 * cross(um, Tv));
                    M33 inner = madd(dT, mscale(madd(XT, mmul(U, dT)), -0.5));
                    inner = madd(inner, mscale(madd(madd(XuT, mmul(U, XT)), mmul(U2, dT)), 1.0 / 12.0));
                    B = madd(meye(1.0), mscale(inner, -c.cR));
                }
            }
        }
    }
    return B;
}

// ---------------------------------------------------------------- banded J0
// The robot-arm rows f^3_m involve every u_n with n <= m.  Replacing them by
// differences D_1 = f^3_1 - f^1, D_m = f^3_m - f^3_{m-1} (an invertible row
// operation) leaves, in the interleaved order of 3-blocks
//   columns: Y_1, u_0, Lambda_0, u_1, Lambda_1, ..., Lambda_{N-2}, u_{N-1}
//   rows:    f^1, f^2_0, D_1,  f^2_1, D_2, ...,     D_{N-1},     f^2_{N-1}
// a block-pentadiagonal matrix: scalar bandwidths kl = ku = 8.  Its LU with
// partial pivoting (upper bandwidth kl + ku after fill-in) is computed once per
// step and applied in every Broyden iteration; J0^{-1} v = (L J0)^{-1} (L v).
__device__ __forceinline__ int orig_col(int C, int N) {
    return C == 0 ? 0 : ((C & 1) ? 1 + (C - 1) / 2 : N + 1 + (C - 2) / 2);
}
// offset in the [6N] unknown / residual layout of interleaved 3-block P (column view)
__device__ __forceinline__ int slot_of(int P, int N) {
    return P == 0 ? 0 : ((P & 1) ? 3 + 3 * ((P - 1) / 2) : 3 + 3 * N + 3 * ((P - 2) / 2));
}

__global__ void __launch_bounds__(256) j0_band_assemble_kernel(SimDev d, BdfCoef bc, const double* __restrict__ X,
                                                             const double* __restrict__ qc,
                                                             const double* __restrict__ Tint, double tt,
                                                             const int32_t* __restrict__ active,
                                                             double* __restrict__ AB) {
    const int64_t f = blockIdx.x;
    if (!active[d.fil_susp[f]]) return;
    const int64_t S = d.S;
    const int64_t s0 = d.seg_off[f];
    const int N = (int)(d.seg_off[f + 1] - s0);
    const int n6 = 6 * N;
    double* ab = AB + 6 * s0 * kBandW;
    __shared__ double sh[kMaxSeg][15];  // t, mu, nu, u, T
    const double* Xf = X + 6 * s0;
    const int teth = d.tether[f];
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const Q4 q = ldq(qc, S, s0 + n);
        const V3 t = frame_t(q), mu = frame_mu(q), nu = frame_nu(q);
        V3 u = ldx(Xf, 3 + 3 * n);
        if ((teth == 1 || teth == 3) && n == 0) u = v3(0, 0, 0);
        const V3 Tm = ld3(Tint, S, s0 + n);
        const double v[15] = {t.x, t.y, t.z, mu.x, mu.y, mu.z, nu.x, nu.y, nu.z, u.x, u.y, u.z, Tm.x, Tm.y, Tm.z};
        for (int i = 0; i < 15; i++) sh[n][i] = v[i];
    }
    for (int e = threadIdx.x; e < n6 * kBandW; e += blockDim.x) ab[e] = 0.0;
    __syncthreads();
    const double dts = d.spar[kSpar * d.fil_susp[f]];
    J0Ctx c{sh, Xf, N, teth, f, tt, bc.b * dts / (6.0 * kPi * d.eta * d.a),
            bc.b * dts / (8.0 * kPi * d.eta * d.a * d.a * d.a)};
    const int nb = 2 * N;
    for (int item = threadIdx.x; item < nb * 5; item += blockDim.x) {
        const int R = item / 5, C = R + item % 5 - 2;
        if (C < 0 || C >= nb) continue;
        const int Jo = orig_col(C, N);
        M33 B;
        if (R == 0) B = j0_block(d, c, 0, Jo);
        else if (R & 1) B = j0_block(d, c, 1 + (R - 1) / 2, Jo);
        else {
            const int m = R / 2;
            B = madd(j0_block(d, c, N + m, Jo), mscale(j0_block(d, c, m == 1 ? 0 : N + m - 1, Jo), -1.0));
        }
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                const int i = 3 * R + a, j = 3 * C + b;
                ab[(int64_t)i * kBandW + (j - i + kKL)] = B.m[3 * a + b];
            }
    }
}



// 1 / x: hardware reciprocal and two Newton steps
__device__ __forceinline__ double rcp_f64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// LU with partial pivoting of every filament's banded system, one wave each, in a
// register window: lane l holds column j + l (l <= kKL + kKU) of rows j .. j + kKL,
// the only rows and columns step j reads or writes (row p <= j + kKL has no
// entries right of column j + kKL + kKU, before or after fill-in).  Step j takes
// the pivot from lane 0's column (broadcast), swaps rows inside every lane, writes
// row j of U and column j of L, updates the window and shifts it one column left /
// one row down; the row entering at the bottom comes from global memory, requested
// a few steps earlier (a queue unrolled by its depth, each load unconditional at a
// clamped address and masked when used, so that it stays in flight).
// kStaged: the results (U rows, L columns, pivots, reciprocal pivots) are kept in
// LDS and written out in band layout at the end, so the only memory counter the row
// loop waits on is that of its own queued loads; the loop runs a multiple of the
// queue depth with the surplus steps inert, so it has no exit inside.  Without
// staging (no LDS, so that every filament of a large ensemble can be resident at
// once) the results go straight to the band, every store unconditional.
template <bool kStaged>
__global__ void __launch_bounds__(64) j0_band_factor_kernel(SimDev d, const int32_t* __restrict__ active,
                                                          double* __restrict__ AB, int32_t* __restrict__ ipiv,
                                                          double* __restrict__ rdiag, int32_t* __restrict__ flag,
                                                          int64_t coff) {
    constexpr int kWin = kKL + kKU + 1;  // window columns (17)
    constexpr int QD = kStaged ? 8 : 4;  // queue depth
    const int64_t f = d.cls_fil[coff + blockIdx.x];
    if (!active[d.fil_susp[f]]) return;
    const int64_t s0 = d.seg_off[f];
    const int n = 6 * (int)(d.seg_off[f + 1] - s0);
    double* const gab = AB + 6 * s0 * kBandW;
    const int l = threadIdx.x;
    const bool lw = l < kWin;
    // LDS (staged): U rows [n][kWin] | L columns [n][kKL] | reciprocal pivots [n] | pivot rows [n]
    extern __shared__ double fac_lds[];
    double* const Ur = fac_lds;
    double* const Lm = Ur + (size_t)n * kWin;
    double* const rd = kStaged ? Lm + (size_t)n * kKL : rdiag + 6 * s0;
    int32_t* const ip = kStaged ? reinterpret_cast<int32_t*>(rd + n) : ipiv + 6 * s0;
    // element (r, c) of the band (0 outside the matrix); the band stores columns r-kKL .. r+kKL+kKU
    auto at = [&](int r, int c) {
        return (lw && r < n && c < n && c - r >= -kKL && c - r <= kKL + kKU)
                   ? gab[(int64_t)r * kBandW + (c - r + kKL)]
                   : 0.0;
    };
    double W[kKL + 1];
#pragma unroll
    for (int r = 0; r <= kKL; r++) W[r] = at(r, l);
    auto at_queued = [&](int r, int c, bool& ok) {
        ok = lw && r < n && c < n && c - r >= -kKL && c - r <= kKL + kKU;
        return gab[ok ? (int64_t)r * kBandW + (c - r + kKL) : 0];
    };
    double Q[QD];
    bool Qok[QD];
#pragma unroll
    for (int q = 0; q < QD; q++) Q[q] = at_queued(kKL + 1 + q, l + 1 + q, Qok[q]);
    int bad = 0;
    // slot qs is consumed at steps j = qs (mod QD) and refilled in place
    for (int j0 = 0; j0 < n; j0 += QD) {
#pragma unroll
        for (int qs = 0; qs < QD; qs++) {
            const int j = j0 + qs;
            if (!kStaged && j >= n) break;
            // pivot column j (lane 0) broadcast to the wave
            double col[kKL + 1];
#pragma unroll
            for (int r = 0; r <= kKL; r++) col[r] = readlane_f64(W[r], 0);
            // reciprocal pivot and multipliers as if row j were its own pivot (the usual
            // case for these blocks), beside the test of that: lane 0's |W[0]| is at least
            // every |W[r]| of its column
            double rp = rcp_f64(col[0]);
            double m[kKL + 1];
#pragma unroll
            for (int r = 1; r <= kKL; r++) m[r] = col[r] * rp;
            const double mx = fmax(fmax(fmax(fmax(fabs(W[0]), fabs(W[1])), fmax(fabs(W[2]), fabs(W[3]))),
                                        fmax(fmax(fabs(W[4]), fabs(W[5])), fmax(fabs(W[6]), fabs(W[7])))),
                                   fabs(W[8]));
            const int keep = __builtin_amdgcn_readfirstlane((int)(fabs(W[0]) >= mx));
            int pr = 0;
            if (__builtin_expect(!keep, 0)) {
                // pivot row: the first maximum of |W[r]| in every lane's own column (lane
                // 0's is used), a pairwise tree in which a later row wins only when
                // strictly larger; then the exchange (wave-uniform: selects) and the
                // reciprocal and multipliers again
                double bv[kKL + 1];
                int ix[kKL + 1];
#pragma unroll
                for (int r = 0; r <= kKL; r++) {
                    bv[r] = W[r];
                    ix[r] = r;
                }
#pragma unroll
                for (int w = 1; w <= kKL; w *= 2)
#pragma unroll
                    for (int r = 0; r + w <= kKL; r += 2 * w)
                        if (fabs(bv[r + w]) > fabs(bv[r])) {
                            bv[r] = bv[r + w];
                            ix[r] = ix[r + w];
                        }
                pr = __builtin_amdgcn_readfirstlane(ix[0]);
                const double w0 = W[0], c0 = col[0];
                double wp = w0, cp = c0;
#pragma unroll
                for (int r = 1; r <= kKL; r++) {
                    const bool sw = pr == r;
                    wp = sw ? W[r] : wp;
                    W[r] = sw ? w0 : W[r];
                    cp = sw ? col[r] : cp;
                    col[r] = sw ? c0 : col[r];
                }
                W[0] = wp;
                col[0] = cp;
                rp = rcp_f64(col[0]);
#pragma unroll
                for (int r = 1; r <= kKL; r++) m[r] = col[r] * rp;
            }
            const bool su = lw && j + l < n;
            if (kStaged) {
                // row j of U (lanes 0..16); lane 0 keeps column j of L, the pivot row and
                // the reciprocal pivot.  Steps past n write nothing.
                if (su) Ur[(int64_t)j * kWin + l] = W[0];
                if (l == 0 && j < n) {
                    double2* lj = reinterpret_cast<double2*>(Lm + (int64_t)j * kKL);
#pragma unroll
                    for (int r = 1; r <= kKL; r += 2) lj[r / 2] = make_double2(m[r], m[r + 1]);
                    ip[j] = j + pr;
                    rd[j] = rp;
                }
                if (j < n && !(fabs(col[0]) > 0.0)) bad = 1;
            } else {
                // final row j of U (lanes 0..16) and column j of L (lane r holds m[r]) in
                // the band.  The stores are unconditional so that the memory counter stays
                // static and the queued row loads remain in flight: a lane with nothing to
                // store writes the reciprocal pivot to its slot, as every lane does.
                double* const rslot = rd + j;
                *(su ? gab + (int64_t)j * kBandW + kKL + l : rslot) = su ? W[0] : rp;
                double ml = 0.0;
#pragma unroll
                for (int r = 1; r <= kKL; r++) ml = l == r ? m[r] : ml;
                const bool sm = l >= 1 && l <= kKL && j + l < n;
                *(sm ? gab + (int64_t)(j + l) * kBandW + kKL - l : rslot) = sm ? ml : rp;
                ip[j] = j + pr;
                if (!(fabs(col[0]) > 0.0)) bad = 1;
            }
            // rank-1 update of the window's lower rows (lane 0's column is done)
#pragma unroll
            for (int r = 1; r <= kKL; r++) W[r] = fma(-m[r], W[0], W[r]);
            // shift: lane l takes column j+1+l, rows j+1 .. j+1+kKL (lanes past the window hold
            // zeros, which is what rows j+1 .. j+kKL of column j+1+kKL+kKU are: beyond the
            // original upper bandwidth and untouched so far); the entering bottom row comes
            // from the queue, refilled with the row needed QD shifts later
#pragma unroll
            for (int r = 0; r < kKL; r++) W[r] = wave_next_f64(W[r + 1]);
            W[kKL] = Qok[qs] ? Q[qs] : 0.0;
            Q[qs] = at_queued(j + 1 + kKL + QD, j + 1 + QD + l, Qok[qs]);
        }
    }
    if (kStaged) {
        __syncthreads();
        // band row r, slot k: k < kKL is L(r, c), c = r - kKL + k (column c's multiplier
        // r - c); k >= kKL is U(r, r + k - kKL); slots outside the matrix are zero
        const int ne = n * kBandW;
        auto band_out = [&](int e) {
            const int r = e / kBandW, k = e - r * kBandW;
            if (k < kKL) {
                const int c = r - kKL + k;
                return c >= 0 ? Lm[(int64_t)c * kKL + (kKL - 1 - k)] : 0.0;
            }
            return r + (k - kKL) < n ? Ur[(int64_t)r * kWin + (k - kKL)] : 0.0;
        };
        int e = l;
        for (; e + 7 * 64 < ne; e += 8 * 64) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = band_out(e + u * 64);
#pragma unroll
            for (int u = 0; u < 8; u++) gab[e + u * 64] = v[u];
        }
        for (; e < ne; e += 64) gab[e] = band_out(e);
        for (int i = l; i < n; i += 64) {
            rdiag[6 * s0 + i] = rd[i];
            ipiv[6 * s0 + i] = ip[i];
        }
    }
    if (l == 0) flag[f] = bad;
}

// launch choice: MI355X has 256 CUs with 160 KB of LDS each; the unstaged factor's
// register use allows 20 of its waves per CU; staging is taken while a class needs at
// most 4 rounds of resident workgroups
constexpr int64_t kNumCU = 256, kFacWavesPerCU = 20, kFacStagedRounds = 4;
constexpr size_t kLdsPerCU = 160 * 1024;

// LDS of the staged factor of a filament of n unknowns
__host__ __device__ constexpr size_t factor_lds_bytes(int n) {
    return (size_t)n * (kKL + kKU + 1 + kKL + 1) * sizeof(double) + (size_t)n * sizeof(int32_t);
}


// Forward and backward sweeps of one banded LU solve by one wave, the solution
// vector y in LDS and a ring of lanes holding the active rows (16 forward, 32
// backward).  The band factor ab is read from global memory: each lane's
// coefficient for the next kSweepAhead steps is already in flight (lane queue);
// pivots ip and reciprocal diagonal rd are in LDS.
constexpr int kSweepAhead = 6;
__device__ __forceinline__ void band_sweeps(const double* __restrict__ ab, const int* ip, const double* rd, double* y,
                                            int n, int lane) {
    double w = (lane < 16 && lane < n) ? y[lane] : 0.0;
    // queued coefficients are loaded unconditionally (clamped address) and masked when
    // used, so each load stays in flight for kSweepAhead steps
    auto fwd_mult = [&](int jj, bool& ok) {
        const int off = (lane - (jj & 15)) & 15;
        ok = lane < 16 && off >= 1 && off <= kKL && jj + off < n;
        return ab[ok ? (int64_t)(jj + off) * kBandW + (kKL - off) : 0];
    };
    double Lq[kSweepAhead];
    bool Lok[kSweepAhead];
#pragma unroll
    for (int q = 0; q < kSweepAhead; q++) Lq[q] = fwd_mult(q, Lok[q]);
    int ipn = ip[0];
    double yin = y[min(16, n - 1)];
    // unrolled by the queue depth: slot q is consumed at steps j = q (mod depth) and
    // refilled in place, so each load has kSweepAhead steps to arrive
    for (int j0 = 0; j0 < n; j0 += kSweepAhead) {
#pragma unroll
        for (int q = 0; q < kSweepAhead; q++) {
            const int j = j0 + q;
            if (j < n) {
                const int h = j & 15;
                const int hp = __builtin_amdgcn_readfirstlane(ipn) & 15;
                const double L = Lok[q] ? Lq[q] : 0.0;
                Lq[q] = fwd_mult(j + kSweepAhead, Lok[q]);
                const double yi = j + 16 < n ? yin : 0.0;
                ipn = ip[min(j + 1, n - 1)];
                yin = y[min(j + 17, n - 1)];
                const double vh = readlane_f64(w, h), vp = readlane_f64(w, hp);
                w = lane == hp ? vh : w;
                w -= L * vp;  // vp: the pivot row now at the head; L = 0 off the kKL entries below it
                y[j] = vp;
                w = lane == h ? yi : w;
            }
        }
    }
    constexpr int kU = kKL + kKU;
    w = 0.0;
    if (lane < 32) {
        const int pos = (n - 1) - (((n - 1) - lane) & 31);
        w = pos >= 0 ? y[pos] : 0.0;
    }
    auto bwd_coef = [&](int ii, bool& ok) {
        const int off = ((ii & 31) - lane) & 31;
        ok = lane < 32 && off >= 1 && off <= kU && ii - off >= 0;
        return ab[ok ? (int64_t)(ii - off) * kBandW + (off + kKL) : 0];
    };
    double Uq[kSweepAhead];
    bool Uok[kSweepAhead];
#pragma unroll
    for (int q = 0; q < kSweepAhead; q++) Uq[q] = bwd_coef(n - 1 - q, Uok[q]);
    double zin = y[max(n - 33, 0)];
    for (int i0 = n - 1; i0 >= 0; i0 -= kSweepAhead) {
#pragma unroll
        for (int q = 0; q < kSweepAhead; q++) {
            const int i = i0 - q;
            if (i >= 0) {
                const int h = i & 31;
                const double U = Uok[q] ? Uq[q] : 0.0, dv = rd[i];
                Uq[q] = bwd_coef(i - kSweepAhead, Uok[q]);
                const double zi = i - 32 >= 0 ? zin : 0.0;
                zin = y[max(i - 33, 0)];
                const double xi = readlane_f64(w, h) * dv;
                w -= U * xi;  // U = 0 off the kKL + kKU entries above the head
                y[i] = xi;
                w = lane == h ? zi : w;
            }
        }
    }
}

// L v in the interleaved order for right-hand side v (X layout, filament block)
__device__ __forceinline__ double diff_rhs(const double* vf, int i, int N) {
    const int R = i / 3, a = i % 3;
    if (R == 0 || (R & 1)) return vf[slot_of(R, N) + a];
    const int m = R / 2;  // D_m = f^3_m - (m == 1 ? f^1 : f^3_{m-1})
    const double prev = m == 1 ? vf[a] : vf[3 + 3 * N + 3 * (m - 2) + a];
    return vf[3 + 3 * N + 3 * (m - 1) + a] - prev;
}
// the same for the unit vector e_c
__device__ __forceinline__ double diff_unit(int c, int i, int N) {
    const int R = i / 3, a = i % 3;
    if (R == 0 || (R & 1)) return slot_of(R, N) + a == c ? 1.0 : 0.0;
    const int m = R / 2;
    const int prev = m == 1 ? a : 3 + 3 * N + 3 * (m - 2) + a;
    return (3 + 3 * N + 3 * (m - 1) + a == c ? 1.0 : 0.0) - (prev == c ? 1.0 : 0.0);
}



// Explicit inverse for the dense per-iteration product.  Block (f, g) owns cb
// columns c = g*cb + t of filament f's J0^{-1}, one per thread: the thread
// solves (D J0) y = D e_c (D the row differencing) through the band factor
// with its column held in a sliding register window (kKL + 1 rows forward,
// kKL + kKU + 1 rows backward), so each sweep step is a few FMAs on registers.
// The band (between zero rows, so that no coefficient read needs a bounds test),
// the reciprocal pivots and the pivot rows are staged in LDS and shared by all
// threads.  A step's coefficients are read two steps ahead into one of two
// register sets (even and odd steps), and the pivot rows of 64 steps sit in one
// register (lane k: step 64q + k) read by lane index, so no step waits on LDS for
// its own data.  Forward results wait in LDS for the backward sweep, whose results
// are then written as row c of Ainv^T.
// zero band rows before / after the filament: the reads two steps past either end stay inside
constexpr int kInvPadLo = kKL + kKU + 2, kInvPadHi = kKL + 2;

// the (at most two) nonzero entries of D e_c in the interleaved order, c in the
// original unknown order: Y_1 and the multipliers are row-differenced, u is not
__device__ __forceinline__ void diff_unit_nonzeros(int c, int N, int& ia, double& va, int& ib, double& vb) {
    ia = ib = -1;
    va = 1.0;
    vb = -1.0;
    if (c < 3) {  // Y_1: block row 0, and minus in block row 2 (the first multiplier difference)
        ia = c;
        if (N >= 2) ib = 6 + c;
    } else if (c < 3 + 3 * N) {  // u_k: block row 2k + 1
        const int k = (c - 3) / 3, a = (c - 3) % 3;
        ia = 3 * (2 * k + 1) + a;
    } else {  // Lambda_q: plus in block row 2q + 2, minus in block row 2q + 4
        const int q = (c - 3 - 3 * N) / 3, a = (c - 3 - 3 * N) % 3;
        ia = 3 * (2 * q + 2) + a;
        if (q + 2 <= N - 1) ib = 3 * (2 * q + 4) + a;
    }
}

template <int CB>
__global__ void __launch_bounds__(64) j0_inverse_cols_kernel(SimDev d, const double* __restrict__ AB,
                                                            const int32_t* __restrict__ ipiv,
                                                            const double* __restrict__ rdiag,
                                                            const int32_t* __restrict__ active,
                                                            double* __restrict__ AinvT, int64_t coff) {
    constexpr int kU = kKL + kKU;
    const int64_t f = d.cls_fil[coff + blockIdx.x];
    if (!active[d.fil_susp[f]]) return;
    const int64_t s0 = d.seg_off[f];
    const int N = (int)(d.seg_off[f + 1] - s0);
    const int n = 6 * N;
    const int c0 = blockIdx.y * CB;
    if (c0 >= n) return;
    // LDS: band rows [-kInvPadLo, n + kInvPadHi) | forward results [n][CB + 1] (rows padded
    // by one so that a column read across lanes spreads over the banks) | reciprocal
    // pivots [n] | pivot rows [n]
    extern __shared__ double lds[];
    const int nrows = n + kInvPadLo + kInvPadHi;
    double* ab = lds + (size_t)kInvPadLo * kBandW;  // ab[i * kBandW + k] for i in [-kInvPadLo, n + kInvPadHi)
    double* ybuf = lds + (size_t)nrows * kBandW;
    constexpr int YS = CB + 1;  // row stride of the forward results
    double* rd = ybuf + (size_t)n * YS;
    int* ip = reinterpret_cast<int*>(rd + n);
    const int t = threadIdx.x;
    const int c = c0 + t;
    const bool live = t < CB && c < n;
    {
        // the band rows are contiguous: zero the padding, copy n * kBandW values with
        // eight loads in flight per thread
        const double* gab = AB + 6 * s0 * kBandW;
        for (int e = t; e < kInvPadLo * kBandW; e += 64) lds[e] = 0.0;
        for (int e = t; e < kInvPadHi * kBandW; e += 64) ab[(int64_t)n * kBandW + e] = 0.0;
        const int ne = n * kBandW;
        int e = t;
        for (; e + 7 * 64 < ne; e += 8 * 64) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = gab[e + u * 64];
#pragma unroll
            for (int u = 0; u < 8; u++) ab[e + u * 64] = v[u];
        }
        for (; e < ne; e += 64) ab[e] = gab[e];
        for (int e = t; e < n; e += blockDim.x) {
            ip[e] = ipiv[6 * s0 + e];
            rd[e] = rdiag[6 * s0 + e];
        }
        __syncthreads();
    }
    int ia, ib;
    double va, vb;
    diff_unit_nonzeros(live ? c : 0, N, ia, va, ib, vb);
    if (!live) ia = ib = -1;
    auto rhs = [&](int i) { return (i == ia ? va : 0.0) + (i == ib ? vb : 0.0); };
    // ---- forward: W[k] = y[j + k]
    double W[kKL + 1];
#pragma unroll
    for (int k = 0; k <= kKL; k++) W[k] = rhs(k);
    // L(j+k, j) = ab[(j + k) * kBandW + kKL - k], k = 1..kKL (zero rows past n)
    auto load_fwd = [&](int j, double (&Lv)[kKL]) {
        const double* col = ab + (int64_t)j * kBandW + kKL;
#pragma unroll
        for (int k = 1; k <= kKL; k++) Lv[k - 1] = col[k * (kBandW - 1)];
    };
    int ipc = ip[min(t, n - 1)], ipn = ip[min(64 + t, n - 1)];
    auto fwd_step = [&](int j, const double (&L)[kKL]) {
        if ((j & 63) == 0 && j > 0) {
            ipc = ipn;
            ipn = ip[min(j + 64 + t, n - 1)];
        }
        const int pc = __builtin_amdgcn_readlane(ipc, j & 63) - j;  // 0..kKL, wave-uniform
        if (__builtin_expect(pc != 0, 0)) {
            const double w0 = W[0];
            double wp = w0;
#pragma unroll
            for (int k = 1; k <= kKL; k++) {
                const bool s = pc == k;
                wp = s ? W[k] : wp;
                W[k] = s ? w0 : W[k];
            }
            W[0] = wp;
        }
        const double yj = W[0];
        if (t < CB) ybuf[(int64_t)j * YS + t] = yj;
#pragma unroll
        for (int k = 0; k < kKL; k++) W[k] = fma(-L[k], yj, W[k + 1]);
        W[kKL] = rhs(j + kKL + 1);
    };
    {
        double LA[kKL], LB[kKL];
        load_fwd(0, LA);
        load_fwd(1, LB);
        for (int j = 0; j < n; j += 2) {
            fwd_step(j, LA);
            load_fwd(j + 2, LA);
            if (j + 1 < n) {
                fwd_step(j + 1, LB);
                load_fwd(j + 3, LB);
            }
        }
    }
    __syncthreads();
    // ---- backward: B[k] = y[i - kU + k]
    double B[kU + 1];
    const int i0 = n - 1;
    const int tt = t < CB ? t : 0;
#pragma unroll
    for (int k = 0; k <= kU; k++) {
        const int r = i0 - kU + k;
        B[k] = (r >= 0 && t < CB) ? ybuf[(int64_t)r * YS + t] : 0.0;
    }
    // U(i-k, i) = ab[(i - k) * kBandW + kKL + k] (zero rows before 0) and 1 / U(i, i);
    // y[i - kU - 1], the value entering the window after step i
    auto load_bwd = [&](int i, double (&Uv)[kU + 1], double& bn) {
        const double* row = ab + (int64_t)i * kBandW + kKL;
        Uv[0] = rd[max(i, 0)];
#pragma unroll
        for (int k = 1; k <= kU; k++) Uv[k] = row[k - (int64_t)k * kBandW];
        bn = ybuf[(int64_t)max(i - kU - 1, 0) * YS + tt];
    };
    auto bwd_step = [&](int i, const double (&U)[kU + 1], double bn) {
        const double xi = B[kU] * U[0];
#pragma unroll
        for (int k = kU; k > 0; k--) B[k] = fma(-U[kU - k + 1], xi, B[k - 1]);
        if (t < CB) ybuf[(int64_t)i * YS + t] = xi;
        B[0] = i - kU - 1 >= 0 ? bn : 0.0;
    };
    {
        double UA[kU + 1], UB[kU + 1];
        double bA, bB;
        load_bwd(i0, UA, bA);
        load_bwd(i0 - 1, UB, bB);
        for (int i = i0; i >= 0; i -= 2) {
            bwd_step(i, UA, bA);
            load_bwd(i - 2, UA, bA);
            if (i - 1 >= 0) {
                bwd_step(i - 1, UB, bB);
                load_bwd(i - 3, UB, bB);
            }
        }
    }
    __syncthreads();
    // ---- row c of Ainv^T (original unknown order): column by column, lane t taking
    // rows t, t + 64, ... whose destination slots it computes once
    constexpr int kRowsPerLane = (6 * kMaxSeg + 63) / 64;
    int sl[kRowsPerLane];
#pragma unroll
    for (int q = 0; q < kRowsPerLane; q++) {
        const int i = t + 64 * q;
        sl[q] = i < n ? slot_of(i / 3, N) + i % 3 : 0;
    }
    const int ncols = min(CB, n - c0);
    double* base = AinvT + d.dense_off[f] + (int64_t)c0 * n;
    // four columns per pass: their LDS reads are issued before any of the stores
    for (int cb = 0; cb < ncols; cb += 4) {
        double v[4][kRowsPerLane];
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int q = 0; q < kRowsPerLane; q++) {
                const int i = t + 64 * q;
                v[u][q] = i < n ? ybuf[(int64_t)i * YS + min(cb + u, CB - 1)] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (cb + u >= ncols) break;
            double* row = base + (int64_t)(cb + u) * n;
#pragma unroll
            for (int q = 0; q < kRowsPerLane; q++)
                if (t + 64 * q < n) row[sl[q]] = v[u][q];
        }
    }
}

// Dynamic LDS beyond 64 KB has to be granted to a kernel (gfx950 has 160 KB per
// workgroup); granted once per kernel, before any launch that is captured.
template <class Kernel>
int allow_lds(Kernel kernel, size_t bytes) {
    static std::mutex mu;
    static std::map<const void*, size_t> granted;
    if (bytes <= 65536) return FIL_OK;
    const void* k = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    auto it = granted.find(k);
    if (it != granted.end() && it->second >= bytes) return FIL_OK;
    FIL_HIP_TRY(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    granted[k] = bytes;
    return FIL_OK;
}

// Column records of the band factor for the grouped sweeps (kBcW doubles per column).
// The first half of record i holds the lane of the pivot row ip[i] in a row of 16 lanes (4 x
// (ip[i] mod 16) in the low word, at position i mod 16) and the multipliers of column i, L(i + off, i) for off = 1 .. kKL, at position
// (i + off) mod 16 (zeros elsewhere); the second half holds the entries of U in column i
// divided by the pivot, U(i - 1 - k, i) / U(i, i) for k = 0 .. 15, at position (i - 1 - k)
// mod 16; zero outside the filament.  With these rotations the lane of a sweep that holds
// row r of the 16-row window (lane r mod 16) reads the same position of every record, so
// one address per lane serves every step with an immediate offset.
__global__ void __launch_bounds__(256) band_columns_kernel(SimDev d, const int32_t* __restrict__ active,
                                                          const double* __restrict__ AB,
                                                          const int32_t* __restrict__ ipiv,
                                                          const double* __restrict__ rdiag, double* __restrict__ BC) {
    static_assert(kKL + kKU == 16 && kKL < 16 && kBcW == 32, "two 16-slot halves");
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= 6 * d.S * kBcW) return;
    const int64_t e = t / kBcW;
    const int k = (int)(t - e * kBcW);
    const int64_t f = d.seg_fil[e / 6];
    if (!active[d.fil_susp[f]]) return;
    const int64_t e0 = 6 * d.seg_off[f];
    const int n = 6 * (int)(d.seg_off[f + 1] - d.seg_off[f]);
    const int i = (int)(e - e0);
    const double* ab = AB + e0 * kBandW;
    double v = 0.0;
    if (k < 16) {
        const int off = (k - i) & 15;  // L(i + off, i) at column offset -off of row i + off
        if (off == 0) v = __hiloint2double(0, (ipiv[e] & 15) << 2);  // the pivot row's lane, as a byte offset
        else if (off <= kKL && i + off < n) v = ab[(int64_t)(i + off) * kBandW + (kKL - off)];
    } else {
        const int off = ((i - (k - 16) - 1) & 15) + 1;  // U(i - off, i) at column offset off of row i - off
        if (i - off >= 0) v = ab[(int64_t)(i - off) * kBandW + (kKL + off)] * rdiag[e];
    }
    BC[t] = v;
}

int j0_factor_launch(const SimDev& d, const BdfCoef& bc, const double* X, const double* qc, const double* Tint,
                     double tt, const int32_t* active, double* AB, int32_t* ipiv, double* rdiag, int32_t* flag,
                     double* AinvT, double* BC, hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    j0_band_assemble_kernel<<<(unsigned)d.M, 256, 0, st>>>(d, bc, X, qc, Tint, tt, active, AB);
    // filaments grouped by size so that each launch's LDS fits its own largest filament
    for (int k = 0; k < d.ncls; k++) {
        const int64_t coff = d.cls_off[k], cnt = d.cls_off[k + 1] - coff;
        if (cnt == 0) continue;
        const int nc = d.cls_n[k];
        // the staged factor while the class's filaments fit on the chip in at most
        // kFacStagedRounds rounds of resident workgroups, else the one without LDS (all
        // resident at once)
        const size_t fl = factor_lds_bytes(nc);
        const int64_t per_cu = std::min<int64_t>(kFacWavesPerCU, (int64_t)(kLdsPerCU / fl));
        if (!d.factor_unstaged && per_cu > 0 && cnt <= kFacStagedRounds * kNumCU * per_cu) {
            if (int rc = allow_lds(j0_band_factor_kernel<true>, fl)) return rc;
            j0_band_factor_kernel<true><<<(unsigned)cnt, 64, fl, st>>>(d, active, AB, ipiv, rdiag, flag, coff);
        } else {
            j0_band_factor_kernel<false><<<(unsigned)cnt, 64, 0, st>>>(d, active, AB, ipiv, rdiag, flag, coff);
        }
        if (!AinvT) continue;
        // one thread per inverse column; a block's columns (the most of 64, 32 or 16 whose
        // band, pivots and forward results fit in one CU's LDS: a block holds one CU either
        // way, so the widest block does the most columns per CU; 500 x 32 suspension: 64
        // columns 0.40 ms against 0.72 ms for 32) share the staged factor
        auto lds = [nc](int cb) {
            return ((size_t)(nc + kInvPadLo + kInvPadHi) * kBandW + (size_t)nc * (cb + 2)) * sizeof(double) +
                   (size_t)nc * sizeof(int);
        };
        if (lds(64) <= kLdsPerCU) {
            const dim3 grid((unsigned)cnt, (unsigned)ceil_div(nc, 64));
            if (int rc = allow_lds(j0_inverse_cols_kernel<64>, lds(64))) return rc;
            j0_inverse_cols_kernel<64><<<grid, 64, lds(64), st>>>(d, AB, ipiv, rdiag, active, AinvT, coff);
        } else if (lds(32) <= kLdsPerCU) {
            const dim3 grid((unsigned)cnt, (unsigned)ceil_div(nc, 32));
            if (int rc = allow_lds(j0_inverse_cols_kernel<32>, lds(32))) return rc;
            j0_inverse_cols_kernel<32><<<grid, 64, lds(32), st>>>(d, AB, ipiv, rdiag, active, AinvT, coff);
        } else {
            const dim3 grid((unsigned)cnt, (unsigned)ceil_div(nc, 16));
            if (int rc = allow_lds(j0_inverse_cols_kernel<16>, lds(16))) return rc;
            j0_inverse_cols_kernel<16><<<grid, 64, lds(16), st>>>(d, AB, ipiv, rdiag, active, AinvT, coff);
        }
    }
    if (BC)
        band_columns_kernel<<<(unsigned)ceil_div(6 * d.S * kBcW, (int64_t)256), 256, 0, st>>>(d, active, AB, ipiv,
                                                                                           rdiag, BC);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// ---------------------------------------------------------------- Broyden update + state
// One workgroup per filament, after the residual kernel of the same evaluation:
//  1. with a judge: the convergence test of the filament's suspension from the
//     maxima the residual kernel left (max|f|/a <= tol ends it when this evaluation
//     may end a step; a non-finite value or it >= kmax fails it).  Every workgroup
//     of the suspension takes the same decision; the one of its first filament logs
//     it and clears the suspension's flag.  A singular J0 block (first step) fails
//     its suspension.
//  2. the suspension's dot products, summed over its filaments in a fixed order (so
//     every workgroup of the suspension holds the same values);
//  3. g = J0^{-1} f for the filament's rows: explicit inverse (P threads per row over
//     contiguous column ranges), or the banded sweeps by the first wave;
//  4. the bad-Broyden update (Alg. 2): g += sum_{h<k} c_h (d_h . f) (R threads per row,
//     thread q over h = q, q + R, ...); c_k = -g/|df|, d_k = df/|df|,
//     step = g + c_k (d_k . f), or for the first step (k < 0) step = g; then
//     fprev <- f and X <- X - step;
//  5. the configuration and internal forces at the new X.
// Every load that does not depend on the kernel's own results (the thread's columns of
// the inverse and history terms when they fit in registers, the rows of f, fprev and
// X, q^j) is issued first, so the phases do not wait for memory one after another.
// Partial sums are combined in a fixed order.
constexpr int kPreCols = 16;  // inverse columns per thread held in registers
constexpr int kPreHist = 4;   // history terms per thread held in registers

template <int NT>
__global__ void __launch_bounds__(NT) broyden_state_kernel(SimDev d, UpdateArgs u, JudgeArgs jg,
                                                         int32_t* __restrict__ active) {
    constexpr int NW = NT / 64;
    const int64_t f = blockIdx.x;
    const int32_t isus = d.fil_susp[f];
    if (!active[isus]) return;
    const int64_t s0 = d.seg_off[f];
    const int N = (int)(d.seg_off[f + 1] - s0);
    const int n = 6 * N;
    const int64_t e0 = 6 * s0, n6 = 6 * d.S;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    // threads per row (inverse columns, history terms); P <= n keeps every column range non-empty
    const int P = max(1, min(min(kSplit, NT / n), n));
    const int pq = t / n, pi = t - pq * n;      // this thread's share: part pq of row pi
    const bool part_thr = t < P * n;
    // ---- loads issued before any use
    const double* A = u.AinvT ? u.AinvT + d.dense_off[f] : nullptr;
    const int cb = (n * pq) / P, ce = (n * (pq + 1)) / P;
    // (only in the 1024-thread form, used for few filaments: the register cost would
    // lower the occupancy the many-filament form relies on)
    const bool areg = NT >= 1024 && A && P * n <= NT && (n + P - 1) / P <= kPreCols;  // uniform
    double ap[kPreCols];
    if (areg && part_thr) {
#pragma unroll
        for (int q = 0; q < kPreCols; q++) ap[q] = A[(int64_t)min(cb + q, ce - 1) * n + pi];  // masked at use
    }
    const bool hreg = NT >= 1024 && P * n <= NT && u.k <= kPreHist * P;  // uniform
    double hp[kPreHist];
    if (hreg && part_thr && u.k > 0) {
#pragma unroll
        for (int m = 0; m < kPreHist; m++) hp[m] = u.Chist[(int64_t)min(pq + m * P, u.k - 1) * n6 + e0 + pi];
    }
    double fr = 0.0, fp = 0.0, xr = 0.0;
    if (t < n) {
        fr = u.fnew[e0 + t];
        fp = u.fprev[e0 + t];
        xr = u.X[e0 + t];
    }
    const Q4 qjn = t < N ? ldq(u.qj, d.S, s0 + t) : Q4{1.0, 0.0, 0.0, 0.0};
    // the suspension's partial dots of this wave's first two dots, for up to 128 filaments
    const int64_t sg0 = d.susp_fil_off[isus], sg1 = d.susp_fil_off[isus + 1];
    const int nd = u.k + 2;
    const int h0 = wave, h1 = wave + NW;
    const bool ppre = NT >= 1024 && u.k >= 0 && sg1 - sg0 <= 128;  // uniform
    double pd0[2] = {0.0, 0.0}, pd1[2] = {0.0, 0.0};
    if (ppre) {
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const int64_t g = min(sg0 + lane + 64 * r, sg1 - 1);  // clamped; masked when summed
            if (h0 < nd) pd0[r] = u.dpart[g * d.max_dots + h0];
            if (h1 < nd) pd1[r] = u.dpart[g * d.max_dots + h1];
        }
    }
    if (jg.log) {
        const double r = __longlong_as_double((long long)jg.resbits[isus]) * jg.inv_a;
        int32_t state = 0;
        if (!(r <= 1.7976931348623157e308)) state = -1;  // NaN or infinite
        else if (r <= jg.tol && jg.can_converge) state = 1;
        else if (jg.it >= jg.kmax) state = -1;
        if (jg.jflag && jg.jflag[f] && threadIdx.x == 0) {
            // singular J0 block: the suspension fails (every such workgroup writes the same)
            jg.log[isus].state = -2;
            active[isus] = 0;
        }
        if (jg.jflag && jg.jflag[f]) return;
        if (threadIdx.x == 0 && f == d.susp_fil_off[isus]) {
            SuspLog& L = jg.log[isus];
            L.it = jg.it;
            L.evals += 1;
            L.evals_hi += jg.can_converge;
            L.last = r;
            if (state && L.state == 0) L.state = state;
            if (state) active[isus] = 0;
            if (!state && jg.notnear) {
                const double vm = __longlong_as_double((long long)jg.resbits[d.nsusp + isus]) * jg.inv_a;
                if (!(r <= fmax(jg.near_tol, jg.near_coef * vm))) atomicAdd(jg.notnear, 1);
            }
        }
        if (state) return;
    }
    __shared__ double sf[6 * kMaxSeg], sg[6 * kMaxSeg], sx[6 * kMaxSeg];
    __shared__ double sdots[kMaxDots];
    __shared__ double red[lds_rows(NT)];
    for (int e = t; e < n; e += NT) sf[e] = e == t ? fr : u.fnew[e0 + e];
    if (u.k >= 0) {
        // dot h by wave h mod NW, two per pass, over the filaments' partials in order
        for (int q0 = h0; q0 < nd; q0 += 2 * NW) {
            const int q1 = q0 + NW;
            double a0 = 0.0, a1 = 0.0;
            if (ppre && q0 == h0) {  // the first pass from the values read ahead
#pragma unroll
                for (int r = 0; r < 2; r++)
                    if (sg0 + lane + 64 * r < sg1) {
                        a0 += pd0[r];
                        a1 += pd1[r];
                    }
            } else {
                for (int64_t g = sg0 + lane; g < sg1; g += 64) {
                    a0 += u.dpart[g * d.max_dots + q0];
                    if (q1 < nd) a1 += u.dpart[g * d.max_dots + q1];
                }
            }
            a0 = wave_sum(a0);
            a1 = wave_sum(a1);
            if (lane == 0) {
                sdots[q0] = a0;
                if (q1 < nd) sdots[q1] = a1;
            }
        }
    }
    __syncthreads();
    if (A) {
        // g_i = sum_c Ainv^T[c][i] f_c
        for (int e = t; e < P * n; e += NT) {
            const int p = e / n, i = e - p * n;
            const int c1 = (n * p) / P, c2 = (n * (p + 1)) / P;
            double acc = 0.0;
            if (areg) {
                double a8[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < kPreCols; q++)
                    if (c1 + q < c2) a8[q & 3] = fma(ap[q], sf[c1 + q], a8[q & 3]);
                acc = (a8[0] + a8[1]) + (a8[2] + a8[3]);
            } else {
                double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                int c = c1;
                for (; c + 8 <= c2; c += 8)
#pragma unroll
                    for (int q = 0; q < 8; q++) a8[q] = fma(A[(int64_t)(c + q) * n + i], sf[c + q], a8[q]);
                for (; c < c2; c++) a8[0] = fma(A[(int64_t)c * n + i], sf[c], a8[0]);
                acc = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
            }
            red[e] = acc;
        }
        __syncthreads();
        for (int i = t; i < n; i += NT) {
            double acc = red[i];
            for (int p = 1; p < P; p++) acc += red[p * n + i];
            sg[i] = acc;
        }
    } else if (u.gsolve) {
        for (int i = t; i < n; i += NT) sg[i] = u.gsolve[e0 + i];
    } else {
        // L f in the interleaved order, then the sweeps through the band factor
        __shared__ double y[6 * kMaxSeg], rd[6 * kMaxSeg];
        __shared__ int ip[6 * kMaxSeg];
        const double* ab = u.AB + e0 * kBandW;
        for (int i = t; i < n; i += NT) {
            y[i] = diff_rhs(sf, i, N);
            rd[i] = u.rdiag[e0 + i];
            ip[i] = u.ipiv[e0 + i];
        }
        __syncthreads();
        if (wave == 0) band_sweeps(ab, ip, rd, y, n, lane);
        __syncthreads();
        for (int i = t; i < n; i += NT) sg[slot_of(i / 3, N) + i % 3] = y[i];
    }
    __syncthreads();
    if (u.k >= 0) {
        // sum_{h<k} c_h (d_h . f) per row
        for (int e = t; e < P * n; e += NT) {
            const int q = e / n, i = e - q * n;
            double acc = 0.0;
            if (hreg) {
                double a2[2] = {0.0, 0.0};
#pragma unroll
                for (int m = 0; m < kPreHist; m++) {
                    const int h = q + m * P;
                    if (h < u.k) a2[m & 1] = fma(hp[m], sdots[h], a2[m & 1]);
                }
                acc = a2[0] + a2[1];
            } else {
                double a0 = 0.0, a1 = 0.0;
                int h = q;
                for (; h + P < u.k; h += 2 * P) {
                    a0 = fma(u.Chist[(int64_t)h * n6 + e0 + i], sdots[h], a0);
                    a1 = fma(u.Chist[(int64_t)(h + P) * n6 + e0 + i], sdots[h + P], a1);
                }
                if (h < u.k) a0 = fma(u.Chist[(int64_t)h * n6 + e0 + i], sdots[h], a0);
                acc = a0 + a1;
            }
            red[e] = acc;
        }
        __syncthreads();
    }
    for (int e = t; e < n; e += NT) {
        const int64_t ge = e0 + e;
        // rows past the first NT were not read ahead
        const double fe = e == t ? fr : sf[e], pe = e == t ? fp : u.fprev[ge], xe = e == t ? xr : u.X[ge];
        double hn;
        if (u.k >= 0) {
            const double nrm = sqrt(sdots[u.k]);
            const double inrm = nrm > 0.0 ? 1.0 / nrm : 0.0;
            const double dfdot = sdots[u.k + 1] * inrm;
            double g = red[e];
            for (int q = 1; q < P; q++) g += red[q * n + e];
            g += sg[e];
            const double c = -g * inrm;
            u.Chist[(int64_t)u.k * n6 + ge] = c;
            u.Dhist[(int64_t)u.k * n6 + ge] = (fe - pe) * inrm;
            hn = fma(c, dfdot, g);
        } else {
            hn = sg[e];
        }
        u.fprev[ge] = fe;
        const double xn = xe - hn;
        u.X[ge] = xn;
        sx[e] = xn;
        if (u.dXout) u.dXout[ge] = -hn;
    }
    __syncthreads();
    filament_state(d, f, sx, qjn, *u.tt, u.Yc, u.qc, u.F, u.T, u.box);
}

// compile-time loop over the 16 lanes of a row (the DPP lane selects are immediates)
template <int H = 0, class Fn>
__device__ __forceinline__ void for_row_lanes(Fn&& fn) {
    if constexpr (H < 16) {
        fn(std::integral_constant<int, H>{});
        for_row_lanes<H + 1>(fn);
    }
}

// the right-hand side row i of L v (as diff_rhs) with both loads issued unconditionally
__device__ __forceinline__ double diff_rhs_nobranch(const double* vf, int i, int N) {
    const int R = i / 3, a = i % 3, m = R / 2;
    const bool plain = R == 0 || (R & 1);
    const int i1 = plain ? slot_of(R, N) + a : 3 + 3 * N + 3 * (m - 1) + a;
    const int i2 = plain ? i1 : (m == 1 ? a : 3 + 3 * N + 3 * (m - 2) + a);
    const double v1 = vf[i1], v2 = vf[i2];
    return plain ? v1 : v1 - v2;
}

// J0^{-1} f for many filaments at once: four filaments per wave, one per row of 16 lanes,
// the rows stepping together through the forward sweep (the factor's row interchanges and
// its kKL multipliers per column) and the backward sweep (U, kKL + kKU entries above the
// diagonal).  Each sweep keeps a 16-row window of the right-hand side in registers, row r
// in lane r mod 16 of its row: a step broadcasts the head row inside the row of lanes
// (DPP), updates the rows below (above) it with one multiply-add from the column record,
// and the freed lane takes the row that enters the window.  Each lane reads one slot of
// every record (band_columns_kernel rotates them so), into a ring of 16 registers: the
// slot for step s + 16 is requested as soon as step s has used its own, so loads have 16
// steps to arrive.  Records past either end of a filament (the next ones, or the zero pads)
// are read but only ever multiply rows outside it, which are zero and never written out.
// A wave's rows of lanes with shorter filaments (or finished suspensions) step along on
// zero rows; in the backward sweep they are aligned at the top, so every row of lanes has
// the same head lane.  The backward sweep leaves U(i, i) x_i, scaled at the output.
__global__ void __launch_bounds__(64) band_solve_kernel(SimDev d, const double* __restrict__ BC,
                                                        const double* __restrict__ rdiag,
                                                        const int32_t* __restrict__ active,
                                                        const double* __restrict__ fX, double* __restrict__ g) {
    static_assert(kKL + kKU == 16 && kKL < 16 && kBcW == 32, "16-row windows, two 16-slot halves");
    constexpr int kRows = 6 * kMaxSeg;
    const int lane = threadIdx.x, gl = lane & 15, grp = lane >> 4, gb = lane & 48;
    const int64_t f = (int64_t)blockIdx.x * 4 + grp;
    const int64_t fc = f < d.M ? f : d.M - 1;
    const bool on = f < d.M && active[d.fil_susp[fc]];
    const int64_t s0 = d.seg_off[fc];
    const int N = (int)(d.seg_off[fc + 1] - s0);
    const int n = on ? 6 * N : 0;
    const int nl = 6 * N - 1;  // last row of the (clamped) filament
    const int64_t e0 = 6 * s0;
    const int nmax = max(max(__builtin_amdgcn_readlane(n, 0), __builtin_amdgcn_readlane(n, 16)),
                         max(__builtin_amdgcn_readlane(n, 32), __builtin_amdgcn_readlane(n, 48)));
    if (nmax == 0) return;
    const double* col = BC + e0 * kBcW;
    // the first 16 forward records, requested before the right-hand side is staged
    const double* pf = col + gl;  // position gl of every record's first half
    double R[16];
#pragma unroll
    for (int h = 0; h < 16; h++) R[h] = pf[h * kBcW];
    // the right-hand side (every load issued before the first is used) into the window store
    __shared__ double ys[4][kRows + 16];  // a spare tail for the last block's rows past nmax
    double* y = ys[grp];
    constexpr int kPer = kRows / 32;  // rows per lane in each of two rounds
#pragma unroll
    for (int r0 = 0; r0 < kRows; r0 += 16 * kPer) {
        double sv[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) sv[q] = diff_rhs_nobranch(fX + e0, min(r0 + gl + 16 * q, nl), N);
#pragma unroll
        for (int q = 0; q < kPer; q++)
            if (r0 + gl + 16 * q < n) y[r0 + gl + 16 * q] = sv[q];
    }
    __syncthreads();

    // ---- forward sweep; step j: rows j .. j+15 in the window, head lane j mod 16.  Rows
    // past n are zero (their multipliers are zero), so steps past n move and add zeros; a
    // lane keeps the row it heads (yo) until the end of the block.
    const int gl4 = gl << 2, gb4 = gb << 2;
    double w = y[min(gl, kRows - 1)];
    w = gl < n ? w : 0.0;
    double yo = 0.0;
    for (int jb = 0; jb < nmax; jb += 16) {
        const int ie = jb + 16 + gl;  // the row that enters this lane at its step
        const double yr = y[min(ie, kRows - 1)];
        const double ye = ie < n ? yr : 0.0;
        const double* pn = pf + (int64_t)(jb + 16) * kBcW;
        for_row_lanes([&](auto hc) {
            constexpr int h = decltype(hc)::value;
            if (jb + h < nmax) {
                // lane h's slot of the record holds the pivot's lane; its multiply-add is discarded
                const int p4 = dpp_i32<kDppRowBcast + h>(__double2loint(R[h])) & 60;
                const double vh = dpp64_f64<kDppRowBcast + h>(w);
                const int a = gb4 | p4;
                const double vp = __hiloint2double(__builtin_amdgcn_ds_bpermute(a, __double2hiint(w)),
                                                   __builtin_amdgcn_ds_bpermute(a, __double2loint(w)));
                const bool head = gl == h;
                w = gl4 == p4 ? vh : w;  // row interchange
                w = fma(-R[h], vp, w);
                yo = head ? vp : yo;
                w = head ? ye : w;
            }
            R[h] = pn[h * kBcW];
        });
        y[jb + gl] = yo;  // rows past n land in the store's spare tail or are never read
    }

    // ---- backward sweep in virtual rows v = i + dl (dl = nmax - n): head lane v mod 16
    const int dl = nmax - n;
    {
        const int r = n - 16 + ((gl - nmax) & 15);  // rows n-16 .. n-1
        const double yr = y[max(r, 0)];
        w = r >= 0 ? yr : 0.0;
    }
    // position (gl - dl) mod 16 of the second halves: this lane's U entry at every step
    const double* pb = col + 16 + ((gl - dl) & 15) - (int64_t)dl * kBcW;
    int kb = (nmax - 1) >> 4;
    {
        const double* pk = pb + (int64_t)16 * kb * kBcW;
#pragma unroll
        for (int h = 0; h < 16; h++) R[h] = pk[h * kBcW];
    }
    for (; kb >= 0; kb--) {
        const int ie = 16 * kb + gl - dl - 16;  // the row that enters this lane at its step
        const double yr = y[max(ie, 0)];
        const double ye = ie >= 0 ? yr : 0.0;
        const double* pn = pb + (int64_t)16 * (kb - 1) * kBcW;
        for_row_lanes([&](auto sc) {
            constexpr int h = 15 - decltype(sc)::value;
            if (16 * kb + h < nmax) {
                const double wi = dpp64_f64<kDppRowBcast + h>(w);  // U(i, i) x_i of the head row i
                const bool head = gl == h;
                yo = head ? wi : yo;
                w = fma(-R[h], wi, head ? ye : w);
            }
            R[h] = pn[h * kBcW];
        });
        const int i = 16 * kb + gl - dl;  // the row this lane headed
        if (i >= 0 && 16 * kb + gl < nmax) y[i] = yo;
    }
    __syncthreads();
#pragma unroll
    for (int r0 = 0; r0 < kRows; r0 += 16 * kPer) {
        double rv[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) rv[q] = rdiag[e0 + min(r0 + gl + 16 * q, nl)];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const int i = r0 + gl + 16 * q;
            if (i < n) g[e0 + slot_of(i / 3, N) + i % 3] = y[i] * rv[q];
        }
    }
}

__global__ void __launch_bounds__(256) f32_switch_kernel(int32_t* __restrict__ active, SuspLog* __restrict__ log,
                                                       int* __restrict__ notnear, int64_t ns, int it, int kmax) {
    const int cnt = *notnear;
    __syncthreads();  // every thread has read the count before it is cleared
    if (threadIdx.x == 0) *notnear = 0;
    if (it < 0 || !(cnt == 0 || 2 * (it - 1) >= kmax)) return;
    for (int64_t i = threadIdx.x; i < ns; i += blockDim.x)
        if (active[i]) {
            active[i] = 0;
            log[i].state = 2;
        }
}

int f32_switch_launch(int32_t* active, SuspLog* log, int* notnear, int64_t nsusp, int it, int kmax, hipStream_t st) {
    f32_switch_kernel<<<1, 256, 0, st>>>(active, log, notnear, nsusp, it, kmax);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

int broyden_state_launch(const SimDev& d, const UpdateArgs& u, const JudgeArgs& jg, int32_t* active, hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    if (u.gsolve && !u.AinvT)
        band_solve_kernel<<<(unsigned)ceil_div(d.M, (int64_t)4), 64, 0, st>>>(d, u.BC, u.rdiag, active, u.fnew,
                                                                            u.gsolve);
    if (fil_threads(d) == 1024) broyden_state_kernel<1024><<<(unsigned)d.M, 1024, 0, st>>>(d, u, jg, active);
    else broyden_state_kernel<256><<<(unsigned)d.M, 256, 0, st>>>(d, u, jg, active);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// dot products of an update from a residual the caller provides
template <int NT>
__global__ void __launch_bounds__(NT) update_dots_kernel(SimDev d, const double* __restrict__ fnew,
                                                       const int32_t* __restrict__ active, DotArgs da) {
    const int64_t f = blockIdx.x;
    if (!active[d.fil_susp[f]]) return;
    const int64_t e0 = 6 * d.seg_off[f];
    const int n = 6 * (int)(d.seg_off[f + 1] - d.seg_off[f]);
    __shared__ double sf[6 * kMaxSeg];
    for (int e = threadIdx.x; e < n; e += NT) sf[e] = fnew[e0 + e];
    __syncthreads();
    filament_dots<NT>(d, f, da, sf, n);
}

int update_dots_launch(const SimDev& d, const double* fnew, const int32_t* active, const DotArgs& da,
                       hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    update_dots_kernel<256><<<(unsigned)d.M, 256, 0, st>>>(d, fnew, active, da);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// ---------------------------------------------------------------- finalise
// History shift of converged suspensions: Y^{j-1} <- Y^j, Y^j <- Y(X*), q^j <- q(X*),
// X^{j-1} <- X^j, X^j <- X*.
__global__ void __launch_bounds__(256) finalize_kernel(SimDev d, const int32_t* __restrict__ commit,
                                                     const double* __restrict__ Yc, const double* __restrict__ qc,
                                                     const double* __restrict__ X, double* __restrict__ Yj,
                                                     double* __restrict__ Yjm1, double* __restrict__ qj,
                                                     double* __restrict__ Xj, double* __restrict__ Xjm1,
                                                     double* __restrict__ Xjm2) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.S) return;
    if (commit && !commit[d.fil_susp[d.seg_fil[s]]]) return;
    const int64_t S = d.S;
    for (int i = 0; i < 3; i++) {
        Yjm1[i * S + s] = Yj[i * S + s];
        Yj[i * S + s] = Yc[i * S + s];
    }
    for (int i = 0; i < 4; i++) qj[i * S + s] = qc[i * S + s];
    for (int i = 0; i < 6; i++) {
        if (Xjm2) Xjm2[6 * s + i] = Xjm1[6 * s + i];
        Xjm1[6 * s + i] = Xj[6 * s + i];
        Xj[6 * s + i] = X[6 * s + i];
    }
}

int finalize_launch(const SimDev& d, const int32_t* commit, const double* Yc, const double* qc, const double* X,
                    double* Yj, double* Yjm1, double* qj, double* Xj, double* Xjm1, double* Xjm2, hipStream_t st) {
    if (d.S == 0) return FIL_OK;
    finalize_kernel<<<(unsigned)ceil_div(d.S, 256), 256, 0, st>>>(d, commit, Yc, qc, X, Yj, Yjm1, qj, Xj, Xjm1, Xjm2);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // namespace fil
