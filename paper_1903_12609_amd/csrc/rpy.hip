// RPY mobility apply on gfx950 (Sec. 2.7.1 of arXiv:1903.12609).
//
// Design
//   * Every (target, source) pair is visited once: the sum is split over
//     source chunks ("split-K") so that a launch has far more workgroups than
//     the 256 CUs, and the per-chunk partial (V, Omega) are reduced in a fixed
//     order by a second kernel (deterministic, no float atomics).
//   * All 64 lanes of a wave walk the same source at the same time, so the
//     source record is wave-uniform: it is read with scalar loads into SGPRs
//     and broadcast to the VALU for free.  No LDS staging is needed.
//   * Each lane owns TPL targets (register blocking amortises loop overhead).
//   * FP64 path: the cross-product terms are expanded so that per-source
//     constants (T_m x Y_m, F_m x Y_m) are precomputed:
//         sum_m s^3 T_m x (Y_n - Y_m) = (sum_m s^3 T_m) x Y_n - sum_m s^3 (T_m x Y_m)
//     which leaves 21 FMA-class accumulators per target and ~43 VALU
//     operations per pair.  The coefficient 2a^2/3 s^3 F_m of M^tt is folded
//     into the s^3 F_m accumulator, -1/2 s^3 T_m of M^rr into s^3 T_m.
//   * FP32-tile path: r = Y_n - Y_m is formed in double and rounded once, the
//     pair arithmetic runs in float and each tile of sources is accumulated in
//     float and then added into double accumulators.
//   * Overlapping pairs (r < 2a, the self pair included) take a rarely executed
//     branch with the regularised forms; the far-field weights are zeroed there.
#include "common.h"
#include "kernels.h"

namespace fil {

constexpr int kRpyBlock = 256;

// ------------------------------------------------------------------ packing
// FP64 source record: Y(3) F(3) T(3) TxY(3) FxY(3) pad -> 16 doubles (128 B)
__global__ void __launch_bounds__(256) rpy_pack_f64(int64_t S, const double* __restrict__ Y,
                                                   const double* __restrict__ F, const double* __restrict__ T,
                                                   double* __restrict__ pk) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= S) return;
    const double y0 = Y[m], y1 = Y[S + m], y2 = Y[2 * S + m];
    const double f0 = F[m], f1 = F[S + m], f2 = F[2 * S + m];
    const double t0 = T[m], t1 = T[S + m], t2 = T[2 * S + m];
    double2* o = reinterpret_cast<double2*>(pk + 16 * m);
    o[0] = make_double2(y0, y1);
    o[1] = make_double2(y2, f0);
    o[2] = make_double2(f1, f2);
    o[3] = make_double2(t0, t1);
    o[4] = make_double2(t2, t1 * y2 - t2 * y1);
    o[5] = make_double2(t2 * y0 - t0 * y2, t0 * y1 - t1 * y0);
    o[6] = make_double2(f1 * y2 - f2 * y1, f2 * y0 - f0 * y2);
    o[7] = make_double2(f0 * y1 - f1 * y0, 0.0);
}

// FP32-tile source record: position in double, force and torque in float (64 B)
struct alignas(16) SrcF32 {
    double y[3];
    float f[3];
    float t[3];
    float pad[4];
};
static_assert(sizeof(SrcF32) == 64, "SrcF32 must be 64 bytes");

__global__ void __launch_bounds__(256) rpy_pack_f32(int64_t S, const double* __restrict__ Y,
                                                   const double* __restrict__ F, const double* __restrict__ T,
                                                   SrcF32* __restrict__ pk) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= S) return;
    SrcF32 s;
    for (int i = 0; i < 3; i++) {
        s.y[i] = Y[i * S + m];
        s.f[i] = (float)F[i * S + m];
        s.t[i] = (float)T[i * S + m];
    }
    s.pad[0] = s.pad[1] = s.pad[2] = s.pad[3] = 0.f;
    pk[m] = s;
}

// ------------------------------------------------------------------ FP64 pair
struct AccF64 {
    double G[3];   // sum s F                     (M^tt, 1/r part)
    double R[3];   // sum s^3 F                   (M^tt a^2 part, M^rt)
    double P[3];   // sum s^3 T                   (M^tr, M^rr)
    double Q[3];   // sum s^3 (T x Y_m)           (M^tr)
    double U[3];   // sum s^3 (F x Y_m) - overlap Omega / c
    double Hv[3];  // sum s^3 (1 - 2a^2 s^2)(r.F) r
    double Hw[3];  // sum s^5 (r.T) r
};

// Overlap (r < 2a) contribution divided by c = 1/(8 pi eta).  Equal-radius
// regularised RPY:
//   V/c  += 4/(3a) [(1 - 9r/(32a)) F + 3/(32 a r) (r.F) r] + (1/(2a^2)) (1/a - 3r/(8a^2)) T x r
//   Om/c += 1/a^3 [(1 - 27r/(32a) + 5r^3/(64a^3)) T + (9/(32 a r) - 3r/(64a^3)) (r.T) r]
//           + (1/(2a^2)) (1/a - 3r/(8a^2)) F x r
// Returned by value so that the accumulators never leave registers.
template <typename R>
struct Ovl {
    R v[3], w[3];
};

template <typename R>
__device__ __forceinline__ Ovl<R> rpy_overlap(R rx, R ry, R rz, R r2, R Fx, R Fy, R Fz, R Tx, R Ty, R Tz, R a) {
    const R r = sqrt(r2);
    const R ir = r > R(0) ? R(1) / r : R(0);
    const R ia = R(1) / a, ia3 = ia * ia * ia;
    const R rF = rx * Fx + ry * Fy + rz * Fz, rT = rx * Tx + ry * Ty + rz * Tz;
    const R ctt1 = R(4.0 / 3.0) * ia * (R(1) - R(9.0 / 32.0) * r * ia);
    const R ctt2 = R(0.125) * ia * ia * ir;
    const R ctr = R(0.5) * ia * ia * (ia - R(0.375) * r * ia * ia);
    const R crr1 = ia3 * (R(1) - R(27.0 / 32.0) * r * ia + R(5.0 / 64.0) * r2 * r * ia3);
    const R crr2 = ia3 * (R(9.0 / 32.0) * ia * ir - R(3.0 / 64.0) * r * ia3);
    Ovl<R> o;
    o.v[0] = ctt1 * Fx + ctt2 * rF * rx + ctr * (Ty * rz - Tz * ry);
    o.v[1] = ctt1 * Fy + ctt2 * rF * ry + ctr * (Tz * rx - Tx * rz);
    o.v[2] = ctt1 * Fz + ctt2 * rF * rz + ctr * (Tx * ry - Ty * rx);
    o.w[0] = crr1 * Tx + crr2 * rT * rx + ctr * (Fy * rz - Fz * ry);
    o.w[1] = crr1 * Ty + crr2 * rT * ry + ctr * (Fz * rx - Fx * rz);
    o.w[2] = crr1 * Tz + crr2 * rT * rz + ctr * (Fx * ry - Fy * rx);
    return o;
}

__device__ __forceinline__ void rpy_pair_f64(const double y[3], const double* __restrict__ s, double a,
                                             double four_a2, double two_a2, AccF64& A) {
    const double rx = y[0] - s[0], ry = y[1] - s[1], rz = y[2] - s[2];
    const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const bool near = r2 < four_a2;
    double sv = rsqrt_f64(r2);
    sv = near ? 0.0 : sv;
    const double s2 = sv * sv, s3 = s2 * sv;
    const double Fx = s[3], Fy = s[4], Fz = s[5], Tx = s[6], Ty = s[7], Tz = s[8];
    const double rF = fma(rx, Fx, fma(ry, Fy, rz * Fz));
    const double rT = fma(rx, Tx, fma(ry, Ty, rz * Tz));
    A.G[0] = fma(sv, Fx, A.G[0]);
    A.G[1] = fma(sv, Fy, A.G[1]);
    A.G[2] = fma(sv, Fz, A.G[2]);
    A.R[0] = fma(s3, Fx, A.R[0]);
    A.R[1] = fma(s3, Fy, A.R[1]);
    A.R[2] = fma(s3, Fz, A.R[2]);
    A.P[0] = fma(s3, Tx, A.P[0]);
    A.P[1] = fma(s3, Ty, A.P[1]);
    A.P[2] = fma(s3, Tz, A.P[2]);
    A.Q[0] = fma(s3, s[9], A.Q[0]);
    A.Q[1] = fma(s3, s[10], A.Q[1]);
    A.Q[2] = fma(s3, s[11], A.Q[2]);
    A.U[0] = fma(s3, s[12], A.U[0]);
    A.U[1] = fma(s3, s[13], A.U[1]);
    A.U[2] = fma(s3, s[14], A.U[2]);
    const double Br = s3 * fma(-two_a2, s2, 1.0) * rF;
    A.Hv[0] = fma(Br, rx, A.Hv[0]);
    A.Hv[1] = fma(Br, ry, A.Hv[1]);
    A.Hv[2] = fma(Br, rz, A.Hv[2]);
    const double D = s3 * s2 * rT;
    A.Hw[0] = fma(D, rx, A.Hw[0]);
    A.Hw[1] = fma(D, ry, A.Hw[1]);
    A.Hw[2] = fma(D, rz, A.Hw[2]);
    if (near) {
        // overlap: added to G (velocity), subtracted from U (angular velocity)
        const Ovl<double> o = rpy_overlap<double>(rx, ry, rz, r2, Fx, Fy, Fz, Tx, Ty, Tz, a);
        for (int i = 0; i < 3; i++) {
            A.G[i] += o.v[i];
            A.U[i] -= o.w[i];
        }
    }
}

// Output addressing shared by both precisions.  With K > 1 each chunk k writes
// its partial (V, Omega) to part[(k*6 + c) * S + n]; with K == 1 directly V, W.
struct RpyOut {
    double* part;
    double* V;
    double* W;
};

__device__ __forceinline__ void rpy_store(const RpyOut& o, int64_t S, int K, int k, int64_t n, const double v[3],
                                          const double w[3]) {
    if (K == 1) {
        for (int i = 0; i < 3; i++) {
            o.V[i * S + n] = v[i];
            o.W[i * S + n] = w[i];
        }
    } else {
        double* p = o.part + (int64_t)k * 6 * S + n;
        for (int i = 0; i < 3; i++) {
            p[i * S] = v[i];
            p[(3 + i) * S] = w[i];
        }
    }
}

// blockIdx.x -> (target block tb = bid / K, source chunk k = bid % K); chunks
// adjacent in k land on different XCDs, so each XCD's L2 holds ~K/8 chunks.
template <int TPL>
__global__ void __launch_bounds__(kRpyBlock) rpy_f64_kernel(int64_t S, int64_t chunk, int K,
                                                          const double* __restrict__ pk,
                                                          const double* __restrict__ Y, double a, double c,
                                                          RpyOut out) {
    const int k = (int)(blockIdx.x % (unsigned)K);
    const int64_t tb = blockIdx.x / (unsigned)K;
    const int64_t m0 = (int64_t)k * chunk;
    const int64_t m1 = min(S, m0 + chunk);
    const double four_a2 = 4.0 * a * a, two_a2 = 2.0 * a * a;
    int64_t n[TPL];
    double y[TPL][3];
    AccF64 A[TPL];
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        n[j] = tb * (kRpyBlock * TPL) + j * kRpyBlock + threadIdx.x;
        const int64_t nn = n[j] < S ? n[j] : S - 1;
        y[j][0] = Y[nn];
        y[j][1] = Y[S + nn];
        y[j][2] = Y[2 * S + nn];
        for (int i = 0; i < 3; i++)
            A[j].G[i] = A[j].R[i] = A[j].P[i] = A[j].Q[i] = A[j].U[i] = A[j].Hv[i] = A[j].Hw[i] = 0.0;
    }
    for (int64_t m = m0; m < m1; ++m) {
        const double* s = pk + 16 * m;
#pragma unroll
        for (int j = 0; j < TPL; j++) rpy_pair_f64(y[j], s, a, four_a2, two_a2, A[j]);
    }
    const double c23 = 2.0 * a * a / 3.0;
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        if (n[j] >= S) continue;
        const AccF64& B = A[j];
        const double* yy = y[j];
        double v[3], w[3];
        // V = c [G + 2a^2/3 R + Hv + P x y - Q];  Omega = c [R x y - U + 3/2 Hw - 1/2 P]
        v[0] = c * (B.G[0] + c23 * B.R[0] + B.Hv[0] + (B.P[1] * yy[2] - B.P[2] * yy[1]) - B.Q[0]);
        v[1] = c * (B.G[1] + c23 * B.R[1] + B.Hv[1] + (B.P[2] * yy[0] - B.P[0] * yy[2]) - B.Q[1]);
        v[2] = c * (B.G[2] + c23 * B.R[2] + B.Hv[2] + (B.P[0] * yy[1] - B.P[1] * yy[0]) - B.Q[2]);
        w[0] = c * ((B.R[1] * yy[2] - B.R[2] * yy[1]) - B.U[0] + 1.5 * B.Hw[0] - 0.5 * B.P[0]);
        w[1] = c * ((B.R[2] * yy[0] - B.R[0] * yy[2]) - B.U[1] + 1.5 * B.Hw[1] - 0.5 * B.P[1]);
        w[2] = c * ((B.R[0] * yy[1] - B.R[1] * yy[0]) - B.U[2] + 1.5 * B.Hw[2] - 0.5 * B.P[2]);
        rpy_store(out, S, K, k, n[j], v, w);
    }
}

// ------------------------------------------------------------------ FP32-tile pair
// Accumulates (V, Omega) / c of one pair in float.
__device__ __forceinline__ void rpy_pair_f32(const double y[3], const SrcF32* __restrict__ s, float a, float four_a2,
                                             float two_a2, float c23, float v[3], float w[3]) {
    const float rx = (float)(y[0] - s->y[0]);
    const float ry = (float)(y[1] - s->y[1]);
    const float rz = (float)(y[2] - s->y[2]);
    const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
    const bool near = r2 < four_a2;
    float sv = __builtin_amdgcn_rsqf(r2);
    sv = near ? 0.f : sv;
    const float s2 = sv * sv, s3 = s2 * sv;
    const float Fx = s->f[0], Fy = s->f[1], Fz = s->f[2], Tx = s->t[0], Ty = s->t[1], Tz = s->t[2];
    const float rF = fmaf(rx, Fx, fmaf(ry, Fy, rz * Fz));
    const float rT = fmaf(rx, Tx, fmaf(ry, Ty, rz * Tz));
    const float A = fmaf(c23, s3, sv);                 // s + 2a^2/3 s^3
    const float Br = s3 * fmaf(-two_a2, s2, 1.f) * rF;  // s^3 (1 - 2a^2 s^2) (r.F)
    const float D = 1.5f * s3 * s2 * rT;               // 3/2 s^5 (r.T)
    const float E = -0.5f * s3;
    v[0] = fmaf(A, Fx, fmaf(Br, rx, fmaf(s3, fmaf(Ty, rz, -Tz * ry), v[0])));
    v[1] = fmaf(A, Fy, fmaf(Br, ry, fmaf(s3, fmaf(Tz, rx, -Tx * rz), v[1])));
    v[2] = fmaf(A, Fz, fmaf(Br, rz, fmaf(s3, fmaf(Tx, ry, -Ty * rx), v[2])));
    w[0] = fmaf(E, Tx, fmaf(D, rx, fmaf(s3, fmaf(Fy, rz, -Fz * ry), w[0])));
    w[1] = fmaf(E, Ty, fmaf(D, ry, fmaf(s3, fmaf(Fz, rx, -Fx * rz), w[1])));
    w[2] = fmaf(E, Tz, fmaf(D, rz, fmaf(s3, fmaf(Fx, ry, -Fy * rx), w[2])));
    if (near) {
        const Ovl<float> o = rpy_overlap<float>(rx, ry, rz, r2, Fx, Fy, Fz, Tx, Ty, Tz, a);
        for (int i = 0; i < 3; i++) {
            v[i] += o.v[i];
            w[i] += o.w[i];
        }
    }
}

constexpr int kF32Tile = 64;  // sources accumulated in float before the double flush

template <int TPL>
__global__ void __launch_bounds__(kRpyBlock) rpy_f32_kernel(int64_t S, int64_t chunk, int K,
                                                          const SrcF32* __restrict__ pk,
                                                          const double* __restrict__ Y, double a, double c,
                                                          RpyOut out) {
    const int k = (int)(blockIdx.x % (unsigned)K);
    const int64_t tb = blockIdx.x / (unsigned)K;
    const int64_t m0 = (int64_t)k * chunk;
    const int64_t m1 = min(S, m0 + chunk);
    const float af = (float)a, four_a2 = (float)(4.0 * a * a), two_a2 = (float)(2.0 * a * a);
    const float c23 = (float)(2.0 * a * a / 3.0);
    int64_t n[TPL];
    double y[TPL][3], vd[TPL][3], wd[TPL][3];
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        n[j] = tb * (kRpyBlock * TPL) + j * kRpyBlock + threadIdx.x;
        const int64_t nn = n[j] < S ? n[j] : S - 1;
        for (int i = 0; i < 3; i++) {
            y[j][i] = Y[i * S + nn];
            vd[j][i] = wd[j][i] = 0.0;
        }
    }
    for (int64_t t0 = m0; t0 < m1; t0 += kF32Tile) {
        const int64_t t1 = min(m1, t0 + kF32Tile);
        float v[TPL][3], w[TPL][3];
#pragma unroll
        for (int j = 0; j < TPL; j++)
            for (int i = 0; i < 3; i++) v[j][i] = w[j][i] = 0.f;
        for (int64_t m = t0; m < t1; ++m) {
            const SrcF32* s = pk + m;
#pragma unroll
            for (int j = 0; j < TPL; j++) rpy_pair_f32(y[j], s, af, four_a2, two_a2, c23, v[j], w[j]);
        }
#pragma unroll
        for (int j = 0; j < TPL; j++)
            for (int i = 0; i < 3; i++) {
                vd[j][i] += (double)v[j][i];
                wd[j][i] += (double)w[j][i];
            }
    }
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        if (n[j] >= S) continue;
        double v[3], w[3];
        for (int i = 0; i < 3; i++) {
            v[i] = c * vd[j][i];
            w[i] = c * wd[j][i];
        }
        rpy_store(out, S, K, k, n[j], v, w);
    }
}

// Fixed-order reduction of the K partial results.
__global__ void __launch_bounds__(256) rpy_reduce(int64_t S, int K, const double* __restrict__ part,
                                                 double* __restrict__ V, double* __restrict__ W) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= S) return;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < K; k++) {
        const double* p = part + (int64_t)k * 6 * S + n;
#pragma unroll
        for (int c = 0; c < 6; c++) acc[c] += p[c * S];
    }
    for (int i = 0; i < 3; i++) {
        V[i * S + n] = acc[i];
        W[i * S + n] = acc[3 + i];
    }
}

// ------------------------------------------------------------------ launch plan
constexpr int kTplF64 = 2;
constexpr int kTplF32 = 2;

RpyPlan rpy_plan(int64_t S, int prec) {
    RpyPlan p{};
    p.S = S;
    p.prec = prec;
    p.tpl = prec == FIL_PREC_F64 ? kTplF64 : kTplF32;
    if (S <= 0) return p;
    p.tb = ceil_div(S, (int64_t)kRpyBlock * p.tpl);
    // aim for ~2048 workgroups (8 per CU), chunks of at least 64 sources
    int64_t K = ceil_div(2048, p.tb);
    K = std::min<int64_t>(K, std::max<int64_t>(1, S / 64));
    if (K >= 8) K = ceil_div(K, 8) * 8;
    p.chunk = ceil_div(S, K);
    p.K = (int)ceil_div(S, p.chunk);
    p.pack_bytes = (size_t)S * (prec == FIL_PREC_F64 ? 16 * sizeof(double) : sizeof(SrcF32));
    p.pack_bytes = (p.pack_bytes + 255) & ~(size_t)255;
    p.part_bytes = p.K > 1 ? (size_t)p.K * 6 * S * sizeof(double) : 0;
    return p;
}

int rpy_launch(const RpyPlan& p, const double* Y, const double* F, const double* T, double a, double eta, double* V,
               double* W, void* work, hipStream_t st) {
    if (p.S <= 0) return FIL_OK;
    char* base = static_cast<char*>(work);
    RpyOut out{reinterpret_cast<double*>(base + p.pack_bytes), V, W};
    const double c = 1.0 / (8.0 * kPi * eta);
    const unsigned grid = (unsigned)(p.tb * p.K);
    const unsigned pgrid = (unsigned)ceil_div(p.S, 256);
    if (p.prec == FIL_PREC_F64) {
        double* pk = reinterpret_cast<double*>(base);
        rpy_pack_f64<<<pgrid, 256, 0, st>>>(p.S, Y, F, T, pk);
        rpy_f64_kernel<kTplF64><<<grid, kRpyBlock, 0, st>>>(p.S, p.chunk, p.K, pk, Y, a, c, out);
    } else {
        SrcF32* pk = reinterpret_cast<SrcF32*>(base);
        rpy_pack_f32<<<pgrid, 256, 0, st>>>(p.S, Y, F, T, pk);
        rpy_f32_kernel<kTplF32><<<grid, kRpyBlock, 0, st>>>(p.S, p.chunk, p.K, pk, Y, a, c, out);
    }
    if (p.K > 1) rpy_reduce<<<pgrid, 256, 0, st>>>(p.S, p.K, out.part, V, W);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // namespace fil
