// RPY mobility of equal spheres above a no-slip plane wall z = 0 (the half-space tensor
// the paper uses for its cilia, Sec. 2.7.1 and Sec. 5.2.2): the free-space RPY blocks of
// every pair (with the regularised overlap forms for r < 2a) plus the wall's image part,
// Blake's image system under the Faxen operators of both spheres (wall_image.h, generated
// by gen_wall_image.py).  Self terms: 1/(6 pi eta a) I, 1/(8 pi eta a^3) I plus the image
// part at coincident points.
//
// FP64, one thread per target, sources staged through LDS in tiles; the source range is
// split into K chunks when there are too few targets to fill the chip, the partial sums
// then added in chunk order by a second kernel (deterministic).
#include <cmath>

#include "common.h"
#include "wall_image.h"

namespace fil {

constexpr int kWallBlock = 64;  // targets per workgroup, also the source tile

struct WallArgs {
    int64_t S;
    const double *Y, *F, *T;
    double a, eta;
};

// per-launch constants of the free-space blocks
struct FreeConst {
    double a2, ia, c8, c16, c6a, c8a3, c16a2;
};

__device__ __forceinline__ FreeConst free_const(double a, double eta) {
    FreeConst k;
    k.a2 = a * a;
    k.ia = 1.0 / a;
    k.c8 = 1.0 / (8.0 * kPi * eta);
    k.c16 = 0.5 * k.c8;
    k.c6a = 1.0 / (6.0 * kPi * eta * a);
    k.c8a3 = k.c8 * k.ia * k.ia * k.ia;
    k.c16a2 = k.c16 * k.ia * k.ia;
    return k;
}

// free-space RPY blocks of the pair with separation r = target - source (not the self pair)
__device__ __forceinline__ void free_pair(double rx, double ry, double rz, double a, const FreeConst& k,
                                          const double* Fm, const double* Tm, double* v, double* w) {
    const double d2 = rx * rx + ry * ry + rz * rz;
    const double id = 1.0 / sqrt(d2);
    const double d = d2 * id;
    const double hx = rx * id, hy = ry * id, hz = rz * id;
    double ctt_i, ctt_r, crr_i, crr_r, ctr;
    if (d >= 2.0 * a) {
        const double id2 = id * id;
        const double c = k.c8 * id;
        ctt_i = c * (1.0 + (2.0 / 3.0) * k.a2 * id2);
        ctt_r = c * (1.0 - 2.0 * k.a2 * id2);
        crr_i = -k.c16 * id2 * id;
        crr_r = 3.0 * k.c16 * id2 * id;
        ctr = k.c8 * id2;
    } else {
        const double x = d * k.ia;
        ctt_i = (1.0 - (9.0 / 32.0) * x) * k.c6a;
        ctt_r = ((3.0 / 32.0) * x) * k.c6a;
        crr_i = (1.0 - (27.0 / 32.0) * x + (5.0 / 64.0) * x * x * x) * k.c8a3;
        crr_r = ((9.0 / 32.0) * x - (3.0 / 64.0) * x * x * x) * k.c8a3;
        ctr = (x - 0.375 * x * x) * k.c16a2;
    }
    const double hF = hx * Fm[0] + hy * Fm[1] + hz * Fm[2];
    const double hT = hx * Tm[0] + hy * Tm[1] + hz * Tm[2];
    // V += ctt F + ctr T x rhat,  W += crr T + ctr F x rhat
    v[0] += ctt_i * Fm[0] + ctt_r * hF * hx + ctr * (Tm[1] * hz - Tm[2] * hy);
    v[1] += ctt_i * Fm[1] + ctt_r * hF * hy + ctr * (Tm[2] * hx - Tm[0] * hz);
    v[2] += ctt_i * Fm[2] + ctt_r * hF * hz + ctr * (Tm[0] * hy - Tm[1] * hx);
    w[0] += crr_i * Tm[0] + crr_r * hT * hx + ctr * (Fm[1] * hz - Fm[2] * hy);
    w[1] += crr_i * Tm[1] + crr_r * hT * hy + ctr * (Fm[2] * hx - Fm[0] * hz);
    w[2] += crr_i * Tm[2] + crr_r * hT * hz + ctr * (Fm[0] * hy - Fm[1] * hx);
}

// grid: (target blocks, K source chunks); out: [K][6][S] partials, or V/W when K == 1
__global__ void __launch_bounds__(kWallBlock) rpy_wall_kernel(WallArgs g, int64_t chunk, double* __restrict__ part,
                                                              double* __restrict__ V, double* __restrict__ W) {
    __shared__ double sy[3][kWallBlock], sf[3][kWallBlock], st[3][kWallBlock];
    const int64_t S = g.S;
    const int64_t n = (int64_t)blockIdx.x * kWallBlock + threadIdx.x;
    const bool valid = n < S;
    const int64_t nn = valid ? n : S - 1;
    const double x0 = g.Y[nn], x1 = g.Y[S + nn], x2 = g.Y[2 * S + nn];
    const int64_t m0 = (int64_t)blockIdx.y * chunk;
    const int64_t m1 = m0 + chunk < S ? m0 + chunk : S;
    double v[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    double vi[3] = {0, 0, 0}, wi[3] = {0, 0, 0};  // image part, scaled by 1/(8 pi eta) at the end
    const FreeConst kc = free_const(g.a, g.eta);
    for (int64_t t0 = m0; t0 < m1; t0 += kWallBlock) {
        __syncthreads();
        const int64_t m = t0 + threadIdx.x;
        if (m < m1)
            for (int c = 0; c < 3; c++) {
                sy[c][threadIdx.x] = g.Y[c * S + m];
                sf[c][threadIdx.x] = g.F[c * S + m];
                st[c][threadIdx.x] = g.T[c * S + m];
            }
        __syncthreads();
        const int cnt = (int)(m1 - t0 < kWallBlock ? m1 - t0 : kWallBlock);
        for (int q = 0; q < cnt; q++) {
            const double Fm[3] = {sf[0][q], sf[1][q], sf[2][q]};
            const double Tm[3] = {st[0][q], st[1][q], st[2][q]};
            const double y0 = sy[0][q], y1 = sy[1][q], y2 = sy[2][q];
            if (t0 + q == nn) {
                for (int c = 0; c < 3; c++) {
                    v[c] += kc.c6a * Fm[c];
                    w[c] += kc.c8a3 * Tm[c];
                }
            } else {
                free_pair(x0 - y0, x1 - y1, x2 - y2, g.a, kc, Fm, Tm, v, w);
            }
            double tt[3][3], tr[3][3], rt[3][3], rr[3][3];
            const double Rx = x0 - y0, Ry = x1 - y1, Rz = x2 + y2;
            wall_image_blocks(Rx, Ry, Rz, 1.0 / sqrt(Rx * Rx + Ry * Ry + Rz * Rz), y2, g.a, tt, tr, rt, rr);
            for (int i = 0; i < 3; i++) {
                vi[i] += tt[i][0] * Fm[0] + tt[i][1] * Fm[1] + tt[i][2] * Fm[2] + tr[i][0] * Tm[0] + tr[i][1] * Tm[1] +
                         tr[i][2] * Tm[2];
                wi[i] += rt[i][0] * Fm[0] + rt[i][1] * Fm[1] + rt[i][2] * Fm[2] + rr[i][0] * Tm[0] + rr[i][1] * Tm[1] +
                         rr[i][2] * Tm[2];
            }
        }
    }
    if (!valid) return;
    double out[6];
    for (int c = 0; c < 3; c++) {
        out[c] = v[c] + kc.c8 * vi[c];
        out[3 + c] = w[c] + kc.c8 * wi[c];
    }
    if (part) {
        double* p = part + (int64_t)blockIdx.y * 6 * S;
        for (int c = 0; c < 6; c++) p[c * S + n] = out[c];
    } else {
        for (int c = 0; c < 3; c++) {
            V[c * S + n] = out[c];
            W[c * S + n] = out[3 + c];
        }
    }
}

__global__ void __launch_bounds__(256) rpy_wall_sum_kernel(int64_t S, int K, const double* __restrict__ part,
                                                           double* __restrict__ V, double* __restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= 6 * S) return;
    double s = 0.0;
    for (int k = 0; k < K; k++) s += part[(int64_t)k * 6 * S + e];
    const int64_t c = e / S, n = e - c * S;
    if (c < 3) V[c * S + n] = s;
    else W[(c - 3) * S + n] = s;
}

// source chunks: about 4096 single-wave workgroups (the kernel holds one wave per SIMD,
// 1024 SIMDs), chunks of at least 16 sources, at most 256 chunks.  A chunk past the end
// of the sources is empty and writes zeros.
int wall_chunks(int64_t S) {
    const int64_t tb = ceil_div(S, (int64_t)kWallBlock);
    int64_t K = ceil_div((int64_t)4096, tb);
    const int64_t maxK = ceil_div(S, (int64_t)16);
    if (K > maxK) K = maxK;
    if (K > 256) K = 256;
    return (int)(K < 1 ? 1 : K);
}

int64_t wall_workspace_bytes(int64_t S) {
    const int K = wall_chunks(S);
    return K > 1 ? (int64_t)K * 6 * S * (int64_t)sizeof(double) : 0;
}

int rpy_wall_launch(int64_t S, const double* Y, const double* F, const double* T, double a, double eta, double* V,
                    double* W, void* work, hipStream_t st) {
    if (S <= 0) return FIL_OK;
    const int K = wall_chunks(S);
    const int64_t chunk = ceil_div(S, (int64_t)K);
    const WallArgs g{S, Y, F, T, a, eta};
    dim3 grid((unsigned)ceil_div(S, (int64_t)kWallBlock), (unsigned)K);
    double* part = K > 1 ? static_cast<double*>(work) : nullptr;
    rpy_wall_kernel<<<grid, kWallBlock, 0, st>>>(g, chunk, part, V, W);
    if (K > 1)
        rpy_wall_sum_kernel<<<(unsigned)ceil_div(6 * S, (int64_t)256), 256, 0, st>>>(S, K, part, V, W);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // namespace fil

using namespace fil;

extern "C" {

int64_t fil_rpy_wall_workspace_bytes(int64_t S) { return S > 0 ? wall_workspace_bytes(S) : 0; }

int fil_rpy_wall_apply(int64_t S, const double* Y, const double* F, const double* T, double a, double eta, double* V,
                       double* Omega, void* work, int64_t work_bytes, void* stream) {
    FIL_CHECK_ARG(S >= 0, "fil_rpy_wall_apply: S < 0");
    if (S == 0) return FIL_OK;
    FIL_CHECK_ARG(Y && F && T && V && Omega, "fil_rpy_wall_apply: null array");
    FIL_CHECK_ARG(std::isfinite(a) && a > 0 && std::isfinite(eta) && eta > 0, "fil_rpy_wall_apply: a and eta must be > 0");
    FIL_CHECK_ARG(V != Omega && V != Y && V != F && V != T && Omega != Y && Omega != F && Omega != T,
                  "fil_rpy_wall_apply: outputs alias inputs");
    const int64_t need = wall_workspace_bytes(S);
    FIL_CHECK_ARG(work_bytes >= need && (need == 0 || work), "fil_rpy_wall_apply: workspace too small");
    return rpy_wall_launch(S, Y, F, T, a, eta, V, Omega, work, (hipStream_t)stream);
}

}  // extern "C"
