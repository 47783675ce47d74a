// Force-coupling-method mobility (Sec. 2.7.2) on a periodic grid:
//   f(x) = sum_m F_m Delta_m(x) - 1/2 sum_m T_m x grad Theta_m(x)   (Gaussians of widths
//   sigma_D = a / sqrt(pi), sigma_T = a / (6 sqrt(pi))^(1/3), truncated at cut * sigma),
//   u_k = (I - k k^T / k^2) f_k / (eta k^2) (u_0 = 0; the Nyquist planes of even axes
//   dropped, where the spectral derivative of a real field is undefined),
//   V_n = sum_grid u Delta_n dV  (trapezoidal rule),
//   Omega_n = 1/2 int (curl u) Theta_n dV = 1/2 int u x grad Theta_n dV
//           = 1/2 sum_grid (r x u) Theta_n / sigma_T^2 dV,  r = x - Y_n,
//   the vorticity average integrated by parts over the periodic box: only the three
//   velocity components are transformed back, and the averaging is the exact adjoint of
//   the rotlet spreading (a symmetric discrete mobility).  It differs from averaging the
//   spectral vorticity by the grid's discretisation error, which falls spectrally with
//   the spacing (below 1e-9 of the rotation at h = 0.3a).
// Spreading adds each segment's Gaussian into the grid with atomics (one workgroup per
// segment, the separable 1D factors in LDS); the transforms are hipFFT's; averaging is a
// gather, one workgroup per segment, summed in a fixed order.
#include <hipfft/hipfft.h>

#include <cmath>
#include <vector>

#include "common.h"

namespace fil {

constexpr int kFcmBlock = 256;
constexpr int kFcmMaxP = 32;  // support half-width in grid points per axis at most

struct FcmGrid {
    int n[3];
    int P[3];      // support half-width per axis: ceil(cut sigma_D / h)
    double L[3], h[3];
    double sD, sT, cut, eta;
    int64_t N, Nc;  // real and complex (half-spectrum) points per field
};

// 1D factors of one segment: offsets o in [-P, P] along each axis, grid index and the
// distance of that node from the segment (the nearest image: the support is smaller
// than the box)
struct Factors1D {
    int idx[3][2 * kFcmMaxP + 1];
    double d[3][2 * kFcmMaxP + 1];
    double eD[3][2 * kFcmMaxP + 1];
    double eT[3][2 * kFcmMaxP + 1];
};

__device__ void fcm_factors(const FcmGrid& g, const double y[3], Factors1D& fa) {
    for (int e = threadIdx.x; e < 3 * (2 * kFcmMaxP + 1); e += blockDim.x) {
        const int c = e / (2 * kFcmMaxP + 1), o = e % (2 * kFcmMaxP + 1) - kFcmMaxP;
        if (o < -g.P[c] || o > g.P[c]) continue;
        const double yw = y[c] - g.L[c] * floor(y[c] / g.L[c]);  // wrapped into [0, L)
        const int i0 = (int)floor(yw / g.h[c]);
        int i = i0 + o;
        const double dist = (double)i * g.h[c] - yw;
        i %= g.n[c];
        if (i < 0) i += g.n[c];
        fa.idx[c][o + kFcmMaxP] = i;
        fa.d[c][o + kFcmMaxP] = dist;
        fa.eD[c][o + kFcmMaxP] = exp(-dist * dist / (2.0 * g.sD * g.sD));
        fa.eT[c][o + kFcmMaxP] = exp(-dist * dist / (2.0 * g.sT * g.sT));
    }
}

__global__ void __launch_bounds__(kFcmBlock) fcm_spread_kernel(FcmGrid g, int64_t S, const double* __restrict__ Y,
                                                               const double* __restrict__ F,
                                                               const double* __restrict__ T,
                                                               double* __restrict__ f) {
    const int64_t m = blockIdx.x;
    __shared__ Factors1D fa;
    const double y[3] = {Y[m], Y[S + m], Y[2 * S + m]};
    fcm_factors(g, y, fa);
    __syncthreads();
    const double Fm[3] = {F[m], F[S + m], F[2 * S + m]};
    const double Tm[3] = {T[m], T[S + m], T[2 * S + m]};
    const double nD = pow(2.0 * kPi * g.sD * g.sD, -1.5), nT = pow(2.0 * kPi * g.sT * g.sT, -1.5);
    const double rcD = g.cut * g.sD * g.cut * g.sD, rcT = g.cut * g.sT * g.cut * g.sT;
    const double half_isT2 = 0.5 / (g.sT * g.sT);
    const int wx = 2 * g.P[0] + 1, wy = 2 * g.P[1] + 1, wz = 2 * g.P[2] + 1;
    const int np = wx * wy * wz;
    for (int p = threadIdx.x; p < np; p += kFcmBlock) {
        const int ox = p / (wy * wz), r_ = p - ox * wy * wz, oy = r_ / wz, oz = r_ - oy * wz;
        const int ax = ox - g.P[0] + kFcmMaxP, ay = oy - g.P[1] + kFcmMaxP, az = oz - g.P[2] + kFcmMaxP;
        const double rx = fa.d[0][ax], ry = fa.d[1][ay], rz = fa.d[2][az];
        const double r2 = rx * rx + ry * ry + rz * rz;
        if (r2 >= rcD) continue;  // sigma_T < sigma_D: outside both supports
        const double gD = nD * fa.eD[0][ax] * fa.eD[1][ay] * fa.eD[2][az];
        double c[3] = {Fm[0] * gD, Fm[1] * gD, Fm[2] * gD};
        if (r2 < rcT) {
            // -1/2 T x grad Theta = 1/2 (T x r) Theta / sigma_T^2
            const double s = nT * fa.eT[0][ax] * fa.eT[1][ay] * fa.eT[2][az] * half_isT2;
            c[0] += s * (Tm[1] * rz - Tm[2] * ry);
            c[1] += s * (Tm[2] * rx - Tm[0] * rz);
            c[2] += s * (Tm[0] * ry - Tm[1] * rx);
        }
        const int64_t gi = ((int64_t)fa.idx[0][ax] * g.n[1] + fa.idx[1][ay]) * g.n[2] + fa.idx[2][az];
        atomicAdd(&f[gi], c[0]);
        atomicAdd(&f[g.N + gi], c[1]);
        atomicAdd(&f[2 * g.N + gi], c[2]);
    }
}

__global__ void __launch_bounds__(kFcmBlock) fcm_zero_kernel(int64_t n, double* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * kFcmBlock + threadIdx.x;
    if (i < n) f[i] = 0.0;
}

// Fourier space: fk [3][Nc] -> uk [3][Nc], scaled by 1/N for the unnormalised inverse
// transform
__global__ void __launch_bounds__(kFcmBlock) fcm_solve_kernel(FcmGrid g, const hipfftDoubleComplex* __restrict__ fk,
                                                              hipfftDoubleComplex* __restrict__ uk) {
    const int64_t e = (int64_t)blockIdx.x * kFcmBlock + threadIdx.x;
    if (e >= g.Nc) return;
    const int nzc = g.n[2] / 2 + 1;
    const int ix = (int)(e / ((int64_t)g.n[1] * nzc));
    const int rem = (int)(e - (int64_t)ix * g.n[1] * nzc);
    const int iy = rem / nzc, iz = rem - iy * nzc;
    const int mi[3] = {ix <= g.n[0] / 2 ? ix : ix - g.n[0], iy <= g.n[1] / 2 ? iy : iy - g.n[1], iz};
    bool drop = ix == 0 && iy == 0 && iz == 0;
    for (int c = 0; c < 3; c++) {
        const int idx = c == 0 ? ix : (c == 1 ? iy : iz);
        drop |= (g.n[c] % 2 == 0) && idx == g.n[c] / 2;
    }
    double k[3];
    for (int c = 0; c < 3; c++) k[c] = 2.0 * kPi * (double)mi[c] / g.L[c];
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    double ur[3] = {0, 0, 0}, ui[3] = {0, 0, 0};
    if (!drop) {
        const hipfftDoubleComplex f0 = fk[e], f1 = fk[g.Nc + e], f2 = fk[2 * g.Nc + e];
        const double fr[3] = {f0.x, f1.x, f2.x}, fi[3] = {f0.y, f1.y, f2.y};
        const double kfr = k[0] * fr[0] + k[1] * fr[1] + k[2] * fr[2];
        const double kfi = k[0] * fi[0] + k[1] * fi[1] + k[2] * fi[2];
        const double sc = 1.0 / (g.eta * k2 * (double)g.N);
        for (int c = 0; c < 3; c++) {
            ur[c] = (fr[c] - k[c] * kfr / k2) * sc;
            ui[c] = (fi[c] - k[c] * kfi / k2) * sc;
        }
    }
    for (int c = 0; c < 3; c++) uk[c * g.Nc + e] = hipfftDoubleComplex{ur[c], ui[c]};
}

// V_n = sum u Delta_n dV, Omega_n = 1/2 sum (r x u) Theta_n / sigma_T^2 dV; u [3][N]
__global__ void __launch_bounds__(kFcmBlock) fcm_average_kernel(FcmGrid g, int64_t S, const double* __restrict__ Y,
                                                                const double* __restrict__ u, double* __restrict__ V,
                                                                double* __restrict__ W) {
    const int64_t m = blockIdx.x;
    __shared__ Factors1D fa;
    __shared__ double red[6][kFcmBlock];
    const double y[3] = {Y[m], Y[S + m], Y[2 * S + m]};
    fcm_factors(g, y, fa);
    __syncthreads();
    const double nD = pow(2.0 * kPi * g.sD * g.sD, -1.5), nT = pow(2.0 * kPi * g.sT * g.sT, -1.5);
    const double rcD = g.cut * g.sD * g.cut * g.sD, rcT = g.cut * g.sT * g.cut * g.sT;
    const int wx = 2 * g.P[0] + 1, wy = 2 * g.P[1] + 1, wz = 2 * g.P[2] + 1;
    const int np = wx * wy * wz;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int p = threadIdx.x; p < np; p += kFcmBlock) {
        const int ox = p / (wy * wz), r_ = p - ox * wy * wz, oy = r_ / wz, oz = r_ - oy * wz;
        const int ax = ox - g.P[0] + kFcmMaxP, ay = oy - g.P[1] + kFcmMaxP, az = oz - g.P[2] + kFcmMaxP;
        const double rx = fa.d[0][ax], ry = fa.d[1][ay], rz = fa.d[2][az];
        const double r2 = rx * rx + ry * ry + rz * rz;
        if (r2 >= rcD) continue;
        const int64_t gi = ((int64_t)fa.idx[0][ax] * g.n[1] + fa.idx[1][ay]) * g.n[2] + fa.idx[2][az];
        const double gD = nD * fa.eD[0][ax] * fa.eD[1][ay] * fa.eD[2][az];
        const double u0 = u[gi], u1 = u[g.N + gi], u2 = u[2 * g.N + gi];
        acc[0] = fma(u0, gD, acc[0]);
        acc[1] = fma(u1, gD, acc[1]);
        acc[2] = fma(u2, gD, acc[2]);
        if (r2 < rcT) {
            const double gT = nT * fa.eT[0][ax] * fa.eT[1][ay] * fa.eT[2][az];
            acc[3] = fma(ry * u2 - rz * u1, gT, acc[3]);
            acc[4] = fma(rz * u0 - rx * u2, gT, acc[4]);
            acc[5] = fma(rx * u1 - ry * u0, gT, acc[5]);
        }
    }
    for (int c = 0; c < 6; c++) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    // fixed-order tree over the block
    for (int w = kFcmBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 6; c++) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double dv = g.h[0] * g.h[1] * g.h[2];
        const double wsc = 0.5 * dv / (g.sT * g.sT);
        for (int c = 0; c < 3; c++) {
            V[c * S + m] = red[c][0] * dv;
            W[c * S + m] = red[3 + c][0] * wsc;
        }
    }
}

}  // namespace fil

using namespace fil;

struct fil_fcm {
    FcmGrid g{};
    hipfftHandle fwd = 0, inv = 0;
    bool fwd_ok = false, inv_ok = false;
    double* f = nullptr;                  // [3][N] body force
    hipfftDoubleComplex* fk = nullptr;    // [3][Nc]
    hipfftDoubleComplex* uk = nullptr;    // [3][Nc]
    double* u = nullptr;                  // [3][N] velocity
};

namespace {

void fcm_free(fil_fcm* s) {
    if (!s) return;
    if (s->fwd_ok) (void)hipfftDestroy(s->fwd);
    if (s->inv_ok) (void)hipfftDestroy(s->inv);
    for (void* p : {(void*)s->f, (void*)s->fk, (void*)s->uk, (void*)s->u})
        if (p) (void)hipFree(p);
    delete s;
}

}  // namespace

extern "C" {

int fil_fcm_create(const double* box, const int32_t* grid, double a, double eta, double cut, fil_fcm** out) {
    FIL_CHECK_ARG(out, "fil_fcm_create: null output");
    *out = nullptr;
    FIL_CHECK_ARG(box && grid, "fil_fcm_create: null box or grid");
    FIL_CHECK_ARG(std::isfinite(a) && a > 0 && std::isfinite(eta) && eta > 0, "fil_fcm_create: a and eta must be > 0");
    FIL_CHECK_ARG(std::isfinite(cut) && cut >= 2.0 && cut <= 12.0, "fil_fcm_create: cut must be in [2, 12] widths");
    fil_fcm* s = new fil_fcm();
    FcmGrid& g = s->g;
    g.sD = a / std::sqrt(kPi);
    g.sT = a / std::cbrt(6.0 * std::sqrt(kPi));
    g.cut = cut;
    g.eta = eta;
    for (int c = 0; c < 3; c++) {
        g.n[c] = grid[c];
        g.L[c] = box[c];
        if (!(grid[c] >= 4 && grid[c] <= 4096 && std::isfinite(box[c]) && box[c] > 0)) {
            fcm_free(s);
            set_error("fil_fcm_create: grid sizes in [4, 4096] and box lengths > 0");
            return FIL_EINVAL;
        }
        g.h[c] = box[c] / grid[c];
        g.P[c] = (int)std::ceil(cut * g.sD / g.h[c]);
        if (g.P[c] > kFcmMaxP || 2 * g.P[c] + 1 > g.n[c]) {
            fcm_free(s);
            set_error("fil_fcm_create: the Gaussian support (cut * sigma_D) must span at most 65 grid points per axis "
                      "and fit in the grid");
            return FIL_EINVAL;
        }
    }
    g.N = (int64_t)g.n[0] * g.n[1] * g.n[2];
    g.Nc = (int64_t)g.n[0] * g.n[1] * (g.n[2] / 2 + 1);
    if (hipMalloc(&s->f, 3 * g.N * sizeof(double)) != hipSuccess ||
        hipMalloc(&s->fk, 3 * g.Nc * sizeof(hipfftDoubleComplex)) != hipSuccess ||
        hipMalloc(&s->uk, 3 * g.Nc * sizeof(hipfftDoubleComplex)) != hipSuccess ||
        hipMalloc(&s->u, 3 * g.N * sizeof(double)) != hipSuccess) {
        fcm_free(s);
        set_error("fil_fcm_create: device allocation of the grids failed");
        return FIL_ENOMEM;
    }
    int n[3] = {g.n[0], g.n[1], g.n[2]};
    if (hipfftPlanMany(&s->fwd, 3, n, nullptr, 1, (int)g.N, nullptr, 1, (int)g.Nc, HIPFFT_D2Z, 3) != HIPFFT_SUCCESS) {
        fcm_free(s);
        set_error("fil_fcm_create: hipFFT forward plan failed");
        return FIL_EHIP;
    }
    s->fwd_ok = true;
    if (hipfftPlanMany(&s->inv, 3, n, nullptr, 1, (int)g.Nc, nullptr, 1, (int)g.N, HIPFFT_Z2D, 3) != HIPFFT_SUCCESS) {
        fcm_free(s);
        set_error("fil_fcm_create: hipFFT inverse plan failed");
        return FIL_EHIP;
    }
    s->inv_ok = true;
    *out = s;
    return FIL_OK;
}

void fil_fcm_destroy(fil_fcm* s) { fcm_free(s); }

int fil_fcm_apply(fil_fcm* s, int64_t S, const double* Y, const double* F, const double* T, double* V, double* Omega,
                  void* stream) {
    FIL_CHECK_ARG(s, "fil_fcm_apply: null handle");
    FIL_CHECK_ARG(S >= 0, "fil_fcm_apply: S < 0");
    if (S == 0) return FIL_OK;
    FIL_CHECK_ARG(Y && F && T && V && Omega, "fil_fcm_apply: null array");
    FIL_CHECK_ARG(V != Omega && V != Y && V != F && V != T && Omega != Y && Omega != F && Omega != T,
                  "fil_fcm_apply: outputs alias inputs");
    hipStream_t st = (hipStream_t)stream;
    const FcmGrid& g = s->g;
    // cleared by a kernel (not a memset node) so that the apply can be captured
    fcm_zero_kernel<<<(unsigned)ceil_div(3 * g.N, (int64_t)kFcmBlock), kFcmBlock, 0, st>>>(3 * g.N, s->f);
    fcm_spread_kernel<<<(unsigned)S, kFcmBlock, 0, st>>>(g, S, Y, F, T, s->f);
    FIL_HIP_TRY(hipGetLastError());
    if (hipfftSetStream(s->fwd, st) != HIPFFT_SUCCESS || hipfftExecD2Z(s->fwd, s->f, s->fk) != HIPFFT_SUCCESS) {
        set_error("fil_fcm_apply: forward transform failed");
        return FIL_EHIP;
    }
    fcm_solve_kernel<<<(unsigned)ceil_div(g.Nc, (int64_t)kFcmBlock), kFcmBlock, 0, st>>>(g, s->fk, s->uk);
    FIL_HIP_TRY(hipGetLastError());
    if (hipfftSetStream(s->inv, st) != HIPFFT_SUCCESS || hipfftExecZ2D(s->inv, s->uk, s->u) != HIPFFT_SUCCESS) {
        set_error("fil_fcm_apply: inverse transform failed");
        return FIL_EHIP;
    }
    fcm_average_kernel<<<(unsigned)S, kFcmBlock, 0, st>>>(g, S, Y, s->u, V, Omega);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // extern "C"
