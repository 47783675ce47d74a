// Vector kernels of the Jacobian-free Newton-Krylov solve (Sec. 3.1: Newton steps whose
// linear systems are solved by GMRES with the Jacobian-vector products taken by finite
// differences of the residual), and the product with the block-diagonal J0^{-1}
// (Sec. 3.2.2) used as its left preconditioner.  Every sum runs in a fixed order, so
// a solve is reproducible run to run.
#include "common.h"
#include "solver.h"

namespace fil {

constexpr int kKryBlock = 256;
constexpr int kKryChunk = kKryBlock * 8;  // elements per block of a dot product

// sum over a 256-thread block in a fixed order (wave trees, then the four waves in order)
__device__ __forceinline__ double block_sum_256(double v) {
    __shared__ double wsum[kKryBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) wsum[wave] = v;
    __syncthreads();
    return (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// partial[j][b] = sum over chunk b of V_j[i] w[i]  (grid: chunks x vectors)
__global__ void __launch_bounds__(kKryBlock) multi_dot_partial_kernel(int64_t n, const double* __restrict__ V,
                                                                      int64_t ldv, const double* __restrict__ w,
                                                                      double* __restrict__ partial) {
    const int64_t b = blockIdx.x, j = blockIdx.y, nb = gridDim.x;
    const double* vj = V + j * ldv;
    const int64_t i0 = b * kKryChunk;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < kKryChunk / kKryBlock; e++) {
        const int64_t i = i0 + e * kKryBlock + threadIdx.x;
        if (i < n) acc = fma(vj[i], w[i], acc);
    }
    acc = block_sum_256(acc);
    if (threadIdx.x == 0) partial[j * nb + b] = acc;
}

// out[j] = sum_b partial[j][b] in chunk order (one wave per vector)
__global__ void __launch_bounds__(64) multi_dot_finish_kernel(int nb, const double* __restrict__ partial,
                                                              double* __restrict__ out) {
    const int j = blockIdx.x;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; b++) s += partial[(int64_t)j * nb + b];
        out[j] = s;
    }
}

// w += sign * sum_j coef[j] V_j  (the terms summed in j order per element)
__global__ void __launch_bounds__(kKryBlock) multi_axpy_kernel(int64_t n, int k, const double* __restrict__ V,
                                                               int64_t ldv, const double* __restrict__ coef,
                                                               double sign, double* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * kKryBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; j++) s = fma(coef[j], V[(int64_t)j * ldv + i], s);
    w[i] = fma(sign, s, w[i]);
}

// out = a x + b y  (y may be null: out = a x)
__global__ void __launch_bounds__(kKryBlock) axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                                                          const double* __restrict__ y, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kKryBlock + threadIdx.x;
    if (i >= n) return;
    out[i] = y ? fma(a, x[i], b * y[i]) : a * x[i];
}

// out = d * x elementwise
__global__ void __launch_bounds__(kKryBlock) mul_kernel(int64_t n, const double* __restrict__ d,
                                                        const double* __restrict__ x, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kKryBlock + threadIdx.x;
    if (i < n) out[i] = d[i] * x[i];
}

// y = J0^{-1} w with the explicit per-filament inverses: AinvT holds row c of
// J0_f^{-T} at dense_off[f] + c n, so y_i = sum_c AinvT[c][i] w_c (c in order)
__global__ void __launch_bounds__(kKryBlock) j0_apply_kernel(SimDev d, const double* __restrict__ AinvT,
                                                             const double* __restrict__ w, double* __restrict__ y) {
    const int64_t f = blockIdx.x;
    const int64_t e0 = 6 * d.seg_off[f];
    const int n = (int)(6 * (d.seg_off[f + 1] - d.seg_off[f]));
    const double* A = AinvT + d.dense_off[f];
    __shared__ double sw[6 * kMaxSeg];
    for (int c = threadIdx.x; c < n; c += kKryBlock) sw[c] = w[e0 + c];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kKryBlock) {
        double s = 0.0;
        for (int c = 0; c < n; c++) s = fma(A[(int64_t)c * n + i], sw[c], s);
        y[e0 + i] = s;
    }
}

// the drag-only mobility of f0 (Sec. 3.2.1): V = F / (6 pi eta a), W = T / (8 pi eta a^3)
__global__ void __launch_bounds__(kKryBlock) diag_mobility_kernel(int64_t n3, double ct, double cr,
                                                                  const double* __restrict__ F,
                                                                  const double* __restrict__ T,
                                                                  double* __restrict__ V, double* __restrict__ W) {
    const int64_t i = (int64_t)blockIdx.x * kKryBlock + threadIdx.x;
    if (i >= n3) return;
    V[i] = ct * F[i];
    W[i] = cr * T[i];
}

static unsigned blocks_for(int64_t n) { return (unsigned)ceil_div(n, (int64_t)kKryBlock); }

int multi_dot_launch(int64_t n, const double* V, int64_t ldv, int k, const double* w, double* partial, double* out,
                     hipStream_t st) {
    if (k <= 0) return FIL_OK;
    const int nb = (int)ceil_div(n, (int64_t)kKryChunk);
    multi_dot_partial_kernel<<<dim3((unsigned)nb, (unsigned)k), kKryBlock, 0, st>>>(n, V, ldv, w, partial);
    multi_dot_finish_kernel<<<(unsigned)k, 64, 0, st>>>(nb, partial, out);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

size_t multi_dot_partial_count(int64_t n, int k) { return (size_t)ceil_div(n, (int64_t)kKryChunk) * (size_t)k; }

int multi_axpy_launch(int64_t n, int k, const double* V, int64_t ldv, const double* coef, double sign, double* w,
                      hipStream_t st) {
    if (k <= 0 || n <= 0) return FIL_OK;
    multi_axpy_kernel<<<blocks_for(n), kKryBlock, 0, st>>>(n, k, V, ldv, coef, sign, w);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

int axpby_launch(int64_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t st) {
    if (n <= 0) return FIL_OK;
    axpby_kernel<<<blocks_for(n), kKryBlock, 0, st>>>(n, a, x, b, y, out);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

int mul_launch(int64_t n, const double* dvec, const double* x, double* out, hipStream_t st) {
    if (n <= 0) return FIL_OK;
    mul_kernel<<<blocks_for(n), kKryBlock, 0, st>>>(n, dvec, x, out);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

int diag_mobility_launch(const SimDev& d, const double* F, const double* T, double* V, double* W, hipStream_t st) {
    const int64_t n3 = 3 * d.S;
    if (n3 <= 0) return FIL_OK;
    diag_mobility_kernel<<<blocks_for(n3), kKryBlock, 0, st>>>(n3, 1.0 / (6.0 * kPi * d.eta * d.a),
                                                               1.0 / (8.0 * kPi * d.eta * d.a * d.a * d.a), F, T, V, W);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

int j0_apply_launch(const SimDev& d, const double* AinvT, const double* w, double* y, hipStream_t st) {
    if (d.M == 0) return FIL_OK;
    j0_apply_kernel<<<(unsigned)d.M, kKryBlock, 0, st>>>(d, AinvT, w, y);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // namespace fil
