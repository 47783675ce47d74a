// Per-filament internal forces and torques (Sec. 2.5 and 2.9.2 of arXiv:1903.12609).
// One 64-lane workgroup per filament; lane n handles segments n, n+64, ...
#include "common.h"
#include "kernels.h"
#include "quat.h"

namespace fil {

__device__ __forceinline__ Q4 load_q(const double* __restrict__ q, int64_t S, int64_t s) {
    return Q4{q[s], q[S + s], q[2 * S + s], q[3 * S + s]};
}
__device__ __forceinline__ V3 load_v(const double* __restrict__ v, int64_t ld, int64_t i) {
    return v3(v[i], v[ld + i], v[2 * ld + i]);
}

__global__ void __launch_bounds__(64) internal_forces_kernel(int64_t M, int64_t S, const int64_t* __restrict__ fil_off,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ Lam,
                                                           const double* __restrict__ kap, double dL, double KB,
                                                           double KT, double* __restrict__ F,
                                                           double* __restrict__ T) {
    const int64_t f = blockIdx.x;
    const int64_t s0 = fil_off[f], N = fil_off[f + 1] - s0;
    const int64_t J = S - M;            // joints in total
    const int64_t j0 = s0 - f;          // first joint of this filament
    for (int64_t n = threadIdx.x; n < N; n += 64) {
        const int64_t s = s0 + n;
        const Q4 qn = load_q(q, S, s);
        V3 lp = v3(0, 0, 0), lm = v3(0, 0, 0), mp = v3(0, 0, 0), mm = v3(0, 0, 0);
        if (n + 1 < N) {
            const V3 k = kap ? load_v(kap, J, j0 + n) : v3(0, 0, 0);
            lp = load_v(Lam, J, j0 + n);
            mp = joint_moment(qn, load_q(q, S, s + 1), k, dL, KB, KT);
        }
        if (n > 0) {
            const V3 k = kap ? load_v(kap, J, j0 + n - 1) : v3(0, 0, 0);
            lm = load_v(Lam, J, j0 + n - 1);
            mm = joint_moment(load_q(q, S, s - 1), qn, k, dL, KB, KT);
        }
        const V3 fc = lp - lm;
        const V3 tc = (0.5 * dL) * cross(frame_t(qn), lp + lm) + (mp - mm);
        F[s] += fc.x;
        F[S + s] += fc.y;
        F[2 * S + s] += fc.z;
        T[s] += tc.x;
        T[S + s] += tc.y;
        T[2 * S + s] += tc.z;
    }
}

int internal_forces_launch(int64_t M, int64_t S, const int64_t* fil_off, const double* q, const double* Lam,
                           const double* kap, double dL, double KB, double KT, double* F, double* T,
                           hipStream_t st) {
    if (M <= 0) return FIL_OK;
    internal_forces_kernel<<<(unsigned)M, 64, 0, st>>>(M, S, fil_off, q, Lam, kap, dL, KB, KT, F, T);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // namespace fil
