/*
 * fil.h -- C ABI of the MI355X filament library: the hot path of the implicit
 * quaternion filament method of Schoeller, Townsend, Westwood & Keaveny,
 * "Methods for suspensions of passive and active filaments" (arXiv:1903.12609).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors),
 *     owned by the caller, double precision unless stated.
 *   - Vector fields over S segments are component-major ("SoA"): double[3][S]
 *     (all x, then all y, then all z).  Quaternions are double[4][S] stored
 *     (q0, q1, q2, q3).  Segments are filament-major: filament f owns segments
 *     fil_off[f] .. fil_off[f+1]-1.
 *   - The unknowns of one filament of N segments are the 6N doubles
 *     [ Y_1 (3) | u_1 .. u_N (3N) | Lambda_{3/2} .. Lambda_{N-1/2} (3(N-1)) ]
 *     (reduced system of Sec. 2.9.3), filament f starting at 6*fil_off[f].
 *     A base-clamped filament keeps its tether multipliers lambda_1, lambda_2
 *     in the Y_1 and u_1 slots (tethering constraints of Sec. 5.2.1).
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls only enqueue
 *     work on it; nothing is synchronised unless the entry point says so.
 *   - Every function returns a fil_status.  Argument errors are detected on the
 *     host before anything is enqueued; fil_last_error() then describes them.
 *   - Nothing here calls back into Python or touches host memory unless the
 *     argument is documented as a host pointer.
 */
#ifndef FIL_H
#define FIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FIL_OK = 0,
    FIL_EINVAL = -1,      /* bad argument (null pointer, negative size, a <= 0, ...) */
    FIL_EHIP = -2,        /* a HIP runtime call failed */
    FIL_ENOCONV = -3,     /* Broyden hit its iteration cap before the tolerance */
    FIL_ENONFINITE = -4,  /* a residual became NaN or infinite */
    FIL_ENOMEM = -5       /* device allocation failed */
} fil_status;

typedef enum {
    FIL_PREC_F64 = 0,        /* pair math and accumulation in double */
    FIL_PREC_F32TILE = 1     /* pair math in float on FP64-referenced offsets, FP64 accumulation */
} fil_prec;

/* Message for the most recent non-OK status returned on this thread. */
const char* fil_last_error(void);

/* ------------------------------------------------------------------------ */
/* Mobility: the RPY mobility matrix applied to all forces and torques.       */
/* ------------------------------------------------------------------------ */
/* (V_n, Omega_n) = sum_m [[M^tt, M^tr], [M^rt, M^rr]]_{nm} (F_m, T_m)
 * with the unbounded RPY sub-tensors of Sec. 2.7.1 (self terms 1/(6 pi eta a)
 * and 1/(8 pi eta a^3); (eps . rhat)_{ij} = eps_{ijk} rhat_k), and for
 * overlapping pairs r < 2a the equal-radius regularised RPY forms that the
 * paper cites in the same section (they meet the far field at r = 2a in value
 * and slope).
 *   S          number of segments (S >= 0; S = 0 is a no-op)
 *   Y, F, T    positions, forces, torques: device double[3][S]
 *   a, eta     segment radius and viscosity (> 0)
 *   prec       FIL_PREC_F64 or FIL_PREC_F32TILE
 *   V, Omega   outputs, device double[3][S]; may not alias the inputs
 *   work       device scratch of at least fil_rpy_workspace_bytes(S, prec)
 *              bytes (NULL allowed when that size is 0); contents are
 *              overwritten; two calls in flight must not share it.
 * The result is deterministic: the same inputs give bitwise the same output. */
int64_t fil_rpy_workspace_bytes(int64_t S, int prec);
int fil_rpy_mobility_apply(int64_t S, const double* Y, const double* F, const double* T, double a, double eta,
                           int prec, double* V, double* Omega, void* work, int64_t work_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Filament mechanics                                                        */
/* ------------------------------------------------------------------------ */
/* Adds the internal forces and torques of every filament (Sec. 2.5, 2.9.2):
 *   F_n += Lambda_{n+1/2} - Lambda_{n-1/2}
 *   T_n += dL/2 t_n x (Lambda_{n+1/2} + Lambda_{n-1/2}) + M_{n+1/2} - M_{n-1/2}
 * with M_{n+1/2} = R(q_{n+1/2}) D (2[q_{n+1/2}^* . (q_{n+1} - q_n)/dL]_{R^3} - kappa),
 * q_{n+1/2} = (q_{n+1} . q_n^*)^{1/2} . q_n, D = diag(KT, KB, KB) and free-end
 * values Lambda = M = 0 at both ends.
 *   M, S       number of filaments (>= 0) and segments (S = fil_off[M])
 *   fil_off    DEVICE int64[M+1], non-decreasing, fil_off[0] = 0, every filament >= 1 segment
 *   q          device double[4][S] unit quaternions
 *   Lambda     device double[3][S-M]: joint k of filament f is column fil_off[f]-f+k
 *   kappa      device double[3][S-M] (gamma0, kappa_mu, kappa_nu) per joint, or NULL for 0
 *   F, T       device double[3][S], accumulated into (+=) */
int fil_filament_internal_forces(int64_t M, int64_t S, const int64_t* fil_off, const double* q,
                                 const double* Lambda, const double* kappa, double dL, double KB, double KT,
                                 double* F, double* T, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FIL_H */
