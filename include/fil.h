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
 *     in the Y_1 and u_1 slots (tethering constraints of Sec. 5.2.1); a pinned one
 *     keeps lambda_1 in the Y_1 slot and its u_1.
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

/* The same apply with its main pair kernel bracketed by two caller-created HIP events
 * (hipEvent_t, NULL for none): ev_start is stamped when the pair kernel starts and ev_end
 * when it ends (extended launch), so hipEventElapsedTime(ev_start, ev_end) is that kernel's
 * own duration; for profiling.  Arguments and errors otherwise as fil_rpy_mobility_apply. */
int fil_rpy_mobility_apply_timed(int64_t S, const double* Y, const double* F, const double* T, double a, double eta,
                                 int prec, double* V, double* Omega, void* work, int64_t work_bytes, void* ev_start,
                                 void* ev_end, void* stream);

/* The same apply for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): no workspace argument,
 * no hipMalloc, hipFree or allocating library call.  Its scratch (source records, FP32
 * tile records, split-K partials) is a static device array of 256 MiB, one per GPU, held by
 * each GPU the library runs on until the process ends (fil_rpy_noalloc_scratch_bytes
 * returns its size).  Every S up to 160,000 fits in both precisions; an S whose
 * fil_rpy_workspace_bytes exceeds the array is refused with FIL_EINVAL.  Nothing in the
 * array needs to start at zero: every apply writes what it reads.  All calls on one GPU
 * share the array, so calls that overlap on one GPU (other streams, other threads) race;
 * calls on one stream are ordered.  The first call on a device looks up the array's device
 * address (FIL_EHIP if that fails).  Other arguments and errors as fil_rpy_mobility_apply;
 * bitwise the same result. */
int fil_rpy_mobility_apply_noalloc(int64_t S, const double* Y, const double* F, const double* T, double a,
                                   double eta, int prec, double* V, double* Omega, void* stream);
int64_t fil_rpy_noalloc_scratch_bytes(void);

/* RPY mobility of the segments above a no-slip plane wall z = 0 (the half-space tensor
 * the paper uses for its cilia, Sec. 2.7.1 and Sec. 5.2.2): the unbounded tensor of
 * fil_rpy_mobility_apply (same overlap forms) plus the wall's image part, Blake's image
 * system for a point force above a wall under the Faxen operators of both spheres
 *   tt = (1 + a^2/6 lap_x)(1 + a^2/6 lap_y) G^im,  rt = 1/2 curl_x (1 + a^2/6 lap_y) G^im,
 *   tr = 1/2 curl_y (1 + a^2/6 lap_x) G^im,  rr = 1/4 curl_x curl_y G^im   (over 8 pi eta),
 * whose self terms are the Rotne-Prager-Blake wall corrections (e.g. 1 - 9a/16h + a^3/8h^3
 * - a^5/16h^5 for translation parallel to the wall).  Valid for centres at z >= a (spheres
 * not crossing the wall); smaller heights are evaluated with the same formulas.
 *   S, Y, F, T, a, eta, V, Omega  as fil_rpy_mobility_apply
 *   prec   FIL_PREC_F64, or FIL_PREC_F32TILE: the pair arithmetic (free-space and image
 *          parts) in float on coordinates relative to an FP64 origin per 16 sources, float
 *          sums of each 16 added to FP64 sums per target; self terms in FP64
 *   work   device scratch of fil_rpy_wall_workspace_bytes(S) bytes (NULL when 0; the same
 *          for both precisions)
 * Deterministic: the partial sums over source chunks are added in a fixed order.
 * FIL_EINVAL on a bad argument or precision, or a workspace too small. */
int64_t fil_rpy_wall_workspace_bytes(int64_t S);
int fil_rpy_wall_apply(int64_t S, const double* Y, const double* F, const double* T, double a, double eta, int prec,
                       double* V, double* Omega, void* work, int64_t work_bytes, void* stream);

/* Force-coupling-method mobility (Sec. 2.7.2) in a periodic box: the forces and
 * torques enter the Stokes equations as Gaussian monopoles F_m Delta_m and rotlets
 * -1/2 T_m x grad Theta_m (widths sigma_D = a / sqrt(pi), sigma_T = a / (6 sqrt(pi))^(1/3),
 * truncated at distance cut * sigma), the equations are solved spectrally on a regular
 * grid, and V_n, Omega_n are the Gaussian-weighted averages of the velocity and half the
 * vorticity (trapezoidal rule), the latter integrated by parts over the box,
 * Omega_n = 1/2 sum (r x u) Theta_n / sigma_T^2 dV (r = x - Y_n): the exact adjoint of the
 * rotlet spreading, equal to the vorticity average up to the grid's discretisation error.
 * The zero mode and the Nyquist planes of even axes are dropped.  The mean force is not
 * balanced: the result is the periodic mobility.
 *   box   HOST double[3]: box lengths (positions are wrapped into [0, L))
 *   grid  HOST int32[3]: grid points per axis (4 .. 4096); the support 2 ceil(cut sigma_D
 *         / h) + 1 must fit in the grid and in 65 points
 *   cut   truncation radius in Gaussian widths, in [2, 12] (7.5: tails below 1e-12)
 * fil_fcm_create allocates the grids and the FFT plans (FIL_ENOMEM, FIL_EHIP on failure);
 * fil_fcm_apply then allocates nothing: S segments, Y, F, T device double[3][S], outputs
 * V, Omega device double[3][S] (not aliasing the inputs), asynchronous on stream.  Two
 * applies in flight must not share a handle.  Spreading adds with atomics, so results
 * may differ between runs in the last bits. */
typedef struct fil_fcm fil_fcm;
int fil_fcm_create(const double* box, const int32_t* grid, double a, double eta, double cut, fil_fcm** out);
int fil_fcm_apply(fil_fcm* fcm, int64_t S, const double* Y, const double* F, const double* T, double* V,
                  double* Omega, void* stream);
void fil_fcm_destroy(fil_fcm* fcm);

/* Batched form: nsusp independent suspensions in one launch; suspension i owns
 * segments susp_off[i] .. susp_off[i+1]-1 and interacts only with itself.  A plan holds
 * the work list of one set of offsets and one precision: fil_rpy_batch_create builds and
 * sorts it on the host, allocates its device copy on the current device and copies it there
 * (synchronously; FIL_ENOMEM, FIL_EHIP on failure).  The apply then only enqueues work on
 * `stream`: no allocation, no host copy and no synchronisation.
 *   susp_off   HOST int64[nsusp+1], non-decreasing, susp_off[0] = 0 (copied)
 *   prec       FIL_PREC_F64 or FIL_PREC_F32TILE
 * fil_rpy_batch_workspace_bytes: device scratch of one apply (source records, FP32 tile
 *   records, split-K partials and the counter its workgroups take work items from, which
 *   the apply clears first), -1 for a null plan.
 * fil_rpy_mobility_apply_batched: Y, F, T, a, eta, V, Omega as fil_rpy_mobility_apply over
 *   S = susp_off[nsusp] segments, on the device the plan was created on; work of at least
 *   fil_rpy_batch_workspace_bytes(plan) bytes (NULL when 0).  Applies in flight may share a
 *   plan but not a workspace.  Deterministic.
 * fil_rpy_batch_destroy frees the plan (after the applies that use it have completed). */
typedef struct fil_rpy_batch fil_rpy_batch;
int fil_rpy_batch_create(int64_t nsusp, const int64_t* susp_off, int prec, fil_rpy_batch** out);
int64_t fil_rpy_batch_workspace_bytes(const fil_rpy_batch* plan);
int fil_rpy_mobility_apply_batched(const fil_rpy_batch* plan, const double* Y, const double* F, const double* T,
                                   double a, double eta, double* V, double* Omega, void* work, int64_t work_bytes,
                                   void* stream);
void fil_rpy_batch_destroy(fil_rpy_batch* plan);

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

/* ------------------------------------------------------------------------ */
/* The implicit step (Sec. 2.9.3 system, Alg. 2 bad Broyden with the explicit */
/* block-diagonal J0 of Sec. 3.2.2 / Appendix B.2).                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double a, eta, dL, KB, KT;
    double chi, FS;             /* steric barrier (Sec. 2.6); FS = 0 switches it off */
    double grav[3];             /* external force on every segment */
    double dt, tol;             /* time step; stop when max|f| / a <= tol */
    int32_t kmax;               /* Broyden iteration cap per step (<= 255) */
    int32_t prec;               /* fil_prec of the mobility apply */
    int32_t j0_mode;            /* how J0^{-1} is applied: 0 auto (explicit inverse up to 256 MB),
                                   1 banded LU sweeps, 2 explicit inverse */
    int32_t j0_factor;          /* form of the banded LU kernel: 0 auto (rows staged in LDS while a
                                   filament size class fits in four rounds of resident workgroups,
                                   else without LDS), 1 always without LDS.  Both give the same
                                   factor; 1 exists to check the large-ensemble form on small cases */
    double K0, kw, omega;       /* kappa_nu(s,t) = K0 sin(kw s - omega t + phase_f) */
} fil_params;

typedef struct {
    int32_t iters;              /* Broyden updates taken */
    int32_t mobility_applies;   /* residual evaluations (one mobility apply each) */
    int32_t converged;          /* 1 if max|f|/a <= tol */
    int32_t applies_f64;        /* of which with the FP64 mobility (all of them in FIL_PREC_F64 mode) */
    double resid;               /* final max|f| / a */
    int32_t used_learned;       /* 1 if the step started from the learned warm start */
    int32_t pad;
} fil_step_report;

typedef struct fil_sim fil_sim;

/* Creates a simulation of nsusp independent suspensions on the current device.
 * All arrays here are HOST pointers, copied in:
 *   susp_fil_off int64[nsusp+1]   filaments of suspension i: susp_fil_off[i] .. [i+1]-1
 *   fil_seg_off  int64[M+1]       segments of filament f (M = susp_fil_off[nsusp])
 *   Y0  double[S][3], q0 double[S][4]   initial positions (constraints met) and unit quaternions
 *   phase  double[M] or NULL      per-filament phase of the preferred curvature
 *   tether int32[M] or NULL       1 = base clamped at its initial Y_1 and q_1; 2 = base
 *                                 pinned at its initial Y_1, its rotation free (the cilia
 *                                 bases of Sec. 5.2.2): lambda_1 in the Y_1 slot, u_1 kept; 3 = base on
 *                                 the rotating motor of fil_set_motor (Sec. 5.2.1)
 * The library allocates all device state and workspace here (FIL_ENOMEM on failure). */
int fil_create(const fil_params* p, int64_t nsusp, const int64_t* susp_fil_off, const int64_t* fil_seg_off,
               const double* Y0, const double* q0, const double* phase, const int32_t* tether, fil_sim** out);
void fil_destroy(fil_sim* sim);

/* Per-suspension parameters for ensembles of independent suspensions whose time
 * step, gravity force (Sec. 5.4: W depends on each suspension's L) or steric
 * strength F^S (Sec. 2.6) differ.  HOST arrays, each may be NULL to keep the
 * value from fil_params: dt double[nsusp] (> 0), grav double[nsusp][3],
 * FS double[nsusp] (>= 0).  Only before the first step.  Differing time steps
 * need K0 = 0 (the time of the preferred curvature is the global step count x
 * fil_params.dt).  FIL_EINVAL on a bad value, nothing changed. */
int fil_set_suspension_params(fil_sim* sim, const double* dt, const double* grav, const double* FS);

/* A further external force on every segment, added to the gravity force in the force
 * balance of each segment (the external forces of Sec. 2.5, e.g. the end load of the
 * clamped filament of Sec. 4.1).  HOST array double[S][3], copied in; NULL removes it.
 * Only before the first step (captured iterations read the force's address).  Not
 * part of checkpoints.  FIL_EINVAL on a non-finite value, FIL_ENOMEM if the device
 * copy cannot be allocated. */
int fil_set_external_forces(fil_sim* sim, const double* Fext);

/* The suspension in a periodic box, its mobility the force-coupling method
 * (fil_fcm_create's box, grid and cut; Sec. 2.7.2) in place of the unbounded RPY
 * tensor, and its steric barrier (Sec. 2.6) between nearest periodic images.  Positions
 * stay unwrapped.  Only before the first step, for one suspension (nsusp == 1) in
 * FIL_PREC_F64; every box length must exceed 4 chi a (the steric cutoff is below half the
 * box).  The iterations of later steps then run from the host (no captured graphs), one
 * FCM apply per residual evaluation; the Newton-Krylov steps and fil_residual use it too.
 * The mobility timing of fil_set_timing then times whole FCM applies.  FIL_EINVAL on a
 * bad argument, and fil_fcm_create's errors. */
int fil_set_periodic_fcm(fil_sim* sim, const double* box, const int32_t* grid, double cut);

/* The rotating motor of Sec. 5.2.1 for every tether-3 filament: its base moves on the circle
 * of radius d0 about the z axis through (initial Y_1) - (d0, 0, 0), at angle omega t, and
 * turns by u_1 = (0, 0, omega dt) per step; lambda_1, lambda_2 fill the Y_1, u_1 slots and
 * act on the first segment as F^C = lambda_1, T^C = D^T lambda_2 (D = dexpinv at u_1).  J0
 * keeps the clamped base's rows.  Only before the first step.  FIL_EINVAL on d0 < 0 or a
 * non-finite value. */
int fil_set_motor(fil_sim* sim, double d0, double omega);

/* Geometric-switch driving torque of model cilia (Sec. 5.2.2) on every pinned filament
 * (tether 2): a torque about the unit axis drives the base until the angle theta between
 * the unit wall normal and the base tangent (signed about the axis, atan2 form) reaches
 * +theta_max or -theta_max, where it reverses; its magnitude is tau_pos while driving
 * towards +theta_max and tau_neg towards -theta_max.  At a switch the torque passes to
 * the new value along a logistic curve over n_transition steps (0: at once).  Decided at
 * the start of each step (and of each Newton-Krylov step) from the committed base
 * orientation; a step that fails keeps the switch state it started with advanced.  All
 * filaments start driving towards +theta_max at tau_pos.  axis, normal: HOST double[3],
 * orthogonal unit vectors.  Only before the first step.  FIL_EINVAL on a bad argument.
 * fil_read_switch copies each filament's direction (+1 / -1) into HOST int32[M]
 * (synchronising). */
int fil_set_geometric_switch(fil_sim* sim, const double* axis, const double* normal, double theta_max,
                             double tau_pos, double tau_neg, int n_transition);
int fil_read_switch(fil_sim* sim, int32_t* dir);

/* The suspension above a no-slip plane wall at z = 0: every residual evaluation applies
 * the wall-bounded RPY mobility of fil_rpy_wall_apply in place of the unbounded one (the
 * steric barrier and everything else unchanged; no wall repulsion, so segments must stay
 * above z = a).  Only before the first step, for one suspension, and not with
 * fil_set_periodic_fcm.  In FIL_PREC_F32TILE the evaluations before the FP64 finish use
 * the wall apply's FP32-tile form.  Graph blocks and the Newton-Krylov steps use it too.
 * FIL_EINVAL on a bad call, FIL_ENOMEM if the workspace cannot be allocated. */
int fil_set_wall(fil_sim* sim);

/* One time step: warm start, J0 and its inverse, Broyden iterations on the
 * device (one mobility apply each), then q^{j+1} = exp(u) . q^j, the robot-arm
 * positions and the history shift.  The first step is BDF1, later ones BDF2.
 * In FIL_PREC_F32TILE mode the step's first mobility applies use FP32 pair
 * tiles; once every running suspension's residual is within 10 tol, or within
 * 3000x the FP32 rounding floor (3e-8 x max|b dt V|), later applies use FP64, the
 * Broyden history restarting there (Alg. 2 from the current iterate, same J0), and
 * only an FP64 residual ends a step (the FP32 floor can exceed tol).
 * report: HOST fil_step_report[nsusp] (may be NULL).  Host-driven iterations
 * (graph execution off) synchronise the stream once per iteration to test
 * convergence; see fil_set_graph for the device-driven form, in which the switch
 * to FP64 applies is decided on the device as well.  On success the commit of the new state may still be running when the
 * call returns: work on the simulation's stream is ordered after it, other
 * streams synchronise first (fil_read_state does).  Returns FIL_ENOCONV or
 * FIL_ENONFINITE if a suspension failed; its state is then left at step j. */
int fil_bdf2_step(fil_sim* sim, fil_step_report* report);

/* One time step solved by Jacobian-free Newton-Krylov instead of bad Broyden (the
 * comparison method of Sec. 3.1 and 3.3.1): Newton iterations X <- X + dX until
 * max|f|/a <= fil_params.tol (at most fil_params.kmax of them), each solving
 * J(X) dX = -f(X) by restarted GMRES (restart length min(krylov_max, 100)) to a
 * relative residual krylov_tol (the paper's 1e-4), the products J v taken as
 * (f(X + fd_delta v) - f(X)) / fd_delta (the paper's delta = 1e-7), one mobility
 * apply each.  precond: 0 none; 1 right preconditioner P_dt, applied as its inverse
 * (the multiplier unknowns scaled by 6 pi eta a / dt); 2 left preconditioner J0^{-1}
 * (the block-diagonal J0 of the step's initial guess; needs the explicit inverse,
 * fil_params.j0_mode 0 within its size limit, or 2).  One suspension, FP64 mobility.
 * The step starts from the same warm start as fil_bdf2_step and commits the same way;
 * on failure the state stays at the previous step (FIL_ENOCONV, FIL_ENONFINITE).
 * report: HOST, may be NULL.  Synchronises the stream several times per Krylov
 * iteration (the Arnoldi coefficients go to the host). */
typedef struct {
    int32_t newton_iters;       /* Newton updates taken (Broyden updates for fil_jfb_step) */
    int32_t krylov_iters;       /* GMRES iterations over all Newton steps */
    int32_t mobility_applies;   /* residual evaluations (one mobility apply each) */
    int32_t converged;
    double resid;               /* final max|f| / a */
} fil_jfnk_report;
int fil_jfnk_step(fil_sim* sim, int precond, double krylov_tol, double fd_delta, int krylov_max,
                  fil_jfnk_report* report);

/* One time step solved by the Jacobian-free good Broyden method JFB-g (Sec. 3.2.1,
 * Alg. 1, compared in Sec. 3.3.2): Broyden iterations dX = -[J0 + sum_i c_i d_i^T]^{-1}
 * f(X_k), c = f(X_{k+1}) / |dX|, d = dX / |dX|, until max|f|/a <= fil_params.tol (at
 * most fil_params.kmax iterations).  J0 = grad f0 at the step's initial guess, with f0
 * the residual computed with the drag-only mobility diag(M) and without steric or
 * external forces; its products are taken as (f0(X0 + fd_delta v) - f0(X0)) / fd_delta,
 * and each system is solved by restarted GMRES to relative residual krylov_tol.  One
 * mobility apply per Broyden iteration.  precond, the restart, the report (with
 * newton_iters holding the Broyden iterations), the refusals and the state on failure
 * as fil_jfnk_step. */
int fil_jfb_step(fil_sim* sim, int precond, double krylov_tol, double fd_delta, int krylov_max,
                 fil_jfnk_report* report);

/* One bad-Broyden update (Alg. 2) on the simulation's current iterate, given
 * the residual f_new = f(X_{k+1}) (device double[6S]):
 *   c_{k+1} = -H_k f_new / |f_new - f_k|,  d_{k+1} = (f_new - f_k) / |f_new - f_k|,
 *   dX_out = -H_{k+1} f_new,  X += dX_out
 * with H_k = J0^{-1} + sum_i c_i d_i^T.  Call fil_broyden_begin first (it
 * evaluates J0 at X0, inverts it and sets f_0). */
/* fil_broyden_begin: X <- X0 (device double[6S]), f_0 = f(X0) (copied to f0_out
 * if not NULL), J0 at X0 and its inverse, then the first step X <- X0 - J0^{-1} f_0.
 * fil_broyden_update: the caller evaluates f_new = f(X) at the current iterate
 * (fil_residual with X from fil_get_state) and passes it in; dX_out (device
 * double[6S]) may be NULL.  At most kmax - 1 updates follow one begin. */
int fil_broyden_begin(fil_sim* sim, const double* X0, double* f0_out);
int fil_broyden_update(fil_sim* sim, const double* f_new, double* dX_out);
/* Residual f(X) of the reduced system at the current step (device arrays). */
int fil_residual(fil_sim* sim, const double* X, double* f_out);

/* Device pointers to the committed state of step j (Y^j [3][S], q^j [4][S],
 * X^j [6S]) and to the current Broyden iterate X [6S]; valid until fil_destroy.
 * Any pointer argument may be NULL. */
int fil_get_state(fil_sim* sim, const double** Y, const double** q, const double** Xj, const double** X, int64_t* S,
                  double* t, int64_t* step);

/* Synchronising copy of the committed state to HOST buffers in the caller's
 * array-of-structures layout: Y double[S][3], q double[S][4], Xj double[6S];
 * any may be NULL. */
int fil_read_state(fil_sim* sim, double* Y, double* q, double* Xj);

/* Checkpoint of the committed state (time, step count, Y^j, Y^{j-1}, q^j, X^j,
 * X^{j-1}, X^{j-2}, the per-suspension parameters and, when fil_set_geometric_switch
 * was called, each filament's switch direction, steps since its last switch and torque
 * at that switch) to a file (HOST path), and its restore into a simulation created with
 * the same filament and suspension layout and the same settings (wall, motor, switch,
 * external forces: they are not in the file); a restored simulation continues exactly as
 * the saved one would (Broyden histories do not outlive a step).  Synchronises the
 * stream.  FIL_EINVAL when the file cannot be opened, written or read, is not a
 * checkpoint, belongs to another layout, holds switch state the simulation has no switch
 * for (or lacks the state of its switch) or holds non-finite values; the simulation is
 * then unchanged. */
int fil_checkpoint(fil_sim* sim, const char* path);
int fil_restore(fil_sim* sim, const char* path);

/* Timing of the mobility pair kernel inside fil_bdf2_step: when enabled, HIP
 * events on the simulation's stream bracket every launch of the main pair
 * kernel; fil_get_timing returns the summed duration (ms) and the launch count
 * since the last fil_set_timing call, HOST arrays of 2: [0] the FP64 kernel,
 * [1] the FP32-tile kernel (either may be NULL).  Enabling resets the counters;
 * fil_get_timing synchronises the stream. */
int fil_set_timing(fil_sim* sim, int enable);
int fil_get_timing(fil_sim* sim, double* rpy_ms, int64_t* rpy_launches);

/* Stream the simulation enqueues on (set before stepping). */
int fil_set_stream(fil_sim* sim, void* stream);

/* Graph execution of the Broyden iterations (the batched-execution form; not
 * part of the paper): with iters_per_launch = U > 0, fil_bdf2_step runs the
 * iterations in blocks of U, each block (per iteration: the residual
 * evaluation with its mobility apply, a device-side convergence test and the
 * bad-Broyden update) captured once into a HIP graph on a private stream and
 * replayed on the simulation's stream.  Every test, the first included, then
 * runs on the device; the host reads a block's log while the next block runs,
 * so a block launched after the end only runs kernels that find their
 * suspension finished.  In FIL_PREC_F32TILE mode the FP32-tile iterations run in
 * blocks too: a one-workgroup kernel before each decides the switch to FP64 from
 * the previous test and stops the suspensions there; FP64 blocks continue from
 * that iteration.  Results are identical to U = 0 (the default, one host test
 * per iteration).  Graphs are cached per (first iteration, U, precision,
 * iteration of the last history restart) and freed by fil_destroy.  U in [0, 64].
 * fil_set_timing then times only the host-driven evaluations (the first of each
 * step); captured blocks carry no timing events. */
int fil_set_graph(fil_sim* sim, int iters_per_launch);

/* ------------------------------------------------------------------------ */
/* Learned warm start.  Not part of the paper's method: a per-filament       */
/* network predicts, from the committed state of step j, how far the         */
/* converged unknowns of step j+1 (Y_1, the Lie-algebra increments u_n and  */
/* the multipliers Lambda) lie from the extrapolated first iterate of the    */
/* warm start (Sec. 3.3.3 notes that the iteration count depends on that     */
/* guess).  The network works around a base guess: the extrapolated first   */
/* iterate plus the last step's own correction (its converged unknowns minus */
/* its extrapolation: second differences of Y_1 and Lambda, first            */
/* differences of u).  The prediction is added to that base; if Broyden then */
/* fails, the step is re-solved from the plain guess, and convergence is     */
/* always judged by the same residual tolerance.                             */
/*                                                                           */
/* Network: 19N inputs -> `depth` SiLU hidden layers of `width` -> 6N        */
/* outputs for filaments of N segments; BF16 weights and activations with    */
/* FP32 accumulation on the matrix cores, FP32 master weights, Adam.         */
/* Dimensions are padded to multiples of 32 (n_in_pad, n_out_pad); the flat  */
/* FP32 parameter vector holds, layer by layer, W [out_pad][in_pad]          */
/* (row-major) then b [out_pad].  Loss: mean of (Y - T)^2 over the valid      */
/* rows and n_out columns, T the standardised targets.                       */
/* ------------------------------------------------------------------------ */
typedef struct fil_mlp fil_mlp;

/* Creates the network on the current device with a seeded uniform (He)
 * initialisation; max_batch bounds B of every call.  FIL_EINVAL for
 * n_seg outside [2, 64], width not a multiple of 32, depth outside [1, 16]. */
int fil_mlp_create(int32_t n_seg, int32_t width, int32_t depth, int32_t max_batch, uint64_t seed, fil_mlp** out);
void fil_mlp_destroy(fil_mlp* mlp);
/* The FP32 master parameters and the normalisation to a file (HOST path), and back
 * into a network of the same architecture (batch capacity may differ; Adam moments
 * restart).  Synchronising.  FIL_EINVAL on an unreadable, incomplete or mismatched file. */
int fil_mlp_save(const fil_mlp* mlp, const char* path);
int fil_mlp_load(fil_mlp* mlp, const char* path);
/* dims (HOST int32[8]): n_in, n_in_pad, n_out, n_out_pad, width, depth, max_batch, n_seg;
 * n_params: length of the flat parameter vector.  Either may be NULL. */
int fil_mlp_dims(const fil_mlp* mlp, int32_t* dims, int64_t* n_params);
/* HOST float[n_params] in / out.  Setting resets the Adam moments. */
int fil_mlp_set_params(fil_mlp* mlp, const float* params);
int fil_mlp_get_params(const fil_mlp* mlp, float* params);
/* Standardisation (HOST float[2 (n_in_pad + n_out_pad)]): mu_in, sd_in, mu_out, sd_out. */
int fil_mlp_set_norm(fil_mlp* mlp, const float* norm);
int fil_mlp_get_norm(const fil_mlp* mlp, float* norm);
/* Fits the standardisation to n samples: feat DEVICE float[n][n_in], targ
 * DEVICE float[n][n_out] (column means and population standard deviations;
 * a constant column gets sd = 1). */
int fil_mlp_fit_norm(fil_mlp* mlp, int64_t n, const float* feat, const float* targ, void* stream);
/* xb (DEVICE bf16 as uint16[n][n_in_pad]) = (feat - mu_in) / sd_in, zero padded;
 * t (DEVICE float[n][n_out_pad]) = (targ - mu_out) / sd_out.  Either pair may be NULL. */
int fil_mlp_standardize(fil_mlp* mlp, int64_t n, const float* feat, const float* targ, uint16_t* xb, float* t,
                        void* stream);
/* Y (DEVICE float[B][n_out_pad]) = network(X), X DEVICE bf16 [B][n_in_pad], B <= max_batch. */
int fil_mlp_forward(fil_mlp* mlp, int32_t B, const uint16_t* X, float* Y, void* stream);
/* Loss and gradient of the minibatch of rows `rows` (DEVICE int32[B]; NULL:
 * rows 0..B-1) of X (DEVICE bf16 [*][n_in_pad]) and T (DEVICE float
 * [*][n_out_pad], standardised).  grad_out (DEVICE float[n_params]) and loss
 * (DEVICE double) may be NULL.  The gradient is kept for fil_mlp_adam_step. */
int fil_mlp_backward(fil_mlp* mlp, int32_t B, const int32_t* rows, const uint16_t* X, const float* T,
                     float* grad_out, double* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the last gradient. */
int fil_mlp_adam_step(fil_mlp* mlp, float lr, void* stream);
/* fil_mlp_backward followed by fil_mlp_adam_step. */
int fil_mlp_train_step(fil_mlp* mlp, int32_t B, const int32_t* rows, const uint16_t* X, const float* T, float lr,
                       double* loss, void* stream);

/* Simulation side (every filament of the simulation must have N segments):
 * fil_sim_features: the 19N raw features of every filament at the committed
 *   state (DEVICE float[M][19N]); valid after at least one step.
 * fil_sim_step_target: the scaled difference between the converged unknowns of
 *   the last step and the base of its learned first iterate (the extrapolated
 *   first iterate plus, from the fourth step on, the correction of the step
 *   before), scaled like the last 6N features (DEVICE float[M][6N]).
 * fil_sim_set_mlp: use the network for the first iterate of every step from
 *   the fourth on (it needs three committed steps of history); tethered
 *   filaments keep the plain guess.  The network must outlive its use and have
 *   max_batch >= M.  enable = 0 switches it off.
 * fil_sim_fallbacks: steps re-solved from the plain guess so far. */
int fil_sim_features(fil_sim* sim, float* out);
int fil_sim_step_target(fil_sim* sim, float* out);
int fil_sim_set_mlp(fil_sim* sim, fil_mlp* mlp, int enable);
int fil_sim_fallbacks(fil_sim* sim, int64_t* n);

#ifdef __cplusplus
}
#endif
#endif /* FIL_H */
