// Device-side view of a simulation and launchers of the implicit-step kernels.
#pragma once
#include "common.h"

namespace fil {

constexpr int kMaxSeg = 64;       // segments per filament (one lane per segment in the steric pass)
constexpr int kKL = 8;            // sub-diagonals of the row-differenced J0 in interleaved order
constexpr int kKU = 8;            // super-diagonals (kKL + kKU after pivoting fill-in)
constexpr int kBandW = 2 * kKL + kKU + 1;
// column records of the band factor (many-filament path), 32 doubles per column: two
// halves of 16 slots, the multipliers below the diagonal and the entries of U above it,
// each rotated by the column index (see band_columns_kernel); kBcPad records of zeros
// before and after the 6S records
constexpr int kBcW = 32;
constexpr int64_t kBcPad = 512;
// explicit J0^{-1} used up to this total size: streaming it in each update beats the
// banded sweeps (latency-bound, 6N sequential steps) up to a few hundred MB
constexpr size_t kDenseInvBytes = size_t(256) << 20;
constexpr int kMaxIter = 256;     // Broyden history capacity
constexpr int kMaxDots = kMaxIter + 2;
constexpr int kSpar = 5;          // per-suspension parameters: dt, gravity force (3), F^S
constexpr int kMaxCls = 6;        // filament size classes: N <= 16, 24, 32, 40, 48, 64
constexpr int kStericWaves = 4;   // waves per filament in the steric pass

// BDF coefficients: y - a1 y^j - a2 y^{j-1} - b dt v = 0, u - g u^j - b dt dexpinv(Omega) = 0
struct BdfCoef {
    double a1, a2, b, g;
};

// Plain-old-data view of the simulation passed by value to kernels.
struct SimDev {
    int64_t S, M, nsusp;
    const int64_t* seg_off;        // [M+1]
    const int32_t* fil_susp;       // [M]
    const int32_t* seg_fil;        // [S]
    const int64_t* susp_seg_off;   // [nsusp+1]
    const int32_t* tether;         // [M]
    const double* base;            // [M][3]
    const double* phase;           // [M] or null
    const int64_t* susp_fil_off;   // [nsusp+1]
    const int64_t* dense_off;      // [M] offsets of the explicit inverses, or null
    int max_seg;                   // largest filament
    int max_dots;                  // dot products per Broyden update at most (kmax + 2)
    const double* spar;            // [nsusp][5] per suspension: dt, gravity force (3), steric strength F^S
    const double* fext;            // [3][S] further external force per segment, or null
    const double* text;            // [3][S] further external torque per segment, or null
    // rotating motor of tether-3 bases: distance of the base from the motor's z axis and its
    // rotation rate (the axis passes through the initial base position minus (d0, 0, 0))
    double motor_d0, motor_w;
    // periodic box lengths of the steric pass (minimum-image distances); periodic == 0:
    // unbounded
    double per[3];
    int periodic;
    // filaments by size class (for launches whose LDS scales with 6N): class k holds
    // cls_fil[cls_off[k] .. cls_off[k+1]), all with 6N <= cls_n[k]
    const int32_t* cls_fil;
    int ncls;
    int factor_unstaged;           // 1: the band LU never stages rows in LDS (fil_params.j0_factor)
    int64_t cls_off[kMaxCls + 1];
    int cls_n[kMaxCls];
    double a, eta, dL, KB, KT, chi, K0, kw, omega;
};

// configuration from X, internal forces (F = F^C + gravity, T = T^C + T^E) and filament boxes
// tt: device pointer to the time t^{j+1} of the step
int state_forces_launch(const SimDev& d, const double* X, const double* qj, const double* tt, const int32_t* active,
                        double* Yc, double* qc, double* F, double* T, double* box, hipStream_t st);
// geometric-switch base torques of pinned filaments (cilia.hip): per filament the switch
// direction and the steps since the last switch, updated from the committed base
// orientations qj at the start of a step; writes the base torques into text
struct SwitchArgs {
    double axis[3], normal[3];
    double theta_max, tau_pos, tau_neg;
    int n_tr;
    int32_t* dir;   // [M] +1 / -1
    int32_t* age;   // [M] steps since the last switch
    double* tau0;   // [M] signed torque before the last switch
};
int switch_torque_launch(const SimDev& d, const SwitchArgs& a, const double* qj, double* text, hipStream_t st);

// RPY mobility above the no-slip wall z = 0 (rpy_wall.hip); work of wall_workspace_bytes(S)
int64_t wall_workspace_bytes(int64_t S);
int rpy_wall_launch(int64_t S, const double* Y, const double* F, const double* T, double a, double eta, int prec,
                    double* V, double* W, void* work, hipStream_t st);
// adds the steric barrier into F and, when prec is FIL_PREC_F64, writes the mobility source records
int steric_pack_launch(const SimDev& d, const double* Yc, const double* box, const int32_t* active, double* F,
                       const double* T, int prec, void* pk, hipStream_t st);
// Dot products of Broyden update k (k < 0: none): per filament f, dpart[f][h] holds
// its share of h < k: d_h . f;  h = k: |f - fprev|^2;  h = k+1: (f - fprev) . f
struct DotArgs {
    int k;
    const double* Dhist;  // [kmax][6S]
    const double* fprev;  // [6S]
    double* dpart;        // [M][max_dots]
};
// residual rows; max|f| per suspension into resbits[0, nsusp) and max|b dt (V, dexpinv Omega)| into
// resbits[nsusp, 2 nsusp) (zeroed by the previous call, which also zeroes resbits_next);
// velocities from the K mobility partials `part` when non-null (then also stored to V, W), else from V, W;
// and the dot products of update da.k
int residual_launch(const SimDev& d, const BdfCoef& bc, const double* X, const double* Xj, const double* Yc,
                    const double* Yj, const double* Yjm1, double* V, double* W, const double* part, int K,
                    const int32_t* active, double* f, unsigned long long* resbits, unsigned long long* resbits_next,
                    const DotArgs& da, hipStream_t st);
// the same dot products for a residual given by the caller
int update_dots_launch(const SimDev& d, const double* fnew, const int32_t* active, const DotArgs& da,
                       hipStream_t st);
// Per-suspension record of a solve run by the device
struct SuspLog {
    int32_t state;     // 0 running, 1 converged, -1 failed, -2 failed on a singular J0 block,
                       // 2 done with FP32-tile evaluations (to continue in FP64)
    int32_t it;        // last iteration tested
    int32_t evals;     // residual evaluations (mobility applies)
    int32_t evals_hi;  // of which in FP64
    double last;       // max|f|/a of the last evaluation
};
// Convergence test of the evaluation just made, for iterations that run without the host
// (captured in a graph).  log null: no test.
struct JudgeArgs {
    SuspLog* log;                       // [nsusp]
    const unsigned long long* resbits;  // the maxima that evaluation left
    const int32_t* jflag;  // [M] singular-J0 flags (first step only; null: not checked): fail the suspension
    double tol, inv_a;
    int it, kmax, can_converge;
    // FP32-tile evaluations (notnear non-null): a running suspension whose max|f|/a exceeds
    // max(near_tol, near_coef max|b dt (V, dexpinv Omega)|/a) adds one to *notnear
    int* notnear;
    double near_tol, near_coef;
};
// Before FP32-tile iteration `it` of captured blocks: when no running suspension counted
// itself not near after iteration it - 1 (or 2 (it - 1) >= kmax), every running suspension
// stops (active 0, log state 2) to continue with FP64 evaluations; *notnear is cleared.
// it < 0: only the clearing.
int f32_switch_launch(int32_t* active, SuspLog* log, int* notnear, int64_t nsusp, int it, int kmax, hipStream_t st);
// Broyden update k (k < 0: first step X <- X - J0^{-1} f) and the state at the new X
struct UpdateArgs {
    int k;
    const double* AB;      // band factor (used when AinvT is null)
    const int32_t* ipiv;
    const double* rdiag;   // reciprocal pivots of the band factor
    const double* AinvT;   // explicit inverses, or null
    const double* dpart;   // partial dot products of update k
    double* Chist;         // [kmax][6S]
    double* Dhist;
    const double* fnew;    // residual at the current iterate
    double* fprev;         // <- fnew
    double* X;             // <- X - step
    double* dXout;         // -step, or null
    const double* qj;      // state at the new X, as state_forces_launch
    const double* tt;
    double *Yc, *qc, *F, *T, *box;
    // band path with many filaments: J0^{-1} fnew is formed first by a kernel of four
    // filaments per wave into gsolve [6S] (X layout) from the column records BC
    // [6S x kBcW]; null: the update kernel's own sweeps
    double* gsolve;
    const double* BC;
};
int broyden_state_launch(const SimDev& d, const UpdateArgs& u, const JudgeArgs& jg, int32_t* active, hipStream_t st);
// Start of a step: the first iterate X0 (and its copy X0c) for every suspension, the base
// of the learned first iterate Xb (X0 plus the last step's correction, from step 3 on),
// every suspension marked running, the device log cleared and the device time set to tt.
int initial_guess_launch(const SimDev& d, int64_t step, const double* Yj, const double* Yjm1, const double* Xj,
                         const double* Xjm1, const double* Xjm2, double* X0, double* X0c, double* Xb, int32_t* active,
                         SuspLog* log, double* time_d, double tt, hipStream_t st);
// copies the device log to pinned host slot (*counter mod 2) and advances *counter
int log_export_launch(const SuspLog* log, int64_t ns, SuspLog* slot0, SuspLog* slot1, int64_t* counter,
                      hipStream_t st);
// J0 at X in row-differenced banded form (6N x kBandW per filament at 6*seg_off[f]*kBandW),
// factorised with partial pivoting (ipiv at 6*seg_off[f]); flag[f] = 1 for a zero pivot
// When AinvT is non-null the explicit inverse is also built (transposed, at dense_off[f]);
// when BC is non-null the column records of the factor are written there (6S x kBcW).
int j0_factor_launch(const SimDev& d, const BdfCoef& bc, const double* X, const double* qc, const double* Tint,
                     double tt, const int32_t* active, double* AB, int32_t* ipiv, double* rdiag, int32_t* flag,
                     double* AinvT, double* BC, hipStream_t st);
// commits the step of the suspensions flagged in commit (null: all): Y, q from the
// converged state; X history shifted (Xjm2 may be null)
int finalize_launch(const SimDev& d, const int32_t* commit, const double* Yc, const double* qc, const double* X,
                    double* Yj, double* Yjm1, double* qj, double* Xj, double* Xjm1, double* Xjm2, hipStream_t st);

// Vector kernels of the Newton-Krylov solve (krylov.hip).  out[j] = V_j . w for the k
// rows of V (row stride ldv), through partial[multi_dot_partial_count(n, k)], summed in
// a fixed order; w += sign sum_j coef[j] V_j; out = a x + b y (y null: a x);
// out = dvec * x; y = J0^{-1} w with the explicit inverses (dense_off must be set).
int multi_dot_launch(int64_t n, const double* V, int64_t ldv, int k, const double* w, double* partial, double* out,
                     hipStream_t st);
size_t multi_dot_partial_count(int64_t n, int k);
int multi_axpy_launch(int64_t n, int k, const double* V, int64_t ldv, const double* coef, double sign, double* w,
                      hipStream_t st);
int axpby_launch(int64_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t st);
int mul_launch(int64_t n, const double* dvec, const double* x, double* out, hipStream_t st);
int j0_apply_launch(const SimDev& d, const double* AinvT, const double* w, double* y, hipStream_t st);
// V = F / (6 pi eta a), W = T / (8 pi eta a^3) on [3][S] (the mobility of f0)
int diag_mobility_launch(const SimDev& d, const double* F, const double* T, double* V, double* W, hipStream_t st);

}  // namespace fil
