// Device-side view of a simulation and launchers of the implicit-step kernels.
#pragma once
#include "common.h"

namespace fil {

constexpr int kMaxSeg = 64;       // segments per filament (one lane per segment in the steric pass)
constexpr int kKL = 8;            // sub-diagonals of the row-differenced J0 in interleaved order
constexpr int kKU = 8;            // super-diagonals (kKL + kKU after pivoting fill-in)
constexpr int kBandW = 2 * kKL + kKU + 1;
constexpr size_t kDenseInvBytes = size_t(64) << 20;  // explicit J0^{-1} used up to this total size
constexpr int kMaxIter = 256;     // Broyden history capacity
constexpr int kMaxDots = kMaxIter + 2;
constexpr int kVecBlock = 256;    // residual-vector elements per Broyden vector block
constexpr int kSpar = 5;
constexpr int kResSeg = 64;
constexpr int kFusedJudgeBlocks = 64;  // residual grids up to this size run the convergence test themselves
constexpr int kMaxCls = 6;        // filament size classes: N <= 16, 24, 32, 40, 48, 64
constexpr int kStericWaves = 4;   // waves per filament in the steric pass       // segments per residual workgroup (six waves sum the partials)          // per-suspension parameters: dt, gravity force (3), F^S

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
    // vector blocks over the 6S unknowns (never straddling suspensions)
    int64_t nvblk;
    const int32_t* vblk_susp;      // [nvblk]
    const int64_t* vblk_start;     // [nvblk+1]
    const int64_t* susp_vblk_off;  // [nsusp+1]
    int max_dots;
    const double* spar;            // [nsusp][5] per suspension: dt, gravity force (3), steric strength F^S
    // filaments by size class (for launches whose LDS scales with 6N): class k holds
    // cls_fil[cls_off[k] .. cls_off[k+1]), all with 6N <= cls_n[k]
    const int32_t* cls_fil;
    int ncls;
    int64_t cls_off[kMaxCls + 1];
    int cls_n[kMaxCls];
    double a, eta, dL, KB, KT, chi, K0, kw, omega;
};

// configuration from X, internal forces (F = F^C + gravity, T = T^C + T^E) and filament boxes
// tt: device pointer to the time t^{j+1} of the step
int state_forces_launch(const SimDev& d, const double* X, const double* qj, const double* tt, const int32_t* active,
                        double* Yc, double* qc, double* F, double* T, double* box, hipStream_t st);
// adds the steric barrier into F and writes the mobility source records (precision prec)
int steric_pack_launch(const SimDev& d, const double* Yc, const double* box, const int32_t* active, double* F,
                       const double* T, int prec, void* pk, hipStream_t st);
// device-side convergence test fused into the residual kernel (graph-captured iterations)
struct JudgeArgs {
    unsigned int* ticket;  // zero-initialised counter; null: no test
    int32_t* active;       // per suspension, cleared when it ends
    int32_t* log;          // [nsusp][4] state (0 running, 1 converged, -1 failed), last iteration, evaluations,
                           // FP64 evaluations
    double* last;          // [nsusp] max|f|/a of the last evaluation
    double tol, inv_a;
    int it, kmax, can_converge;
};

// residual rows; max|f| per suspension into resbits[0, nsusp) and max|b dt (V, dexpinv Omega)| into
// resbits[nsusp, 2 nsusp) (zeroed by the previous call, which also zeroes resbits_next);
// velocities from the K mobility partials `part` when non-null (then also stored to V, W), else from V, W
int residual_launch(const SimDev& d, const BdfCoef& bc, const double* X, const double* Xj, const double* Yc,
                    const double* Yj, const double* Yjm1, double* V, double* W, const double* part, int K,
                    const int32_t* active, double* f, unsigned long long* resbits, unsigned long long* resbits_next,
                    hipStream_t st, const JudgeArgs* judge = nullptr);
int initial_guess_launch(const SimDev& d, int64_t step, const double* Yj, const double* Yjm1, const double* Xj,
                         const double* Xjm1, const int32_t* active, double* X0, hipStream_t st);
// J0 at X in row-differenced banded form (6N x kBandW per filament at 6*seg_off[f]*kBandW),
// factorised with partial pivoting (ipiv at 6*seg_off[f]); flag[f] = 1 for a zero pivot
// When AinvT is non-null the explicit inverse is also built (transposed, at dense_off[f]).
int j0_factor_launch(const SimDev& d, const BdfCoef& bc, const double* X, const double* qc, const double* Tint,
                     double tt, const int32_t* active, double* AB, int32_t* ipiv, int32_t* flag, double* AinvT,
                     hipStream_t st);
// out = J0^{-1} v: dense product when AinvT is non-null, else the banded sweeps
int j0_solve_launch(const SimDev& d, const double* AB, const int32_t* ipiv, const double* AinvT, const double* v,
                    const int32_t* active, double* out, hipStream_t st);
int broyden_update_launch(const SimDev& d, int k, const double* AB, const int32_t* ipiv, const double* AinvT,
                          double* Chist, double* Dhist, const double* fnew, double* fprev, double* g0, double* hvec,
                          double* part, double* X, double* dXout, const int32_t* active, hipStream_t st);
int first_step_launch(const SimDev& d, const double* h, const double* f, double* fprev, double* X, double* dXout,
                      const int32_t* active, hipStream_t st);
// commits the step: Y, q from the converged state; X history shifted (Xjm2 may be null)
int finalize_launch(const SimDev& d, const int32_t* commit, const double* Yc, const double* qc, const double* X,
                    double* Yj, double* Yjm1, double* qj, double* Xj, double* Xjm1, double* Xjm2, hipStream_t st);

}  // namespace fil
