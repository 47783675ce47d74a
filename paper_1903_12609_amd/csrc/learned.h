// Launchers of the learned warm start's simulation-side kernels (learned.hip).
#pragma once
#include "common.h"
#include "mlp.h"
#include "solver.h"

namespace fil {

// raw features [M][19N] of every filament at the committed state (all filaments have N segments)
int learned_features_launch(const SimDev& d, int N, const double* Yj, const double* qj, const double* F,
                            const double* V, const double* Xj, const double* Xjm1, const double* Xjm2, float* out,
                            hipStream_t st);
// scaled targets [M][6N]: converged unknowns of the last step minus the base Xb of its learned first iterate
int learned_target_launch(const SimDev& d, int N, const double* Xj, const double* Xb, float* out, hipStream_t st);
// X = Xb + de-standardised prediction for the free filaments of N segments in active suspensions
int learned_apply_launch(const SimDev& d, int N, int out_pad, const float* Y, const float* mu, const float* sd,
                         const int32_t* active, const double* Xb, double* X, hipStream_t st);

}  // namespace fil
