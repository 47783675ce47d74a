// Internal interface of the learned warm start's network (mlp.hip) used by the
// simulation (sim.hip).
#pragma once
#include "common.h"

namespace fil {

// features per segment: position (3), quaternion (4), force (3), velocity (3),
// history of the six unknowns the segment owns (6)
constexpr int kMlpFeatPerSeg = 19;

int mlp_forward_rows(fil_mlp* m, int rows, const uint16_t* X, float* Y, hipStream_t st);
int mlp_standardize(fil_mlp* m, int64_t n, const float* feat, const float* targ, uint16_t* xb, float* t,
                    hipStream_t st);
const float* mlp_norm(const fil_mlp* m);  // device [mu_in | sd_in | mu_out | sd_out] (padded dims)
int mlp_segments(const fil_mlp* m);
int mlp_in_pad(const fil_mlp* m);
int mlp_out_pad(const fil_mlp* m);
int mlp_max_batch(const fil_mlp* m);

}  // namespace fil
