// Host-side launchers of the filament library's kernels.
#pragma once
#include "common.h"

namespace fil {

struct RpyPlan {
    int64_t S;
    int prec;
    int tpl;
    int64_t tb;
    int K;
    int64_t chunk;
    size_t pack_bytes;
    size_t part_bytes;
    size_t total() const { return pack_bytes + part_bytes; }
};
RpyPlan rpy_plan(int64_t S, int prec);
int rpy_launch(const RpyPlan& p, const double* Y, const double* F, const double* T, double a, double eta, double* V,
               double* W, void* work, hipStream_t st);
int internal_forces_launch(int64_t M, int64_t S, const int64_t* fil_off, const double* q, const double* Lam,
                           const double* kap, double dL, double KB, double KT, double* F, double* T, hipStream_t st);


}  // namespace fil
