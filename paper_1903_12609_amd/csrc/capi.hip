// extern "C" entry points of the filament library: argument checking, workspace
// sizing and dispatch to the kernels' launchers.
#include <cmath>
#include <string>

#include "common.h"
#include "kernels.h"

namespace fil {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace fil

using namespace fil;

extern "C" {

const char* fil_last_error(void) { return g_last_error.c_str(); }

int64_t fil_rpy_workspace_bytes(int64_t S, int prec) {
    if (S < 0 || (prec != FIL_PREC_F64 && prec != FIL_PREC_F32TILE)) return -1;
    return (int64_t)rpy_plan(S, prec).total();
}

int fil_rpy_mobility_apply(int64_t S, const double* Y, const double* F, const double* T, double a, double eta,
                           int prec, double* V, double* Omega, void* work, int64_t work_bytes, void* stream) {
    FIL_CHECK_ARG(S >= 0, "fil_rpy_mobility_apply: S < 0");
    FIL_CHECK_ARG(prec == FIL_PREC_F64 || prec == FIL_PREC_F32TILE, "fil_rpy_mobility_apply: unknown precision");
    FIL_CHECK_ARG(std::isfinite(a) && a > 0 && std::isfinite(eta) && eta > 0,
                  "fil_rpy_mobility_apply: a and eta must be finite and > 0");
    if (S == 0) return FIL_OK;
    FIL_CHECK_ARG(Y && F && T && V && Omega, "fil_rpy_mobility_apply: null array");
    FIL_CHECK_ARG(V != Omega && V != Y && V != F && V != T && Omega != Y && Omega != F && Omega != T,
                  "fil_rpy_mobility_apply: outputs alias inputs");
    const RpyPlan p = rpy_plan(S, prec);
    FIL_CHECK_ARG(work_bytes >= (int64_t)p.total() && (work || p.total() == 0),
                  "fil_rpy_mobility_apply: workspace smaller than fil_rpy_workspace_bytes()");
    return rpy_launch(p, Y, F, T, a, eta, V, Omega, work, (hipStream_t)stream);
}

int64_t fil_rpy_batched_workspace_bytes(int64_t nsusp, const int64_t* susp_off, int prec) {
    if (nsusp < 1 || !susp_off || susp_off[0] != 0 || (prec != FIL_PREC_F64 && prec != FIL_PREC_F32TILE)) return -1;
    for (int64_t i = 0; i < nsusp; i++)
        if (susp_off[i + 1] < susp_off[i]) return -1;
    return (int64_t)rpy_batch_plan(nsusp, susp_off, prec).total();
}

int fil_rpy_mobility_apply_batched(int64_t nsusp, const int64_t* susp_off, const double* Y, const double* F,
                                   const double* T, double a, double eta, int prec, double* V, double* Omega,
                                   void* work, int64_t work_bytes, void* stream) {
    FIL_CHECK_ARG(nsusp >= 1 && susp_off && susp_off[0] == 0, "fil_rpy_mobility_apply_batched: bad offsets");
    for (int64_t i = 0; i < nsusp; i++)
        FIL_CHECK_ARG(susp_off[i + 1] >= susp_off[i], "fil_rpy_mobility_apply_batched: offsets must not decrease");
    FIL_CHECK_ARG(prec == FIL_PREC_F64 || prec == FIL_PREC_F32TILE,
                  "fil_rpy_mobility_apply_batched: unknown precision");
    FIL_CHECK_ARG(std::isfinite(a) && a > 0 && std::isfinite(eta) && eta > 0,
                  "fil_rpy_mobility_apply_batched: a and eta must be finite and > 0");
    const int64_t S = susp_off[nsusp];
    if (S == 0) return FIL_OK;
    FIL_CHECK_ARG(Y && F && T && V && Omega, "fil_rpy_mobility_apply_batched: null array");
    FIL_CHECK_ARG(V != Omega && V != Y && V != F && V != T && Omega != Y && Omega != F && Omega != T,
                  "fil_rpy_mobility_apply_batched: outputs alias inputs");
    const RpyBatchPlan p = rpy_batch_plan(nsusp, susp_off, prec);
    FIL_CHECK_ARG(work && work_bytes >= (int64_t)p.total(),
                  "fil_rpy_mobility_apply_batched: workspace smaller than fil_rpy_batched_workspace_bytes()");
    int rc = rpy_batch_upload(p, work, (hipStream_t)stream);
    if (rc) return rc;
    rc = rpy_batch_launch(p, Y, F, T, a, eta, V, Omega, work, (hipStream_t)stream);
    if (rc) return rc;
    // the host-side lists must outlive the asynchronous upload
    FIL_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    return FIL_OK;
}

int fil_filament_internal_forces(int64_t M, int64_t S, const int64_t* fil_off, const double* q,
                                 const double* Lambda, const double* kappa, double dL, double KB, double KT,
                                 double* F, double* T, void* stream) {
    FIL_CHECK_ARG(M >= 0 && S >= M, "fil_filament_internal_forces: need 0 <= M <= S");
    FIL_CHECK_ARG(std::isfinite(dL) && dL > 0, "fil_filament_internal_forces: dL must be > 0");
    if (M == 0) return FIL_OK;
    FIL_CHECK_ARG(fil_off && q && F && T && (Lambda || S == M), "fil_filament_internal_forces: null array");
    return internal_forces_launch(M, S, fil_off, q, Lambda, kappa, dL, KB, KT, F, T, (hipStream_t)stream);
}

}  // extern "C"
