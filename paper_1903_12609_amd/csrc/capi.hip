// extern "C" entry points of the filament library: argument checking, workspace
// sizing and dispatch to the kernels' launchers.
#include <cmath>
#include <map>
#include <mutex>
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
    return fil_rpy_mobility_apply_timed(S, Y, F, T, a, eta, prec, V, Omega, work, work_bytes, nullptr, nullptr,
                                        stream);
}

int fil_rpy_mobility_apply_timed(int64_t S, const double* Y, const double* F, const double* T, double a, double eta,
                                 int prec, double* V, double* Omega, void* work, int64_t work_bytes, void* ev_start,
                                 void* ev_end, void* stream) {
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
    return rpy_launch(p, Y, F, T, a, eta, V, Omega, work, (hipStream_t)stream, (hipEvent_t)ev_start,
                      (hipEvent_t)ev_end);
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free apply
// The workspace of fil_rpy_mobility_apply_noalloc: a static device array, one copy per GPU
// (each GPU holds it until the process ends).  Host code never passes the array's name to a
// kernel: it uses the device address hipGetSymbolAddress returns, looked up once per device.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

int scratch_address(void** out) {
    int dev = 0;
    FIL_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        FIL_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return FIL_OK;
}
}  // namespace

extern "C" {

int fil_rpy_mobility_apply_noalloc(int64_t S, const double* Y, const double* F, const double* T, double a,
                                   double eta, int prec, double* V, double* Omega, void* stream) {
    FIL_CHECK_ARG(S >= 0, "fil_rpy_mobility_apply_noalloc: S < 0");
    FIL_CHECK_ARG(prec == FIL_PREC_F64 || prec == FIL_PREC_F32TILE,
                  "fil_rpy_mobility_apply_noalloc: unknown precision");
    FIL_CHECK_ARG(std::isfinite(a) && a > 0 && std::isfinite(eta) && eta > 0,
                  "fil_rpy_mobility_apply_noalloc: a and eta must be finite and > 0");
    if (S == 0) return FIL_OK;
    FIL_CHECK_ARG(Y && F && T && V && Omega, "fil_rpy_mobility_apply_noalloc: null array");
    FIL_CHECK_ARG(V != Omega && V != Y && V != F && V != T && Omega != Y && Omega != F && Omega != T,
                  "fil_rpy_mobility_apply_noalloc: outputs alias inputs");
    const RpyPlan p = rpy_plan(S, prec);
    FIL_CHECK_ARG(p.total() <= kNoAllocScratchBytes,
                  "fil_rpy_mobility_apply_noalloc: S = " + std::to_string(S) + " needs " +
                      std::to_string(p.total()) + " bytes of scratch; the static buffer holds " +
                      std::to_string(kNoAllocScratchBytes) + " (use fil_rpy_mobility_apply with a workspace)");
    void* ptr = nullptr;
    if (int rc = scratch_address(&ptr)) return rc;
    return rpy_launch(p, Y, F, T, a, eta, V, Omega, ptr, (hipStream_t)stream);
}

int64_t fil_rpy_noalloc_scratch_bytes(void) { return (int64_t)kNoAllocScratchBytes; }

}  // extern "C"

struct fil_rpy_batch {
    RpyBatchPlan p;
    void* lists = nullptr;  // device copy of the work list
};

extern "C" {

int fil_rpy_batch_create(int64_t nsusp, const int64_t* susp_off, int prec, fil_rpy_batch** out) {
    FIL_CHECK_ARG(out, "fil_rpy_batch_create: out is null");
    *out = nullptr;
    FIL_CHECK_ARG(nsusp >= 1 && susp_off && susp_off[0] == 0, "fil_rpy_batch_create: bad offsets");
    for (int64_t i = 0; i < nsusp; i++)
        FIL_CHECK_ARG(susp_off[i + 1] >= susp_off[i], "fil_rpy_batch_create: offsets must not decrease");
    FIL_CHECK_ARG(susp_off[nsusp] <= ((int64_t)1 << 31) - 1, "fil_rpy_batch_create: more than 2^31 - 1 segments");
    FIL_CHECK_ARG(prec == FIL_PREC_F64 || prec == FIL_PREC_F32TILE, "fil_rpy_batch_create: unknown precision");
    fil_rpy_batch* b = new fil_rpy_batch();
    b->p = rpy_batch_plan(nsusp, susp_off, prec);
    const size_t nb = b->p.lists_bytes();
    if (nb > 0) {
        if (hipMalloc(&b->lists, nb) != hipSuccess) {
            delete b;
            set_error("fil_rpy_batch_create: out of device memory");
            return FIL_ENOMEM;
        }
        int rc = rpy_batch_upload(b->p, b->lists, nullptr);
        if (rc == FIL_OK && hipStreamSynchronize(nullptr) != hipSuccess) {
            set_error("fil_rpy_batch_create: copy of the work list failed");
            rc = FIL_EHIP;
        }
        if (rc) {
            (void)hipFree(b->lists);
            delete b;
            return rc;
        }
    }
    *out = b;
    return FIL_OK;
}

int64_t fil_rpy_batch_workspace_bytes(const fil_rpy_batch* plan) {
    return plan ? (int64_t)plan->p.work_bytes() : -1;
}

int fil_rpy_mobility_apply_batched(const fil_rpy_batch* plan, const double* Y, const double* F, const double* T,
                                   double a, double eta, double* V, double* Omega, void* work, int64_t work_bytes,
                                   void* stream) {
    FIL_CHECK_ARG(plan, "fil_rpy_mobility_apply_batched: null plan");
    FIL_CHECK_ARG(std::isfinite(a) && a > 0 && std::isfinite(eta) && eta > 0,
                  "fil_rpy_mobility_apply_batched: a and eta must be finite and > 0");
    const RpyBatchPlan& p = plan->p;
    if (p.Sg == 0) return FIL_OK;
    FIL_CHECK_ARG(Y && F && T && V && Omega, "fil_rpy_mobility_apply_batched: null array");
    FIL_CHECK_ARG(V != Omega && V != Y && V != F && V != T && Omega != Y && Omega != F && Omega != T,
                  "fil_rpy_mobility_apply_batched: outputs alias inputs");
    FIL_CHECK_ARG(work_bytes >= (int64_t)p.work_bytes() && (work || p.work_bytes() == 0),
                  "fil_rpy_mobility_apply_batched: workspace smaller than fil_rpy_batch_workspace_bytes()");
    return rpy_batch_launch(p, plan->lists, Y, F, T, a, eta, V, Omega, work, (hipStream_t)stream);
}

void fil_rpy_batch_destroy(fil_rpy_batch* plan) {
    if (!plan) return;
    if (plan->lists) (void)hipFree(plan->lists);
    delete plan;
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
