// Host-side launchers of the filament library's kernels.
#pragma once
#include "common.h"

#include <vector>

namespace fil {

// FP32-tile source record: position in double, force and torque in float (64 B)
struct alignas(16) SrcF32 {
    double y[3];
    float f[3];
    float t[3];
    float pad[4];
};
static_assert(sizeof(SrcF32) == 64, "SrcF32 must be 64 bytes");

// Writes the mobility source record of segment m: FP64 records are 16 doubles
// [Y, F, T, T x Y, F x Y, 0]; FP32-tile records are SrcF32.
__device__ __forceinline__ void rpy_pack_record(int prec, void* pk, int64_t m, double y0, double y1, double y2,
                                                double f0, double f1, double f2, double t0, double t1, double t2) {
    if (prec == FIL_PREC_F64) {
        double2* o = reinterpret_cast<double2*>(static_cast<double*>(pk) + 16 * m);
        o[0] = make_double2(y0, y1);
        o[1] = make_double2(y2, f0);
        o[2] = make_double2(f1, f2);
        o[3] = make_double2(t0, t1);
        o[4] = make_double2(t2, t1 * y2 - t2 * y1);
        o[5] = make_double2(t2 * y0 - t0 * y2, t0 * y1 - t1 * y0);
        o[6] = make_double2(f1 * y2 - f2 * y1, f2 * y0 - f0 * y2);
        o[7] = make_double2(f0 * y1 - f1 * y0, 0.0);
    } else {
        SrcF32 s;
        s.y[0] = y0; s.y[1] = y1; s.y[2] = y2;
        s.f[0] = (float)f0; s.f[1] = (float)f1; s.f[2] = (float)f2;
        s.t[0] = (float)t0; s.t[1] = (float)t1; s.t[2] = (float)t2;
        s.pad[0] = s.pad[1] = s.pad[2] = s.pad[3] = 0.f;
        static_cast<SrcF32*>(pk)[m] = s;
    }
}

// Work item of the persistent RPY launch: a target block x source chunk of one suspension.
struct RpyItem {
    int64_t base;   // first global segment of the suspension
    int64_t part;   // offset (doubles) of the suspension's partial results
    int32_t S;      // segments of the suspension
    int32_t tb;     // target block
    int32_t k;      // source chunk
    int32_t K;      // chunks of the suspension
    int64_t chunk;  // sources per chunk
    int32_t susp;   // suspension index
    int32_t pad;
};
struct RpySusp {
    int64_t base, part;
    int32_t S, K;
};

// Batched (ragged) plan: host-side lists, uploaded into the workspace.
struct RpyBatchPlan {
    int prec = 0;
    int64_t Sg = 0;
    std::vector<RpyItem> items;
    std::vector<RpySusp> sus;
    std::vector<int32_t> seg_susp;
    size_t pack_bytes = 0, part_bytes = 0, items_bytes = 0, sus_bytes = 0, segs_bytes = 0;
    bool any_reduce = false;
    size_t total() const { return pack_bytes + part_bytes + items_bytes + sus_bytes + segs_bytes; }
};
RpyBatchPlan rpy_batch_plan(int64_t nsusp, const int64_t* susp_off, int prec);
// copies the plan's lists into `work` (host -> device, on `st`)
int rpy_batch_upload(const RpyBatchPlan& p, void* work, hipStream_t st);
int rpy_batch_launch(const RpyBatchPlan& p, const double* Y, const double* F, const double* T, double a, double eta,
                     double* V, double* W, void* work, hipStream_t st, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr, bool packed = false, const int32_t* active = nullptr);

struct RpyPlan {
    int64_t S;
    int prec;
    int tpl;        // targets per lane
    int ws;         // waves sharing one target group (splitting its sources)
    int64_t tb;
    int K;
    int64_t chunk;
    size_t pack_bytes;
    size_t part_bytes;
    size_t total() const { return pack_bytes + part_bytes; }
};
RpyPlan rpy_plan(int64_t S, int prec);
// ev0/ev1 (may be null) are recorded on `st` just before and after the main pair kernel.
// packed: the source records are already in the workspace (Y, F, T unused).
// reduce: false leaves the K partials in the workspace (rpy_partials) for the caller.
// active: optional device flag of the (single) suspension; when it is 0 the pair kernel exits at once.
int rpy_launch(const RpyPlan& p, const double* Y, const double* F, const double* T, double a, double eta, double* V,
               double* W, void* work, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
               bool packed = false, bool reduce = true, const int32_t* active = nullptr);
inline double* rpy_partials(const RpyPlan& p, void* work) {
    return reinterpret_cast<double*>(static_cast<char*>(work) + p.pack_bytes);
}
int internal_forces_launch(int64_t M, int64_t S, const int64_t* fil_off, const double* q, const double* Lam,
                           const double* kap, double dL, double KB, double KT, double* F, double* T, hipStream_t st);


}  // namespace fil
