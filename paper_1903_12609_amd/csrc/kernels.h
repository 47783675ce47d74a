// Host-side launchers of the filament library's kernels.
#pragma once
#include "common.h"

#include <vector>

namespace fil {

// FP32-tile source record (64 B, all float): the source's offset from the origin of its
// tile (kF32Tile consecutive sources by global index), its force, its torque, and the cross
// products of torque and force with that offset (the parts of T x r and F x r that do not
// depend on the target, formed once per source)
constexpr int kF32Tile = 16;
struct alignas(16) SrcF32 {
    float sp[3];   // fl(Y_m - O_tile)
    float f[3];    // F_m
    float t[3];    // T_m
    float ct[3];   // T_m x sp
    float cf[3];   // 2/3 F_m x sp
    float pad;
};
static_assert(sizeof(SrcF32) == 64, "SrcF32 must be 64 bytes");
// Tile record (32 B): origin (centre of the tile's bounding box) and radius (half the box
// diagonal) in double
struct alignas(16) TileF32 {
    double o[3];
    double rad;
};
static_assert(sizeof(TileF32) == 32, "TileF32 must be 32 bytes");

// Writes the FP64 mobility source record of segment m: 16 doubles [Y, F, T, T x Y, 2/3 F x Y, 0].
__device__ __forceinline__ void rpy_pack_record_f64(double* pk, int64_t m, double y0, double y1, double y2,
                                                    double f0, double f1, double f2, double t0, double t1, double t2) {
    double2* o = reinterpret_cast<double2*>(pk + 16 * m);
    constexpr double k23 = 2.0 / 3.0;
    o[0] = make_double2(y0, y1);
    o[1] = make_double2(y2, f0);
    o[2] = make_double2(f1, f2);
    o[3] = make_double2(t0, t1);
    o[4] = make_double2(t2, t1 * y2 - t2 * y1);
    o[5] = make_double2(t2 * y0 - t0 * y2, t0 * y1 - t1 * y0);
    o[6] = make_double2(k23 * (f1 * y2 - f2 * y1), k23 * (f2 * y0 - f0 * y2));
    o[7] = make_double2(k23 * (f0 * y1 - f1 * y0), 0.0);
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

// Batched (ragged) plan: the work list, built and sorted on the host once; its device copy
// (lists_bytes(), filled by rpy_batch_upload) is read by every launch.  Each launch also takes
// a workspace of work_bytes(): source records, FP32 tile records and split-K partials.
struct RpyBatchPlan {
    int prec = 0;
    int64_t Sg = 0;
    std::vector<RpyItem> items;
    std::vector<RpySusp> sus;
    std::vector<int32_t> seg_susp;
    size_t pack_bytes = 0, tile_bytes = 0, part_bytes = 0;
    size_t ctr_bytes = 256;  // the work-item counter of one apply (cleared at its start)
    size_t items_bytes = 0, sus_bytes = 0, segs_bytes = 0;
    bool any_reduce = false;
    size_t work_bytes() const { return pack_bytes + tile_bytes + part_bytes + ctr_bytes; }
    size_t lists_bytes() const { return items_bytes + sus_bytes + segs_bytes; }
};
RpyBatchPlan rpy_batch_plan(int64_t nsusp, const int64_t* susp_off, int prec);
// copies the plan's lists into `lists` (device, lists_bytes()), host -> device on `st`; the
// plan's host vectors must stay alive until the copy has completed
int rpy_batch_upload(const RpyBatchPlan& p, void* lists, hipStream_t st);
// counter_clear: the work-item counter in `work` is known to be zero (cleared when the
// workspace was made and by every apply of a plan that sums partials); else it is cleared first
int rpy_batch_launch(const RpyBatchPlan& p, const void* lists, const double* Y, const double* F, const double* T,
                     double a, double eta, double* V, double* W, void* work, hipStream_t st, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr, bool packed = false, const int32_t* active = nullptr,
                     bool counter_clear = false);
// byte offset of the work-item counter in an apply's workspace
inline size_t rpy_batch_counter_offset(const RpyBatchPlan& p) { return p.pack_bytes + p.tile_bytes + p.part_bytes; }

struct RpyPlan {
    int64_t S;
    int prec;
    int tpl;        // targets per lane
    int ws;         // waves sharing one target group (splitting its sources)
    int64_t tb;
    int K;
    int64_t chunk;
    size_t pack_bytes;
    size_t tile_bytes;  // FP32-tile tile records (0 in FP64)
    size_t part_bytes;
    size_t total() const { return pack_bytes + tile_bytes + part_bytes; }
};
RpyPlan rpy_plan(int64_t S, int prec);
// ev0/ev1 (may be null) are recorded on `st` just before and after the main pair kernel.
// packed: the FP64 source records are already in the workspace (F, T unused; the FP32-tile
// records are always written here, from Y, F, T).
// reduce: false leaves the K partials in the workspace (rpy_partials) for the caller.
// active: optional device flag of the (single) suspension; when it is 0 the pair kernel exits at once.
int rpy_launch(const RpyPlan& p, const double* Y, const double* F, const double* T, double a, double eta, double* V,
               double* W, void* work, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
               bool packed = false, bool reduce = true, const int32_t* active = nullptr);
inline double* rpy_partials(const RpyPlan& p, void* work) {
    return reinterpret_cast<double*>(static_cast<char*>(work) + p.pack_bytes + p.tile_bytes);
}
int internal_forces_launch(int64_t M, int64_t S, const int64_t* fil_off, const double* q, const double* Lam,
                           const double* kap, double dL, double KB, double KT, double* F, double* T, hipStream_t st);


}  // namespace fil
