// Host orchestration of the implicit step (fil_sim): device state, workspace,
// the Broyden loop and the extern "C" entry points declared in fil.h.
//
// One step (Sec. 2.9.3, Alg. 2, Sec. 3.2.2):
//   X0 = warm start; f0 = f(X0); J0 = df0/dX at X0 (Appendix B.2), inverted per
//   filament; X1 = X0 - J0^{-1} f0; then for k = 1, 2, ...: f_k = f(X_k)
//   (one mobility apply), stop when max|f_k|/a <= tol, else the bad-Broyden
//   update reusing H_{k-1} f_k for both c_k and the next step.
// Convergence is tested on the host once per iteration (one small D2H copy),
// or, with graph execution on, on the device: blocks of U iterations (each an
// evaluation, the convergence test and the Broyden update) are captured once
// into a HIP graph and replayed, and the host reads the per-suspension state
// once per block.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "learned.h"
#include "solver.h"

using namespace fil;

struct fil_sim {
    fil_params p{};
    int64_t S = 0, M = 0, nsusp = 0;
    hipStream_t st = nullptr;
    std::vector<void*> dev_allocs;
    std::vector<void*> host_allocs;
    SimDev d{};
    double *Yj = nullptr, *Yjm1 = nullptr, *qj = nullptr, *Xj = nullptr, *Xjm1 = nullptr, *Xjm2 = nullptr;
    double* X0p = nullptr;  // extrapolated first iterate of the last step (the plain warm start)
    double* Xb = nullptr;   // base of the learned first iterate of the last step
    double *X = nullptr, *f = nullptr, *fprev = nullptr;
    double *Yc = nullptr, *qc = nullptr, *F = nullptr, *T = nullptr, *V = nullptr, *W = nullptr;
    double *AB = nullptr, *AinvT = nullptr, *Chist = nullptr, *Dhist = nullptr, *part = nullptr;
    double* gsolve = nullptr;  // J0^{-1} f formed before the update (band path, many filaments)
    double* BC = nullptr;      // the band factor's column records for that solve
    double* rdiag = nullptr;  // reciprocal pivots of the band factor [6S]
    double* box = nullptr;
    double* spar = nullptr;  // [nsusp][kSpar]
    int32_t *ipiv = nullptr, *active_d = nullptr, *jflag_d = nullptr;
    unsigned long long* resbits_d = nullptr;
    int32_t *active_h = nullptr, *jflag_h = nullptr;
    unsigned long long* resbits_h = nullptr;
    // mobility plans and workspaces: [0] FP64, [1] FP32-tile (only when prec is FP32-tile)
    void* rpy_work[2] = {nullptr, nullptr};
    void* rpy_lists[2] = {nullptr, nullptr};  // device work lists of the batched plans
    RpyPlan rplan[2]{};
    RpyBatchPlan bplan[2];
    int cur = 0;  // plan of the next residual evaluation
    int rb = 0;   // which half of resbits_d the last residual evaluation wrote
    bool batched = false;
    // device time t^{j+1} (read by the state kernel) and its pinned staging slot
    double *time_d = nullptr, *time_h = nullptr;
    // graph execution of the Broyden iterations
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;
        int rb_end = 0;
    };
    int graph_iters = 0;  // iterations per captured block; 0 runs every iteration from the host
    int pred_iters = 0;   // iterations the last device-driven solve took (0: none yet)
    int pred_iters32 = 0;  // the same for the FP32-tile iterations of FP32-tile mode
    int* notnear_d = nullptr;  // FP32-tile iterations: running suspensions not near the switch
    int koff = 0;         // iteration at which the Broyden history last restarted (update k = it - 1 - koff)
    hipStream_t cap_st = nullptr;  // private stream the blocks are captured on (launches go to st)
    double* fext_d = nullptr;      // [3][S] external forces per segment (null until set)
    // force-coupling-method mobility of a periodic box (null: the unbounded RPY mobility);
    // its iterations run host-driven (the FFTs are not captured)
    fil_fcm* fcm = nullptr;
    // geometric-switch base torques of pinned filaments (their state on the device)
    bool sw = false;
    SwitchArgs swa{};
    double* text_d = nullptr;  // [3][S] external torques the switch writes
    // the RPY mobility above a no-slip wall at z = 0 in place of the unbounded one
    bool wall = false;
    void* wall_work = nullptr;
    // Newton-Krylov workspace (allocated on first use): Krylov basis [(m+1)][6S], residuals
    // at the Newton point and a perturbed point, work vectors, P^{-1} diagonal, dot partials
    int kry_m = 0;
    double *kry_V = nullptr, *kry_f0 = nullptr, *kry_fp = nullptr, *kry_Xp = nullptr, *kry_w = nullptr,
           *kry_u = nullptr, *kry_x = nullptr, *kry_pinv = nullptr, *kry_partial = nullptr, *kry_dots_d = nullptr,
           *kry_coef_d = nullptr;
    double *kry_dots_h = nullptr, *kry_coef_h = nullptr;
    double *kry_f00 = nullptr, *kry_spar0 = nullptr;  // f0 at the initial guess; parameters without external forces
    unsigned long long* kry_rb = nullptr;              // maxima of f0 evaluations (unused, two alternating pairs)
    int kry_rbi = 0;
    std::map<std::array<int, 6>, GraphEntry> graphs;
    SuspLog* log_d = nullptr;  // device log of the current solve [nsusp]
    SuspLog* log_h = nullptr;  // staging of the host's counts when the device takes over a solve
    // two pinned slots for the logs of graph blocks in flight, each with its export's event
    SuspLog* log_slot[2] = {nullptr, nullptr};
    SuspLog* log_slot_dev[2] = {nullptr, nullptr};  // the same slots as the device addresses them
    hipEvent_t log_ev[2] = {nullptr, nullptr};
    int64_t* exports_d = nullptr;  // exports so far (device; selects the slot), mirrored by exports_h
    int64_t exports_h = 0;
    // learned warm start
    fil_mlp* mlp = nullptr;
    bool use_mlp = false;
    int seg_uniform = 0;           // N when every filament has N segments, else 0
    float* feat = nullptr;         // [M][19N] raw features
    uint16_t* featb = nullptr;     // [M][in_pad] standardised BF16 features
    float* pred = nullptr;         // [M][out_pad] network output
    int feat_in_pad = 0, feat_out_pad = 0;
    int64_t fallbacks = 0;
    double t = 0.0;
    int64_t step = 0;
    int k = 0;
    BdfCoef bc{};
    std::vector<int64_t> susp_seg_off;
    std::vector<int64_t> fil_seg_off_h;  // filament offsets (host copy, for checkpoint checks)
    bool has_motor = false;   // some filament's base sits on the rotating motor (tether 3)
    bool dt_differ = false;   // fil_set_suspension_params gave a suspension its own time step
    // optional timing of the main mobility kernel: one event pair per apply of a step
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int nev = 0;
    std::vector<int> ev_prec;  // plan of each recorded launch
    double rpy_ms[2] = {0.0, 0.0};
    int64_t rpy_launches[2] = {0, 0};
    int64_t pairs_per_apply = 0;
};

namespace {

template <class T>
int dalloc(fil_sim* s, T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    void* q = nullptr;
    if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) {
        set_error("fil_create: device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
        return FIL_ENOMEM;
    }
    s->dev_allocs.push_back(q);
    *p = static_cast<T*>(q);
    return FIL_OK;
}
template <class T>
int halloc(fil_sim* s, T** p, size_t n) {
    void* q = nullptr;
    if (hipHostMalloc(&q, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault) != hipSuccess) {
        set_error("fil_create: pinned host allocation failed");
        return FIL_ENOMEM;
    }
    s->host_allocs.push_back(q);
    *p = static_cast<T*>(q);
    return FIL_OK;
}
template <class T>
int upload(T* dst, const std::vector<T>& src) {
    if (!src.empty()) FIL_HIP_TRY(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return FIL_OK;
}

#define TRY(x)                \
    do {                      \
        int _rc = (x);        \
        if (_rc) return _rc;  \
    } while (0)

BdfCoef coefs(int64_t step) {
    if (step == 0) return BdfCoef{1.0, 0.0, 1.0, 0.0};  // BDF1 start
    return BdfCoef{4.0 / 3.0, -1.0 / 3.0, 2.0 / 3.0, 1.0 / 3.0};
}

// FP32-tile mode: the switch to FP64 evaluations happens once every running
// suspension has max|f|/a <= max(kSwitchTol tol, kNoiseMargin kF32Floor max|b dt V|/a),
// kF32Floor being the measured rounding floor of an FP32-tile apply relative to
// the size of its mobility term.  The margin keeps the FP32 secant pairs well above
// that floor (at 30x the noise they slowed the FP64 finish: 500 x 32 suspension 42.6
// iterations per step against 33.5 in FP64), and the Broyden history restarts at the
// switch (Alg. 2 from the current iterate with the same J0): 31.4 iterations, 16.5 ms
// against 18.9 ms per step in FP64.
constexpr double kSwitchTol = 10.0;
constexpr double kF32Floor = 3e-8;
constexpr double kNoiseMargin = 3000.0;
// timing events of mobility launches not yet read (read when the pool is this full, or on request)
constexpr int kMaxPendingTimings = 256;
// from this many filaments on, the band path forms J0^{-1} f in a kernel of its own before
// the update (inside the update kernel the sweeps run six per CU, a latency-bound chain of
// ~570 cycles per row: 256-suspension ensemble, 8684 filaments, 580 us per update)
constexpr int64_t kLaneSolveMinFil = 256;

// adds the recorded mobility-kernel durations (stream already synchronised)
int collect_timing(fil_sim* s) {
    for (int i = 0; i < s->nev; i++) {
        float ms = 0.f;
        FIL_HIP_TRY(hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]));
        s->rpy_ms[s->ev_prec[i]] += ms;
        s->rpy_launches[s->ev_prec[i]]++;
    }
    s->nev = 0;
    return FIL_OK;
}

// Forgets the captured graph blocks: they hold the device view and the mobility path as
// they were when captured, so every setter that changes either drops them.
void drop_graphs(fil_sim* s) {
    for (auto& kv : s->graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    s->graphs.clear();
    s->pred_iters = s->pred_iters32 = 0;
}

void free_sim(fil_sim* s) {
    if (!s) return;
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->log_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& kv : s->graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (s->cap_st) (void)hipStreamDestroy(s->cap_st);
    if (s->fcm) fil_fcm_destroy(s->fcm);
    for (void* p : s->dev_allocs) (void)hipFree(p);
    for (void* p : s->host_allocs) (void)hipHostFree(p);
    delete s;
}

// a pair of timing events from the pool (null when timing is off)
int pool_events(fil_sim* s, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!s->timing) return FIL_OK;
    while ((int)s->ev.size() < 2 * (s->nev + 1)) {
        hipEvent_t e;
        FIL_HIP_TRY(hipEventCreate(&e));
        s->ev.push_back(e);
    }
    *e0 = s->ev[2 * s->nev];
    *e1 = s->ev[2 * s->nev + 1];
    if ((int)s->ev_prec.size() <= s->nev) s->ev_prec.resize(s->nev + 1);
    s->ev_prec[s->nev] = s->cur;
    s->nev++;
    return FIL_OK;
}

// the time t^{j+1} of the current step, on the device
int set_time(fil_sim* s) {
    FIL_HIP_TRY(hipStreamSynchronize(s->st));  // the staging slot may still feed an earlier copy
    s->time_h[0] = s->t + s->p.dt;
    FIL_HIP_TRY(hipMemcpyAsync(s->time_d, s->time_h, sizeof(double), hipMemcpyHostToDevice, s->st));
    return FIL_OK;
}

// f = f(X) for the active suspensions: the state at X first when `state` (else the
// update kernel left it), then the steric pass, the mobility apply and the residual
// kernel, which also leaves the dot products of Broyden update dots_k (< 0: none).
// resbits receives max|f| per suspension; e0/e1 (may be null) bracket the mobility
// pair kernel.
int eval_residual(fil_sim* s, const double* X, double* fout, hipEvent_t e0, hipEvent_t e1, bool state, int dots_k) {
    if (state)
        TRY(state_forces_launch(s->d, X, s->qj, s->time_d, s->active_d, s->Yc, s->qc, s->F, s->T, s->box, s->st));
    // the source records sit at the start of the mobility workspace in both plans
    const int c = s->cur;
    TRY(steric_pack_launch(s->d, s->Yc, s->box, s->active_d, s->F, s->T, c ? FIL_PREC_F32TILE : FIL_PREC_F64,
                           s->rpy_work[c], s->st));
    const double* part = nullptr;
    int K = 1;
    if (s->fcm) {
        if (e0) FIL_HIP_TRY(hipEventRecord(e0, s->st));
        TRY(fil_fcm_apply(s->fcm, s->S, s->Yc, s->F, s->T, s->V, s->W, s->st));
        if (e1) FIL_HIP_TRY(hipEventRecord(e1, s->st));
    } else if (s->wall) {
        if (e0) FIL_HIP_TRY(hipEventRecord(e0, s->st));
        TRY(rpy_wall_launch(s->S, s->Yc, s->F, s->T, s->p.a, s->p.eta, c ? FIL_PREC_F32TILE : FIL_PREC_F64, s->V,
                            s->W, s->wall_work, s->st));
        if (e1) FIL_HIP_TRY(hipEventRecord(e1, s->st));
    } else if (s->batched) {
        TRY(rpy_batch_launch(s->bplan[c], s->rpy_lists[c], s->Yc, s->F, s->T, s->p.a, s->p.eta, s->V, s->W,
                             s->rpy_work[c], s->st, e0, e1, true, s->active_d, true));
    } else {
        // the split-K partials are summed inside the residual kernel
        TRY(rpy_launch(s->rplan[c], s->Yc, s->F, s->T, s->p.a, s->p.eta, s->V, s->W, s->rpy_work[c], s->st, e0, e1,
                       true, false, s->active_d));
        if (s->rplan[c].K > 1) {
            part = rpy_partials(s->rplan[c], s->rpy_work[c]);
            K = s->rplan[c].K;
        }
    }
    s->rb ^= 1;
    const DotArgs da{dots_k, s->Dhist, s->fprev, s->part};
    TRY(residual_launch(s->d, s->bc, X, s->Xj, s->Yc, s->Yj, s->Yjm1, s->V, s->W, part, K, s->active_d, fout,
                        s->resbits_d + 2 * s->rb * s->nsusp, s->resbits_d + 2 * (1 - s->rb) * s->nsusp, da, s->st));
    return FIL_OK;
}

// Broyden update k (k < 0: the first step) from the residual fnew, then the state at the new X
UpdateArgs update_args(fil_sim* s, int k, const double* fnew, double* dXout) {
    return UpdateArgs{k,     s->AB,    s->ipiv, s->rdiag, s->AinvT, s->part, s->Chist, s->Dhist, fnew, s->fprev,
                      s->X,  dXout,    s->qj,   s->time_d, s->Yc,   s->qc,   s->F,     s->T,     s->box, s->gsolve, s->BC};
}

// the device-side test of iteration it (jflag: singular-J0 flags, first iteration only);
// FP32-tile evaluations cannot end a step and count the suspensions not yet near the switch
JudgeArgs judge_args(fil_sim* s, int it, const int32_t* jflag) {
    const bool f32 = s->cur == 1;
    return JudgeArgs{s->log_d,
                     s->resbits_d + 2 * s->rb * s->nsusp,
                     jflag,
                     s->p.tol,
                     1.0 / s->p.a,
                     it,
                     s->p.kmax,
                     f32 ? 0 : 1,
                     f32 ? s->notnear_d : nullptr,
                     kSwitchTol * s->p.tol,
                     kNoiseMargin * kF32Floor};
}

// max|f|/a and max|b dt (V, dexpinv Omega)| per suspension of the last evaluation
int read_resid(fil_sim* s, std::vector<double>& res, std::vector<double>* vmax = nullptr) {
    const int64_t ns = s->nsusp;
    FIL_HIP_TRY(hipMemcpyAsync(s->resbits_h, s->resbits_d + 2 * s->rb * ns, 2 * ns * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s->st));
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    res.resize(ns);
    if (vmax) vmax->resize(ns);
    for (int64_t i = 0; i < ns; i++) {
        double v;
        std::memcpy(&v, &s->resbits_h[i], sizeof v);
        res[i] = v / s->p.a;
        if (vmax) {
            std::memcpy(&v, &s->resbits_h[ns + i], sizeof v);
            (*vmax)[i] = v / s->p.a;
        }
    }
    return FIL_OK;
}

int upload_flags(fil_sim* s, int32_t* dst, const int32_t* src) {
    FIL_HIP_TRY(hipMemcpyAsync(dst, src, s->nsusp * sizeof(int32_t), hipMemcpyHostToDevice, s->st));
    return FIL_OK;
}

// J0 at the configuration of X (state buffers already filled by eval_residual), factorised
// (and inverted explicitly when the inverses fit)
int begin_solve(fil_sim* s) {
    const double tt = s->t + s->p.dt;
    TRY(j0_factor_launch(s->d, s->bc, s->X, s->qc, s->T, tt, s->active_d, s->AB, s->ipiv, s->rdiag, s->jflag_d,
                         s->AinvT, s->BC, s->st));
    s->k = 0;
    return FIL_OK;
}

// Iterations it0 .. it0+U-1 (evaluation, device-side convergence test, bad-Broyden
// update with k = it-1 and the state at the new iterate) as one HIP graph, captured on first use for this
// (it0, U, precision, resbits parity, first-step coefficients) and replayed on
// the simulation's stream.  The captured work holds no memset, no host copy and
// no timing event (the mobility kernel is timed only in host-driven iterations).
using GraphEntry = fil_sim::GraphEntry;
int capture_block(fil_sim* s, int it0, int U, GraphEntry& g) {
    const int64_t ns = s->nsusp;
    const int rb0 = s->rb;
    // captured on a private stream (the simulation's may be the null stream, which cannot be captured)
    if (!s->cap_st) FIL_HIP_TRY(hipStreamCreateWithFlags(&s->cap_st, hipStreamNonBlocking));
    hipStream_t run_st = s->st;
    s->st = s->cap_st;
    if (hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        s->st = run_st;
        set_error("graph capture could not start");
        return FIL_EHIP;
    }
    int rc = FIL_OK;
    for (int i = 0; i < U && rc == FIL_OK; i++) {
        const int it = it0 + i;
        // FP32-tile iterations: the switch to FP64 is decided on the device before each
        if (s->cur == 1) rc = f32_switch_launch(s->active_d, s->log_d, s->notnear_d, ns, it, s->p.kmax, s->st);
        if (rc == FIL_OK) rc = eval_residual(s, s->X, s->f, nullptr, nullptr, false, it - 1 - s->koff);
        const JudgeArgs jg = judge_args(s, it, nullptr);
        if (rc == FIL_OK)
            rc = broyden_state_launch(s->d, update_args(s, it - 1 - s->koff, s->f, nullptr), jg, s->active_d, s->st);
    }
    // the block ends by exporting its log to the next pinned slot
    if (rc == FIL_OK)
        rc = log_export_launch(s->log_d, ns, s->log_slot_dev[0], s->log_slot_dev[1], s->exports_d, s->st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s->st, &graph);
    s->st = run_st;
    g.rb_end = s->rb;
    s->rb = rb0;
    if (rc == FIL_OK && e != hipSuccess) {
        set_error(std::string("graph capture: ") + hipGetErrorString(e));
        rc = FIL_EHIP;
    }
    if (rc == FIL_OK && hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("graph instantiation failed");
        rc = FIL_EHIP;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != FIL_OK) {
        (void)hipGetLastError();
        g.exec = nullptr;
    }
    return rc;
}

int graph_block(fil_sim* s, int it0, int U) {
    const std::array<int, 6> key{it0, U, s->cur, s->rb, s->step == 0 ? 1 : 0, s->koff};
    auto itg = s->graphs.find(key);
    if (itg == s->graphs.end()) {
        GraphEntry g;
        TRY(capture_block(s, it0, U, g));
        itg = s->graphs.emplace(key, std::move(g)).first;
    }
    FIL_HIP_TRY(hipGraphLaunch(itg->second.exec, s->st));
    s->rb = itg->second.rb_end;
    return FIL_OK;
}

struct SolveLog {
    std::vector<int32_t> state, iters, applies, applies_hi;  // state: 0 running, 1 converged, -1 failed
    std::vector<double> last;
    bool singular = false;
    explicit SolveLog(int64_t ns) : state(ns, 0), iters(ns, 0), applies(ns, 0), applies_hi(ns, 0), last(ns, 0.0) {}
};

// Graph blocks from iteration `it` until every suspension has ended (the device log
// holds the counts so far).  The next block is launched before the log of the
// previous one is read, so the GPU never waits for the host; a block launched after
// the end runs only kernels that find their suspension finished.  Blocks are full
// up to the iteration count of the previous solve and single iterations beyond it,
// which bounds that waste.
int device_iterations(fil_sim* s, SolveLog& L, int it, int& pred_out) {
    const int64_t ns = s->nsusp;
    const int pred = pred_out;
    int pending = 0;
    int rslot = (int)(s->exports_h & 1);
    for (;;) {
        while (pending < 2 && it <= s->p.kmax) {
            int U = s->graph_iters;
            if (pred > 0) U = it <= pred ? std::min(U, pred - it + 1) : 1;
            U = std::min(U, s->p.kmax - it + 1);
            TRY(graph_block(s, it, U));  // ends with the log export to slot (exports so far) mod 2
            it += U;
            s->k += U;
            const int wslot = (int)(s->exports_h++ & 1);
            FIL_HIP_TRY(hipEventRecord(s->log_ev[wslot], s->st));
            pending++;
        }
        if (pending == 0) break;  // every iteration up to kmax has run (its test failed what was left)
        FIL_HIP_TRY(hipEventSynchronize(s->log_ev[rslot]));
        bool any = false;
        for (int64_t i = 0; i < ns; i++) {
            const SuspLog& q = s->log_slot[rslot][i];
            L.state[i] = q.state;
            L.iters[i] = q.it;
            L.applies[i] = q.evals;
            L.applies_hi[i] = q.evals_hi;
            L.last[i] = q.last;
            s->active_h[i] = q.state == 0;
            any |= q.state == 0;
        }
        rslot ^= 1;
        pending--;
        if (!any) break;
    }
    pred_out = *std::max_element(L.iters.begin(), L.iters.end());
    return FIL_OK;
}

// Alg. 2 from the iterate in s->X for every active suspension: f_0 = f(X_0), J0
// at X_0 and its inverse, X_1 = X_0 - J0^{-1} f_0, then one evaluation and one
// bad-Broyden update per iteration until every suspension has converged or failed.
// The iterations run in captured graph blocks when enabled, with every test on the
// device (the first one included) and no host round trip between blocks, or one by one
// from the host.  In FP32-tile mode the evaluations start in FP32 and switch to FP64 once
// every running suspension is near the tolerance or near the FP32 rounding floor (in
// graph blocks the switch is decided on the device before each iteration and the FP64
// blocks take over from the host at the switch); only an FP64 residual can end a step.
int solve(fil_sim* s, SolveLog& L) {
    const int64_t ns = s->nsusp;
    s->cur = s->p.prec == FIL_PREC_F32TILE ? 1 : 0;
    s->koff = 0;
    std::vector<double> res, vmx;
    bool changed = false;
    auto count = [&]() {
        for (int64_t i = 0; i < ns; i++)
            if (s->active_h[i]) {
                L.applies[i]++;
                L.applies_hi[i] += s->cur == 0;
            }
    };
    auto judge = [&](int it) -> bool {
        bool any = false, near = true;
        for (int64_t i = 0; i < ns; i++) {
            if (!s->active_h[i]) continue;
            L.iters[i] = it;
            L.last[i] = res[i];
            if (!std::isfinite(res[i])) L.state[i] = -1;
            else if (res[i] <= s->p.tol && s->cur == 0) L.state[i] = 1;
            else if (it >= s->p.kmax) L.state[i] = -1;
            if (L.state[i] != 0) {
                s->active_h[i] = 0;
                changed = true;
                continue;
            }
            any = true;
            near &= res[i] <= std::max(kSwitchTol * s->p.tol, kNoiseMargin * kF32Floor * vmx[i]);
        }
        if (s->cur == 1 && any && (near || 2 * it >= s->p.kmax)) s->cur = 0;
        return any;
    };
    auto singular = [&]() {
        for (int64_t f = 0; f < s->M; f++)
            if (s->jflag_h[f]) {
                set_error("fil_bdf2_step: approximate Jacobian block of filament " + std::to_string(f) + " is singular");
                std::fill(L.state.begin(), L.state.end(), -1);
                L.singular = true;
                return true;
            }
        return false;
    };
    hipEvent_t e0, e1;
    TRY(pool_events(s, &e0, &e1));
    TRY(eval_residual(s, s->X, s->f, e0, e1, true, -1));
    TRY(begin_solve(s));
    const bool graphs = s->graph_iters > 0 && !s->fcm;
    if (graphs) {
        // the first test runs in the first-step kernel (the log was cleared at the start
        // of the step), which also fails a suspension with a singular J0 block
        if (s->cur == 1) TRY(f32_switch_launch(s->active_d, s->log_d, s->notnear_d, ns, -1, s->p.kmax, s->st));
        TRY(broyden_state_launch(s->d, update_args(s, -1, s->f, nullptr), judge_args(s, 0, s->jflag_d), s->active_d,
                                 s->st));
        if (s->cur == 1) {
            // FP32-tile iterations until the device switches; the switched suspensions then
            // continue with FP64 evaluations from the next iteration, the Broyden history
            // restarting there (as in the host-driven loop below)
            TRY(device_iterations(s, L, 1, s->pred_iters32));
            int its = -1;
            for (int64_t i = 0; i < ns; i++)
                if (L.state[i] == 2) {
                    its = L.iters[i] + 1;
                    L.state[i] = 0;
                }
            if (its > 0) {
                for (int64_t i = 0; i < ns; i++) {
                    s->active_h[i] = L.state[i] == 0;
                    s->log_h[i] = SuspLog{L.state[i], L.iters[i], L.applies[i], L.applies_hi[i], L.last[i]};
                }
                FIL_HIP_TRY(hipMemcpyAsync(s->log_d, s->log_h, ns * sizeof(SuspLog), hipMemcpyHostToDevice, s->st));
                TRY(upload_flags(s, s->active_d, s->active_h));
                s->cur = 0;
                s->koff = its;
                TRY(device_iterations(s, L, its, s->pred_iters));
            }
        } else {
            TRY(device_iterations(s, L, 1, s->pred_iters));
        }
        for (int64_t i = 0; i < ns; i++)
            if (L.state[i] == -2) {
                set_error("fil_bdf2_step: an approximate Jacobian block of suspension " + std::to_string(i) +
                          " is singular");
                std::fill(L.state.begin(), L.state.end(), -1);
                L.singular = true;
                break;
            }
        return FIL_OK;
    }
    count();
    TRY(read_resid(s, res, &vmx));
    FIL_HIP_TRY(hipMemcpyAsync(s->jflag_h, s->jflag_d, s->M * sizeof(int32_t), hipMemcpyDeviceToHost, s->st));
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    bool any = judge(0);
    if (singular()) {
        for (int64_t i = 0; i < ns; i++) s->active_h[i] = 0;
        changed = true;
        any = false;
    }
    if (changed) TRY(upload_flags(s, s->active_d, s->active_h));
    if (any) TRY(broyden_state_launch(s->d, update_args(s, -1, s->f, nullptr), JudgeArgs{}, s->active_d, s->st));
    bool restart = false;  // the evaluation of this iteration is the first FP64 one after FP32 tiles
    for (int it = 1; any;) {
        count();
        TRY(pool_events(s, &e0, &e1));
        TRY(eval_residual(s, s->X, s->f, e0, e1, false, restart ? -1 : s->k));
        TRY(read_resid(s, res, &vmx));
        changed = false;
        const int cur_before = s->cur;
        any = judge(it);
        if (!any) break;
        if (changed) TRY(upload_flags(s, s->active_d, s->active_h));
        // a restart takes Alg. 2's first step X <- X - J0^{-1} f from the first FP64 residual
        TRY(broyden_state_launch(s->d, update_args(s, restart ? -1 : s->k, s->f, nullptr), JudgeArgs{}, s->active_d,
                                 s->st));
        s->k = restart ? 0 : s->k + 1;
        restart = cur_before == 1 && s->cur == 0;
        it++;
    }
    return FIL_OK;
}

int ensure_learned_buffers(fil_sim* s, int in_pad, int out_pad) {
    if (!s->feat) TRY(dalloc(s, &s->feat, (size_t)s->M * kMlpFeatPerSeg * s->seg_uniform));
    if (in_pad && (!s->featb || s->feat_in_pad != in_pad || s->feat_out_pad != out_pad)) {
        TRY(dalloc(s, &s->featb, (size_t)s->M * in_pad));
        TRY(dalloc(s, &s->pred, (size_t)s->M * out_pad));
        s->feat_in_pad = in_pad;
        s->feat_out_pad = out_pad;
    }
    return FIL_OK;
}

// X = Xb + the network's prediction for every free filament (Xb: X0 plus the last step's correction)
int learned_guess(fil_sim* s) {
    fil_mlp* m = s->mlp;
    const int N = s->seg_uniform;
    TRY(learned_features_launch(s->d, N, s->Yj, s->qj, s->F, s->V, s->Xj, s->Xjm1, s->Xjm2, s->feat, s->st));
    TRY(mlp_standardize(m, s->M, s->feat, nullptr, s->featb, nullptr, s->st));
    TRY(mlp_forward_rows(m, (int)s->M, s->featb, s->pred, s->st));
    const float* nrm = mlp_norm(m);
    const float* mu = nrm + 2 * mlp_in_pad(m);
    TRY(learned_apply_launch(s->d, N, mlp_out_pad(m), s->pred, mu, mu + mlp_out_pad(m), s->active_d, s->Xb, s->X,
                             s->st));
    return FIL_OK;
}

}  // namespace

extern "C" {

int fil_create(const fil_params* p, int64_t nsusp, const int64_t* susp_fil_off, const int64_t* fil_seg_off,
               const double* Y0, const double* q0, const double* phase, const int32_t* tether, fil_sim** out) {
    FIL_CHECK_ARG(out, "fil_create: out is null");
    *out = nullptr;
    FIL_CHECK_ARG(p && susp_fil_off && fil_seg_off && Y0 && q0, "fil_create: null argument");
    FIL_CHECK_ARG(nsusp >= 1, "fil_create: nsusp must be >= 1");
    FIL_CHECK_ARG(p->a > 0 && p->eta > 0 && p->dL > 0 && p->dt > 0 && p->tol > 0 && std::isfinite(p->dt),
                  "fil_create: a, eta, dL, dt and tol must be > 0");
    FIL_CHECK_ARG(p->kmax >= 1 && p->kmax < kMaxIter, "fil_create: kmax must be in [1, 255]");
    FIL_CHECK_ARG(p->prec == FIL_PREC_F64 || p->prec == FIL_PREC_F32TILE, "fil_create: unknown precision");
    FIL_CHECK_ARG(p->j0_mode >= 0 && p->j0_mode <= 2, "fil_create: j0_mode must be 0, 1 or 2");
    FIL_CHECK_ARG(p->j0_factor == 0 || p->j0_factor == 1, "fil_create: j0_factor must be 0 or 1");
    FIL_CHECK_ARG(p->FS == 0.0 || p->chi > 1.0, "fil_create: the steric range chi must exceed 1");
    FIL_CHECK_ARG(susp_fil_off[0] == 0, "fil_create: susp_fil_off[0] must be 0");
    for (int64_t i = 0; i < nsusp; i++)
        FIL_CHECK_ARG(susp_fil_off[i + 1] > susp_fil_off[i], "fil_create: every suspension needs >= 1 filament");
    const int64_t M = susp_fil_off[nsusp];
    if (tether)
        for (int64_t f = 0; f < M; f++)
            FIL_CHECK_ARG(tether[f] >= 0 && tether[f] <= 3,
                          "fil_create: tether values are 0, 1 (clamped), 2 (pinned) or 3 (rotating motor)");
    FIL_CHECK_ARG(fil_seg_off[0] == 0, "fil_create: fil_seg_off[0] must be 0");
    for (int64_t f = 0; f < M; f++) {
        const int64_t N = fil_seg_off[f + 1] - fil_seg_off[f];
        FIL_CHECK_ARG(N >= 1 && N <= kMaxSeg, "fil_create: filaments need 1..64 segments");
    }
    const int64_t S = fil_seg_off[M];
    for (int64_t i = 0; i < 4 * S; i++) FIL_CHECK_ARG(std::isfinite(q0[i]), "fil_create: non-finite quaternion");
    for (int64_t i = 0; i < 3 * S; i++) FIL_CHECK_ARG(std::isfinite(Y0[i]), "fil_create: non-finite position");

    fil_sim* s = new fil_sim();
    s->p = *p;
    s->S = S;
    s->M = M;
    s->nsusp = nsusp;
    if (tether)
        for (int64_t f = 0; f < M; f++) s->has_motor |= tether[f] == 3;
    // ---- host-side index lists
    std::vector<int64_t> seg_off(fil_seg_off, fil_seg_off + M + 1);
    std::vector<int32_t> fil_susp(M), seg_fil(S), teth(M, 0);
    std::vector<int64_t> susp_seg_off(nsusp + 1);
    for (int64_t i = 0; i < nsusp; i++) {
        susp_seg_off[i] = seg_off[susp_fil_off[i]];
        for (int64_t f = susp_fil_off[i]; f < susp_fil_off[i + 1]; f++) fil_susp[f] = (int32_t)i;
    }
    susp_seg_off[nsusp] = S;
    for (int64_t f = 0; f < M; f++) {
        for (int64_t x = seg_off[f]; x < seg_off[f + 1]; x++) seg_fil[x] = (int32_t)f;
        if (tether) teth[f] = tether[f];
    }
    s->seg_uniform = (int)(seg_off[1] - seg_off[0]);
    for (int64_t f = 0; f < M; f++)
        if (seg_off[f + 1] - seg_off[f] != s->seg_uniform) s->seg_uniform = 0;
    std::vector<double> base(3 * M);
    for (int64_t f = 0; f < M; f++)
        for (int i = 0; i < 3; i++) base[3 * f + i] = Y0[3 * seg_off[f] + i];
    int max_seg = 1;
    std::vector<int64_t> dense_off(M);
    int64_t dense_tot = 0;
    for (int64_t f = 0; f < M; f++) {
        const int64_t N = seg_off[f + 1] - seg_off[f];
        max_seg = std::max<int>(max_seg, (int)N);
        dense_off[f] = dense_tot;
        dense_tot += 36 * N * N;
    }
    const bool dense = p->j0_mode == 2 || (p->j0_mode == 0 && (size_t)dense_tot * sizeof(double) <= kDenseInvBytes);
    std::vector<int64_t> sfo(susp_fil_off, susp_fil_off + nsusp + 1);
    s->susp_seg_off = susp_seg_off;
    s->fil_seg_off_h = seg_off;

    // ---- device allocations
    int rc = FIL_OK;
    int64_t *d_seg_off, *d_susp_seg_off, *d_susp_fil_off, *d_dense_off = nullptr;
    int32_t *d_fil_susp, *d_seg_fil, *d_teth, *d_cls_fil;
    // size classes of the filaments
    const int cls_bound[kMaxCls] = {16, 24, 32, 40, 48, kMaxSeg};
    std::vector<int32_t> cls_fil;
    int64_t cls_off[kMaxCls + 1];
    int cls_n[kMaxCls];
    for (int k = 0; k < kMaxCls; k++) {
        cls_off[k] = (int64_t)cls_fil.size();
        int nmx = 0;
        for (int64_t f = 0; f < M; f++) {
            const int N = (int)(seg_off[f + 1] - seg_off[f]);
            if (N <= cls_bound[k] && (k == 0 || N > cls_bound[k - 1])) {
                cls_fil.push_back((int32_t)f);
                nmx = std::max(nmx, 6 * N);
            }
        }
        cls_n[k] = nmx;
    }
    cls_off[kMaxCls] = (int64_t)cls_fil.size();
    double *d_base, *d_phase = nullptr;
    const size_t n6 = 6 * (size_t)S;
    const int max_dots = p->kmax + 2;
#define A(ptr, n)                                  \
    if (rc == FIL_OK) rc = dalloc(s, &(ptr), (n));
    A(d_seg_off, M + 1) A(d_susp_seg_off, nsusp + 1) A(d_susp_fil_off, nsusp + 1)
    A(d_fil_susp, M) A(d_seg_fil, S) A(d_teth, M) A(d_cls_fil, M)
    A(d_base, 3 * M)
    if (phase) A(d_phase, M)
    A(s->Yj, 3 * S) A(s->Yjm1, 3 * S) A(s->qj, 4 * S) A(s->Xj, n6) A(s->Xjm1, n6) A(s->Xjm2, n6) A(s->X0p, n6) A(s->Xb, n6)
    A(s->X, n6) A(s->f, n6) A(s->fprev, n6)
    A(s->Yc, 3 * S) A(s->qc, 4 * S) A(s->F, 3 * S) A(s->T, 3 * S) A(s->V, 3 * S) A(s->W, 3 * S)
    A(s->AB, n6 * kBandW) A(s->ipiv, n6) A(s->rdiag, n6)
    if (dense) { A(s->AinvT, dense_tot) A(d_dense_off, M) }
    if (!dense && M >= kLaneSolveMinFil) { A(s->gsolve, n6) A(s->BC, (n6 + 2 * kBcPad) * kBcW) }
    A(s->Chist, (size_t)p->kmax * n6) A(s->Dhist, (size_t)p->kmax * n6) A(s->part, (size_t)M * max_dots)
    A(s->box, 6 * M) A(s->spar, kSpar * nsusp) A(s->time_d, 1) A(s->log_d, nsusp) A(s->exports_d, 1)
    A(s->active_d, nsusp) A(s->jflag_d, M) A(s->resbits_d, 4 * nsusp) A(s->notnear_d, 1)
#undef A
    // the column records' zero pads (a sweep of a shorter filament beside a longer one reads
    // past its own records); the records themselves are rewritten at every factorisation
    if (rc == FIL_OK && s->BC) {
        if (hipMemset(s->BC, 0, (n6 + 2 * kBcPad) * kBcW * sizeof(double)) != hipSuccess) {
            set_error("fil_create: clearing the band records failed");
            rc = FIL_EHIP;
        }
        s->BC += kBcPad * kBcW;
    }
    if (rc == FIL_OK) rc = halloc(s, &s->active_h, nsusp);
    if (rc == FIL_OK) rc = halloc(s, &s->jflag_h, M);
    if (rc == FIL_OK) rc = halloc(s, &s->resbits_h, 2 * nsusp);
    if (rc == FIL_OK) rc = halloc(s, &s->time_h, 1);
    if (rc == FIL_OK) rc = halloc(s, &s->log_h, nsusp);
    for (int i = 0; i < 2; i++) {
        if (rc == FIL_OK) rc = halloc(s, &s->log_slot[i], nsusp);
        if (rc == FIL_OK && hipHostGetDevicePointer((void**)&s->log_slot_dev[i], s->log_slot[i], 0) != hipSuccess) {
            set_error("fil_create: no device address for a pinned log slot");
            rc = FIL_EHIP;
        }
        if (rc == FIL_OK && hipEventCreateWithFlags(&s->log_ev[i], hipEventDisableTiming) != hipSuccess) {
            set_error("fil_create: event creation failed");
            rc = FIL_EHIP;
        }
    }
    if (rc) {
        free_sim(s);
        return rc;
    }
    // mobility workspaces: FP64 always (the FP32-tile mode finishes every step in FP64)
    s->batched = nsusp > 1;
    const int nplan = p->prec == FIL_PREC_F32TILE ? 2 : 1;
    for (int c = 0; c < nplan; c++) {
        const int pr = c ? FIL_PREC_F32TILE : FIL_PREC_F64;
        size_t wbytes;
        if (s->batched) {
            s->bplan[c] = rpy_batch_plan(nsusp, susp_seg_off.data(), pr);
            wbytes = s->bplan[c].work_bytes() + s->bplan[c].lists_bytes();
        } else {
            s->rplan[c] = rpy_plan(S, pr);
            wbytes = s->rplan[c].total();
        }
        char* wk = nullptr;
        if ((rc = dalloc(s, &wk, wbytes))) {
            free_sim(s);
            return rc;
        }
        s->rpy_work[c] = wk;
        if (s->batched) {
            s->rpy_lists[c] = wk + s->bplan[c].work_bytes();
            // the work-item counter starts at zero; every apply that sums partials clears it again
            if (hipMemset(wk + rpy_batch_counter_offset(s->bplan[c]), 0, s->bplan[c].ctr_bytes) != hipSuccess) {
                set_error("fil_create: clearing the mobility work counter failed");
                free_sim(s);
                return FIL_EHIP;
            }
        }
    }
    // ---- uploads
    std::vector<double> Ysoa(3 * S), qsoa(4 * S);
    for (int64_t x = 0; x < S; x++) {
        for (int i = 0; i < 3; i++) Ysoa[i * S + x] = Y0[3 * x + i];
        double nq = 0;
        for (int i = 0; i < 4; i++) nq += q0[4 * x + i] * q0[4 * x + i];
        nq = 1.0 / std::sqrt(nq);
        for (int i = 0; i < 4; i++) qsoa[i * S + x] = q0[4 * x + i] * nq;
    }
    std::vector<double> zeros(n6, 0.0);
    std::vector<double> spar(kSpar * nsusp);
    for (int64_t i = 0; i < nsusp; i++) {
        const double v[kSpar] = {p->dt, p->grav[0], p->grav[1], p->grav[2], p->FS};
        for (int c = 0; c < kSpar; c++) spar[kSpar * i + c] = v[c];
    }
    auto up = [&]() -> int {
        TRY(upload(s->spar, spar));
        TRY(upload(d_seg_off, seg_off));
        TRY(upload(d_susp_seg_off, susp_seg_off));
        TRY(upload(d_susp_fil_off, sfo));
        if (dense) TRY(upload(d_dense_off, dense_off));
        TRY(upload(d_fil_susp, fil_susp));
        TRY(upload(d_seg_fil, seg_fil));
        TRY(upload(d_teth, teth));
        TRY(upload(d_cls_fil, cls_fil));
        TRY(upload(d_base, base));
        if (phase) TRY(upload(d_phase, std::vector<double>(phase, phase + M)));
        TRY(upload(s->Yj, Ysoa));
        TRY(upload(s->Yjm1, Ysoa));
        TRY(upload(s->qj, qsoa));
        TRY(upload(s->Xj, zeros));
        TRY(upload(s->Xjm1, zeros));
        TRY(upload(s->Xjm2, zeros));
        TRY(upload(s->X0p, zeros));
        TRY(upload(s->Xb, zeros));
        TRY(upload(s->exports_d, std::vector<int64_t>(1, 0)));
        TRY(upload(s->X, zeros));
        TRY(upload(s->resbits_d, std::vector<unsigned long long>(4 * nsusp, 0ull)));
        if (s->batched) {
            for (int c = 0; c < nplan; c++) TRY(rpy_batch_upload(s->bplan[c], s->rpy_lists[c], nullptr));
            FIL_HIP_TRY(hipDeviceSynchronize());
        }
        return FIL_OK;
    };
    if ((rc = up())) {
        free_sim(s);
        return rc;
    }
    SimDev& d = s->d;
    d.S = S;
    d.M = M;
    d.nsusp = nsusp;
    d.seg_off = d_seg_off;
    d.fil_susp = d_fil_susp;
    d.seg_fil = d_seg_fil;
    d.susp_seg_off = d_susp_seg_off;
    d.tether = d_teth;
    d.base = d_base;
    d.phase = d_phase;
    d.susp_fil_off = d_susp_fil_off;
    d.dense_off = d_dense_off;
    d.max_seg = max_seg;
    d.max_dots = max_dots;
    d.a = p->a;
    d.eta = p->eta;
    d.dL = p->dL;
    d.KB = p->KB;
    d.KT = p->KT;
    d.chi = p->chi;
    d.spar = s->spar;
    d.cls_fil = d_cls_fil;
    d.ncls = kMaxCls;
    d.factor_unstaged = p->j0_factor;
    for (int k = 0; k <= kMaxCls; k++) d.cls_off[k] = cls_off[k];
    for (int k = 0; k < kMaxCls; k++) d.cls_n[k] = cls_n[k];
    d.K0 = p->K0;
    d.kw = p->kw;
    d.omega = p->omega;
    *out = s;
    return FIL_OK;
}

void fil_destroy(fil_sim* sim) {
    if (sim) (void)hipStreamSynchronize(sim->st);
    free_sim(sim);
}

int fil_set_stream(fil_sim* sim, void* stream) {
    FIL_CHECK_ARG(sim, "fil_set_stream: null sim");
    sim->st = (hipStream_t)stream;
    return FIL_OK;
}

int fil_set_suspension_params(fil_sim* s, const double* dt, const double* grav, const double* FS) {
    FIL_CHECK_ARG(s, "fil_set_suspension_params: null sim");
    FIL_CHECK_ARG(s->step == 0, "fil_set_suspension_params: only before the first step");
    const int64_t ns = s->nsusp;
    std::vector<double> sp(kSpar * ns);
    FIL_HIP_TRY(hipMemcpy(sp.data(), s->spar, sp.size() * sizeof(double), hipMemcpyDeviceToHost));
    bool differ = false;
    for (int64_t i = 0; i < ns; i++) {
        if (dt) {
            FIL_CHECK_ARG(dt[i] > 0 && std::isfinite(dt[i]), "fil_set_suspension_params: dt must be finite and > 0");
            sp[kSpar * i] = dt[i];
            differ |= dt[i] != s->p.dt;
        }
        if (grav)
            for (int c = 0; c < 3; c++) {
                FIL_CHECK_ARG(std::isfinite(grav[3 * i + c]), "fil_set_suspension_params: non-finite gravity");
                sp[kSpar * i + 1 + c] = grav[3 * i + c];
            }
        if (FS) {
            FIL_CHECK_ARG(FS[i] >= 0 && std::isfinite(FS[i]), "fil_set_suspension_params: F^S must be >= 0");
            FIL_CHECK_ARG(FS[i] == 0.0 || s->p.chi > 1.0, "fil_set_suspension_params: steric range chi must exceed 1");
            sp[kSpar * i + 4] = FS[i];
        }
    }
    for (int64_t i = 0; i < ns; i++) differ |= sp[kSpar * i] != s->p.dt;  // also from an earlier call
    FIL_CHECK_ARG(!differ || s->p.K0 == 0.0,
                  "fil_set_suspension_params: per-suspension dt needs a time-independent preferred curvature (K0 = 0)");
    FIL_CHECK_ARG(!differ || !s->has_motor || s->d.motor_w == 0.0,
                  "fil_set_suspension_params: per-suspension dt with a turning motor (the motor's angle follows one "
                  "global time)");
    s->dt_differ = differ;
    drop_graphs(s);
    FIL_HIP_TRY(hipMemcpy(s->spar, sp.data(), sp.size() * sizeof(double), hipMemcpyHostToDevice));
    return FIL_OK;
}

int fil_set_external_forces(fil_sim* s, const double* Fext) {
    FIL_CHECK_ARG(s, "fil_set_external_forces: null sim");
    FIL_CHECK_ARG(s->step == 0, "fil_set_external_forces: only before the first step");
    drop_graphs(s);
    if (!Fext) {
        s->d.fext = nullptr;
        return FIL_OK;
    }
    const int64_t S = s->S;
    std::vector<double> soa(3 * S);
    for (int64_t n = 0; n < S; n++)
        for (int c = 0; c < 3; c++) {
            FIL_CHECK_ARG(std::isfinite(Fext[3 * n + c]), "fil_set_external_forces: non-finite force");
            soa[c * S + n] = Fext[3 * n + c];
        }
    if (!s->fext_d) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(1, soa.size()) * sizeof(double)) != hipSuccess) {
            set_error("fil_set_external_forces: out of device memory");
            return FIL_ENOMEM;
        }
        s->dev_allocs.push_back(p);
        s->fext_d = static_cast<double*>(p);
    }
    FIL_HIP_TRY(hipMemcpy(s->fext_d, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice));
    s->d.fext = s->fext_d;
    return FIL_OK;
}

int fil_set_periodic_fcm(fil_sim* s, const double* box, const int32_t* grid, double cut) {
    FIL_CHECK_ARG(s, "fil_set_periodic_fcm: null sim");
    FIL_CHECK_ARG(s->step == 0, "fil_set_periodic_fcm: only before the first step");
    FIL_CHECK_ARG(!s->fcm, "fil_set_periodic_fcm: the periodic box is already set");
    FIL_CHECK_ARG(s->nsusp == 1, "fil_set_periodic_fcm: one suspension per periodic box");
    FIL_CHECK_ARG(s->p.prec == FIL_PREC_F64, "fil_set_periodic_fcm: needs FIL_PREC_F64");
    FIL_CHECK_ARG(box && grid, "fil_set_periodic_fcm: null box or grid");
    for (int c = 0; c < 3; c++)
        FIL_CHECK_ARG(std::isfinite(box[c]) && 4.0 * s->p.chi * s->p.a < box[c],
                      "fil_set_periodic_fcm: every box length must exceed twice the steric range 2 chi a");
    fil_fcm* f = nullptr;
    TRY(fil_fcm_create(box, grid, s->p.a, s->p.eta, cut, &f));
    s->fcm = f;
    for (int c = 0; c < 3; c++) s->d.per[c] = box[c];
    s->d.periodic = 1;
    drop_graphs(s);
    return FIL_OK;
}

int fil_set_geometric_switch(fil_sim* s, const double* axis, const double* normal, double theta_max,
                             double tau_pos, double tau_neg, int n_transition) {
    FIL_CHECK_ARG(s, "fil_set_geometric_switch: null sim");
    FIL_CHECK_ARG(s->step == 0, "fil_set_geometric_switch: only before the first step");
    FIL_CHECK_ARG(!s->sw, "fil_set_geometric_switch: already set");
    FIL_CHECK_ARG(axis && normal, "fil_set_geometric_switch: null axis or normal");
    FIL_CHECK_ARG(std::isfinite(theta_max) && theta_max > 0 && theta_max < kPi,
                  "fil_set_geometric_switch: theta_max in (0, pi)");
    FIL_CHECK_ARG(std::isfinite(tau_pos) && std::isfinite(tau_neg) && tau_pos >= 0 && tau_neg >= 0,
                  "fil_set_geometric_switch: torque magnitudes >= 0");
    FIL_CHECK_ARG(n_transition >= 0 && n_transition <= 100000, "fil_set_geometric_switch: n_transition in [0, 1e5]");
    double na = 0, nn = 0, an = 0;
    for (int c = 0; c < 3; c++) {
        na += axis[c] * axis[c];
        nn += normal[c] * normal[c];
        an += axis[c] * normal[c];
    }
    FIL_CHECK_ARG(std::fabs(na - 1.0) < 1e-12 && std::fabs(nn - 1.0) < 1e-12 && std::fabs(an) < 1e-12,
                  "fil_set_geometric_switch: axis and normal must be orthogonal unit vectors");
    const int64_t M = s->M;
    TRY(dalloc(s, &s->text_d, (size_t)(3 * s->S)));
    TRY(dalloc(s, &s->swa.dir, (size_t)M));
    TRY(dalloc(s, &s->swa.age, (size_t)M));
    TRY(dalloc(s, &s->swa.tau0, (size_t)M));
    std::vector<int32_t> dir(M, 1), age(M, n_transition);
    std::vector<double> tau0(M, tau_pos);
    TRY(upload(s->swa.dir, dir));
    TRY(upload(s->swa.age, age));
    TRY(upload(s->swa.tau0, tau0));
    FIL_HIP_TRY(hipMemset(s->text_d, 0, 3 * s->S * sizeof(double)));
    for (int c = 0; c < 3; c++) {
        s->swa.axis[c] = axis[c];
        s->swa.normal[c] = normal[c];
    }
    s->swa.theta_max = theta_max;
    s->swa.tau_pos = tau_pos;
    s->swa.tau_neg = tau_neg;
    s->swa.n_tr = n_transition;
    s->d.text = s->text_d;
    s->sw = true;
    drop_graphs(s);
    return FIL_OK;
}

int fil_read_switch(fil_sim* s, int32_t* dir) {
    FIL_CHECK_ARG(s && dir, "fil_read_switch: null argument");
    FIL_CHECK_ARG(s->sw, "fil_read_switch: no geometric switch set");
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    FIL_HIP_TRY(hipMemcpy(dir, s->swa.dir, s->M * sizeof(int32_t), hipMemcpyDeviceToHost));
    return FIL_OK;
}

int fil_set_motor(fil_sim* s, double d0, double omega) {
    FIL_CHECK_ARG(s, "fil_set_motor: null sim");
    FIL_CHECK_ARG(s->step == 0, "fil_set_motor: only before the first step");
    FIL_CHECK_ARG(std::isfinite(d0) && d0 >= 0 && std::isfinite(omega), "fil_set_motor: d0 >= 0 and finite omega");
    FIL_CHECK_ARG(omega == 0.0 || !s->has_motor || !s->dt_differ,
                  "fil_set_motor: the suspensions have their own time steps; the motor turns with one global time");
    s->d.motor_d0 = d0;
    s->d.motor_w = omega;
    drop_graphs(s);
    return FIL_OK;
}

int fil_set_wall(fil_sim* s) {
    FIL_CHECK_ARG(s, "fil_set_wall: null sim");
    FIL_CHECK_ARG(s->step == 0, "fil_set_wall: only before the first step");
    FIL_CHECK_ARG(!s->wall, "fil_set_wall: the wall is already set");
    FIL_CHECK_ARG(!s->fcm, "fil_set_wall: the suspension is in a periodic box");
    FIL_CHECK_ARG(s->nsusp == 1, "fil_set_wall: one suspension per wall");
    const int64_t nb = wall_workspace_bytes(s->S);
    if (nb > 0) {
        double* w = nullptr;
        TRY(dalloc(s, &w, (size_t)(nb / (int64_t)sizeof(double))));
        s->wall_work = w;
    }
    s->wall = true;
    drop_graphs(s);
    return FIL_OK;
}

int fil_bdf2_step(fil_sim* s, fil_step_report* report) {
    FIL_CHECK_ARG(s, "fil_bdf2_step: null sim");
    const int64_t ns = s->nsusp;
    s->bc = coefs(s->step);
    if (s->timing && s->nev >= kMaxPendingTimings) {
        FIL_HIP_TRY(hipStreamSynchronize(s->st));
        TRY(collect_timing(s));
    }
    for (int64_t i = 0; i < ns; i++) s->active_h[i] = 1;
    if (s->sw) TRY(switch_torque_launch(s->d, s->swa, s->qj, s->text_d, s->st));
    // one kernel starts the step: first iterate and its copy, every suspension running,
    // the device log cleared, the time t^{j+1}
    TRY(initial_guess_launch(s->d, s->step, s->Yj, s->Yjm1, s->Xj, s->Xjm1, s->Xjm2, s->X, s->X0p, s->Xb,
                             s->active_d, s->log_d, s->time_d, s->t + s->p.dt, s->st));
    bool learned = s->use_mlp && s->mlp && s->step >= 3;
    if (learned) TRY(learned_guess(s));
    SolveLog L(ns);
    TRY(solve(s, L));
    bool all_ok = std::all_of(L.state.begin(), L.state.end(), [](int32_t v) { return v == 1; });
    if (!all_ok && learned) {
        // the plain warm start is the fallback: the step restarts from it
        s->fallbacks++;
        learned = false;
        for (int64_t i = 0; i < ns; i++) s->active_h[i] = 1;
        TRY(upload_flags(s, s->active_d, s->active_h));
        FIL_HIP_TRY(hipMemsetAsync(s->log_d, 0, ns * sizeof(SuspLog), s->st));
        FIL_HIP_TRY(hipMemcpyAsync(s->X, s->X0p, 6 * s->S * sizeof(double), hipMemcpyDeviceToDevice, s->st));
        SolveLog L2(ns);
        TRY(solve(s, L2));
        for (int64_t i = 0; i < ns; i++) {
            L2.applies[i] += L.applies[i];
            L2.applies_hi[i] += L.applies_hi[i];
        }
        L = L2;
        all_ok = std::all_of(L.state.begin(), L.state.end(), [](int32_t v) { return v == 1; });
    }
    for (int64_t i = 0; i < ns && report; i++) {
        report[i].iters = L.iters[i];
        report[i].mobility_applies = L.applies[i];
        report[i].converged = L.state[i] == 1;
        report[i].applies_f64 = L.applies_hi[i];
        report[i].resid = L.last[i];
        report[i].used_learned = learned ? 1 : 0;
        report[i].pad = 0;
    }
    if (!all_ok) {
        bool nonfinite = false;
        for (int64_t i = 0; i < ns; i++) nonfinite |= !std::isfinite(L.last[i]);
        if (!L.singular)
            set_error(nonfinite ? "fil_bdf2_step: residual became non-finite; state left at the previous step"
                                : "fil_bdf2_step: Broyden did not reach the tolerance; state left at the previous step");
        return nonfinite || L.singular ? FIL_ENONFINITE : FIL_ENOCONV;
    }
    // the commit stays queued on the stream (reads of the state synchronise first)
    TRY(finalize_launch(s->d, nullptr, s->Yc, s->qc, s->X, s->Yj, s->Yjm1, s->qj, s->Xj, s->Xjm1, s->Xjm2, s->st));
    s->t += s->p.dt;
    s->step += 1;
    return FIL_OK;
}

int fil_set_graph(fil_sim* s, int iters_per_launch) {
    FIL_CHECK_ARG(s, "fil_set_graph: null sim");
    FIL_CHECK_ARG(iters_per_launch >= 0 && iters_per_launch <= 64, "fil_set_graph: iterations per launch in [0, 64]");
    s->graph_iters = iters_per_launch;
    return FIL_OK;
}

int fil_sim_set_mlp(fil_sim* s, fil_mlp* m, int enable) {
    FIL_CHECK_ARG(s, "fil_sim_set_mlp: null sim");
    if (enable) {
        FIL_CHECK_ARG(m, "fil_sim_set_mlp: null network");
        FIL_CHECK_ARG(s->seg_uniform == mlp_segments(m),
                      "fil_sim_set_mlp: every filament must have the network's number of segments");
        FIL_CHECK_ARG(s->M <= mlp_max_batch(m), "fil_sim_set_mlp: more filaments than the network's max_batch");
        TRY(ensure_learned_buffers(s, mlp_in_pad(m), mlp_out_pad(m)));
    }
    s->mlp = enable ? m : nullptr;
    s->use_mlp = enable != 0;
    return FIL_OK;
}

int fil_sim_features(fil_sim* s, float* out) {
    FIL_CHECK_ARG(s && out, "fil_sim_features: null argument");
    FIL_CHECK_ARG(s->seg_uniform > 0, "fil_sim_features: filaments of different lengths");
    FIL_CHECK_ARG(s->step >= 1, "fil_sim_features: no step taken yet");
    return learned_features_launch(s->d, s->seg_uniform, s->Yj, s->qj, s->F, s->V, s->Xj, s->Xjm1, s->Xjm2, out,
                                   s->st);
}

int fil_sim_step_target(fil_sim* s, float* out) {
    FIL_CHECK_ARG(s && out, "fil_sim_step_target: null argument");
    FIL_CHECK_ARG(s->seg_uniform > 0, "fil_sim_step_target: filaments of different lengths");
    FIL_CHECK_ARG(s->step >= 1, "fil_sim_step_target: no step taken yet");
    return learned_target_launch(s->d, s->seg_uniform, s->Xj, s->Xb, out, s->st);
}

int fil_sim_fallbacks(fil_sim* s, int64_t* n) {
    FIL_CHECK_ARG(s && n, "fil_sim_fallbacks: null argument");
    *n = s->fallbacks;
    return FIL_OK;
}

int fil_set_timing(fil_sim* s, int enable) {
    FIL_CHECK_ARG(s, "fil_set_timing: null sim");
    s->timing = enable != 0;
    s->rpy_ms[0] = s->rpy_ms[1] = 0.0;
    s->rpy_launches[0] = s->rpy_launches[1] = 0;
    s->nev = 0;
    return FIL_OK;
}

int fil_get_timing(fil_sim* s, double* rpy_ms, int64_t* rpy_launches) {
    FIL_CHECK_ARG(s, "fil_get_timing: null sim");
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    TRY(collect_timing(s));
    for (int c = 0; c < 2; c++) {
        if (rpy_ms) rpy_ms[c] = s->rpy_ms[c];
        if (rpy_launches) rpy_launches[c] = s->rpy_launches[c];
    }
    return FIL_OK;
}

int fil_residual(fil_sim* s, const double* X, double* f_out) {
    FIL_CHECK_ARG(s && X && f_out, "fil_residual: null argument");
    s->bc = coefs(s->step);
    for (int64_t i = 0; i < s->nsusp; i++) s->active_h[i] = 1;
    TRY(upload_flags(s, s->active_d, s->active_h));
    TRY(set_time(s));
    hipEvent_t e0, e1;
    TRY(pool_events(s, &e0, &e1));
    return eval_residual(s, X, f_out, e0, e1, true, -1);
}

int fil_broyden_begin(fil_sim* s, const double* X0, double* f0_out) {
    FIL_CHECK_ARG(s && X0, "fil_broyden_begin: null argument");
    s->bc = coefs(s->step);
    for (int64_t i = 0; i < s->nsusp; i++) s->active_h[i] = 1;
    TRY(upload_flags(s, s->active_d, s->active_h));
    FIL_HIP_TRY(hipMemcpyAsync(s->X, X0, 6 * s->S * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    TRY(set_time(s));
    hipEvent_t e0, e1;
    TRY(pool_events(s, &e0, &e1));
    TRY(eval_residual(s, s->X, s->f, e0, e1, true, -1));
    TRY(begin_solve(s));
    if (f0_out) FIL_HIP_TRY(hipMemcpyAsync(f0_out, s->f, 6 * s->S * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    TRY(broyden_state_launch(s->d, update_args(s, -1, s->f, nullptr), JudgeArgs{}, s->active_d, s->st));
    return FIL_OK;
}

int fil_broyden_update(fil_sim* s, const double* f_new, double* dX_out) {
    FIL_CHECK_ARG(s && f_new, "fil_broyden_update: null argument");
    FIL_CHECK_ARG(s->k + 1 < s->p.kmax, "fil_broyden_update: history full (kmax updates)");
    TRY(update_dots_launch(s->d, f_new, s->active_d, DotArgs{s->k, s->Dhist, s->fprev, s->part}, s->st));
    TRY(broyden_state_launch(s->d, update_args(s, s->k, f_new, dX_out), JudgeArgs{}, s->active_d, s->st));
    s->k++;
    return FIL_OK;
}

int fil_get_state(fil_sim* s, const double** Y, const double** q, const double** Xj, const double** X, int64_t* S,
                  double* t, int64_t* step) {
    FIL_CHECK_ARG(s, "fil_get_state: null sim");
    if (Y) *Y = s->Yj;
    if (q) *q = s->qj;
    if (Xj) *Xj = s->Xj;
    if (X) *X = s->X;
    if (S) *S = s->S;
    if (t) *t = s->t;
    if (step) *step = s->step;
    return FIL_OK;
}

int fil_read_state(fil_sim* s, double* Y, double* q, double* Xj) {
    FIL_CHECK_ARG(s, "fil_read_state: null sim");
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    const int64_t S = s->S;
    std::vector<double> buf(6 * S);
    if (Y) {
        FIL_HIP_TRY(hipMemcpy(buf.data(), s->Yj, 3 * S * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t x = 0; x < S; x++)
            for (int i = 0; i < 3; i++) Y[3 * x + i] = buf[i * S + x];
    }
    if (q) {
        FIL_HIP_TRY(hipMemcpy(buf.data(), s->qj, 4 * S * sizeof(double), hipMemcpyDeviceToHost));
        for (int64_t x = 0; x < S; x++)
            for (int i = 0; i < 4; i++) q[4 * x + i] = buf[i * S + x];
    }
    if (Xj) FIL_HIP_TRY(hipMemcpy(Xj, s->Xj, 6 * S * sizeof(double), hipMemcpyDeviceToHost));
    return FIL_OK;
}

// ---------------------------------------------------------------- checkpoint / restore
// File layout (native byte order): "FILSIM02", int64 S, M, nsusp, step, double t,
// int64 fil_seg_off[M+1], int64 susp_fil_off[nsusp+1], double spar[nsusp][5],
// then Y^j, Y^{j-1} [3][S], q^j [4][S], X^j, X^{j-1}, X^{j-2} [6S], then int64 sw
// (1 when a geometric switch drives the bases) followed, when sw = 1, by its state:
// int32 dir[M], int32 age[M], double tau0[M].  "FILSIM01" files (no switch block) are
// still read, into simulations without a switch.
}  // extern "C"

namespace {
constexpr char kSimMagic[8] = {'F', 'I', 'L', 'S', 'I', 'M', '0', '2'};
constexpr char kSimMagicV1[8] = {'F', 'I', 'L', 'S', 'I', 'M', '0', '1'};

struct FileCloser {
    FILE* f;
    ~FileCloser() {
        if (f) fclose(f);
    }
};

// the committed arrays of a simulation with their element counts
std::vector<std::pair<double*, size_t>> state_arrays(fil_sim* s) {
    const size_t S = (size_t)s->S, n6 = 6 * S;
    return {{s->Yj, 3 * S}, {s->Yjm1, 3 * S}, {s->qj, 4 * S}, {s->Xj, n6}, {s->Xjm1, n6}, {s->Xjm2, n6}};
}
}  // namespace

extern "C" {

int fil_checkpoint(fil_sim* s, const char* path) {
    FIL_CHECK_ARG(s && path, "fil_checkpoint: null argument");
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    FileCloser fc{fopen(path, "wb")};
    FIL_CHECK_ARG(fc.f, std::string("fil_checkpoint: cannot open ") + path);
    const int64_t hdr[4] = {s->S, s->M, s->nsusp, s->step};
    std::vector<int64_t> sfo(s->nsusp + 1);
    FIL_HIP_TRY(hipMemcpy(sfo.data(), s->d.susp_fil_off, sfo.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<double> spar(kSpar * s->nsusp);
    FIL_HIP_TRY(hipMemcpy(spar.data(), s->spar, spar.size() * sizeof(double), hipMemcpyDeviceToHost));
    bool ok = fwrite(kSimMagic, 1, 8, fc.f) == 8 && fwrite(hdr, sizeof(int64_t), 4, fc.f) == 4 &&
              fwrite(&s->t, sizeof(double), 1, fc.f) == 1 &&
              fwrite(s->fil_seg_off_h.data(), sizeof(int64_t), s->fil_seg_off_h.size(), fc.f) ==
                  s->fil_seg_off_h.size() &&
              fwrite(sfo.data(), sizeof(int64_t), sfo.size(), fc.f) == sfo.size() &&
              fwrite(spar.data(), sizeof(double), spar.size(), fc.f) == spar.size();
    std::vector<double> buf;
    for (auto& a : state_arrays(s)) {
        if (!ok) break;
        buf.resize(a.second);
        FIL_HIP_TRY(hipMemcpy(buf.data(), a.first, a.second * sizeof(double), hipMemcpyDeviceToHost));
        ok = fwrite(buf.data(), sizeof(double), a.second, fc.f) == a.second;
    }
    // the geometric switch's state: without it a restored run would restart every switch
    const int64_t sw = s->sw ? 1 : 0;
    ok = ok && fwrite(&sw, sizeof(int64_t), 1, fc.f) == 1;
    if (ok && sw) {
        const size_t M = (size_t)s->M;
        std::vector<int32_t> dir(M), age(M);
        std::vector<double> tau0(M);
        FIL_HIP_TRY(hipMemcpy(dir.data(), s->swa.dir, M * sizeof(int32_t), hipMemcpyDeviceToHost));
        FIL_HIP_TRY(hipMemcpy(age.data(), s->swa.age, M * sizeof(int32_t), hipMemcpyDeviceToHost));
        FIL_HIP_TRY(hipMemcpy(tau0.data(), s->swa.tau0, M * sizeof(double), hipMemcpyDeviceToHost));
        ok = fwrite(dir.data(), sizeof(int32_t), M, fc.f) == M && fwrite(age.data(), sizeof(int32_t), M, fc.f) == M &&
             fwrite(tau0.data(), sizeof(double), M, fc.f) == M;
    }
    ok = ok && fflush(fc.f) == 0;
    FIL_CHECK_ARG(ok, std::string("fil_checkpoint: write to ") + path + " failed");
    return FIL_OK;
}

int fil_restore(fil_sim* s, const char* path) {
    FIL_CHECK_ARG(s && path, "fil_restore: null argument");
    FileCloser fc{fopen(path, "rb")};
    FIL_CHECK_ARG(fc.f, std::string("fil_restore: cannot open ") + path);
    char magic[8];
    int64_t hdr[4];
    double t = 0.0;
    const bool magic_ok = fread(magic, 1, 8, fc.f) == 8;
    const bool v1 = magic_ok && std::memcmp(magic, kSimMagicV1, 8) == 0;
    FIL_CHECK_ARG(magic_ok && (v1 || std::memcmp(magic, kSimMagic, 8) == 0) &&
                      fread(hdr, sizeof(int64_t), 4, fc.f) == 4 && fread(&t, sizeof(double), 1, fc.f) == 1,
                  "fil_restore: not a simulation checkpoint");
    FIL_CHECK_ARG(hdr[0] == s->S && hdr[1] == s->M && hdr[2] == s->nsusp && hdr[3] >= 0,
                  "fil_restore: checkpoint of a different simulation (segments, filaments or suspensions)");
    std::vector<int64_t> off(s->M + 1), sfo(s->nsusp + 1), sfo_d(s->nsusp + 1);
    std::vector<double> spar(kSpar * s->nsusp);
    FIL_CHECK_ARG(fread(off.data(), sizeof(int64_t), off.size(), fc.f) == off.size() &&
                      fread(sfo.data(), sizeof(int64_t), sfo.size(), fc.f) == sfo.size() &&
                      fread(spar.data(), sizeof(double), spar.size(), fc.f) == spar.size(),
                  "fil_restore: truncated checkpoint");
    FIL_HIP_TRY(hipMemcpy(sfo_d.data(), s->d.susp_fil_off, sfo_d.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    FIL_CHECK_ARG(off == s->fil_seg_off_h && sfo == sfo_d,
                  "fil_restore: checkpoint of a different simulation (filament or suspension layout)");
    for (double v : spar) FIL_CHECK_ARG(std::isfinite(v), "fil_restore: non-finite parameter");
    std::vector<std::vector<double>> data;
    for (auto& a : state_arrays(s)) {
        data.emplace_back(a.second);
        FIL_CHECK_ARG(fread(data.back().data(), sizeof(double), a.second, fc.f) == a.second,
                      "fil_restore: truncated checkpoint");
        for (double v : data.back()) FIL_CHECK_ARG(std::isfinite(v), "fil_restore: non-finite state");
    }
    int64_t sw = 0;
    if (!v1) FIL_CHECK_ARG(fread(&sw, sizeof(int64_t), 1, fc.f) == 1 && (sw == 0 || sw == 1),
                           "fil_restore: truncated checkpoint");
    FIL_CHECK_ARG((sw == 1) == s->sw,
                  sw ? "fil_restore: the checkpoint holds a geometric switch's state and the simulation has none"
                     : "fil_restore: the simulation has a geometric switch and the checkpoint holds no state of it");
    const size_t M = (size_t)s->M;
    std::vector<int32_t> dir(sw ? M : 0), age(sw ? M : 0);
    std::vector<double> tau0(sw ? M : 0);
    if (sw) {
        FIL_CHECK_ARG(fread(dir.data(), sizeof(int32_t), M, fc.f) == M && fread(age.data(), sizeof(int32_t), M, fc.f) == M &&
                          fread(tau0.data(), sizeof(double), M, fc.f) == M,
                      "fil_restore: truncated checkpoint");
        for (size_t f = 0; f < M; f++)
            FIL_CHECK_ARG((dir[f] == 1 || dir[f] == -1) && age[f] >= 0 && std::isfinite(tau0[f]),
                          "fil_restore: invalid geometric-switch state");
    }
    // everything read and checked: the simulation is changed only now
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    FIL_HIP_TRY(hipMemcpy(s->spar, spar.data(), spar.size() * sizeof(double), hipMemcpyHostToDevice));
    const auto arrays = state_arrays(s);
    for (size_t i = 0; i < arrays.size(); i++)
        FIL_HIP_TRY(hipMemcpy(arrays[i].first, data[i].data(), arrays[i].second * sizeof(double),
                              hipMemcpyHostToDevice));
    if (sw) {
        FIL_HIP_TRY(hipMemcpy(s->swa.dir, dir.data(), M * sizeof(int32_t), hipMemcpyHostToDevice));
        FIL_HIP_TRY(hipMemcpy(s->swa.age, age.data(), M * sizeof(int32_t), hipMemcpyHostToDevice));
        FIL_HIP_TRY(hipMemcpy(s->swa.tau0, tau0.data(), M * sizeof(double), hipMemcpyHostToDevice));
    }
    s->t = t;
    s->step = hdr[3];
    s->pred_iters = s->pred_iters32 = 0;
    return FIL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- Newton-Krylov and JFB steps
// Two steps whose linear systems are solved by restarted GMRES with Jacobian-free
// products (Sec. 3.1, 3.2.1; compared in Sec. 3.3.1, 3.3.2):
//  * Newton-Krylov: X <- X + dX with J(X) dX = -f(X), J v = (f(X + delta v) - f(X)) / delta
//    (one mobility apply per Krylov iteration);
//  * JFB-g, good Broyden (Alg. 1) with J0 = grad f0 taken the same way from f0, the
//    residual with the drag-only mobility and no steric or external forces, at the
//    step's initial guess: [J0 + sum_i c_i d_i^T] dX = -f(X_k), then c = f(X_{k+1}) /
//    |dX|, d = dX / |dX| (one mobility apply per Broyden iteration; the Krylov
//    iterations evaluate f0 only).
// Preconditioning: none; right, with P_dt^{-1} (multiplier rows scaled by 6 pi eta a /
// dt, the inverse of the Delta t / (6 pi eta a) factor their Jacobian columns carry);
// or left, with the block-diagonal explicit J0^{-1} of the initial guess.
namespace {

struct KryOpts {
    int precond;  // 0 none, 1 right P_dt, 2 left J0
    double rtol, delta;
    int kmax;     // Krylov iterations per linear solve at most
};
using KryOp = std::function<int(const double*, double*)>;

int kry_ensure(fil_sim* s, int m) {
    if (s->kry_V && s->kry_m >= m) return FIL_OK;
    FIL_CHECK_ARG(!s->kry_V, "Krylov solve: the workspace was sized by an earlier call with a smaller krylov_max");
    const size_t n6 = 6 * (size_t)s->S;
    TRY(dalloc(s, &s->kry_V, (size_t)(m + 1) * n6));
    for (double** v : {&s->kry_f0, &s->kry_fp, &s->kry_Xp, &s->kry_w, &s->kry_u, &s->kry_x, &s->kry_pinv, &s->kry_f00})
        TRY(dalloc(s, v, n6));
    TRY(dalloc(s, &s->kry_partial, multi_dot_partial_count((int64_t)n6, std::max(m + 1, s->p.kmax + 1))));
    TRY(dalloc(s, &s->kry_dots_d, (size_t)std::max(m, s->p.kmax) + 2));
    TRY(dalloc(s, &s->kry_coef_d, (size_t)std::max(m, s->p.kmax) + 2));
    TRY(halloc(s, &s->kry_dots_h, (size_t)std::max(m, s->p.kmax) + 2));
    TRY(halloc(s, &s->kry_coef_h, (size_t)std::max(m, s->p.kmax) + 2));
    TRY(dalloc(s, &s->kry_spar0, (size_t)kSpar * s->nsusp));
    TRY(dalloc(s, &s->kry_rb, 4 * (size_t)s->nsusp));
    s->kry_m = m;
    return FIL_OK;
}

// out[0..k) = V_j . w on the host
int kry_dots(fil_sim* s, const double* V, int k, const double* w, double* out) {
    const int64_t n6 = 6 * s->S;
    TRY(multi_dot_launch(n6, V, n6, k, w, s->kry_partial, s->kry_dots_d, s->st));
    FIL_HIP_TRY(hipMemcpyAsync(s->kry_dots_h, s->kry_dots_d, k * sizeof(double), hipMemcpyDeviceToHost, s->st));
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    for (int j = 0; j < k; j++) out[j] = s->kry_dots_h[j];
    return FIL_OK;
}

// w += sign sum_j c[j] V_j with the coefficients uploaded from the host
int kry_axpy(fil_sim* s, const double* V, int k, const double* c, double sign, double* w) {
    const int64_t n6 = 6 * s->S;
    if (k <= 0) return FIL_OK;
    for (int j = 0; j < k; j++) s->kry_coef_h[j] = c[j];
    FIL_HIP_TRY(hipMemcpyAsync(s->kry_coef_d, s->kry_coef_h, k * sizeof(double), hipMemcpyHostToDevice, s->st));
    TRY(multi_axpy_launch(n6, k, V, n6, s->kry_coef_d, sign, w, s->st));
    // the pinned coefficients may be overwritten only after the copy has run
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    return FIL_OK;
}

// restarted GMRES for A x = b (b a device vector, x0 = 0) until the residual norm is at
// most rtol |b| or o.kmax iterations of this solve; x is left in kry_x and the iterations
// are added to kiters.  Gram-Schmidt runs twice per Arnoldi step (classical, for the
// device); the operator may use kry_u, kry_Xp, kry_fp but not V, kry_w, kry_x.
int kry_gmres(fil_sim* s, const KryOpts& o, const KryOp& A, const double* b, int& kiters_total) {
    int kiters = 0;
    struct Add {
        int& total;
        const int& n;
        ~Add() { total += n; }
    } add{kiters_total, kiters};
    const int64_t n6 = 6 * s->S;
    const int m = s->kry_m;
    double* V = s->kry_V;
    FIL_HIP_TRY(hipMemsetAsync(s->kry_x, 0, n6 * sizeof(double), s->st));
    double nb = 0.0;
    TRY(kry_dots(s, b, 1, b, &nb));
    nb = std::sqrt(nb);
    if (!(nb > 0.0)) return std::isfinite(nb) ? FIL_OK : FIL_ENONFINITE;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 2), h2(m + 2);
    bool first = true;
    while (true) {
        double beta;
        if (first) {
            TRY(axpby_launch(n6, 1.0, b, 0.0, nullptr, V, s->st));
            beta = nb;
        } else {
            TRY(A(s->kry_x, s->kry_w));  // r = b - A x
            TRY(axpby_launch(n6, 1.0, b, -1.0, s->kry_w, V, s->st));
            TRY(kry_dots(s, V, 1, V, &beta));
            beta = std::sqrt(beta);
        }
        first = false;
        if (!std::isfinite(beta)) return FIL_ENONFINITE;
        if (beta <= o.rtol * nb || kiters >= o.kmax) return FIL_OK;
        TRY(axpby_launch(n6, 1.0 / beta, V, 0.0, nullptr, V, s->st));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool done = false;
        for (; k < m && kiters < o.kmax; k++) {
            double* vk1 = V + (int64_t)(k + 1) * n6;
            TRY(A(V + (int64_t)k * n6, vk1));
            kiters++;
            // twice classical Gram-Schmidt against V_0 .. V_k
            TRY(kry_dots(s, V, k + 1, vk1, h.data()));
            TRY(kry_axpy(s, V, k + 1, h.data(), -1.0, vk1));
            TRY(kry_dots(s, V, k + 1, vk1, h2.data()));
            TRY(kry_axpy(s, V, k + 1, h2.data(), -1.0, vk1));
            for (int j = 0; j <= k; j++) h[j] += h2[j];
            double hn = 0.0;
            TRY(kry_dots(s, vk1, 1, vk1, &hn));
            hn = std::sqrt(hn);
            if (!std::isfinite(hn)) return FIL_ENONFINITE;
            if (hn > 0.0) TRY(axpby_launch(n6, 1.0 / hn, vk1, 0.0, nullptr, vk1, s->st));
            // Givens rotations of the Hessenberg column
            for (int j = 0; j < k; j++) {
                const double t = cs[j] * h[j] + sn[j] * h[j + 1];
                h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
                h[j] = t;
            }
            const double r = std::hypot(h[k], hn);
            cs[k] = r > 0.0 ? h[k] / r : 1.0;
            sn[k] = r > 0.0 ? hn / r : 0.0;
            h[k] = r;
            for (int j = 0; j <= k; j++) H[(size_t)j * m + k] = h[j];
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (std::fabs(g[k + 1]) <= o.rtol * nb || hn == 0.0) {
                k++;
                done = true;
                break;
            }
        }
        // y = H^{-1} g (upper triangular), x += V y
        for (int i = k - 1; i >= 0; i--) {
            double t = g[i];
            for (int j = i + 1; j < k; j++) t -= H[(size_t)i * m + j] * y[j];
            y[i] = t / H[(size_t)i * m + i];
        }
        TRY(kry_axpy(s, V, k, y.data(), 1.0, s->kry_x));
        if (done || kiters >= o.kmax) return FIL_OK;
    }
}

// f0(X) (drag-only mobility, no steric or external forces) into fout; overwrites the
// state buffers and V, W like an evaluation of f
int eval_f0(fil_sim* s, const double* X, double* fout) {
    SimDev d0 = s->d;
    d0.spar = s->kry_spar0;
    d0.fext = nullptr;
    d0.text = nullptr;
    TRY(state_forces_launch(d0, X, s->qj, s->time_d, s->active_d, s->Yc, s->qc, s->F, s->T, s->box, s->st));
    TRY(diag_mobility_launch(d0, s->F, s->T, s->V, s->W, s->st));
    unsigned long long* rb = s->kry_rb + 2 * s->kry_rbi * s->nsusp;
    unsigned long long* rbn = s->kry_rb + 2 * (1 - s->kry_rbi) * s->nsusp;
    s->kry_rbi ^= 1;
    const DotArgs none{-1, nullptr, nullptr, nullptr};
    return residual_launch(d0, s->bc, X, s->Xj, s->Yc, s->Yj, s->Yjm1, s->V, s->W, nullptr, 1, s->active_d, fout, rb,
                           rbn, none, s->st);
}

// common checks, the warm start, P^{-1} and (left preconditioner) J0 at the initial
// guess; leaves f(X0) in kry_f0 and max|f|/a in res
int kry_begin(fil_sim* s, const char* who, int precond, double krylov_tol, double fd_delta, int krylov_max,
              std::vector<double>& res, int& applies) {
    FIL_CHECK_ARG(s, std::string(who) + ": null sim");
    FIL_CHECK_ARG(s->nsusp == 1, std::string(who) + ": one suspension per simulation");
    FIL_CHECK_ARG(s->p.prec == FIL_PREC_F64, std::string(who) + ": FP64 mobility only");
    FIL_CHECK_ARG(precond >= 0 && precond <= 2, std::string(who) + ": precond must be 0 (none), 1 (P_dt) or 2 (J0)");
    FIL_CHECK_ARG(precond != 2 || s->AinvT,
                  std::string(who) + ": the J0 preconditioner needs the explicit inverse (j0_mode 0 or 2)");
    FIL_CHECK_ARG(krylov_tol > 0.0 && krylov_tol < 1.0 && fd_delta > 0.0 && std::isfinite(fd_delta),
                  std::string(who) + ": krylov_tol in (0, 1), fd_delta > 0");
    FIL_CHECK_ARG(krylov_max >= 1 && krylov_max <= 100000, std::string(who) + ": krylov_max in [1, 100000]");
    const int64_t n6 = 6 * s->S;
    TRY(kry_ensure(s, std::min(krylov_max, 100)));
    if (s->sw) TRY(switch_torque_launch(s->d, s->swa, s->qj, s->text_d, s->st));
    s->bc = coefs(s->step);
    s->cur = 0;
    s->active_h[0] = 1;
    TRY(initial_guess_launch(s->d, s->step, s->Yj, s->Yjm1, s->Xj, s->Xjm1, s->Xjm2, s->X, s->X0p, s->Xb,
                             s->active_d, s->log_d, s->time_d, s->t + s->p.dt, s->st));
    std::vector<double> sp(kSpar * s->nsusp);
    FIL_HIP_TRY(hipMemcpy(sp.data(), s->spar, sp.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (precond == 1) {
        // P^{-1}: 1 on Y_1 and u, 6 pi eta a / dt on the multipliers of each filament
        std::vector<double> pinv(n6, 1.0);
        const double sc = 6.0 * kPi * s->p.eta * s->p.a / sp[0];
        for (int64_t f = 0; f < s->M; f++) {
            const int64_t s0 = s->fil_seg_off_h[f], N = s->fil_seg_off_h[f + 1] - s0;
            for (int64_t e = 3 + 3 * N; e < 6 * N; e++) pinv[6 * s0 + e] = sc;
        }
        FIL_HIP_TRY(hipMemcpy(s->kry_pinv, pinv.data(), n6 * sizeof(double), hipMemcpyHostToDevice));
    }
    // the parameters of f0: gravity and steric strength zero, the same time step
    for (int64_t i = 0; i < s->nsusp; i++)
        for (int c = 1; c < kSpar; c++) sp[kSpar * i + c] = 0.0;
    FIL_HIP_TRY(hipMemcpy(s->kry_spar0, sp.data(), sp.size() * sizeof(double), hipMemcpyHostToDevice));
    TRY(state_forces_launch(s->d, s->X, s->qj, s->time_d, s->active_d, s->Yc, s->qc, s->F, s->T, s->box, s->st));
    if (precond == 2) {
        TRY(j0_factor_launch(s->d, s->bc, s->X, s->qc, s->T, s->t + s->p.dt, s->active_d, s->AB, s->ipiv, s->rdiag,
                             s->jflag_d, s->AinvT, nullptr, s->st));
        FIL_HIP_TRY(hipMemcpyAsync(s->jflag_h, s->jflag_d, s->M * sizeof(int32_t), hipMemcpyDeviceToHost, s->st));
    }
    TRY(eval_residual(s, s->X, s->kry_f0, nullptr, nullptr, false, -1));
    applies++;
    TRY(read_resid(s, res));
    if (precond == 2)
        for (int64_t f = 0; f < s->M; f++)
            if (s->jflag_h[f]) {
                set_error(std::string(who) + ": approximate Jacobian block of filament " + std::to_string(f) +
                          " is singular");
                return FIL_ENONFINITE;
            }
    return FIL_OK;
}

// b = -f (left: -J0^{-1} f) into out
int kry_rhs(fil_sim* s, int precond, const double* f, double* out) {
    const int64_t n6 = 6 * s->S;
    if (precond == 2) {
        TRY(j0_apply_launch(s->d, s->AinvT, f, s->kry_u, s->st));
        return axpby_launch(n6, -1.0, s->kry_u, 0.0, nullptr, out, s->st);
    }
    return axpby_launch(n6, -1.0, f, 0.0, nullptr, out, s->st);
}

int kry_finish(fil_sim* s, const char* who, int rc, int outer, int kiters, int applies, const std::vector<double>& res,
               fil_jfnk_report* report) {
    if (report) {
        report->newton_iters = outer;
        report->krylov_iters = kiters;
        report->mobility_applies = applies;
        report->converged = rc == FIL_OK ? 1 : 0;
        report->resid = res.empty() ? 0.0 : res[0];
    }
    if (rc != FIL_OK) {
        set_error(std::string(who) + (rc == FIL_ENONFINITE ? ": residual became non-finite; state left at the previous step"
                                                          : ": did not reach the tolerance; state left at the previous step"));
        return rc;
    }
    TRY(finalize_launch(s->d, nullptr, s->Yc, s->qc, s->X, s->Yj, s->Yjm1, s->qj, s->Xj, s->Xjm1, s->Xjm2, s->st));
    s->t += s->p.dt;
    s->step += 1;
    return FIL_OK;
}

}  // namespace

extern "C" {

int fil_jfnk_step(fil_sim* s, int precond, double krylov_tol, double fd_delta, int krylov_max,
                  fil_jfnk_report* report) {
    std::vector<double> res;
    int applies = 0, kiters = 0, newton = 0;
    TRY(kry_begin(s, "fil_jfnk_step", precond, krylov_tol, fd_delta, krylov_max, res, applies));
    const int64_t n6 = 6 * s->S;
    const KryOpts o{precond, krylov_tol, fd_delta, krylov_max};
    // (J P^{-1}) v, left-multiplied by J0^{-1} when preconditioned so
    const KryOp A = [&](const double* v, double* w) -> int {
        const double* u = v;
        if (precond == 1) {
            TRY(mul_launch(n6, s->kry_pinv, v, s->kry_u, s->st));
            u = s->kry_u;
        }
        TRY(axpby_launch(n6, 1.0, s->X, o.delta, u, s->kry_Xp, s->st));
        TRY(eval_residual(s, s->kry_Xp, s->kry_fp, nullptr, nullptr, true, -1));
        applies++;
        double* jv = precond == 2 ? s->kry_u : w;
        TRY(axpby_launch(n6, 1.0 / o.delta, s->kry_fp, -1.0 / o.delta, s->kry_f0, jv, s->st));
        if (precond == 2) TRY(j0_apply_launch(s->d, s->AinvT, s->kry_u, w, s->st));
        return FIL_OK;
    };
    int rc = FIL_OK;
    while (!(res[0] <= s->p.tol)) {
        if (!std::isfinite(res[0])) {
            rc = FIL_ENONFINITE;
            break;
        }
        if (newton >= s->p.kmax) {
            rc = FIL_ENOCONV;
            break;
        }
        TRY(kry_rhs(s, precond, s->kry_f0, s->kry_f00));  // b, apart from the operator's buffers
        rc = kry_gmres(s, o, A, s->kry_f00, kiters);
        if (rc != FIL_OK) break;
        if (precond == 1) TRY(mul_launch(n6, s->kry_pinv, s->kry_x, s->kry_x, s->st));
        TRY(axpby_launch(n6, 1.0, s->X, 1.0, s->kry_x, s->X, s->st));
        TRY(eval_residual(s, s->X, s->kry_f0, nullptr, nullptr, true, -1));
        applies++;
        newton++;
        TRY(read_resid(s, res));
    }
    return kry_finish(s, "fil_jfnk_step", rc, newton, kiters, applies, res, report);
}

int fil_jfb_step(fil_sim* s, int precond, double krylov_tol, double fd_delta, int krylov_max,
                 fil_jfnk_report* report) {
    std::vector<double> res;
    int applies = 0, kiters = 0, iters = 0;
    TRY(kry_begin(s, "fil_jfb_step", precond, krylov_tol, fd_delta, krylov_max, res, applies));
    const int64_t n6 = 6 * s->S;
    const KryOpts o{precond, krylov_tol, fd_delta, krylov_max};
    double* C = s->Chist;
    double* D = s->Dhist;
    int k = 0;
    std::vector<double> dd(std::max(1, s->p.kmax));
    // f0 at the initial guess, the base point of J0 = grad f0
    TRY(eval_f0(s, s->X0p, s->kry_f00));
    // ([J0 + C D^T] P^{-1}) v, left-multiplied by J0^{-1} when preconditioned so
    const KryOp A = [&](const double* v, double* w) -> int {
        const double* u = v;
        if (precond == 1) {
            TRY(mul_launch(n6, s->kry_pinv, v, s->kry_u, s->st));
            u = s->kry_u;
        }
        TRY(axpby_launch(n6, 1.0, s->X0p, o.delta, u, s->kry_Xp, s->st));
        TRY(eval_f0(s, s->kry_Xp, s->kry_fp));
        double* jv = precond == 2 ? s->kry_Xp : w;  // kry_Xp is free once f0 has been evaluated
        TRY(axpby_launch(n6, 1.0 / o.delta, s->kry_fp, -1.0 / o.delta, s->kry_f00, jv, s->st));
        if (k > 0) {
            TRY(kry_dots(s, D, k, u, dd.data()));
            TRY(kry_axpy(s, C, k, dd.data(), 1.0, jv));
        }
        if (precond == 2) TRY(j0_apply_launch(s->d, s->AinvT, s->kry_Xp, w, s->st));
        return FIL_OK;
    };
    int rc = FIL_OK;
    while (!(res[0] <= s->p.tol)) {
        if (!std::isfinite(res[0])) {
            rc = FIL_ENONFINITE;
            break;
        }
        if (iters >= s->p.kmax) {
            rc = FIL_ENOCONV;
            break;
        }
        // the right-hand side -f (left: -J0^{-1} f) in the slot of the next d
        double* rhs = D + (int64_t)k * n6;
        TRY(kry_rhs(s, precond, s->kry_f0, rhs));
        rc = kry_gmres(s, o, A, rhs, kiters);
        if (rc != FIL_OK) break;
        if (precond == 1) TRY(mul_launch(n6, s->kry_pinv, s->kry_x, s->kry_x, s->st));
        TRY(axpby_launch(n6, 1.0, s->X, 1.0, s->kry_x, s->X, s->st));
        TRY(eval_residual(s, s->X, s->kry_f0, nullptr, nullptr, true, -1));
        applies++;
        iters++;
        TRY(read_resid(s, res));
        // good-Broyden rank-one term: c = f(X_{k+1}) / |dX|, d = dX / |dX|
        double nx = 0.0;
        TRY(kry_dots(s, s->kry_x, 1, s->kry_x, &nx));
        nx = std::sqrt(nx);
        if (!(nx > 0.0)) continue;
        TRY(axpby_launch(n6, 1.0 / nx, s->kry_f0, 0.0, nullptr, C + (int64_t)k * n6, s->st));
        TRY(axpby_launch(n6, 1.0 / nx, s->kry_x, 0.0, nullptr, D + (int64_t)k * n6, s->st));
        k++;
    }
    return kry_finish(s, "fil_jfb_step", rc, iters, kiters, applies, res, report);
}

}  // extern "C"
