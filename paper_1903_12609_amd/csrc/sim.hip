// Host orchestration of the implicit step (fil_sim): device state, workspace,
// the Broyden loop and the extern "C" entry points declared in fil.h.
//
// One step (Sec. 2.9.3, Alg. 2, Sec. 3.2.2):
//   X0 = warm start; f0 = f(X0); J0 = df0/dX at X0 (Appendix B.2), inverted per
//   filament; X1 = X0 - J0^{-1} f0; then for k = 1, 2, ...: f_k = f(X_k)
//   (one mobility apply), stop when max|f_k|/a <= tol, else the bad-Broyden
//   update reusing H_{k-1} f_k for both c_k and the next step.
// Convergence is tested on the host once per iteration (one small D2H copy).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "solver.h"

using namespace fil;

struct fil_sim {
    fil_params p{};
    int64_t S = 0, M = 0, nsusp = 0;
    hipStream_t st = nullptr;
    std::vector<void*> dev_allocs;
    std::vector<void*> host_allocs;
    SimDev d{};
    double *Yj = nullptr, *Yjm1 = nullptr, *qj = nullptr, *Xj = nullptr, *Xjm1 = nullptr;
    double *X = nullptr, *f = nullptr, *fprev = nullptr, *h = nullptr, *g0 = nullptr;
    double *Yc = nullptr, *qc = nullptr, *F = nullptr, *T = nullptr, *V = nullptr, *W = nullptr;
    double *AB = nullptr, *AinvT = nullptr, *Chist = nullptr, *Dhist = nullptr, *part = nullptr;
    double* box = nullptr;
    int32_t *ipiv = nullptr, *active_d = nullptr, *commit_d = nullptr, *jflag_d = nullptr;
    unsigned long long* resbits_d = nullptr;
    int32_t *active_h = nullptr, *commit_h = nullptr, *jflag_h = nullptr;
    unsigned long long* resbits_h = nullptr;
    void* rpy_work = nullptr;
    int rb = 0;  // which half of resbits_d the last residual evaluation wrote
    RpyPlan rplan{};
    RpyBatchPlan bplan;
    bool batched = false;
    double t = 0.0;
    int64_t step = 0;
    int k = 0;
    BdfCoef bc{};
    std::vector<int64_t> susp_seg_off;
    // optional timing of the main mobility kernel: one event pair per apply of a step
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int nev = 0;
    double rpy_ms = 0.0;
    int64_t rpy_launches = 0;
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

// adds the recorded mobility-kernel durations (stream already synchronised)
int collect_timing(fil_sim* s) {
    for (int i = 0; i < s->nev; i++) {
        float ms = 0.f;
        FIL_HIP_TRY(hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]));
        s->rpy_ms += ms;
        s->rpy_launches++;
    }
    s->nev = 0;
    return FIL_OK;
}

void free_sim(fil_sim* s) {
    if (!s) return;
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    for (void* p : s->dev_allocs) (void)hipFree(p);
    for (void* p : s->host_allocs) (void)hipHostFree(p);
    delete s;
}

// f = f(X) for the active suspensions; resbits receives max|f| per suspension
int eval_residual(fil_sim* s, const double* X, double* fout) {
    const double tt = s->t + s->p.dt;
    TRY(state_forces_launch(s->d, X, s->qj, tt, s->active_d, s->Yc, s->qc, s->F, s->T, s->box, s->st));
    // the source records sit at the start of the mobility workspace in both plans
    TRY(steric_pack_launch(s->d, s->Yc, s->box, s->active_d, s->F, s->T, s->p.prec, s->rpy_work, s->st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s->timing) {
        while ((int)s->ev.size() < 2 * (s->nev + 1)) {
            hipEvent_t e;
            FIL_HIP_TRY(hipEventCreate(&e));
            s->ev.push_back(e);
        }
        e0 = s->ev[2 * s->nev];
        e1 = s->ev[2 * s->nev + 1];
        s->nev++;
    }
    const double* part = nullptr;
    int K = 1;
    if (s->batched) {
        TRY(rpy_batch_launch(s->bplan, s->Yc, s->F, s->T, s->p.a, s->p.eta, s->V, s->W, s->rpy_work, s->st, e0, e1,
                             true));
    } else {
        // the split-K partials are summed inside the residual kernel
        TRY(rpy_launch(s->rplan, s->Yc, s->F, s->T, s->p.a, s->p.eta, s->V, s->W, s->rpy_work, s->st, e0, e1, true,
                       false));
        if (s->rplan.K > 1) {
            part = rpy_partials(s->rplan, s->rpy_work);
            K = s->rplan.K;
        }
    }
    s->rb ^= 1;
    TRY(residual_launch(s->d, s->bc, X, s->Xj, s->Yc, s->Yj, s->Yjm1, s->V, s->W, part, K, s->active_d, fout,
                        s->resbits_d + s->rb * s->nsusp, s->resbits_d + (1 - s->rb) * s->nsusp, s->st));
    return FIL_OK;
}

int read_resid(fil_sim* s, std::vector<double>& res) {
    FIL_HIP_TRY(hipMemcpyAsync(s->resbits_h, s->resbits_d + s->rb * s->nsusp, s->nsusp * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, s->st));
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    res.resize(s->nsusp);
    for (int64_t i = 0; i < s->nsusp; i++) {
        double v;
        std::memcpy(&v, &s->resbits_h[i], sizeof v);
        res[i] = v / s->p.a;
    }
    return FIL_OK;
}

int upload_flags(fil_sim* s, int32_t* dst, const int32_t* src) {
    FIL_HIP_TRY(hipMemcpyAsync(dst, src, s->nsusp * sizeof(int32_t), hipMemcpyHostToDevice, s->st));
    return FIL_OK;
}

// J0 at the configuration of X (state buffers already filled by eval_residual),
// factorised; h = J0^{-1} f.
int begin_solve(fil_sim* s, double* dXout) {
    const double tt = s->t + s->p.dt;
    TRY(j0_factor_launch(s->d, s->bc, s->X, s->qc, s->T, tt, s->active_d, s->AB, s->ipiv, s->jflag_d, s->AinvT,
                         s->st));
    TRY(j0_solve_launch(s->d, s->AB, s->ipiv, s->AinvT, s->f, s->active_d, s->h, s->st));
    s->k = 0;
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
    FIL_CHECK_ARG(p->FS == 0.0 || p->chi > 1.0, "fil_create: the steric range chi must exceed 1");
    FIL_CHECK_ARG(susp_fil_off[0] == 0, "fil_create: susp_fil_off[0] must be 0");
    for (int64_t i = 0; i < nsusp; i++)
        FIL_CHECK_ARG(susp_fil_off[i + 1] > susp_fil_off[i], "fil_create: every suspension needs >= 1 filament");
    const int64_t M = susp_fil_off[nsusp];
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
        if (tether) teth[f] = tether[f] ? 1 : 0;
    }
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
    std::vector<int64_t> vblk_start, susp_vblk_off(nsusp + 1);
    std::vector<int32_t> vblk_susp;
    std::vector<int64_t> sfo(susp_fil_off, susp_fil_off + nsusp + 1);
    for (int64_t i = 0; i < nsusp; i++) {
        susp_vblk_off[i] = (int64_t)vblk_susp.size();
        for (int64_t e = 6 * susp_seg_off[i]; e < 6 * susp_seg_off[i + 1]; e += kVecBlock) {
            vblk_start.push_back(e);
            vblk_susp.push_back((int32_t)i);
        }
    }
    susp_vblk_off[nsusp] = (int64_t)vblk_susp.size();
    const int64_t nvblk = (int64_t)vblk_susp.size();
    vblk_start.push_back(6 * S);
    s->susp_seg_off = susp_seg_off;

    // ---- device allocations
    int rc = FIL_OK;
    int64_t *d_seg_off, *d_susp_seg_off, *d_susp_fil_off, *d_vblk_start, *d_susp_vblk_off, *d_dense_off = nullptr;
    int32_t *d_fil_susp, *d_seg_fil, *d_teth, *d_vblk_susp;
    double *d_base, *d_phase = nullptr;
    const size_t n6 = 6 * (size_t)S;
    const int max_dots = p->kmax + 2;
#define A(ptr, n)                                  \
    if (rc == FIL_OK) rc = dalloc(s, &(ptr), (n));
    A(d_seg_off, M + 1) A(d_susp_seg_off, nsusp + 1) A(d_susp_fil_off, nsusp + 1) A(d_vblk_start, nvblk + 1)
    A(d_susp_vblk_off, nsusp + 1) A(d_fil_susp, M) A(d_seg_fil, S) A(d_teth, M) A(d_vblk_susp, nvblk)
    A(d_base, 3 * M)
    if (phase) A(d_phase, M)
    A(s->Yj, 3 * S) A(s->Yjm1, 3 * S) A(s->qj, 4 * S) A(s->Xj, n6) A(s->Xjm1, n6)
    A(s->X, n6) A(s->f, n6) A(s->fprev, n6) A(s->h, n6) A(s->g0, n6)
    A(s->Yc, 3 * S) A(s->qc, 4 * S) A(s->F, 3 * S) A(s->T, 3 * S) A(s->V, 3 * S) A(s->W, 3 * S)
    A(s->AB, n6 * kBandW) A(s->ipiv, n6)
    if (dense) { A(s->AinvT, dense_tot) A(d_dense_off, M) }
    A(s->Chist, (size_t)p->kmax * n6) A(s->Dhist, (size_t)p->kmax * n6) A(s->part, (size_t)nvblk * max_dots)
    A(s->box, 6 * M) A(s->active_d, nsusp) A(s->commit_d, nsusp) A(s->jflag_d, M) A(s->resbits_d, 2 * nsusp)
#undef A
    if (rc == FIL_OK) rc = halloc(s, &s->active_h, nsusp);
    if (rc == FIL_OK) rc = halloc(s, &s->commit_h, nsusp);
    if (rc == FIL_OK) rc = halloc(s, &s->jflag_h, M);
    if (rc == FIL_OK) rc = halloc(s, &s->resbits_h, nsusp);
    if (rc) {
        free_sim(s);
        return rc;
    }
    // mobility workspace
    s->batched = nsusp > 1;
    size_t wbytes;
    if (s->batched) {
        s->bplan = rpy_batch_plan(nsusp, susp_seg_off.data(), p->prec);
        wbytes = s->bplan.total();
    } else {
        s->rplan = rpy_plan(S, p->prec);
        wbytes = s->rplan.total();
    }
    char* wk = nullptr;
    if ((rc = dalloc(s, &wk, wbytes))) {
        free_sim(s);
        return rc;
    }
    s->rpy_work = wk;
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
    auto up = [&]() -> int {
        TRY(upload(d_seg_off, seg_off));
        TRY(upload(d_susp_seg_off, susp_seg_off));
        TRY(upload(d_susp_fil_off, sfo));
        if (dense) TRY(upload(d_dense_off, dense_off));
        TRY(upload(d_vblk_start, vblk_start));
        TRY(upload(d_susp_vblk_off, susp_vblk_off));
        TRY(upload(d_fil_susp, fil_susp));
        TRY(upload(d_seg_fil, seg_fil));
        TRY(upload(d_teth, teth));
        TRY(upload(d_vblk_susp, vblk_susp));
        TRY(upload(d_base, base));
        if (phase) TRY(upload(d_phase, std::vector<double>(phase, phase + M)));
        TRY(upload(s->Yj, Ysoa));
        TRY(upload(s->Yjm1, Ysoa));
        TRY(upload(s->qj, qsoa));
        TRY(upload(s->Xj, zeros));
        TRY(upload(s->Xjm1, zeros));
        TRY(upload(s->X, zeros));
        TRY(upload(s->resbits_d, std::vector<unsigned long long>(2 * nsusp, 0ull)));
        if (s->batched) {
            TRY(rpy_batch_upload(s->bplan, s->rpy_work, nullptr));
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
    d.nvblk = nvblk;
    d.vblk_susp = d_vblk_susp;
    d.vblk_start = d_vblk_start;
    d.susp_vblk_off = d_susp_vblk_off;
    d.max_dots = max_dots;
    d.a = p->a;
    d.eta = p->eta;
    d.dL = p->dL;
    d.KB = p->KB;
    d.KT = p->KT;
    d.chi = p->chi;
    d.FS = p->FS;
    for (int i = 0; i < 3; i++) d.grav[i] = p->grav[i];
    d.dt = p->dt;
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

int fil_bdf2_step(fil_sim* s, fil_step_report* report) {
    FIL_CHECK_ARG(s, "fil_bdf2_step: null sim");
    const int64_t ns = s->nsusp;
    s->bc = coefs(s->step);
    s->nev = 0;
    std::vector<int32_t> state(ns, 0);  // 0 running, 1 converged, -1 failed
    std::vector<int32_t> iters(ns, 0);
    std::vector<double> res, last(ns, 0.0);
    for (int64_t i = 0; i < ns; i++) s->active_h[i] = 1;
    TRY(upload_flags(s, s->active_d, s->active_h));
    TRY(initial_guess_launch(s->d, s->step, s->Yj, s->Yjm1, s->Xj, s->Xjm1, s->active_d, s->X, s->st));
    TRY(eval_residual(s, s->X, s->f));
    TRY(begin_solve(s, nullptr));
    TRY(read_resid(s, res));
    FIL_HIP_TRY(hipMemcpyAsync(s->jflag_h, s->jflag_d, s->M * sizeof(int32_t), hipMemcpyDeviceToHost, s->st));
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    bool changed = false;
    for (int64_t i = 0; i < ns; i++) {
        last[i] = res[i];
        if (!std::isfinite(res[i])) state[i] = -1;
        else if (res[i] <= s->p.tol) state[i] = 1;
        if (state[i] != 0) {
            s->active_h[i] = 0;
            changed = true;
        }
    }
    for (int64_t f = 0; f < s->M; f++)
        if (s->jflag_h[f]) {
            set_error("fil_bdf2_step: approximate Jacobian block of filament " + std::to_string(f) + " is singular");
            for (int64_t i = 0; i < ns; i++) s->active_h[i] = 0;
            std::fill(state.begin(), state.end(), -1);
            changed = true;
            break;
        }
    bool any = false;
    for (int64_t i = 0; i < ns; i++) any |= s->active_h[i] != 0;
    if (changed) TRY(upload_flags(s, s->active_d, s->active_h));
    if (any) TRY(first_step_launch(s->d, s->h, s->f, s->fprev, s->X, nullptr, s->active_d, s->st));
    for (int it = 1; any; it++) {
        TRY(eval_residual(s, s->X, s->f));
        TRY(read_resid(s, res));
        changed = false;
        any = false;
        for (int64_t i = 0; i < ns; i++) {
            if (!s->active_h[i]) continue;
            iters[i] = it;
            last[i] = res[i];
            if (!std::isfinite(res[i])) state[i] = -1;
            else if (res[i] <= s->p.tol) state[i] = 1;
            else if (it >= s->p.kmax) state[i] = -1;
            if (state[i] != 0) {
                s->active_h[i] = 0;
                changed = true;
            } else {
                any = true;
            }
        }
        if (!any) break;
        if (changed) TRY(upload_flags(s, s->active_d, s->active_h));
        TRY(broyden_update_launch(s->d, s->k, s->AB, s->ipiv, s->AinvT, s->Chist, s->Dhist, s->f, s->fprev, s->g0,
                                  s->h, s->part, s->X, nullptr, s->active_d, s->st));
        s->k++;
    }
    if (s->timing) {
        FIL_HIP_TRY(hipStreamSynchronize(s->st));
        TRY(collect_timing(s));
    }
    bool all_ok = true;
    for (int64_t i = 0; i < ns; i++) {
        all_ok &= state[i] == 1;
        if (report) {
            report[i].iters = iters[i];
            report[i].mobility_applies = iters[i] + 1;
            report[i].converged = state[i] == 1;
            report[i].pad = 0;
            report[i].resid = last[i];
        }
    }
    if (!all_ok) {
        bool nonfinite = false;
        for (int64_t i = 0; i < ns; i++) nonfinite |= !std::isfinite(last[i]);
        set_error(nonfinite ? "fil_bdf2_step: residual became non-finite; state left at the previous step"
                            : "fil_bdf2_step: Broyden did not reach the tolerance; state left at the previous step");
        return nonfinite ? FIL_ENONFINITE : FIL_ENOCONV;
    }
    for (int64_t i = 0; i < ns; i++) s->commit_h[i] = 1;
    TRY(upload_flags(s, s->commit_d, s->commit_h));
    TRY(finalize_launch(s->d, s->commit_d, s->Yc, s->qc, s->X, s->Yj, s->Yjm1, s->qj, s->Xj, s->Xjm1, s->st));
    FIL_HIP_TRY(hipStreamSynchronize(s->st));
    s->t += s->p.dt;
    s->step += 1;
    return FIL_OK;
}

int fil_set_timing(fil_sim* s, int enable) {
    FIL_CHECK_ARG(s, "fil_set_timing: null sim");
    s->timing = enable != 0;
    s->rpy_ms = 0.0;
    s->rpy_launches = 0;
    s->nev = 0;
    return FIL_OK;
}

int fil_get_timing(fil_sim* s, double* rpy_ms, int64_t* rpy_launches) {
    FIL_CHECK_ARG(s, "fil_get_timing: null sim");
    if (rpy_ms) *rpy_ms = s->rpy_ms;
    if (rpy_launches) *rpy_launches = s->rpy_launches;
    return FIL_OK;
}

int fil_residual(fil_sim* s, const double* X, double* f_out) {
    FIL_CHECK_ARG(s && X && f_out, "fil_residual: null argument");
    s->bc = coefs(s->step);
    for (int64_t i = 0; i < s->nsusp; i++) s->active_h[i] = 1;
    TRY(upload_flags(s, s->active_d, s->active_h));
    return eval_residual(s, X, f_out);
}

int fil_broyden_begin(fil_sim* s, const double* X0, double* f0_out) {
    FIL_CHECK_ARG(s && X0, "fil_broyden_begin: null argument");
    s->bc = coefs(s->step);
    for (int64_t i = 0; i < s->nsusp; i++) s->active_h[i] = 1;
    TRY(upload_flags(s, s->active_d, s->active_h));
    FIL_HIP_TRY(hipMemcpyAsync(s->X, X0, 6 * s->S * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    TRY(eval_residual(s, s->X, s->f));
    TRY(begin_solve(s, nullptr));
    if (f0_out) FIL_HIP_TRY(hipMemcpyAsync(f0_out, s->f, 6 * s->S * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    TRY(first_step_launch(s->d, s->h, s->f, s->fprev, s->X, nullptr, s->active_d, s->st));
    return FIL_OK;
}

int fil_broyden_update(fil_sim* s, const double* f_new, double* dX_out) {
    FIL_CHECK_ARG(s && f_new, "fil_broyden_update: null argument");
    FIL_CHECK_ARG(s->k + 1 < s->p.kmax, "fil_broyden_update: history full (kmax updates)");
    TRY(broyden_update_launch(s->d, s->k, s->AB, s->ipiv, s->AinvT, s->Chist, s->Dhist, f_new, s->fprev, s->g0, s->h,
                              s->part, s->X, dX_out, s->active_d, s->st));
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

}  // extern "C"
