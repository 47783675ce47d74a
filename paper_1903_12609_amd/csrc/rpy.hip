// RPY mobility apply on gfx950 (Sec. 2.7.1 of arXiv:1903.12609).
//
// Design
//   * Every (target, source) pair is visited once: the sum is split over
//     source chunks ("split-K") so that a launch has far more workgroups than
//     the 256 CUs, and the per-chunk partial (V, Omega) are reduced in a fixed
//     order by a second kernel (deterministic, no float atomics).
//   * All 64 lanes of a wave walk the same source at the same time, so the
//     source record is wave-uniform: it is read with scalar loads into SGPRs
//     and broadcast to the VALU for free.  No LDS staging is needed.
//   * Each lane owns TPL targets (register blocking amortises loop overhead).
//   * FP64 path: the cross-product terms are expanded so that per-source
//     constants (T_m x Y_m, 2/3 F_m x Y_m) are precomputed:
//         sum_m s^3 T_m x (Y_n - Y_m) = (sum_m s^3 T_m) x Y_n - sum_m s^3 (T_m x Y_m)
//     and the terms that enter V (or Omega) with a fixed coefficient share one sum,
//     which leaves four 3-vector sums per target and ~50 VALU operations per pair.
//     The coefficient 2a^2/3 of s^3 F_m in M^tt and -1/2 of s^3 T_m in M^rr are
//     applied once per target at the end.
//   * FP32-tile path: sources come in tiles of 16 (by global index) with an FP64
//     origin each; a source record holds its FP32 offset s' from that origin and the
//     cross products of its torque and force with s'.  A wave's targets are
//     contiguous; each target's offset y' from the tile origin is rounded once per
//     tile and r = y' - s' is formed in float (an error of a few float ulps of
//     |r| + 2 x tile radius).  The pair arithmetic runs in float, the parts of T x r
//     and F x r that depend on y' are completed once per tile, and each tile's sums
//     are added into double.  Only tiles that may hold a pair closer than 2a to one of
//     the wave's targets take the overlap test.
//   * Overlapping pairs (r < 2a) take a rarely executed branch with the regularised
//     forms; the far-field weights are zeroed there.  The self pair (r = 0) is taken in
//     its closed form 4/(3a) F, T/a^3 (in the FP32-tile path: in double, per target).
#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace fil {

constexpr int kRpyBlock = 256;
constexpr int kMaxChunkSmall = 256;  // most sources per block on the small-size path (64 per wave)

// ------------------------------------------------------------------ packing
__global__ void __launch_bounds__(256) rpy_pack_f64(int64_t S, const double* __restrict__ Y,
                                                   const double* __restrict__ F, const double* __restrict__ T,
                                                   double* __restrict__ pk) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= S) return;
    rpy_pack_record_f64(pk, m, Y[m], Y[S + m], Y[2 * S + m], F[m], F[S + m], F[2 * S + m], T[m], T[S + m],
                        T[2 * S + m]);
}

// FP32-tile records: one thread per source; the 16 lanes of a tile (tiles start at global
// indices that are multiples of 16, and so do the lane groups of every wave) reduce their
// bounding box with lane exchanges, take its centre as the tile origin and write their
// offsets from it.  active: optional flag of the single suspension (0: nothing to do).
__global__ void __launch_bounds__(256) rpy_tile_pack(int64_t S, const double* __restrict__ Y,
                                                    const double* __restrict__ F, const double* __restrict__ T,
                                                    SrcF32* __restrict__ pk, TileF32* __restrict__ tiles,
                                                    const int32_t* __restrict__ active) {
    static_assert(kF32Tile == 16 || kF32Tile == 32, "lane groups of 16 or 32 within a wave");
    if (active && !active[0]) return;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t mm = m < S ? m : S - 1;  // lanes past the end repeat the last source
    double y[3], lo[3], hi[3];
    for (int i = 0; i < 3; i++) y[i] = lo[i] = hi[i] = Y[i * S + mm];
    for (int off = 1; off < kF32Tile; off <<= 1)
        for (int i = 0; i < 3; i++) {
            lo[i] = fmin(lo[i], __shfl_xor(lo[i], off));
            hi[i] = fmax(hi[i], __shfl_xor(hi[i], off));
        }
    if (m >= S) return;
    double o[3], d2 = 0.0;
    for (int i = 0; i < 3; i++) {
        o[i] = 0.5 * (lo[i] + hi[i]);
        d2 = fma(hi[i] - lo[i], hi[i] - lo[i], d2);
    }
    SrcF32 r;
    double sp[3], f[3], t[3];
    for (int i = 0; i < 3; i++) {
        r.sp[i] = (float)(y[i] - o[i]);
        sp[i] = (double)r.sp[i];  // the cross products below use the offset as stored
        f[i] = F[i * S + m];
        t[i] = T[i * S + m];
        r.f[i] = (float)f[i];
        r.t[i] = (float)t[i];
    }
    for (int i = 0; i < 3; i++) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
        r.ct[i] = (float)(t[i1] * sp[i2] - t[i2] * sp[i1]);
        r.cf[i] = (float)((2.0 / 3.0) * (f[i1] * sp[i2] - f[i2] * sp[i1]));
    }
    r.pad = 0.f;
    pk[m] = r;
    if (m % kF32Tile == 0) {
        TileF32 tr;
        for (int i = 0; i < 3; i++) tr.o[i] = o[i];
        tr.rad = 0.5 * sqrt(d2);
        tiles[m / kF32Tile] = tr;
    }
}

// ------------------------------------------------------------------ FP64 pair
// Per target, with r = y - Y_m and s = 1/|r| (V, Omega below are divided by c):
//   V += s F + (1 - 2a^2 s^2)(r.F) s^3 r - s^3 (T x Y_m)   (+ overlap V)
//   R += s^3 F,   P += s^3 T
//   W += s^5 (r.T) r - 2/3 s^3 (F x Y_m)                   (+ 2/3 overlap Omega)
// and at the end V = V + 2a^2/3 R + P x y, Omega = R x y + 3/2 W - 1/2 P (T x Y_m and
// 2/3 F x Y_m come with the source record).
struct AccF64 {
    double V[3], R[3], P[3], W[3];
};

// Overlap (r < 2a) contribution divided by c = 1/(8 pi eta).  Equal-radius
// regularised RPY:
//   V/c  += 4/(3a) [(1 - 9r/(32a)) F + 3/(32 a r) (r.F) r] + (1/(2a^2)) (1/a - 3r/(8a^2)) T x r
//   Om/c += 1/a^3 [(1 - 27r/(32a) + 5r^3/(64a^3)) T + (9/(32 a r) - 3r/(64a^3)) (r.T) r]
//           + (1/(2a^2)) (1/a - 3r/(8a^2)) F x r
// Returned by value so that the accumulators never leave registers.
template <typename R>
struct Ovl {
    R v[3], w[3];
};

template <typename R>
__device__ __forceinline__ Ovl<R> rpy_overlap(R rx, R ry, R rz, R r2, R Fx, R Fy, R Fz, R Tx, R Ty, R Tz, R a) {
    const R r = sqrt(r2);
    const R ir = r > R(0) ? R(1) / r : R(0);
    const R ia = R(1) / a, ia3 = ia * ia * ia;
    const R rF = rx * Fx + ry * Fy + rz * Fz, rT = rx * Tx + ry * Ty + rz * Tz;
    const R ctt1 = R(4.0 / 3.0) * ia * (R(1) - R(9.0 / 32.0) * r * ia);
    const R ctt2 = R(0.125) * ia * ia * ir;
    const R ctr = R(0.5) * ia * ia * (ia - R(0.375) * r * ia * ia);
    const R crr1 = ia3 * (R(1) - R(27.0 / 32.0) * r * ia + R(5.0 / 64.0) * r2 * r * ia3);
    const R crr2 = ia3 * (R(9.0 / 32.0) * ia * ir - R(3.0 / 64.0) * r * ia3);
    Ovl<R> o;
    o.v[0] = ctt1 * Fx + ctt2 * rF * rx + ctr * (Ty * rz - Tz * ry);
    o.v[1] = ctt1 * Fy + ctt2 * rF * ry + ctr * (Tz * rx - Tx * rz);
    o.v[2] = ctt1 * Fz + ctt2 * rF * rz + ctr * (Tx * ry - Ty * rx);
    o.w[0] = crr1 * Tx + crr2 * rT * rx + ctr * (Fy * rz - Fz * ry);
    o.w[1] = crr1 * Ty + crr2 * rT * ry + ctr * (Fz * rx - Fx * rz);
    o.w[2] = crr1 * Tz + crr2 * rT * rz + ctr * (Fx * ry - Fy * rx);
    return o;
}

__device__ __forceinline__ void rpy_pair_f64(const double y[3], const double (&s)[15], double a, double four_a2,
                                             double two_a2, AccF64& A) {
    const double rx = y[0] - s[0], ry = y[1] - s[1], rz = y[2] - s[2];
    const double r2 = fma(rx, rx, fma(ry, ry, rz * rz));
    const bool near = r2 < four_a2;
    double sv = rsqrt_f64(r2);
    sv = near ? 0.0 : sv;
    const double s2 = sv * sv, s3 = s2 * sv;
    const double Fx = s[3], Fy = s[4], Fz = s[5], Tx = s[6], Ty = s[7], Tz = s[8];
    const double rF = fma(rx, Fx, fma(ry, Fy, rz * Fz));
    const double rT = fma(rx, Tx, fma(ry, Ty, rz * Tz));
    const double Br = s3 * fma(-two_a2, s2, 1.0) * rF;
    A.V[0] = fma(sv, Fx, fma(Br, rx, fma(-s3, s[9], A.V[0])));
    A.V[1] = fma(sv, Fy, fma(Br, ry, fma(-s3, s[10], A.V[1])));
    A.V[2] = fma(sv, Fz, fma(Br, rz, fma(-s3, s[11], A.V[2])));
    A.R[0] = fma(s3, Fx, A.R[0]);
    A.R[1] = fma(s3, Fy, A.R[1]);
    A.R[2] = fma(s3, Fz, A.R[2]);
    A.P[0] = fma(s3, Tx, A.P[0]);
    A.P[1] = fma(s3, Ty, A.P[1]);
    A.P[2] = fma(s3, Tz, A.P[2]);
    const double D = s3 * s2 * rT;
    A.W[0] = fma(D, rx, fma(-s3, s[12], A.W[0]));
    A.W[1] = fma(D, ry, fma(-s3, s[13], A.W[1]));
    A.W[2] = fma(D, rz, fma(-s3, s[14], A.W[2]));
    if (near) {
        // overlap: added to V and (times 2/3) to W.  At r = 0 (the self pair) the overlap
        // forms reduce to 4/(3a) F and T/a^3, taken directly
        if (r2 > 0.0) {
            const Ovl<double> o = rpy_overlap<double>(rx, ry, rz, r2, Fx, Fy, Fz, Tx, Ty, Tz, a);
            for (int i = 0; i < 3; i++) {
                A.V[i] += o.v[i];
                A.W[i] = fma(2.0 / 3.0, o.w[i], A.W[i]);
            }
        } else {
            const double cv = 4.0 / (3.0 * a), cw = 2.0 / (3.0 * a * a * a);
            A.V[0] = fma(cv, Fx, A.V[0]);
            A.V[1] = fma(cv, Fy, A.V[1]);
            A.V[2] = fma(cv, Fz, A.V[2]);
            A.W[0] = fma(cw, Tx, A.W[0]);
            A.W[1] = fma(cw, Ty, A.W[1]);
            A.W[2] = fma(cw, Tz, A.W[2]);
        }
    }
}

// Output addressing shared by both precisions.  With K > 1 each chunk k writes
// its partial (V, Omega) to part[(k*6 + c) * S + n]; with K == 1 directly V, W.
struct RpyOut {
    double* part;
    double* V;
    double* W;
    const int32_t* active;  // per-suspension flags (null: always compute); inactive ones are skipped
};

__device__ __forceinline__ void rpy_store(const RpyOut& o, int64_t base, int64_t S, int64_t Sg, int K, int k,
                                          int64_t n, const double v[3], const double w[3]) {
    if (K == 1) {
        for (int i = 0; i < 3; i++) {
            o.V[i * Sg + base + n] = v[i];
            o.W[i * Sg + base + n] = w[i];
        }
    } else {
        double* p = o.part + (int64_t)k * 6 * S + n;
        for (int i = 0; i < 3; i++) {
            p[i * S] = v[i];
            p[(3 + i) * S] = w[i];
        }
    }
}

// Writes the per-target results; with WS > 1 the waves' sums are combined in LDS
// (wave 0 adds waves 1..WS-1 in order) before the store.
template <int TPL, int WS>
__device__ __forceinline__ void rpy_finish(const RpyOut& out, int64_t base, int64_t S, int64_t Sg, int K, int k,
                                           const int64_t (&n)[TPL], double (&vw)[TPL][6]) {
    if (WS > 1) {
        __shared__ double red[WS > 1 ? WS - 1 : 1][TPL * 6][64];
        const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
        if (wave > 0)
#pragma unroll
            for (int j = 0; j < TPL; j++)
                for (int q = 0; q < 6; q++) red[wave - 1][j * 6 + q][lane] = vw[j][q];
        __syncthreads();
        if (wave > 0) return;
#pragma unroll
        for (int j = 0; j < TPL; j++)
            for (int q = 0; q < 6; q++)
                for (int w2 = 0; w2 < WS - 1; w2++) vw[j][q] += red[w2][j * 6 + q][lane];
    }
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        if (n[j] >= S) continue;
        const double v[3] = {vw[j][0], vw[j][1], vw[j][2]}, w[3] = {vw[j][3], vw[j][4], vw[j][5]};
        rpy_store(out, base, S, Sg, K, k, n[j], v, w);
    }
}

// One work item: targets [tb*256*TPL, +256*TPL) x sources [k*chunk, +chunk) of one
// suspension whose segments start at global index `base` (S of them).  Partial
// results go to part[(k*6 + c) * S + n] (suspension-local n) when K > 1.
// WS = 1: the block's four waves own 4 x 64 x TPL different targets.  WS = 4 (small
// sizes): the four waves share 64 x TPL targets and split the chunk's sources
// four ways; their results are combined through LDS in wave order.  SKIP (WS = 1, many
// suspensions of any size): each wave owns 64 x TPL consecutive targets and a wave whose
// targets all lie past the end of the suspension returns at once.
template <int TPL, int WS, bool SKIP = false>
__device__ __forceinline__ void rpy_item_f64(int64_t base, int64_t S, int64_t Sg, int64_t tb, int k, int K,
                                             int64_t chunk, const double* __restrict__ pk,
                                             const double* __restrict__ Y, double a, double c, const RpyOut& out) {
    static_assert(!SKIP || WS == 1, "waves that share targets cannot skip");
    constexpr int kTgtPerBlock = kRpyBlock / WS;  // targets per j-slice
    // the wave index is made visibly wave-uniform so that the source range, the
    // loop and the source addresses stay on the scalar unit
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int tid = WS == 1 ? (int)threadIdx.x : (int)(threadIdx.x % 64);
    const int64_t t_wave = tb * (kTgtPerBlock * TPL) + (int64_t)wave * 64 * TPL;  // SKIP: the wave's first target
    if (SKIP && t_wave >= S) return;
    int64_t m0 = (int64_t)k * chunk;
    int64_t m1 = min(S, m0 + chunk);
    if (WS > 1) {
        const int64_t sub = (m1 - m0 + WS - 1) / WS;
        const int64_t a0 = m0 + wave * sub;
        m1 = min(m1, a0 + sub);
        m0 = min(a0, m1);
    }
    const double four_a2 = 4.0 * a * a, two_a2 = 2.0 * a * a;
    int64_t n[TPL];
    double y[TPL][3];
    AccF64 A[TPL];
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        n[j] = SKIP ? t_wave + j * 64 + (tid & 63) : tb * (kTgtPerBlock * TPL) + j * kTgtPerBlock + tid;
        const int64_t nn = base + (n[j] < S ? n[j] : S - 1);
        y[j][0] = Y[nn];
        y[j][1] = Y[Sg + nn];
        y[j][2] = Y[2 * Sg + nn];
        for (int i = 0; i < 3; i++) A[j].V[i] = A[j].R[i] = A[j].P[i] = A[j].W[i] = 0.0;
    }
    {
        // the next source record is requested before the current one is used, so
        // the scalar-load latency overlaps the pair arithmetic
        // (32-bit, wave-uniform loop arithmetic stays on the scalar unit)
        const double* src = pk + 16 * (base + m0);
        const int cnt = (int)(m1 - m0);
        double cur[15];
        if (cnt > 0) {
            for (int i = 0; i < 15; i++) cur[i] = src[i];
        }
        for (int m = 0; m < cnt; ++m) {
            const int mn = m + 1 < cnt ? m + 1 : m;
            double nxt[15];
            for (int i = 0; i < 15; i++) nxt[i] = src[16 * mn + i];
#pragma unroll
            for (int j = 0; j < TPL; j++) rpy_pair_f64(y[j], cur, a, four_a2, two_a2, A[j]);
            for (int i = 0; i < 15; i++) cur[i] = nxt[i];
        }
    }
    const double c23 = 2.0 * a * a / 3.0;
    double vw[TPL][6];
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        const AccF64& B = A[j];
        const double* yy = y[j];
        // V = c [V + 2a^2/3 R + P x y];  Omega = c [R x y + 3/2 W - 1/2 P]
        vw[j][0] = c * (B.V[0] + c23 * B.R[0] + (B.P[1] * yy[2] - B.P[2] * yy[1]));
        vw[j][1] = c * (B.V[1] + c23 * B.R[1] + (B.P[2] * yy[0] - B.P[0] * yy[2]));
        vw[j][2] = c * (B.V[2] + c23 * B.R[2] + (B.P[0] * yy[1] - B.P[1] * yy[0]));
        vw[j][3] = c * ((B.R[1] * yy[2] - B.R[2] * yy[1]) + 1.5 * B.W[0] - 0.5 * B.P[0]);
        vw[j][4] = c * ((B.R[2] * yy[0] - B.R[0] * yy[2]) + 1.5 * B.W[1] - 0.5 * B.P[1]);
        vw[j][5] = c * ((B.R[0] * yy[1] - B.R[1] * yy[0]) + 1.5 * B.W[2] - 0.5 * B.P[2]);
    }
    rpy_finish<TPL, WS>(out, base, S, Sg, K, k, n, vw);
}

// Single suspension: blockIdx.x -> (target block tb = bid / K, source chunk
// k = bid % K); chunks adjacent in k land on different XCDs, so each XCD's L2
// holds ~K/8 of the sources.
template <int TPL, int WS>
__global__ void __launch_bounds__(kRpyBlock) __attribute__((amdgpu_waves_per_eu(3))) rpy_f64_kernel(int64_t S, int64_t chunk, int K,
                                                          const double* __restrict__ pk,
                                                          const double* __restrict__ Y, double a, double c,
                                                          RpyOut out) {
    if (out.active && !out.active[0]) return;
    const int k = (int)(blockIdx.x % (unsigned)K);
    const int64_t tb = blockIdx.x / (unsigned)K;
    rpy_item_f64<TPL, WS>(0, S, S, tb, k, K, chunk, pk, Y, a, c, out);
}

// Many suspensions in one persistent launch: a fixed grid walks a work list
// sorted by cost (largest first), item i handled by block i mod gridDim.
// The next work item of a persistent workgroup: taken from a counter shared by the launch
// (items are listed largest first, so taking them in order balances the workgroups)
__device__ __forceinline__ int64_t next_item(int* next, int& take) {
    __syncthreads();  // every thread has read the previous item's index
    if (threadIdx.x == 0) take = atomicAdd(next, 1);
    __syncthreads();
    return take;
}

__global__ void __launch_bounds__(32) rpy_items_reset(int* __restrict__ next) {
    if (threadIdx.x == 0) *next = 0;
}

template <int TPL>
__global__ void __launch_bounds__(kRpyBlock) __attribute__((amdgpu_waves_per_eu(3))) rpy_f64_items_kernel(const RpyItem* __restrict__ items, int64_t nitems,
                                                                int64_t Sg, const double* __restrict__ pk,
                                                                const double* __restrict__ Y, double a, double c,
                                                                RpyOut out, int* __restrict__ next) {
    __shared__ int take;
    for (;;) {
        const int64_t it = next_item(next, take);
        if (it >= nitems) break;
        const RpyItem w = items[it];
        if (out.active && !out.active[w.susp]) continue;
        RpyOut o = out;
        o.part = out.part + w.part;
        rpy_item_f64<TPL, 1, true>(w.base, w.S, Sg, w.tb, w.k, w.K, w.chunk, pk, Y, a, c, o);
    }
}

// ------------------------------------------------------------------ FP32-tile pair
// Sums over the sources of one tile, per target, in float.  With r = y_t - s_p (y_t the
// target's and s_p the source's offset from the tile origin), s = 1/|r|:
//   V  += s F + (1 - 2a^2 s^2)(r.F) s^3 r - s^3 (T x s_p)
//   R  += s^3 F
//   P  += s^3 T
//   W  += s^5 (r.T) r - 2/3 s^3 (F x s_p)
// (40 VALU operations per pair, r included; T x s_p and 2/3 F x s_p are stored in the
// source record).  Once per tile the target's (V, Omega) / c take
//   v = V + 2a^2/3 R + P x y_t,   w = R x y_t + 3/2 W - 1/2 P,
// which is s F + 2a^2/3 s^3 F + (1 - 2a^2 s^2)(r.F) s^3 r + s^3 T x r for v and
// s^3 F x r + 3/2 s^5 (r.T) r - 1/2 s^3 T for w, summed over the tile.  NEAR: the overlap
// test and its branch.
struct SrcRegF32 {
    float sp[3], f[3], t[3], ct[3], cf[3];
};
struct AccF32 {
    float V[3], R[3], P[3], W[3];
};
// the whole 64-byte record in one scalar load (it is wave-uniform)
__device__ __forceinline__ SrcRegF32 load_src_f32(const SrcF32* __restrict__ s) {
    const float4* p = reinterpret_cast<const float4*>(s);
    const float4 a = p[0], b = p[1], c = p[2], d = p[3];
    SrcRegF32 r;
    r.sp[0] = a.x; r.sp[1] = a.y; r.sp[2] = a.z;
    r.f[0] = a.w;  r.f[1] = b.x;  r.f[2] = b.y;
    r.t[0] = b.z;  r.t[1] = b.w;  r.t[2] = c.x;
    r.ct[0] = c.y; r.ct[1] = c.z; r.ct[2] = c.w;
    r.cf[0] = d.x; r.cf[1] = d.y; r.cf[2] = d.z;
    return r;
}
template <bool NEAR>
__device__ __forceinline__ void rpy_pair_f32(float rx, float ry, float rz, const SrcRegF32& s, float a,
                                             float four_a2, float two_a2, AccF32& A) {
    const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
    float sv = __builtin_amdgcn_rsqf(r2);
    bool near = false;
    if (NEAR) {
        near = r2 < four_a2;
        sv = near ? 0.f : sv;
    }
    const float s2 = sv * sv, s3 = s2 * sv;
    const float Fx = s.f[0], Fy = s.f[1], Fz = s.f[2], Tx = s.t[0], Ty = s.t[1], Tz = s.t[2];
    const float rF = fmaf(rx, Fx, fmaf(ry, Fy, rz * Fz));
    const float rT = fmaf(rx, Tx, fmaf(ry, Ty, rz * Tz));
    const float s5 = s2 * s3;
    const float Bs3 = fmaf(-two_a2, s5, s3) * rF;  // (1 - 2a^2 s^2)(r.F) s^3
    const float Ds5 = s5 * rT;                      // s^5 (r.T)
    A.V[0] = fmaf(sv, Fx, fmaf(Bs3, rx, fmaf(-s3, s.ct[0], A.V[0])));
    A.V[1] = fmaf(sv, Fy, fmaf(Bs3, ry, fmaf(-s3, s.ct[1], A.V[1])));
    A.V[2] = fmaf(sv, Fz, fmaf(Bs3, rz, fmaf(-s3, s.ct[2], A.V[2])));
    A.R[0] = fmaf(s3, Fx, A.R[0]);
    A.R[1] = fmaf(s3, Fy, A.R[1]);
    A.R[2] = fmaf(s3, Fz, A.R[2]);
    A.P[0] = fmaf(s3, Tx, A.P[0]);
    A.P[1] = fmaf(s3, Ty, A.P[1]);
    A.P[2] = fmaf(s3, Tz, A.P[2]);
    A.W[0] = fmaf(Ds5, rx, fmaf(-s3, s.cf[0], A.W[0]));
    A.W[1] = fmaf(Ds5, ry, fmaf(-s3, s.cf[1], A.W[1]));
    A.W[2] = fmaf(Ds5, rz, fmaf(-s3, s.cf[2], A.W[2]));
    if (NEAR && near && r2 > 0.f) {  // the self pair (r = 0) is added per target, in double, after the loop
        const Ovl<float> o = rpy_overlap<float>(rx, ry, rz, r2, Fx, Fy, Fz, Tx, Ty, Tz, a);
        for (int i = 0; i < 3; i++) {
            A.V[i] += o.v[i];
            A.W[i] = fmaf(2.f / 3.f, o.w[i], A.W[i]);
        }
    }
}

// a wave-uniform double as such (both halves through readfirstlane)
__device__ __forceinline__ double uniform_f64(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One work item of the FP32-tile path: as rpy_item_f64, but the lanes of a wave own
// 64 x TPL consecutive targets (lane + 64 j), so that the wave's targets are close together
// and most tiles are far enough from all of them to skip the overlap test.
template <int TPL, int WS, bool SKIP = false>
__device__ __forceinline__ void rpy_item_f32(int64_t base, int64_t S, int64_t Sg, int64_t tb, int k, int K,
                                             int64_t chunk, const SrcF32* __restrict__ pk,
                                             const TileF32* __restrict__ tiles, const double* __restrict__ Y,
                                             double a, double c, const RpyOut& out) {
    static_assert(!SKIP || WS == 1, "waves that share targets cannot skip");
    constexpr int kTgtPerBlock = kRpyBlock / WS;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x % 64);
    int64_t m0 = (int64_t)k * chunk;
    int64_t m1 = min(S, m0 + chunk);
    if (WS > 1) {
        const int64_t sub = ((m1 - m0 + WS - 1) / WS + kF32Tile - 1) / kF32Tile * kF32Tile;
        const int64_t a0 = m0 + wave * sub;
        m1 = min(m1, a0 + sub);
        m0 = min(a0, m1);
    }
    const float af = (float)a, four_a2 = (float)(4.0 * a * a), two_a2 = (float)(2.0 * a * a);
    const float c23 = (float)(2.0 * a * a / 3.0);
    const int64_t t_first = tb * (kTgtPerBlock * TPL) + (WS == 1 ? (int64_t)wave * 64 * TPL : 0);
    if (SKIP && t_first >= S) return;  // no target of this wave inside the suspension
    int64_t n[TPL];
    double y[TPL][3], vd[TPL][3], wd[TPL][3];
    double lo[3], hi[3];
#pragma unroll
    for (int j = 0; j < TPL; j++) {
        n[j] = t_first + j * 64 + lane;
        const int64_t nn = base + (n[j] < S ? n[j] : S - 1);
        for (int i = 0; i < 3; i++) {
            y[j][i] = Y[i * Sg + nn];
            vd[j][i] = wd[j][i] = 0.0;
            lo[i] = j ? fmin(lo[i], y[j][i]) : y[j][i];
            hi[i] = j ? fmax(hi[i], y[j][i]) : y[j][i];
        }
    }
    // bounding box of the wave's targets: centre cw and radius rw, wave-uniform
    for (int off = 32; off >= 1; off >>= 1)
        for (int i = 0; i < 3; i++) {
            lo[i] = fmin(lo[i], __shfl_xor(lo[i], off));
            hi[i] = fmax(hi[i], __shfl_xor(hi[i], off));
        }
    double cw[3], rw2 = 0.0;
    for (int i = 0; i < 3; i++) {
        cw[i] = uniform_f64(0.5 * (lo[i] + hi[i]));
        rw2 = fma(hi[i] - lo[i], hi[i] - lo[i], rw2);
    }
    const double rw = uniform_f64(0.5 * sqrt(rw2));
    for (int64_t t0 = m0; t0 < m1;) {
        const int64_t g = base + t0;
        const int64_t tile = g / kF32Tile;
        const int64_t t1 = min(m1, (tile + 1) * kF32Tile - base);
        const int cnt = (int)(t1 - t0);
        const TileF32 tr = tiles[tile];
        const double dx = cw[0] - tr.o[0], dy = cw[1] - tr.o[1], dz = cw[2] - tr.o[2];
        // |C_w - O| >= reach: every pair of this tile is at least 2a apart (no overlap test)
        const double reach = rw + tr.rad + 2.0 * a;
        const int far = __builtin_amdgcn_readfirstlane((int)(fma(dx, dx, fma(dy, dy, dz * dz)) >= reach * reach));
        AccF32 acc[TPL];
#pragma unroll
        for (int j = 0; j < TPL; j++)
            for (int i = 0; i < 3; i++) acc[j].V[i] = acc[j].R[i] = acc[j].P[i] = acc[j].W[i] = 0.f;
        // r in float from the target's offset to the tile origin (rounded once per tile) and the
        // source's stored offset: its error is a few float ulps of |r| + 2 rad
        float yt[TPL][3];
#pragma unroll
        for (int j = 0; j < TPL; j++)
            for (int i = 0; i < 3; i++) yt[j][i] = (float)(y[j][i] - tr.o[i]);
        // the next record is requested before the current one is used (latency overlap);
        // 32-bit, wave-uniform loop arithmetic stays on the scalar unit
        const SrcF32* ts = pk + g;
        SrcRegF32 cur = load_src_f32(ts);
        auto sweep = [&](auto near) {
            for (int i = 0; i < cnt; ++i) {
                const SrcRegF32 nxt = load_src_f32(ts + (i + 1 < cnt ? i + 1 : i));
#pragma unroll
                for (int j = 0; j < TPL; j++)
                    rpy_pair_f32<decltype(near)::value>(yt[j][0] - cur.sp[0], yt[j][1] - cur.sp[1],
                                                        yt[j][2] - cur.sp[2], cur, af, four_a2, two_a2, acc[j]);
                cur = nxt;
            }
        };
        if (far) sweep(std::false_type{});
        else sweep(std::true_type{});
#pragma unroll
        for (int j = 0; j < TPL; j++) {
            const AccF32& A = acc[j];
            const float* u = yt[j];
            for (int i = 0; i < 3; i++) {
                const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
                const float v = fmaf(A.P[i1], u[i2], fmaf(-A.P[i2], u[i1], fmaf(c23, A.R[i], A.V[i])));
                const float w = fmaf(A.R[i1], u[i2], fmaf(-A.R[i2], u[i1], fmaf(1.5f, A.W[i], -0.5f * A.P[i])));
                vd[j][i] += (double)v;
                wd[j][i] += (double)w;
            }
        }
        t0 = t1;
    }
    // the self pair (r = 0 in the overlap forms): 4/(3a) F and T / a^3, in double
#pragma unroll
    for (int j = 0; j < TPL; j++)
        if (n[j] >= m0 && n[j] < m1) {
            const SrcF32& sr = pk[base + n[j]];
            const double cv = 4.0 / (3.0 * a), cw3 = 1.0 / (a * a * a);
            for (int i = 0; i < 3; i++) {
                vd[j][i] = fma(cv, (double)sr.f[i], vd[j][i]);
                wd[j][i] = fma(cw3, (double)sr.t[i], wd[j][i]);
            }
        }
    double vw[TPL][6];
#pragma unroll
    for (int j = 0; j < TPL; j++)
        for (int i = 0; i < 3; i++) {
            vw[j][i] = c * vd[j][i];
            vw[j][3 + i] = c * wd[j][i];
        }
    rpy_finish<TPL, WS>(out, base, S, Sg, K, k, n, vw);
}

template <int TPL, int WS>
__global__ void __launch_bounds__(kRpyBlock) __attribute__((amdgpu_waves_per_eu(5))) rpy_f32_kernel(int64_t S, int64_t chunk, int K,
                                                          const SrcF32* __restrict__ pk,
                                                          const TileF32* __restrict__ tiles,
                                                          const double* __restrict__ Y, double a, double c,
                                                          RpyOut out) {
    if (out.active && !out.active[0]) return;
    const int k = (int)(blockIdx.x % (unsigned)K);
    const int64_t tb = blockIdx.x / (unsigned)K;
    rpy_item_f32<TPL, WS>(0, S, S, tb, k, K, chunk, pk, tiles, Y, a, c, out);
}

template <int TPL>
__global__ void __launch_bounds__(kRpyBlock) __attribute__((amdgpu_waves_per_eu(5))) rpy_f32_items_kernel(const RpyItem* __restrict__ items, int64_t nitems,
                                                                int64_t Sg, const SrcF32* __restrict__ pk,
                                                                const TileF32* __restrict__ tiles,
                                                                const double* __restrict__ Y, double a, double c,
                                                                RpyOut out, int* __restrict__ next) {
    __shared__ int take;
    for (;;) {
        const int64_t it = next_item(next, take);
        if (it >= nitems) break;
        const RpyItem w = items[it];
        if (out.active && !out.active[w.susp]) continue;
        RpyOut o = out;
        o.part = out.part + w.part;
        rpy_item_f32<TPL, 1, true>(w.base, w.S, Sg, w.tb, w.k, w.K, w.chunk, pk, tiles, Y, a, c, o);
    }
}

// Fixed-order reduction of the K partial results; one thread per (component, target).
__global__ void __launch_bounds__(256) rpy_reduce(int64_t S, int K, const double* __restrict__ part,
                                                 double* __restrict__ V, double* __restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 6 * S) return;
    const int64_t c = e / S, n = e - c * S;
    // four independent partial sums keep several loads in flight; fixed order
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int k = 0;
    for (; k + 4 <= K; k += 4) {
        a0 += part[((int64_t)k * 6 + c) * S + n];
        a1 += part[((int64_t)(k + 1) * 6 + c) * S + n];
        a2 += part[((int64_t)(k + 2) * 6 + c) * S + n];
        a3 += part[((int64_t)(k + 3) * 6 + c) * S + n];
    }
    for (; k < K; k++) a0 += part[((int64_t)k * 6 + c) * S + n];
    const double acc = (a0 + a1) + (a2 + a3);
    if (c < 3) V[c * S + n] = acc;
    else W[(c - 3) * S + n] = acc;
}

// Reduction for the work-list launch: segment s of suspension i = seg_susp[s]
// sums the K_i partials of its suspension (suspensions with K_i = 1 wrote V, W).
__global__ void __launch_bounds__(256) rpy_reduce_items(int64_t Sg, const int32_t* __restrict__ seg_susp,
                                                       const RpySusp* __restrict__ sus, const double* __restrict__ part,
                                                       double* __restrict__ V, double* __restrict__ W,
                                                       const int32_t* __restrict__ active, int* __restrict__ next) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *next = 0;  // the items kernel has finished: clear its counter
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 6 * Sg) return;
    const int64_t c = e / Sg, s = e - c * Sg;
    if (active && !active[seg_susp[s]]) return;
    const RpySusp u = sus[seg_susp[s]];
    if (u.K <= 1) return;
    const int64_t n = s - u.base;
    double acc = 0.0;
    for (int k = 0; k < u.K; k++) acc += part[u.part + ((int64_t)k * 6 + c) * u.S + n];
    if (c < 3) V[c * Sg + s] = acc;
    else W[(c - 3) * Sg + s] = acc;
}

// Launch of a pair kernel; with timing events, through the extended launch that
// stamps them at the kernel's own start and end (not at separate marker packets).
template <class K, class... A>
void launch_pair(K kernel, unsigned grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, A... args) {
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kRpyBlock), 0, st, ev0, ev1, 0, args...);
    else
        kernel<<<grid, kRpyBlock, 0, st>>>(args...);
}

// ------------------------------------------------------------------ launch plan
constexpr int kTplF64 = 2;
constexpr int kTplF32 = 2;
constexpr int64_t kSmallS = 12000;  // below this, one target per lane and short chunks (latency-bound sizes)

RpyPlan rpy_plan(int64_t S, int prec) {
    RpyPlan p{};
    p.S = S;
    p.prec = prec;
    const bool small = S < kSmallS;
    const bool f32 = prec == FIL_PREC_F32TILE;
    p.tpl = small ? 1 : (f32 ? kTplF32 : kTplF64);
    p.ws = small ? 4 : 1;
    if (S <= 0) return p;
    p.tb = ceil_div(S, (int64_t)(kRpyBlock / p.ws) * p.tpl);
    // aim for ~2048 workgroups (8 per CU; FP32 tiles on the large path: ~8192, whose finer
    // grain balances the end of the launch better than the extra partials cost: S = 32000
    // pair kernel 1.11 -> 1.01 ms); every wave gets >= 16 (small), 64 (FP64) or 128 (FP32
    // tiles) sources; and on the small path no wave walks more than 64 sources
    const bool fine = f32 && !small;
    int64_t K = ceil_div(fine ? 8192 : 2048, p.tb);
    K = std::min<int64_t>(K, std::max<int64_t>(1, S / (small ? 16 * p.ws : (fine ? 128 : 64))));
    if (small) K = std::max<int64_t>(K, ceil_div(S, kMaxChunkSmall));
    if (K >= 8) K = ceil_div(K, 8) * 8;
    p.chunk = ceil_div(S, K);
    if (f32) p.chunk = ceil_div(p.chunk, kF32Tile) * kF32Tile;  // chunks start on tile boundaries
    p.K = (int)ceil_div(S, p.chunk);
    p.pack_bytes = (size_t)S * (f32 ? sizeof(SrcF32) : 16 * sizeof(double));
    p.pack_bytes = (p.pack_bytes + 255) & ~(size_t)255;
    p.tile_bytes = f32 ? ((size_t)ceil_div(S, kF32Tile) * sizeof(TileF32) + 255) & ~(size_t)255 : 0;
    p.part_bytes = p.K > 1 ? (size_t)p.K * 6 * S * sizeof(double) : 0;
    return p;
}

int rpy_launch(const RpyPlan& p, const double* Y, const double* F, const double* T, double a, double eta, double* V,
               double* W, void* work, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, bool packed, bool reduce,
               const int32_t* active) {
    if (p.S <= 0) return FIL_OK;
    char* base = static_cast<char*>(work);
    RpyOut out{reinterpret_cast<double*>(base + p.pack_bytes + p.tile_bytes), V, W, active};
    const double c = 1.0 / (8.0 * kPi * eta);
    const unsigned grid = (unsigned)(p.tb * p.K);
    const unsigned pgrid = (unsigned)ceil_div(p.S, 256);
    if (p.prec == FIL_PREC_F64) {
        double* pk = reinterpret_cast<double*>(base);
        if (!packed) rpy_pack_f64<<<pgrid, 256, 0, st>>>(p.S, Y, F, T, pk);
        const double* src = pk;
        if (p.ws == 4) launch_pair(rpy_f64_kernel<1, 4>, grid, st, ev0, ev1, p.S, p.chunk, p.K, src, Y, a, c, out);
        else launch_pair(rpy_f64_kernel<kTplF64, 1>, grid, st, ev0, ev1, p.S, p.chunk, p.K, src, Y, a, c, out);
    } else {
        SrcF32* pk = reinterpret_cast<SrcF32*>(base);
        TileF32* tiles = reinterpret_cast<TileF32*>(base + p.pack_bytes);
        rpy_tile_pack<<<pgrid, 256, 0, st>>>(p.S, Y, F, T, pk, tiles, active);
        const SrcF32* src = pk;
        const TileF32* tl = tiles;
        if (p.ws == 4)
            launch_pair(rpy_f32_kernel<1, 4>, grid, st, ev0, ev1, p.S, p.chunk, p.K, src, tl, Y, a, c, out);
        else launch_pair(rpy_f32_kernel<kTplF32, 1>, grid, st, ev0, ev1, p.S, p.chunk, p.K, src, tl, Y, a, c, out);
    }
    if (p.K > 1 && reduce) rpy_reduce<<<(unsigned)ceil_div(6 * p.S, 256), 256, 0, st>>>(p.S, p.K, out.part, V, W);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// ------------------------------------------------------------------ batched plan
constexpr int kBatchChunk = 256;
constexpr int kPersistentBlocks = 2048;

RpyBatchPlan rpy_batch_plan(int64_t nsusp, const int64_t* susp_off, int prec) {
    RpyBatchPlan p;
    p.prec = prec;
    p.Sg = susp_off[nsusp];
    const bool f32 = prec == FIL_PREC_F32TILE;
    const int tpl = f32 ? kTplF32 : kTplF64;
    int64_t part = 0;
    p.sus.resize(nsusp);
    p.seg_susp.resize(p.Sg);
    for (int64_t i = 0; i < nsusp; i++) {
        const int64_t base = susp_off[i], S = susp_off[i + 1] - base;
        for (int64_t s = base; s < base + S; s++) p.seg_susp[s] = (int32_t)i;
        RpySusp u{base, 0, (int32_t)S, 1};
        if (S > 0) {
            const int64_t tb = ceil_div(S, (int64_t)kRpyBlock * tpl);
            int64_t K = std::max<int64_t>(1, ceil_div(S, kBatchChunk));
            const int64_t chunk = ceil_div(S, K);
            K = ceil_div(S, chunk);
            u.K = (int32_t)K;
            if (K > 1) {
                u.part = part;
                part += K * 6 * S;
                p.any_reduce = true;
            }
            for (int64_t t = 0; t < tb; t++)
                for (int64_t k = 0; k < K; k++) p.items.push_back(RpyItem{base, u.part, (int32_t)S, (int32_t)t,
                                                                          (int32_t)k, (int32_t)K, chunk,
                                                                          (int32_t)i, 0});
        }
        p.sus[i] = u;
    }
    // largest items first: workgroups taking them in order from a shared counter balance
    auto cost = [tpl](const RpyItem& w) {
        const int64_t nt = std::min<int64_t>((int64_t)kRpyBlock * tpl, w.S - (int64_t)w.tb * kRpyBlock * tpl);
        const int64_t ns = std::min<int64_t>(w.chunk, w.S - (int64_t)w.k * w.chunk);
        return nt * ns;
    };
    std::stable_sort(p.items.begin(), p.items.end(),
                     [&](const RpyItem& x, const RpyItem& y) { return cost(x) > cost(y); });
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    p.pack_bytes = al((size_t)p.Sg * (f32 ? sizeof(SrcF32) : 16 * sizeof(double)));
    p.tile_bytes = f32 ? al((size_t)ceil_div(p.Sg, kF32Tile) * sizeof(TileF32)) : 0;
    p.part_bytes = al((size_t)part * sizeof(double));
    p.items_bytes = al(p.items.size() * sizeof(RpyItem));
    p.sus_bytes = al(p.sus.size() * sizeof(RpySusp));
    p.segs_bytes = al(p.seg_susp.size() * sizeof(int32_t));
    return p;
}

int rpy_batch_upload(const RpyBatchPlan& p, void* lists, hipStream_t st) {
    char* base = static_cast<char*>(lists);
    if (!p.items.empty())
        FIL_HIP_TRY(hipMemcpyAsync(base, p.items.data(), p.items.size() * sizeof(RpyItem), hipMemcpyHostToDevice, st));
    base += p.items_bytes;
    if (!p.sus.empty())
        FIL_HIP_TRY(hipMemcpyAsync(base, p.sus.data(), p.sus.size() * sizeof(RpySusp), hipMemcpyHostToDevice, st));
    base += p.sus_bytes;
    if (!p.seg_susp.empty())
        FIL_HIP_TRY(hipMemcpyAsync(base, p.seg_susp.data(), p.seg_susp.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
    return FIL_OK;
}

int rpy_batch_launch(const RpyBatchPlan& p, const void* lists, const double* Y, const double* F, const double* T,
                     double a, double eta, double* V, double* W, void* work, hipStream_t st, hipEvent_t ev0,
                     hipEvent_t ev1, bool packed, const int32_t* active, bool counter_clear) {
    if (p.Sg <= 0) return FIL_OK;
    char* base = static_cast<char*>(work);
    RpyOut out{reinterpret_cast<double*>(base + p.pack_bytes + p.tile_bytes), V, W, active};
    const char* lb = static_cast<const char*>(lists);
    const RpyItem* items = reinterpret_cast<const RpyItem*>(lb);
    const RpySusp* sus = reinterpret_cast<const RpySusp*>(lb + p.items_bytes);
    const int32_t* segs = reinterpret_cast<const int32_t*>(lb + p.items_bytes + p.sus_bytes);
    const double c = 1.0 / (8.0 * kPi * eta);
    const int64_t nitems = (int64_t)p.items.size();
    const unsigned grid = (unsigned)std::min<int64_t>(nitems, kPersistentBlocks);
    const unsigned pgrid = (unsigned)ceil_div(p.Sg, 256);
    int* next = reinterpret_cast<int*>(base + p.pack_bytes + p.tile_bytes + p.part_bytes);
    // the counter starts at zero: cleared here, or (counter_clear, a plan with partials to sum)
    // by the previous apply's sum of the partials
    if (nitems && !(counter_clear && p.any_reduce)) rpy_items_reset<<<1, 32, 0, st>>>(next);
    if (p.prec == FIL_PREC_F64) {
        double* pk = reinterpret_cast<double*>(base);
        if (!packed) rpy_pack_f64<<<pgrid, 256, 0, st>>>(p.Sg, Y, F, T, pk);
        const double* src = pk;
        if (nitems)
            launch_pair(rpy_f64_items_kernel<kTplF64>, grid, st, ev0, ev1, items, nitems, p.Sg, src, Y, a, c, out, next);
    } else {
        SrcF32* pk = reinterpret_cast<SrcF32*>(base);
        TileF32* tiles = reinterpret_cast<TileF32*>(base + p.pack_bytes);
        rpy_tile_pack<<<pgrid, 256, 0, st>>>(p.Sg, Y, F, T, pk, tiles, nullptr);
        const SrcF32* src = pk;
        const TileF32* tl = tiles;
        if (nitems)
            launch_pair(rpy_f32_items_kernel<kTplF32>, grid, st, ev0, ev1, items, nitems, p.Sg, src, tl, Y, a, c, out,
                        next);
    }
    if (!nitems) {  // nothing launched: the timing events still mark this point
        if (ev0) FIL_HIP_TRY(hipEventRecord(ev0, st));
        if (ev1) FIL_HIP_TRY(hipEventRecord(ev1, st));
    }
    if (p.any_reduce)
        rpy_reduce_items<<<(unsigned)ceil_div(6 * p.Sg, 256), 256, 0, st>>>(p.Sg, segs, sus, out.part, V, W, active,
                                                                            next);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // namespace fil
