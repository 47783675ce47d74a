// Learned warm start: a per-filament multilayer perceptron (SiLU hidden layers,
// BF16 weights and activations, FP32 accumulation on the MFMA matrix cores),
// its training (mean-squared error, backpropagation, Adam with FP32 master
// weights) and the feature statistics.  Every product is one "NT" GEMM,
// C[M x N] = A[M x K] B[N x K]^T with both operands K-contiguous BF16, computed
// by v_mfma_f32_16x16x32_bf16 tiles; transposed copies of activations and
// weights are written by the producing kernels so every operand is read with
// 16-byte loads along K.
//
// Layer l maps din[l] -> dout[l] (dims padded to multiples of 32 with zeros):
//   Z_l = A_{l-1} W_l^T + b_l,  A_l = SiLU(Z_l) (hidden),  Y = Z_{L-1} (output)
// Loss: mean over the B valid rows and n_out valid columns of (Y - T)^2.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include <cstdio>
#include <string>
#include "common.h"
#include "mlp.h"

using namespace fil;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 32;  // output tile per wave (2 x 2 MFMA 16x16 blocks), also the K step

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                            // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float silu(float z) { return z / (1.f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.f / (1.f + __expf(-z));
    return s * (1.f + z * (1.f - s));
}

enum Epi { kEpiHidden = 0, kEpiOut = 1, kEpiBackHidden = 2, kEpiStore = 3 };

struct EpiArgs {
    const float* bias;  // [N] (forward)
    float* Z;           // pre-activations [M][N] f32 (hidden forward: written; backward: read)
    uint16_t* Ab;       // bf16 result [M][N]
    uint16_t* AT;       // bf16 result transposed [N][ldT] (may be null)
    int ldT;
    float* C;           // f32 result [M][N] (output layer, weight gradient)
};

// One 64-lane wave per 32 x 32 output tile.  Lane l loads rows (l mod 16) of
// the two 16-row A and B blocks, 8 consecutive K elements (16 B) at K offset
// 8 (l / 16); the accumulator of block (a, b) holds C[16a + 4 (l/16) + r][16b + l mod 16].
template <int EPI>
__global__ void __launch_bounds__(64) gemm_nt_kernel(int M, int N, int K, const uint16_t* __restrict__ A, int lda,
                                                     const uint16_t* __restrict__ B, int ldb, EpiArgs e) {
    const int lane = threadIdx.x;
    const int m0 = blockIdx.x * kTile, n0 = blockIdx.y * kTile;
    const int li = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint4 zero = make_uint4(0, 0, 0, 0);
    for (int k0 = 0; k0 < K; k0 += kTile) {
        uint4 af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; a++) {
            const int r = m0 + 16 * a + li;
            af[a] = r < M ? *reinterpret_cast<const uint4*>(A + (int64_t)r * lda + k0 + kq) : zero;
        }
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int c = n0 + 16 * b + li;
            bfr[b] = c < N ? *reinterpret_cast<const uint4*>(B + (int64_t)c * ldb + k0 + kq) : zero;
        }
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[a]),
                                                                    __builtin_bit_cast(bf16x8, bfr[b]), acc[a][b],
                                                                    0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const int n = n0 + 16 * b + li;
            if (n >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + 16 * a + 4 * (lane >> 4) + r;
                if (m >= M) continue;
                const int64_t o = (int64_t)m * N + n;
                float v = acc[a][b][r];
                if (EPI == kEpiHidden) {
                    v += e.bias[n];
                    e.Z[o] = v;
                    const uint16_t h = to_bf16(silu(v));
                    e.Ab[o] = h;
                    if (e.AT) e.AT[(int64_t)n * e.ldT + m] = h;
                } else if (EPI == kEpiOut) {
                    e.C[o] = v + e.bias[n];
                } else if (EPI == kEpiBackHidden) {
                    const uint16_t h = to_bf16(v * dsilu(e.Z[o]));
                    e.Ab[o] = h;
                    e.AT[(int64_t)n * e.ldT + m] = h;
                } else {
                    e.C[o] = v;
                }
            }
        }
}

template <int EPI>
int gemm(int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb, const EpiArgs& e,
         hipStream_t st) {
    if (M == 0 || N == 0) return FIL_OK;
    dim3 grid((unsigned)ceil_div(M, kTile), (unsigned)ceil_div(N, kTile));
    gemm_nt_kernel<EPI><<<grid, 64, 0, st>>>(M, N, K, A, lda, B, ldb, e);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

// Minibatch assembly: rows[r] (r < B) of the standardised sample arrays, zero
// rows up to Bp; X is also written transposed (for the first layer's gradient).
__global__ void __launch_bounds__(256) gather_kernel(int B, int Bp, int nin, int nout, const int32_t* __restrict__ rows,
                                                     const uint16_t* __restrict__ Xall,
                                                     const float* __restrict__ Tall, uint16_t* __restrict__ X,
                                                     uint16_t* __restrict__ XT, float* __restrict__ T) {
    const int r = blockIdx.x;
    const int64_t src = r < B ? (rows ? (int64_t)rows[r] : (int64_t)r) : -1;
    for (int c = threadIdx.x; c < nin; c += blockDim.x) {
        const uint16_t h = src >= 0 ? Xall[src * nin + c] : (uint16_t)0;
        X[(int64_t)r * nin + c] = h;
        XT[(int64_t)c * Bp + r] = h;
    }
    for (int c = threadIdx.x; c < nout; c += blockDim.x) T[(int64_t)r * nout + c] = src >= 0 ? Tall[src * nout + c] : 0.f;
}

// dY = 2 (Y - T) / (B n_out) on the valid block (zero elsewhere), in both layouts, and
// the squared errors summed per workgroup (rows blockIdx.x, blockIdx.x + kLossBlocks, ...)
// by a fixed-order block reduction; loss_sum_kernel adds the workgroups' sums in order.
constexpr int kLossBlocks = 64;
__global__ void __launch_bounds__(256) loss_kernel(int B, int Bp, int nout, int nout_pad, const float* __restrict__ Y,
                                                   const float* __restrict__ T, uint16_t* __restrict__ dY,
                                                   uint16_t* __restrict__ dYT, double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    const float scale = 2.f / ((float)B * (float)nout);
    for (int r = blockIdx.x; r < Bp; r += gridDim.x)
        for (int c = threadIdx.x; c < nout_pad; c += blockDim.x) {
            const int64_t e = (int64_t)r * nout_pad + c;
            float g = 0.f;
            if (r < B && c < nout) {
                const float d = Y[e] - T[e];
                acc += (double)d * d;
                g = scale * d;
            }
            const uint16_t h = to_bf16(g);
            dY[e] = h;
            dYT[(int64_t)c * Bp + r] = h;
        }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(64) loss_sum_kernel(int n, const double* __restrict__ part, double inv,
                                                      double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; i++) s += part[i];
    *loss = s * inv;
}

// db[n] = sum over the batch of dZ[b][n], from the transposed BF16 copy; one wave per n.
__global__ void __launch_bounds__(64) colsum_kernel(int N, int Bp, const uint16_t* __restrict__ dZT,
                                                    float* __restrict__ db) {
    const int n = blockIdx.x;
    float s = 0.f;
    for (int b = threadIdx.x; b < Bp; b += 64) s += from_bf16(dZT[(int64_t)n * Bp + b]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) db[n] = s;
}

// Adam (Kingma & Ba) on one layer's FP32 master parameters [W (out x in), b (out)];
// refreshes the BF16 weights and their transpose.
__global__ void __launch_bounds__(256) adam_kernel(int64_t count, int out, int in, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2, const float* __restrict__ g,
                                                   float* __restrict__ p, float* __restrict__ m,
                                                   float* __restrict__ v, uint16_t* __restrict__ Wb,
                                                   uint16_t* __restrict__ WT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    if (i < (int64_t)out * in) {
        const uint16_t h = to_bf16(pi);
        Wb[i] = h;
        WT[(i % in) * out + i / in] = h;
    }
}

// BF16 copies of a layer's weights from the master parameters
__global__ void __launch_bounds__(256) cast_weights_kernel(int out, int in, const float* __restrict__ p,
                                                           uint16_t* __restrict__ Wb, uint16_t* __restrict__ WT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)out * in) return;
    const uint16_t h = to_bf16(p[i]);
    Wb[i] = h;
    WT[(i % in) * out + i / in] = h;
}

// column mean and standard deviation (population) of a [n][ncol] array, one block per column;
// a (near-)constant column gets sd = 1
__global__ void __launch_bounds__(256) colstats_kernel(int64_t n, int ncol, const float* __restrict__ x,
                                                       float* __restrict__ mu, float* __restrict__ sd) {
    __shared__ double s1[256], s2[256];
    const int c = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double v = x[r * ncol + c];
        a += v;
        b += v * v;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = s1[0] / (double)n;
        const double var = fmax(0.0, s2[0] / (double)n - mean * mean);
        const double s = sqrt(var);
        mu[c] = (float)mean;
        sd[c] = (float)(s > 1e-12 * fmax(1.0, fabs(mean)) ? s : 1.0);
    }
}

// xb = bf16((feat - mu) / sd) (zero in the padding columns), t = (targ - mu) / sd
__global__ void __launch_bounds__(256) standardize_kernel(int64_t n, int nin, int nin_pad, int nout, int nout_pad,
                                                          const float* __restrict__ feat,
                                                          const float* __restrict__ targ,
                                                          const float* __restrict__ norm, uint16_t* __restrict__ xb,
                                                          float* __restrict__ t) {
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    const float* mu_in = norm;
    const float* sd_in = norm + nin_pad;
    const float* mu_out = norm + 2 * nin_pad;
    const float* sd_out = mu_out + nout_pad;
    if (feat && xb)
        for (int c = threadIdx.x; c < nin_pad; c += blockDim.x)
            xb[r * nin_pad + c] = c < nin ? to_bf16((feat[r * nin + c] - mu_in[c]) / sd_in[c]) : (uint16_t)0;
    if (targ && t)
        for (int c = threadIdx.x; c < nout_pad; c += blockDim.x)
            t[r * nout_pad + c] = c < nout ? (targ[r * nout + c] - mu_out[c]) / sd_out[c] : 0.f;
}

template <class T>
int dalloc(fil_mlp* m, T** p, size_t n);

}  // namespace

struct fil_mlp {
    int N = 0, n_in = 0, n_in_pad = 0, n_out = 0, n_out_pad = 0, width = 0, depth = 0, L = 0, Bmax = 0, Bp = 0;
    std::vector<int> din, dout;
    std::vector<int64_t> poff;  // flat parameter offset of layer l (W, then b)
    int64_t nparams = 0;
    float *P = nullptr, *Mo = nullptr, *Ve = nullptr, *G = nullptr, *norm = nullptr;
    std::vector<uint16_t*> Wb, WT;
    uint16_t *X = nullptr, *XT = nullptr;
    std::vector<float*> Z;
    std::vector<uint16_t*> A, AT;
    float *Y = nullptr, *T = nullptr;
    uint16_t *dZ[2] = {nullptr, nullptr}, *dZT[2] = {nullptr, nullptr};
    double* loss = nullptr;
    double* lpart = nullptr;  // per-workgroup squared-error sums of the loss kernel
    int64_t adam_t = 0;
    bool has_grad = false;
    std::vector<void*> allocs;
};

namespace {
template <class T>
int dalloc(fil_mlp* m, T** p, size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        set_error("fil_mlp_create: device allocation failed");
        return FIL_ENOMEM;
    }
    m->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return FIL_OK;
}

void free_mlp(fil_mlp* m) {
    if (!m) return;
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
}

int round32(int x) { return (x + 31) / 32 * 32; }

// forward pass over Bp rows of m->X; when `train`, activations are also stored transposed
int forward(fil_mlp* m, int rows, const uint16_t* X, float* Y, bool train, hipStream_t st) {
    const uint16_t* a = X;
    for (int l = 0; l < m->L; l++) {
        EpiArgs e{};
        e.bias = m->P + m->poff[l] + (int64_t)m->dout[l] * m->din[l];
        if (l + 1 < m->L) {
            e.Z = m->Z[l];
            e.Ab = m->A[l];
            e.AT = train ? m->AT[l] : nullptr;
            e.ldT = m->Bp;
            int rc = gemm<kEpiHidden>(rows, m->dout[l], m->din[l], a, m->din[l], m->Wb[l], m->din[l], e, st);
            if (rc) return rc;
            a = m->A[l];
        } else {
            e.C = Y;
            int rc = gemm<kEpiOut>(rows, m->dout[l], m->din[l], a, m->din[l], m->Wb[l], m->din[l], e, st);
            if (rc) return rc;
        }
    }
    return FIL_OK;
}

// loss and gradient of the minibatch in m->X / m->T (B valid rows of Bp) into m->G
int backward(fil_mlp* m, int B, double* loss, hipStream_t st) {
    const int Bp = m->Bp;
    int rc = forward(m, Bp, m->X, m->Y, true, st);
    if (rc) return rc;
    loss_kernel<<<kLossBlocks, 256, 0, st>>>(B, Bp, m->n_out, m->n_out_pad, m->Y, m->T, m->dZ[0], m->dZT[0],
                                             m->lpart);
    if (loss) loss_sum_kernel<<<1, 64, 0, st>>>(kLossBlocks, m->lpart, 1.0 / ((double)B * m->n_out), loss);
    FIL_HIP_TRY(hipGetLastError());
    int cur = 0;
    for (int l = m->L - 1; l >= 0; l--) {
        const uint16_t* inT = l == 0 ? m->XT : m->AT[l - 1];
        float* gW = m->G + m->poff[l];
        float* gb = gW + (int64_t)m->dout[l] * m->din[l];
        EpiArgs e{};
        e.C = gW;
        if ((rc = gemm<kEpiStore>(m->dout[l], m->din[l], Bp, m->dZT[cur], Bp, inT, Bp, e, st))) return rc;
        colsum_kernel<<<m->dout[l], 64, 0, st>>>(m->dout[l], Bp, m->dZT[cur], gb);
        FIL_HIP_TRY(hipGetLastError());
        if (l == 0) break;
        EpiArgs d{};
        d.Z = m->Z[l - 1];
        d.Ab = m->dZ[1 - cur];
        d.AT = m->dZT[1 - cur];
        d.ldT = Bp;
        if ((rc = gemm<kEpiBackHidden>(Bp, m->din[l], m->dout[l], m->dZ[cur], m->dout[l], m->WT[l], m->dout[l], d,
                                       st)))
            return rc;
        cur = 1 - cur;
    }
    m->has_grad = true;
    return FIL_OK;
}

int adam(fil_mlp* m, float lr, hipStream_t st) {
    m->adam_t++;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->adam_t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->adam_t));
    for (int l = 0; l < m->L; l++) {
        const int64_t cnt = (int64_t)m->dout[l] * m->din[l] + m->dout[l];
        const int64_t o = m->poff[l];
        adam_kernel<<<(unsigned)ceil_div(cnt, 256), 256, 0, st>>>(cnt, m->dout[l], m->din[l], lr, b1, b2, eps, bc1,
                                                                  bc2, m->G + o, m->P + o, m->Mo + o, m->Ve + o,
                                                                  m->Wb[l], m->WT[l]);
        FIL_HIP_TRY(hipGetLastError());
    }
    return FIL_OK;
}

int gather(fil_mlp* m, int B, const int32_t* rows, const uint16_t* Xall, const float* Tall, hipStream_t st) {
    gather_kernel<<<m->Bp, 256, 0, st>>>(B, m->Bp, m->n_in_pad, m->n_out_pad, rows, Xall, Tall, m->X, m->XT, m->T);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

}  // namespace

namespace fil {
int mlp_forward_rows(fil_mlp* m, int rows, const uint16_t* X, float* Y, hipStream_t st) {
    return forward(m, rows, X, Y, false, st);
}
int mlp_standardize(fil_mlp* m, int64_t n, const float* feat, const float* targ, uint16_t* xb, float* t,
                    hipStream_t st) {
    if (n == 0) return FIL_OK;
    standardize_kernel<<<(unsigned)n, 256, 0, st>>>(n, m->n_in, m->n_in_pad, m->n_out, m->n_out_pad, feat, targ,
                                                    m->norm, xb, t);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}
const float* mlp_norm(const fil_mlp* m) { return m->norm; }
int mlp_segments(const fil_mlp* m) { return m->N; }
int mlp_in_pad(const fil_mlp* m) { return m->n_in_pad; }
int mlp_out_pad(const fil_mlp* m) { return m->n_out_pad; }
int mlp_max_batch(const fil_mlp* m) { return m->Bmax; }
}  // namespace fil

extern "C" {

int fil_mlp_create(int32_t n_seg, int32_t width, int32_t depth, int32_t max_batch, uint64_t seed, fil_mlp** out) {
    FIL_CHECK_ARG(out, "fil_mlp_create: out is null");
    *out = nullptr;
    FIL_CHECK_ARG(n_seg >= 2 && n_seg <= 64, "fil_mlp_create: n_seg must be in [2, 64]");
    FIL_CHECK_ARG(width >= 32 && width % 32 == 0 && width <= 4096, "fil_mlp_create: width must be a multiple of 32");
    FIL_CHECK_ARG(depth >= 1 && depth <= 16, "fil_mlp_create: depth must be in [1, 16]");
    FIL_CHECK_ARG(max_batch >= 1 && max_batch <= (1 << 20), "fil_mlp_create: max_batch must be in [1, 2^20]");
    fil_mlp* m = new fil_mlp();
    m->N = n_seg;
    m->n_in = kMlpFeatPerSeg * n_seg;
    m->n_out = 6 * n_seg;
    m->n_in_pad = round32(m->n_in);
    m->n_out_pad = round32(m->n_out);
    m->width = width;
    m->depth = depth;
    m->L = depth + 1;
    m->Bmax = max_batch;
    m->Bp = round32(max_batch);
    for (int l = 0; l < m->L; l++) {
        m->din.push_back(l == 0 ? m->n_in_pad : width);
        m->dout.push_back(l + 1 < m->L ? width : m->n_out_pad);
        m->poff.push_back(m->nparams);
        m->nparams += (int64_t)m->dout[l] * m->din[l] + m->dout[l];
    }
    int rc = FIL_OK;
    const size_t Bp = m->Bp;
#define A(ptr, n) \
    if (rc == FIL_OK) rc = dalloc(m, &(ptr), (n));
    A(m->P, m->nparams) A(m->Mo, m->nparams) A(m->Ve, m->nparams) A(m->G, m->nparams)
    A(m->norm, 2 * (size_t)(m->n_in_pad + m->n_out_pad)) A(m->X, Bp * m->n_in_pad) A(m->XT, Bp * m->n_in_pad)
    A(m->Y, Bp * m->n_out_pad) A(m->T, Bp * m->n_out_pad) A(m->loss, 1) A(m->lpart, kLossBlocks)
    const size_t wmax = std::max(width, m->n_out_pad);
    for (int i = 0; i < 2; i++) { A(m->dZ[i], Bp * wmax) A(m->dZT[i], Bp * wmax) }
    m->Wb.resize(m->L);
    m->WT.resize(m->L);
    for (int l = 0; l < m->L; l++) {
        A(m->Wb[l], (size_t)m->dout[l] * m->din[l]) A(m->WT[l], (size_t)m->dout[l] * m->din[l])
    }
    m->Z.resize(depth);
    m->A.resize(depth);
    m->AT.resize(depth);
    for (int l = 0; l < depth; l++) { A(m->Z[l], Bp * width) A(m->A[l], Bp * width) A(m->AT[l], Bp * width) }
#undef A
    if (rc) {
        free_mlp(m);
        return rc;
    }
    // He-style uniform initialisation (seeded, host), zero biases, unit normalisation
    std::vector<float> P(m->nparams, 0.f);
    uint64_t state = seed * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
    auto next = [&]() {  // splitmix64
        uint64_t z = (state += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int l = 0; l < m->L; l++) {
        const int fan_in = l == 0 ? m->n_in : width;
        const double lim = std::sqrt(6.0 / fan_in) * (l + 1 < m->L ? 1.0 : 0.1);
        const int rows = l + 1 < m->L ? m->dout[l] : m->n_out;
        for (int o = 0; o < rows; o++)
            for (int i = 0; i < fan_in; i++) {
                const double u = (double)(next() >> 11) * (1.0 / 9007199254740992.0);
                P[m->poff[l] + (int64_t)o * m->din[l] + i] = (float)((2.0 * u - 1.0) * lim);
            }
    }
    std::vector<float> nrm(2 * (size_t)(m->n_in_pad + m->n_out_pad), 0.f);
    std::fill(nrm.begin() + m->n_in_pad, nrm.begin() + 2 * m->n_in_pad, 1.f);
    std::fill(nrm.begin() + 2 * m->n_in_pad + m->n_out_pad, nrm.end(), 1.f);
    auto up = [&]() -> int {
        FIL_HIP_TRY(hipMemcpy(m->norm, nrm.data(), nrm.size() * sizeof(float), hipMemcpyHostToDevice));
        FIL_HIP_TRY(hipMemset(m->Mo, 0, m->nparams * sizeof(float)));
        FIL_HIP_TRY(hipMemset(m->Ve, 0, m->nparams * sizeof(float)));
        FIL_HIP_TRY(hipMemset(m->G, 0, m->nparams * sizeof(float)));
        FIL_HIP_TRY(hipMemset(m->X, 0, Bp * m->n_in_pad * sizeof(uint16_t)));
        FIL_HIP_TRY(hipMemset(m->XT, 0, Bp * m->n_in_pad * sizeof(uint16_t)));
        return FIL_OK;
    };
    if ((rc = up()) || (rc = fil_mlp_set_params(m, P.data()))) {
        free_mlp(m);
        return rc;
    }
    *out = m;
    return FIL_OK;
}

void fil_mlp_destroy(fil_mlp* m) {
    if (m) (void)hipDeviceSynchronize();
    free_mlp(m);
}

int fil_mlp_dims(const fil_mlp* m, int32_t* dims, int64_t* n_params) {
    FIL_CHECK_ARG(m, "fil_mlp_dims: null mlp");
    if (dims) {
        dims[0] = m->n_in;
        dims[1] = m->n_in_pad;
        dims[2] = m->n_out;
        dims[3] = m->n_out_pad;
        dims[4] = m->width;
        dims[5] = m->depth;
        dims[6] = m->Bmax;
        dims[7] = m->N;
    }
    if (n_params) *n_params = m->nparams;
    return FIL_OK;
}

int fil_mlp_set_params(fil_mlp* m, const float* P) {
    FIL_CHECK_ARG(m && P, "fil_mlp_set_params: null argument");
    for (int64_t i = 0; i < m->nparams; i++) FIL_CHECK_ARG(std::isfinite(P[i]), "fil_mlp_set_params: non-finite");
    FIL_HIP_TRY(hipDeviceSynchronize());
    FIL_HIP_TRY(hipMemcpy(m->P, P, m->nparams * sizeof(float), hipMemcpyHostToDevice));
    FIL_HIP_TRY(hipMemset(m->Mo, 0, m->nparams * sizeof(float)));
    FIL_HIP_TRY(hipMemset(m->Ve, 0, m->nparams * sizeof(float)));
    m->adam_t = 0;
    for (int l = 0; l < m->L; l++) {
        const int64_t cnt = (int64_t)m->dout[l] * m->din[l];
        cast_weights_kernel<<<(unsigned)ceil_div(cnt, 256), 256>>>(m->dout[l], m->din[l], m->P + m->poff[l], m->Wb[l],
                                                                   m->WT[l]);
        FIL_HIP_TRY(hipGetLastError());
    }
    FIL_HIP_TRY(hipDeviceSynchronize());
    return FIL_OK;
}

int fil_mlp_get_params(const fil_mlp* m, float* P) {
    FIL_CHECK_ARG(m && P, "fil_mlp_get_params: null argument");
    FIL_HIP_TRY(hipDeviceSynchronize());
    FIL_HIP_TRY(hipMemcpy(P, m->P, m->nparams * sizeof(float), hipMemcpyDeviceToHost));
    return FIL_OK;
}

int fil_mlp_set_norm(fil_mlp* m, const float* norm) {
    FIL_CHECK_ARG(m && norm, "fil_mlp_set_norm: null argument");
    const size_t n = 2 * (size_t)(m->n_in_pad + m->n_out_pad);
    for (size_t i = 0; i < n; i++) FIL_CHECK_ARG(std::isfinite(norm[i]), "fil_mlp_set_norm: non-finite value");
    for (int c = 0; c < m->n_in_pad; c++) FIL_CHECK_ARG(norm[m->n_in_pad + c] > 0, "fil_mlp_set_norm: sd must be > 0");
    for (int c = 0; c < m->n_out_pad; c++)
        FIL_CHECK_ARG(norm[2 * m->n_in_pad + m->n_out_pad + c] > 0, "fil_mlp_set_norm: sd must be > 0");
    FIL_HIP_TRY(hipDeviceSynchronize());
    FIL_HIP_TRY(hipMemcpy(m->norm, norm, n * sizeof(float), hipMemcpyHostToDevice));
    return FIL_OK;
}

int fil_mlp_get_norm(const fil_mlp* m, float* norm) {
    FIL_CHECK_ARG(m && norm, "fil_mlp_get_norm: null argument");
    FIL_HIP_TRY(hipDeviceSynchronize());
    FIL_HIP_TRY(hipMemcpy(norm, m->norm, 2 * (size_t)(m->n_in_pad + m->n_out_pad) * sizeof(float),
                          hipMemcpyDeviceToHost));
    return FIL_OK;
}

int fil_mlp_fit_norm(fil_mlp* m, int64_t n, const float* feat, const float* targ, void* stream) {
    FIL_CHECK_ARG(m && feat && targ && n >= 2, "fil_mlp_fit_norm: null argument or fewer than 2 samples");
    hipStream_t st = (hipStream_t)stream;
    float* nrm = m->norm;
    // padding columns keep mu = 0, sd = 1
    colstats_kernel<<<m->n_in, 256, 0, st>>>(n, m->n_in, feat, nrm, nrm + m->n_in_pad);
    FIL_HIP_TRY(hipGetLastError());
    colstats_kernel<<<m->n_out, 256, 0, st>>>(n, m->n_out, targ, nrm + 2 * m->n_in_pad,
                                              nrm + 2 * m->n_in_pad + m->n_out_pad);
    FIL_HIP_TRY(hipGetLastError());
    return FIL_OK;
}

int fil_mlp_standardize(fil_mlp* m, int64_t n, const float* feat, const float* targ, uint16_t* xb, float* t,
                        void* stream) {
    FIL_CHECK_ARG(m && n >= 0, "fil_mlp_standardize: bad argument");
    FIL_CHECK_ARG((feat != nullptr) == (xb != nullptr) && (targ != nullptr) == (t != nullptr),
                  "fil_mlp_standardize: inputs and outputs must be given in pairs");
    return mlp_standardize(m, n, feat, targ, xb, t, (hipStream_t)stream);
}

int fil_mlp_forward(fil_mlp* m, int32_t B, const uint16_t* X, float* Y, void* stream) {
    FIL_CHECK_ARG(m && X && Y, "fil_mlp_forward: null argument");
    FIL_CHECK_ARG(B >= 0 && B <= m->Bmax, "fil_mlp_forward: batch exceeds max_batch");
    return forward(m, B, X, Y, false, (hipStream_t)stream);
}

int fil_mlp_backward(fil_mlp* m, int32_t B, const int32_t* rows, const uint16_t* X, const float* T, float* grad_out,
                     double* loss, void* stream) {
    FIL_CHECK_ARG(m && X && T, "fil_mlp_backward: null argument");
    FIL_CHECK_ARG(B >= 1 && B <= m->Bmax, "fil_mlp_backward: batch must be in [1, max_batch]");
    hipStream_t st = (hipStream_t)stream;
    int rc = gather(m, B, rows, X, T, st);
    if (rc) return rc;
    if ((rc = backward(m, B, loss ? loss : m->loss, st))) return rc;
    if (grad_out)
        FIL_HIP_TRY(hipMemcpyAsync(grad_out, m->G, m->nparams * sizeof(float), hipMemcpyDeviceToDevice, st));
    return FIL_OK;
}

int fil_mlp_adam_step(fil_mlp* m, float lr, void* stream) {
    FIL_CHECK_ARG(m, "fil_mlp_adam_step: null mlp");
    FIL_CHECK_ARG(m->has_grad, "fil_mlp_adam_step: no gradient (call fil_mlp_backward first)");
    FIL_CHECK_ARG(std::isfinite(lr) && lr >= 0, "fil_mlp_adam_step: lr must be finite and >= 0");
    return adam(m, lr, (hipStream_t)stream);
}

int fil_mlp_train_step(fil_mlp* m, int32_t B, const int32_t* rows, const uint16_t* X, const float* T, float lr,
                       double* loss, void* stream) {
    int rc = fil_mlp_backward(m, B, rows, X, T, nullptr, loss, stream);
    if (rc) return rc;
    return fil_mlp_adam_step(m, lr, stream);
}

// File layout (native byte order): "FILMLP01", int32 dims[8] as fil_mlp_dims,
// int64 number of parameters, int64 number of normalisation values, then the FP32
// master parameters and the normalisation (mu, sd of inputs, then of outputs).
static const char kMlpMagic[8] = {'F', 'I', 'L', 'M', 'L', 'P', '0', '1'};

int fil_mlp_save(const fil_mlp* m, const char* path) {
    FIL_CHECK_ARG(m && path, "fil_mlp_save: null argument");
    int32_t dims[8];
    int64_t np = 0;
    if (int rc = fil_mlp_dims(m, dims, &np)) return rc;
    const int64_t nn = 2 * (int64_t)(m->n_in_pad + m->n_out_pad);
    std::vector<float> P(np), nrm(nn);
    if (int rc = fil_mlp_get_params(m, P.data())) return rc;
    if (int rc = fil_mlp_get_norm(m, nrm.data())) return rc;
    FILE* fp = fopen(path, "wb");
    FIL_CHECK_ARG(fp, std::string("fil_mlp_save: cannot open ") + path);
    bool ok = fwrite(kMlpMagic, 1, 8, fp) == 8 && fwrite(dims, sizeof(int32_t), 8, fp) == 8 &&
              fwrite(&np, sizeof(int64_t), 1, fp) == 1 && fwrite(&nn, sizeof(int64_t), 1, fp) == 1 &&
              fwrite(P.data(), sizeof(float), P.size(), fp) == P.size() &&
              fwrite(nrm.data(), sizeof(float), nrm.size(), fp) == nrm.size();
    ok = (fclose(fp) == 0) && ok;
    FIL_CHECK_ARG(ok, std::string("fil_mlp_save: write to ") + path + " failed");
    return FIL_OK;
}

int fil_mlp_load(fil_mlp* m, const char* path) {
    FIL_CHECK_ARG(m && path, "fil_mlp_load: null argument");
    int32_t want[8];
    int64_t np_want = 0;
    if (int rc = fil_mlp_dims(m, want, &np_want)) return rc;
    FILE* fp = fopen(path, "rb");
    FIL_CHECK_ARG(fp, std::string("fil_mlp_load: cannot open ") + path);
    char magic[8];
    int32_t dims[8];
    int64_t np = 0, nn = 0;
    bool ok = fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
              fread(dims, sizeof(int32_t), 8, fp) == 8 && fread(&np, sizeof(int64_t), 1, fp) == 1 &&
              fread(&nn, sizeof(int64_t), 1, fp) == 1;
    // the architecture must match (the batch capacity, dims[6], may differ)
    const bool same = ok && dims[0] == want[0] && dims[1] == want[1] && dims[2] == want[2] && dims[3] == want[3] &&
                      dims[4] == want[4] && dims[5] == want[5] && dims[7] == want[7] && np == np_want &&
                      nn == 2 * (int64_t)(m->n_in_pad + m->n_out_pad);
    std::vector<float> P(same ? np : 0), nrm(same ? nn : 0);
    if (same)
        ok = fread(P.data(), sizeof(float), P.size(), fp) == P.size() &&
             fread(nrm.data(), sizeof(float), nrm.size(), fp) == nrm.size();
    fclose(fp);
    FIL_CHECK_ARG(ok, std::string("fil_mlp_load: ") + path + " is not a complete network file");
    FIL_CHECK_ARG(same, "fil_mlp_load: network of a different architecture");
    if (int rc = fil_mlp_set_params(m, P.data())) return rc;
    return fil_mlp_set_norm(m, nrm.data());
}

}  // extern "C"
