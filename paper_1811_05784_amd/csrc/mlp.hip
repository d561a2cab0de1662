// Late-tail surrogate: a ReLU multilayer perceptron with BF16 weights and
// activations, FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16), FP32 master weights updated by Adam, and the
// feature / target transforms between the image-source histograms and the
// network.  Not part of the paper: it extends the paper's remark that late
// image sources are reached by few rays (section "Discrete model") by
// predicting the decay of the full trace from the first reflection orders.
//
// Parameter layout (theta, theta_bf16, gradients, Adam moments): layer after
// layer, W_l [w_{l+1}, w_l] row-major followed by b_l [w_{l+1}].
#include "common.h"

#include <cmath>

namespace rtac {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxLayers = 8;
constexpr int kMaxWidth = 4096;
constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdsK = kBK + 8;   // row stride in LDS (bf16), 80 B: spreads the 16-B fragment reads over banks
constexpr int kGemmThreads = 256;

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even (finite inputs)
__device__ inline uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

enum Layout { kRowK = 0, kRowMN = 1 };   // operand stored [rows][K] or [K][rows]

enum Epi {
    kEpiBiasRelu = 0,   // bf16 out = relu(acc + bias)
    kEpiBias = 1,       // f32 out = acc + bias
    kEpiMask = 2,       // bf16 out = acc * (mask_act > 0)
    kEpiStore = 3,      // f32 out = acc
};

struct GemmArgs {
    const uint16_t* A;   // logical [M, K]
    const uint16_t* B;   // logical [N, K] (the product is A B^T)
    int64_t lda, ldb;    // row stride of the stored array
    int64_t M, N, K;
    const float* bias;          // [N] (f32 master bias) for the bias epilogues
    const uint16_t* bias_bf16;  // [N] bf16 bias (used when bias == nullptr)
    const uint16_t* mask_act;   // [M, N] bf16 activation whose sign masks (kEpiMask)
    void* out;                  // [M, N]
    int64_t ldo;
};

// Stage a 64 x 32 tile of a logical [rows, K] operand into LDS as [row][k].
template <int kLayout>
__device__ inline void load_tile(uint16_t (*dst)[kLdsK], const uint16_t* src, int64_t ld, int64_t rows, int64_t K,
                                 int64_t r0, int64_t k0, int t) {
    if (kLayout == kRowK) {
        // memory [rows][K], K contiguous: thread t loads row t/4, 8 k from (t%4)*8
        const int r = t >> 2, kc = (t & 3) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (r0 + r < rows && k0 + kc < K) v = *reinterpret_cast<const uint4*>(src + (r0 + r) * ld + k0 + kc);
        *reinterpret_cast<uint4*>(&dst[r][kc]) = v;
    } else {
        // memory [K][rows], rows contiguous: thread t loads k t/8, 8 rows from (t%8)*8
        const int k = t >> 3, rc = (t & 7) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (k0 + k < K && r0 + rc < rows) v = *reinterpret_cast<const uint4*>(src + (k0 + k) * ld + r0 + rc);
        const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
        for (int i = 0; i < 8; i++) dst[rc + i][k] = e[i];
    }
}

// C[M, N] = A[M, K] B[N, K]^T with a fused epilogue.  256 threads = 4
// wavefronts in a 2 x 2 grid; each wavefront owns a 32 x 32 block of 2 x 2
// MFMA 16 x 16 tiles.  Fragment layout of v_mfma_f32_16x16x32_bf16: lane l
// supplies row (l % 16) of A and column (l % 16) of B^T at k = 8 (l / 16) ..
// + 7, and receives C rows 4 (l / 16) .. + 3 of column l % 16.
template <int kLA, int kLB, int kEpi>
__global__ __launch_bounds__(kGemmThreads) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kLdsK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kLdsK];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int64_t m0 = (int64_t)blockIdx.y * kBM, n0 = (int64_t)blockIdx.x * kBN;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    for (int64_t k0 = 0; k0 < g.K; k0 += kBK) {
        load_tile<kLA>(As, g.A, g.lda, g.M, g.K, m0, k0, t);
        load_tile<kLB>(Bs, g.B, g.ldb, g.N, g.K, n0, k0, t);
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; i++) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + i * 16 + fr][fk]);
#pragma unroll
        for (int j = 0; j < 2; j++) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + j * 16 + fr][fk]);
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // epilogue
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int64_t n = n0 + wn * 32 + j * 16 + fr;
            if (n >= g.N) continue;
            float bias = 0.f;
            if (kEpi == kEpiBiasRelu || kEpi == kEpiBias)
                bias = g.bias ? g.bias[n] : bf16_to_f32(g.bias_bf16[n]);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
                if (m >= g.M) continue;
                float v = acc[i][j][r];
                if (kEpi == kEpiBiasRelu) {
                    v = fmaxf(v + bias, 0.f);
                    reinterpret_cast<uint16_t*>(g.out)[m * g.ldo + n] = f32_to_bf16(v);
                } else if (kEpi == kEpiBias) {
                    reinterpret_cast<float*>(g.out)[m * g.ldo + n] = v + bias;
                } else if (kEpi == kEpiMask) {
                    const bool on = bf16_to_f32(g.mask_act[m * g.ldo + n]) > 0.f;
                    reinterpret_cast<uint16_t*>(g.out)[m * g.ldo + n] = f32_to_bf16(on ? v : 0.f);
                } else {
                    reinterpret_cast<float*>(g.out)[m * g.ldo + n] = v;
                }
            }
        }
}

template <int kLA, int kLB, int kEpi>
void gemm(const GemmArgs& g, hipStream_t st) {
    dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM));
    hipLaunchKernelGGL((k_gemm<kLA, kLB, kEpi>), grid, dim3(kGemmThreads), 0, st, g);
}

// dLoss terms: d = y - t; g = 2 m d (bf16, unscaled); per-block FP64 partial
// sums of m d^2 and m, reduced in a fixed order by k_loss_final.
constexpr int kRedThreads = 256;
__global__ __launch_bounds__(kRedThreads) void k_mse(const float* y, const float* tgt, const float* mask, int64_t n,
                                                     uint16_t* gy, double* partial) {
    __shared__ double s0[kRedThreads], s1[kRedThreads];
    double a0 = 0.0, a1 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kRedThreads;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
        const float m = mask ? mask[i] : 1.f;
        const float d = y[i] - tgt[i];
        gy[i] = f32_to_bf16(2.f * m * d);
        a0 += (double)m * (double)d * (double)d;
        a1 += (double)m;
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s0[threadIdx.x] += s0[threadIdx.x + s];
            s1[threadIdx.x] += s1[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s0[0];
        partial[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ void k_loss_final(const double* partial, int nb, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a0 = 0.0, a1 = 0.0;
        for (int b = 0; b < nb; b++) {
            a0 += partial[2 * b];
            a1 += partial[2 * b + 1];
        }
        out[0] = a0;
        out[1] = a1;
    }
}

// bias gradient: db[n] = sum over rows of g[m, n] (bf16 in, FP32 sum in row order)
__global__ void k_colsum(const uint16_t* g, int64_t M, int64_t N, float* db) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int64_t m = 0; m < M; m++) s += bf16_to_f32(g[m * N + n]);
    db[n] = s;
}

struct AdamArgs {
    float* theta;
    uint16_t* theta_bf16;
    const float* grad;
    float* m;
    float* v;
    const double* loss_terms;
    int64_t n;
    float lr, b1, b2, eps, c1, c2;
};

__global__ void k_adam(AdamArgs a) {
    float gs = 1.f;
    if (a.loss_terms) {
        const double w = a.loss_terms[1];
        gs = w > 0.0 ? (float)(1.0 / w) : 0.f;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const float g = a.grad[i] * gs;
        const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
        const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
        a.m[i] = m;
        a.v[i] = v;
        const float mh = m * a.c1, vh = v * a.c2;
        const float th = a.theta[i] - a.lr * mh / (sqrtf(vh) + a.eps);
        a.theta[i] = th;
        if (a.theta_bf16) a.theta_bf16[i] = f32_to_bf16(th);
    }
}

__global__ void k_to_bf16(const float* x, int64_t n, uint16_t* y) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = f32_to_bf16(x[i]);
}

__global__ void k_features(const float* h, int64_t n, float floor_db, float off_db, float scale_db, uint16_t* x) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float e = h[i];
        float db = e > 0.f ? 10.f * log10f(e) : floor_db;
        db = fmaxf(db, floor_db);
        x[i] = f32_to_bf16((db + off_db) / scale_db);
    }
}

// Backward (Schroeder) integration per row, one wavefront per row: lane l
// owns a chunk of consecutive bins; chunk totals are suffix-summed across
// lanes, then each lane walks its chunk from the end.  FP64 sums; dB
// relative to the row total, clamped at floor_db.
__global__ __launch_bounds__(256) void k_edc(const float* h, int64_t rows, int32_t bins, float floor_db,
                                             float* out) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= rows) return;
    const float* hr = h + row * bins;
    float* orow = out + row * bins;
    const int chunk = (bins + 63) / 64;
    const int b0 = lane * chunk;
    const int b1 = b0 + chunk < bins ? b0 + chunk : bins;
    double own = 0.0;
    for (int b = b0; b < b1; b++) own += (double)hr[b];
    // suffix sum over lanes: after[l] = sum of chunks of lanes > l
    double incl = own;
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_down(incl, d, 64);
        if (lane + d < 64) incl += o;
    }
    double after = __shfl_down(incl, 1, 64);   // chunks of the lanes after this one
    if (lane == 63) after = 0.0;
    // total = the suffix sum at bin 0, summed in the same order as below, so
    // that the first bin is exactly 0 dB
    double run = after;
    for (int b = b1 - 1; b >= b0; b--) run += (double)hr[b];
    const double tot = __shfl(run, 0, 64);
    run = after;
    for (int b = b1 - 1; b >= b0; b--) {
        run += (double)hr[b];
        float v = floor_db;
        if (tot > 0.0 && run > 0.0) v = (float)(10.0 * log10(run / tot));
        orow[b] = v > floor_db ? v : floor_db;
    }
}

unsigned grid_for(int64_t n, int threads, int cap_per_cu = 8) {
    int64_t b = (n + threads - 1) / threads;
    const int64_t cap = (int64_t)device_sm_count() * cap_per_cu;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace
}  // namespace rtac

struct rt_mlp {
    int device = 0;
    int n_layers = 0;                 // weight layers
    int32_t width[rtac::kMaxLayers + 1] = {};
    int64_t param_off[rtac::kMaxLayers + 1] = {};   // start of W_l; b_l follows W_l
    int64_t n_params = 0;
    int64_t max_batch = 0;
    int64_t act_off[rtac::kMaxLayers + 1] = {};     // start of hidden activation l (1..L-1) in acts
    rtac::Buf acts, gbuf[2], partial, loss_tmp;
    int64_t last_batch = -1;
};

using namespace rtac;

extern "C" int rt_mlp_create(const int32_t* widths, int32_t n_layers, int64_t max_batch, rt_mlp** out) {
    RT_CHECK(out && widths, RT_EINVAL, "rt_mlp_create: null argument");
    *out = nullptr;
    RT_CHECK(n_layers >= 1 && n_layers <= kMaxLayers, RT_EINVAL, "rt_mlp_create: n_layers must be in [1, %d]",
             kMaxLayers);
    RT_CHECK(max_batch >= 1 && max_batch <= (1 << 20), RT_EINVAL, "rt_mlp_create: max_batch must be in [1, 2^20]");
    for (int l = 0; l <= n_layers; l++)
        RT_CHECK(widths[l] >= 64 && widths[l] <= kMaxWidth && widths[l] % 64 == 0, RT_EINVAL,
                 "rt_mlp_create: width %d = %d (must be a multiple of 64 in [64, %d])", l, widths[l], kMaxWidth);
    int device = 0;
    RT_HIP(hipGetDevice(&device));
    rt_mlp* n = new rt_mlp();
    n->device = device;
    n->n_layers = n_layers;
    int64_t off = 0, aoff = 0, wmax = 0;
    for (int l = 0; l <= n_layers; l++) {
        n->width[l] = widths[l];
        if (widths[l] > wmax) wmax = widths[l];
    }
    for (int l = 0; l < n_layers; l++) {
        n->param_off[l] = off;
        off += (int64_t)widths[l] * widths[l + 1] + widths[l + 1];
    }
    n->param_off[n_layers] = off;
    n->n_params = off;
    for (int l = 1; l < n_layers; l++) {
        n->act_off[l] = aoff;
        aoff += max_batch * widths[l];
    }
    n->act_off[n_layers] = aoff;
    n->max_batch = max_batch;
    const int nb = (int)grid_for(max_batch * wmax, kRedThreads);
    if (n->acts.ensure(2 * (size_t)(aoff > 0 ? aoff : 1)) || n->gbuf[0].ensure(2 * (size_t)max_batch * wmax) ||
        n->gbuf[1].ensure(2 * (size_t)max_batch * wmax) || n->partial.ensure(16 * (size_t)nb)) {
        n->acts.release();
        n->gbuf[0].release();
        n->gbuf[1].release();
        n->partial.release();
        delete n;
        return RT_ENOMEM;
    }
    *out = n;
    return RT_OK;
}

extern "C" int rt_mlp_destroy(rt_mlp* n) {
    if (!n) return RT_OK;
    n->acts.release();
    n->gbuf[0].release();
    n->gbuf[1].release();
    n->partial.release();
    n->loss_tmp.release();
    delete n;
    return RT_OK;
}

extern "C" int rt_mlp_info(const rt_mlp* n, int64_t* info) {
    RT_CHECK(n && info, RT_EINVAL, "rt_mlp_info: null argument");
    info[0] = n->n_params;
    info[1] = n->n_layers;
    info[2] = n->max_batch;
    info[3] = n->act_off[n->n_layers];
    return RT_OK;
}

extern "C" int rt_mlp_forward(rt_mlp* n, const uint16_t* theta_bf16, const float* theta_f32, const uint16_t* x,
                              int64_t batch, float* y, void* stream) {
    RT_CHECK(n && theta_bf16 && x && y, RT_EINVAL, "rt_mlp_forward: null argument");
    RT_CHECK(((uintptr_t)theta_bf16 & 15u) == 0 && ((uintptr_t)x & 15u) == 0, RT_EINVAL,
             "rt_mlp_forward: theta_bf16 and x must be 16-byte aligned");
    RT_CHECK(batch >= 0 && batch <= n->max_batch, RT_EINVAL, "rt_mlp_forward: batch %lld not in [0, %lld]",
             (long long)batch, (long long)n->max_batch);
    if (batch == 0) return RT_OK;
    hipStream_t st = (hipStream_t)stream;
    uint16_t* acts = n->acts.as<uint16_t>();
    const uint16_t* in = x;
    for (int l = 0; l < n->n_layers; l++) {
        GemmArgs g{};
        g.A = in;
        g.lda = n->width[l];
        g.B = theta_bf16 + n->param_off[l];
        g.ldb = n->width[l];
        g.M = batch;
        g.N = n->width[l + 1];
        g.K = n->width[l];
        const int64_t boff = n->param_off[l] + (int64_t)n->width[l] * n->width[l + 1];
        g.bias = theta_f32 ? theta_f32 + boff : nullptr;
        g.bias_bf16 = theta_bf16 + boff;
        g.ldo = g.N;
        if (l + 1 < n->n_layers) {
            g.out = acts + n->act_off[l + 1];
            gemm<kRowK, kRowK, kEpiBiasRelu>(g, st);
            in = acts + n->act_off[l + 1];
        } else {
            g.out = y;
            gemm<kRowK, kRowK, kEpiBias>(g, st);
        }
    }
    n->last_batch = batch;
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" int rt_mlp_backward(rt_mlp* n, const uint16_t* theta_bf16, const uint16_t* x, int64_t batch,
                               const float* y, const float* target, const float* mask, float* grad,
                               double* loss_terms, void* stream) {
    RT_CHECK(n && theta_bf16 && x && y && target && grad && loss_terms, RT_EINVAL, "rt_mlp_backward: null argument");
    RT_CHECK(batch >= 1 && batch <= n->max_batch, RT_EINVAL, "rt_mlp_backward: batch %lld not in [1, %lld]",
             (long long)batch, (long long)n->max_batch);
    RT_CHECK(((uintptr_t)theta_bf16 & 15u) == 0 && ((uintptr_t)x & 15u) == 0, RT_EINVAL,
             "rt_mlp_backward: theta_bf16 and x must be 16-byte aligned");
    RT_CHECK(batch == n->last_batch, RT_EINVAL,
             "rt_mlp_backward: must follow rt_mlp_forward on the same input (batch %lld, last forward %lld)",
             (long long)batch, (long long)n->last_batch);
    hipStream_t st = (hipStream_t)stream;
    const int L = n->n_layers;
    const int64_t ny = batch * n->width[L];
    const unsigned nb = grid_for(ny, kRedThreads);
    uint16_t* gcur = n->gbuf[0].as<uint16_t>();
    uint16_t* gnext = n->gbuf[1].as<uint16_t>();
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kRedThreads), 0, st, y, target, mask, ny, gcur,
                       n->partial.as<double>());
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, n->partial.as<double>(), (int)nb, loss_terms);
    const uint16_t* acts = n->acts.as<uint16_t>();
    for (int l = L - 1; l >= 0; l--) {
        const int64_t O = n->width[l + 1], I = n->width[l];
        const uint16_t* a_in = l == 0 ? x : acts + n->act_off[l];
        // dW_l [O, I] = g^T [O, B] a_in [B, I]
        GemmArgs gw{};
        gw.A = gcur;          // stored [B][O]: logical [O, K=B] with rows contiguous
        gw.lda = O;
        gw.B = a_in;          // stored [B][I]: logical [I, K=B] with rows contiguous
        gw.ldb = I;
        gw.M = O;
        gw.N = I;
        gw.K = batch;
        gw.out = grad + n->param_off[l];
        gw.ldo = I;
        gemm<kRowMN, kRowMN, kEpiStore>(gw, st);
        hipLaunchKernelGGL(k_colsum, dim3((unsigned)((O + 255) / 256)), dim3(256), 0, st, gcur, batch, O,
                           grad + n->param_off[l] + O * I);
        if (l > 0) {
            // g_{l-1} [B, I] = (g [B, O] W_l [O, I]) * (a_in > 0)
            GemmArgs gx{};
            gx.A = gcur;      // [B][O], K = O contiguous
            gx.lda = O;
            gx.B = theta_bf16 + n->param_off[l];   // stored [O][I]: logical [I, K=O] with rows contiguous
            gx.ldb = I;
            gx.M = batch;
            gx.N = I;
            gx.K = O;
            gx.mask_act = a_in;
            gx.out = gnext;
            gx.ldo = I;
            gemm<kRowK, kRowMN, kEpiMask>(gx, st);
            uint16_t* t = gcur;
            gcur = gnext;
            gnext = t;
        }
    }
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" int rt_mlp_adam(int64_t n_params, float* theta, uint16_t* theta_bf16, const float* grad, float* m,
                           float* v, const double* loss_terms, int32_t step, float lr, float beta1, float beta2,
                           float eps, void* stream) {
    RT_CHECK(theta && grad && m && v, RT_EINVAL, "rt_mlp_adam: null argument");
    RT_CHECK(n_params >= 0, RT_EINVAL, "rt_mlp_adam: n_params < 0");
    RT_CHECK(step >= 1, RT_EINVAL, "rt_mlp_adam: step must be >= 1");
    RT_CHECK(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f, RT_EINVAL,
             "rt_mlp_adam: betas must be in [0, 1)");
    if (n_params == 0) return RT_OK;
    AdamArgs a{theta, theta_bf16, grad, m, v, loss_terms, n_params, lr, beta1, beta2, eps, 0.f, 0.f};
    a.c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    a.c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n_params, 256)), dim3(256), 0, (hipStream_t)stream, a);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" int rt_to_bf16(const float* x, int64_t n, uint16_t* y, void* stream) {
    RT_CHECK(n >= 0 && (n == 0 || (x && y)), RT_EINVAL, "rt_to_bf16: null argument");
    if (n == 0) return RT_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, x, n, y);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" int rt_hist_features(const float* hist, int64_t n, float floor_db, float offset_db, float scale_db,
                                uint16_t* x, void* stream) {
    RT_CHECK(n >= 0 && (n == 0 || (hist && x)), RT_EINVAL, "rt_hist_features: null argument");
    RT_CHECK(scale_db != 0.f, RT_EINVAL, "rt_hist_features: scale_db is 0");
    if (n == 0) return RT_OK;
    hipLaunchKernelGGL(k_features, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, hist, n, floor_db,
                       offset_db, scale_db, x);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

extern "C" int rt_edc_db(const float* hist, int64_t rows, int32_t bins, float floor_db, float* edc, void* stream) {
    RT_CHECK(rows >= 0 && bins >= 1 && bins <= (1 << 20), RT_EINVAL, "rt_edc_db: bad sizes");
    RT_CHECK(rows == 0 || (hist && edc), RT_EINVAL, "rt_edc_db: null argument");
    if (rows == 0) return RT_OK;
    RT_CHECK((rows + 3) / 4 < ((int64_t)1 << 31), RT_EINVAL, "rt_edc_db: too many rows");
    hipLaunchKernelGGL(k_edc, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, (hipStream_t)stream, hist, rows, bins,
                       floor_db, edc);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
