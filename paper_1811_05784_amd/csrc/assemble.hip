// Impulse response from image sources (rt_assemble_ir) and the absorption
// adjoint (rt_band_energy_adjoint).
//
// Energy of an image source per octave band (eq. for E_s with air
// absorption): n/N exp(-beta d) prod_j (1 - alpha_j), FP64.  Arrival bin
// floor(d fs / c).  The histogram is built without floating-point atomics:
// sources are sorted by (receiver, bin) and every bin is summed by one thread
// in sorted order, so results are bitwise reproducible.  Pressure sqrt(E) is
// taken per bin and filtered per band.
//
// The 'same'-mode FIR y[n] = sum_j h[j] x[n + c - j] (c = (K-1)/2) runs on
// the FP32 matrix cores as a Toeplitz x Hankel product: a 16x16 output tile
// Y[i][q] = y[n0 + i + 16 q] = sum_kk A[i][kk] B[kk][q] with
// A[i][kk] = h[i + K - 1 - kk] and B[kk][q] = x[n0 + 16 q + kk - c].  Taps
// and the signal window (sqrt applied on load) are staged in LDS; the window
// is stored 20 floats per 16 samples so that the 64 lanes of one B fragment
// hit 64 different banks.
#include <initializer_list>

#include "common.h"

namespace rtac {

namespace {

struct IsArgs {
    const int32_t* key;
    const int32_t* count;
    const double* dist;
    const int64_t* n_is;
    int64_t is_cap;
    int32_t R1;
    int64_t n_rays;
    int32_t n_rcv;
    const float* alpha;
    const float* beta;
    const int32_t* plane_mat;
    int64_t n_tri;
    double c, fs;
    int64_t L;
    uint64_t invalid;   // sort key of sources outside the IR (n_rcv * L)
    // batched calls: global receiver row -> job -> scene (materials, rays)
    const int32_t* rcv_job;
    const DevJob* jobs;
    const DevScene* scenes;
};

// Material table view and ray count for image sources of receiver row m.
struct MatView {
    const int32_t* plane_mat;
    int64_t n_tri;
    int32_t mat_off;
    int64_t n_rays;
};
__device__ inline MatView mat_view(const IsArgs& a, int32_t m) {
    if (a.rcv_job) {
        const DevJob& jb = a.jobs[a.rcv_job[m]];
        const DevScene& sc = a.scenes[jb.scene];
        return MatView{sc.plane_mat, sc.n_tri, sc.mat_off, jb.n_rays};
    }
    return MatView{a.plane_mat, a.n_tri, 0, a.n_rays};
}

__device__ inline int64_t is_count_of(const IsArgs& a) {
    int64_t n = *a.n_is;
    if (n < 0) n = 0;
    return n > a.is_cap ? a.is_cap : n;
}

// Energy per band and (receiver, bin) sort key; invalid / late -> a.invalid.
__global__ void k_is_energy(IsArgs a, double* __restrict__ E, uint64_t* __restrict__ skey) {
    const int64_t n = is_count_of(a);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* row = a.key + i * (int64_t)(a.R1 + 1);
        const int32_t m = row[0], k = row[1];
        const double d = a.dist[i];
        double e[8];
        bool ok = m >= 0 && m < a.n_rcv && k >= 0 && k < a.R1;
        const MatView mv = mat_view(a, ok ? m : 0);
        const double base = (double)a.count[i] / (double)mv.n_rays;
        for (int b = 0; b < 8; b++) e[b] = base * exp(-(double)a.beta[b] * d);
        // planes and their materials fetched eight at a time, factors applied in order (a row
        // with an invalid plane is dropped from the histogram, whatever its factors)
        for (int j0 = 0; ok && j0 < k; j0 += 8) {
            int32_t p[8], mt[8];
#pragma unroll
            for (int q = 0; q < 8; q++) p[q] = j0 + q < k ? row[2 + j0 + q] : 0;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const bool valid = p[q] >= 0 && p[q] < mv.n_tri;
                if (j0 + q < k && !valid) ok = false;
                mt[q] = (j0 + q < k && valid) ? mv.mat_off + mv.plane_mat[p[q]] : -1;
            }
#pragma unroll
            for (int q = 0; q < 8; q++)
                if (mt[q] >= 0)
                    for (int b = 0; b < 8; b++) e[b] *= 1.0 - (double)a.alpha[8 * mt[q] + b];
        }
        for (int b = 0; b < 8; b++) E[8 * i + b] = e[b];
        const double sb = floor(d * a.fs / a.c);
        uint64_t key = a.invalid;
        if (ok && sb >= 0.0 && sb < (double)a.L) key = (uint64_t)m * (uint64_t)a.L + (uint64_t)sb;
        skey[i] = key;
    }
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One thread per run of equal (receiver, bin): sum in sorted order (FP64).
__global__ void k_bin_sum(IsArgs a, const uint64_t* __restrict__ skey, const uint32_t* __restrict__ idx,
                          const double* __restrict__ E, float* __restrict__ hist) {
    const int64_t n = is_count_of(a);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = skey[i];
        if (key == a.invalid) continue;
        if (i > 0 && skey[i - 1] == key) continue;
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t j = i; j < n && skey[j] == key; j++) {
            const uint32_t q = idx[j];
            for (int b = 0; b < 8; b++) s[b] += E[8 * (int64_t)q + b];
        }
        const int64_t m = (int64_t)(key / (uint64_t)a.L), bin = (int64_t)(key % (uint64_t)a.L);
        for (int b = 0; b < 8; b++) hist[(m * 8 + b) * a.L + bin] = (float)s[b];
    }
}

// band_energy[r, b] = sum over bins (FP64 tree reduction, fixed order).
// Band energies: each signal is cut into kBandChunks chunks (one workgroup
// each, so the whole GPU works on the 8 n_rcv signals), summed in FP64 in a
// fixed order; k_band_final adds a signal's chunk sums in order.
constexpr int kBandChunks = 16;
__global__ void __launch_bounds__(256) k_band_partial(const float* __restrict__ hist, int64_t L,
                                                      double* __restrict__ part) {
    __shared__ double red[256];
    const int64_t sig = blockIdx.y;
    const int c = blockIdx.x;
    const int64_t len = (L + kBandChunks - 1) / kBandChunks;
    const int64_t lo = c * len, hi = lo + len < L ? lo + len : L;
    const float* h = hist + sig * L;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += (double)h[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[sig * kBandChunks + c] = red[0];
}

__global__ void k_band_final(const double* __restrict__ part, int64_t n_sig, float* __restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sig) return;
    double a = 0.0;
    for (int c = 0; c < kBandChunks; c++) a += part[s * kBandChunks + c];
    out[s] = (float)a;
}

// ---------------------------------------------------------------------------
// FIR on MFMA (v_mfma_f32_16x16x4_f32)
// ---------------------------------------------------------------------------
constexpr int kFirWaves = 4;
constexpr int kFirTiles = 4;                                    // 16x16 tiles per wave
constexpr int kFirOut = kFirWaves * kFirTiles * 256;            // outputs per workgroup

__device__ inline int win_addr(int p) { return (p >> 4) * 20 + (p & 15); }

typedef float floatx4 __attribute__((ext_vector_type(4)));

// grid: (ceil(L / kFirOut), n_rcv * 8).  taps padded: hp[u] = h[u - 48] for
// u - 48 in [0, K), else 0, length Kpad = K + 112.
__global__ void __launch_bounds__(256) k_fir_mfma(const float* __restrict__ hist, const float* __restrict__ fir, int K,
                                                  int64_t L, float* __restrict__ band_ir) {
    extern __shared__ float smem[];
    const int sig = blockIdx.y;
    const int band = sig & 7;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = (K - 1) / 2;
    const int64_t n0 = (int64_t)blockIdx.x * kFirOut;
    // signal window: positions [w0, w0 + W) with w0 = floor16(n0 - c)
    const int64_t s0 = n0 - c;
    const int64_t w0 = s0 >= 0 ? (s0 & ~(int64_t)15) : -((-s0 + 15) & ~(int64_t)15);
    const int delta = (int)(s0 - w0);                            // 0..15
    const int S = (K + 15 + delta + 3) / 4;                      // MFMA steps (kk' in [0, 4S))
    const int W = kFirOut + 4 * S + 16;                          // window samples
    const int Kpad = K + 112;
    float* hp = smem;                                            // [Kpad]
    float* xw = smem + Kpad;                                     // [win_addr(W) + 20]
    const float* taps = fir + (int64_t)band * K;
    for (int u = tid; u < Kpad; u += 256) {
        const int j = u - 48;
        hp[u] = (j >= 0 && j < K) ? taps[j] : 0.f;
    }
    const float* x = hist + (int64_t)sig * L;
    for (int p = tid; p < W; p += 256) {
        const int64_t g = w0 + p;
        const float v = (g >= 0 && g < L) ? x[g] : 0.f;
        xw[win_addr(p)] = sqrtf(v);
    }
    __syncthreads();
    const int i = lane & 15, kq = lane >> 4;
    floatx4 acc[kFirTiles];
    for (int t = 0; t < kFirTiles; t++) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    // A[i][kk'] = h[i + K - 1 + delta - kk'], kk' = 4s + kq  -> hp index + 48
    const int abase = i + K - 1 + delta - kq + 48;
    // B[kk'][q] = x[w0 + tile_off + 16 q + kk'], q = lane & 15
    const int bbase = wave * (kFirTiles * 256) + 16 * i + kq;
    for (int s = 0; s < S; s++) {
        const int ai = abase - 4 * s;
        const float av = (ai >= 0 && ai < Kpad) ? hp[ai] : 0.f;
#pragma unroll
        for (int t = 0; t < kFirTiles; t++) {
            const float bv = xw[win_addr(bbase + t * 256 + 4 * s)];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
        }
    }
    // D[i][q]: lane = q + 16 * (i / 4), element i % 4 -> y[n0 + tile + i + 16 q]
    float* y = band_ir + (int64_t)sig * L;
    const int q = lane & 15, ib = 4 * (lane >> 4);
    for (int t = 0; t < kFirTiles; t++) {
        const int64_t o = n0 + wave * (kFirTiles * 256) + t * 256 + 16 * q + ib;
        for (int e = 0; e < 4; e++)
            if (o + e < L) y[o + e] = acc[t][e];
    }
}

// ---------------------------------------------------------------------------
// FIR by FFT (overlap-save) for long filters
// ---------------------------------------------------------------------------
// N = 4^7-point transforms held in LDS, in place: the forward transform is
// radix-4 decimation in frequency (output in base-4 digit-reversed order),
// the inverse is its exact stage-by-stage inverse (decimation in time from
// digit-reversed input to natural order), so the pointwise product with a
// filter spectrum computed the same way needs no permutation.  Two
// consecutive segments of one band signal ride as the real and imaginary
// parts of one transform (the taps are real).  A segment of N samples yields
// N - K + 1 outputs of the 'same'-aligned convolution.
constexpr int kFftLog4 = 7;
constexpr int kFftN = 1 << (2 * kFftLog4);
constexpr int kFftThreads = 1024;
constexpr int kFirFftMinK = 1024;

__device__ inline float2 cmulf(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cmulf_conj(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline float2 addf2(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 subf2(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// tw[m] = exp(-2 pi i m / N), FP64 rounded once
__global__ void k_fft_twiddles(float2* __restrict__ tw) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= kFftN) return;
    double s, c;
    sincos(-2.0 * 3.14159265358979323846 * (double)m / (double)kFftN, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
}

// Stage s works on blocks of M = N / 4^s with quarter q = M / 4; output k of
// the butterfly at offset j gets the twiddle w_M^(j k) = tw[j k 4^s].
__device__ inline void fft_dif(float2* x, const float2* __restrict__ tw) {
    for (int s = 0; s < kFftLog4; s++) {
        const int lq = 2 * (kFftLog4 - 1 - s);   // log2 q
        const int q = 1 << lq;
        for (int u = threadIdx.x; u < kFftN / 4; u += kFftThreads) {
            const int j = u & (q - 1);
            const int base = ((u >> lq) << (lq + 2)) + j;
            const float2 a0 = x[base], a1 = x[base + q], a2 = x[base + 2 * q], a3 = x[base + 3 * q];
            const float2 t0 = addf2(a0, a2), t1 = subf2(a0, a2), t2 = addf2(a1, a3), d = subf2(a1, a3);
            const float2 t3 = make_float2(d.y, -d.x);   // -i d
            const int e = j << (2 * s);
            x[base] = addf2(t0, t2);
            x[base + q] = cmulf(addf2(t1, t3), tw[e]);
            x[base + 2 * q] = cmulf(subf2(t0, t2), tw[2 * e]);
            x[base + 3 * q] = cmulf(subf2(t1, t3), tw[3 * e]);
        }
        __syncthreads();
    }
}

// Inverse of fft_dif up to the factor N (undo the twiddles, 4-point inverse
// transform, stages in reverse order).
__device__ inline void fft_dit_inv(float2* x, const float2* __restrict__ tw) {
    for (int s = kFftLog4 - 1; s >= 0; s--) {
        const int lq = 2 * (kFftLog4 - 1 - s);
        const int q = 1 << lq;
        for (int u = threadIdx.x; u < kFftN / 4; u += kFftThreads) {
            const int j = u & (q - 1);
            const int base = ((u >> lq) << (lq + 2)) + j;
            const int e = j << (2 * s);
            const float2 a0 = x[base];
            const float2 a1 = cmulf_conj(x[base + q], tw[e]);
            const float2 a2 = cmulf_conj(x[base + 2 * q], tw[2 * e]);
            const float2 a3 = cmulf_conj(x[base + 3 * q], tw[3 * e]);
            const float2 t0 = addf2(a0, a2), t1 = subf2(a0, a2), t2 = addf2(a1, a3), d = subf2(a1, a3);
            const float2 t3 = make_float2(-d.y, d.x);   // i d
            x[base] = addf2(t0, t2);
            x[base + q] = addf2(t1, t3);
            x[base + 2 * q] = subf2(t0, t2);
            x[base + 3 * q] = subf2(t1, t3);
        }
        __syncthreads();
    }
}

// spec[b] = forward transform of the zero-padded taps of band b, times 1 / N
__global__ void __launch_bounds__(kFftThreads) k_fir_spectrum(const float* __restrict__ fir, int K,
                                                               const float2* __restrict__ tw,
                                                               float2* __restrict__ spec) {
    extern __shared__ float2 xs[];
    const int b = blockIdx.x;
    for (int i = threadIdx.x; i < kFftN; i += kFftThreads)
        xs[i] = make_float2(i < K ? fir[(int64_t)b * K + i] : 0.f, 0.f);
    __syncthreads();
    fft_dif(xs, tw);
    const float inv = 1.0f / (float)kFftN;
    for (int i = threadIdx.x; i < kFftN; i += kFftThreads)
        spec[(int64_t)b * kFftN + i] = make_float2(xs[i].x * inv, xs[i].y * inv);
}

// grid: (ceil(n_seg / 2), n_rcv * 8); segment g covers outputs [g B, g B + B)
// with B = N - K + 1 and reads samples from g B - (K - 1) / 2.
__global__ void __launch_bounds__(kFftThreads) k_fir_fft(const float* __restrict__ hist,
                                                          const float2* __restrict__ spec,
                                                          const float2* __restrict__ tw, int K, int64_t L,
                                                          float* __restrict__ band_ir) {
    extern __shared__ float2 xs[];
    const int sig = blockIdx.y;
    const int band = sig & 7;
    const int64_t B = kFftN - K + 1;
    const int c = (K - 1) / 2;
    const int64_t n0a = (int64_t)(2 * blockIdx.x) * B, n0b = n0a + B;
    const float* x = hist + (int64_t)sig * L;
    for (int i = threadIdx.x; i < kFftN; i += kFftThreads) {
        const int64_t ga = n0a - c + i, gb = n0b - c + i;
        const float va = (ga >= 0 && ga < L) ? sqrtf(x[ga]) : 0.f;
        const float vb = (n0b < L && gb >= 0 && gb < L) ? sqrtf(x[gb]) : 0.f;
        xs[i] = make_float2(va, vb);
    }
    __syncthreads();
    fft_dif(xs, tw);
    const float2* hs = spec + (int64_t)band * kFftN;
    for (int i = threadIdx.x; i < kFftN; i += kFftThreads) xs[i] = cmulf(xs[i], hs[i]);
    __syncthreads();
    fft_dit_inv(xs, tw);
    float* y = band_ir + (int64_t)sig * L;
    for (int64_t t = threadIdx.x; t < B; t += kFftThreads) {
        const float2 v = xs[K - 1 + t];
        if (n0a + t < L) y[n0a + t] = v.x;
        if (n0b + t < L) y[n0b + t] = v.y;
    }
}

__global__ void k_sum_bands(const float* __restrict__ band_ir, int64_t L, int32_t n_rcv, float* __restrict__ ir) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_rcv * L) return;
    const int64_t m = i / L, s = i % L;
    float acc = 0.f;
    for (int b = 0; b < 8; b++) acc += band_ir[(m * 8 + b) * L + s];
    ir[i] = acc;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
constexpr int kAdjThreads = 256;

constexpr int kAdjDistinct = 16;   // distinct materials of one path kept in LDS (more: the path is rescanned)

// partial[block][m][b]: per-block sums in a fixed order.  Each image source
// first lists the distinct materials of its path with their multiplicities
// (once), and the block marks the materials that occur; a material absent
// from the block gets a zero partial without a reduction.  For a present one,
// d/d alpha_(mat,b) of prod_j (1 - alpha_(m_j,b)) = -c (1 - alpha_(mat,b))^(c-1)
// x the product over the path's other materials is summed over the
// wavefront by a butterfly of lane exchanges and over the block's four
// wavefronts in order (bitwise reproducible).
__global__ void __launch_bounds__(kAdjThreads) k_adjoint_partial(IsArgs a, int32_t n_mat, const float* __restrict__ g,
                                                                 double* __restrict__ partial) {
    __shared__ double red[kAdjThreads / kWave][8];
    __shared__ uint32_t present[128];   // materials on the block's paths (n_mat <= 4096)
    __shared__ int32_t dmat[kAdjDistinct][kAdjThreads];
    __shared__ int32_t dcnt[kAdjDistinct][kAdjThreads];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (int w = tid; w < 128; w += kAdjThreads) present[w] = 0u;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kAdjThreads + tid;
    const int64_t n = is_count_of(a);
    bool ok = i < n;
    const int32_t* row = ok ? a.key + i * (int64_t)(a.R1 + 1) : nullptr;
    int32_t m = 0, k = 0, nd = 0;
    bool rescan = false;   // more distinct materials than the list holds
    double base[8];
    MatView mv{a.plane_mat, a.n_tri, 0, a.n_rays};
    if (ok) {
        m = row[0];
        k = row[1];
        ok = m >= 0 && m < a.n_rcv && k >= 0 && k < a.R1;
        if (ok) mv = mat_view(a, m);
        const double d = a.dist[i];
        const double sb = floor(d * a.fs / a.c);
        ok = ok && sb >= 0.0 && sb < (double)a.L;
        for (int j = 0; ok && j < k; j++) ok = row[2 + j] >= 0 && row[2 + j] < mv.n_tri;
        for (int b = 0; b < 8; b++)
            base[b] = ok ? (double)a.count[i] / (double)mv.n_rays * exp(-(double)a.beta[b] * d) * (double)g[8 * m + b]
                         : 0.0;
    }
    if (ok) {
        for (int j = 0; j < k; j++) {
            const int32_t mt = mv.mat_off + mv.plane_mat[row[2 + j]];
            if (mt < 0 || mt >= n_mat) continue;   // not a differentiated material
            int f = -1;
            for (int q = 0; q < nd; q++)
                if (dmat[q][tid] == mt) f = q;
            if (f >= 0) {
                dcnt[f][tid]++;
            } else if (nd < kAdjDistinct) {
                dmat[nd][tid] = mt;
                dcnt[nd][tid] = 1;
                nd++;
            } else {
                rescan = true;
            }
            atomicOr(&present[mt >> 5], 1u << (mt & 31));
        }
    }
    __syncthreads();
    for (int mat = 0; mat < n_mat; mat++) {
        if (((present[mat >> 5] >> (mat & 31)) & 1u) == 0u) {
            if (tid < 8) partial[((int64_t)blockIdx.x * n_mat + mat) * 8 + tid] = 0.0;
            continue;
        }
        int cm = 0;
        if (ok) {
            if (rescan) {
                for (int j = 0; j < k; j++) cm += mv.mat_off + mv.plane_mat[row[2 + j]] == mat;
            } else {
                for (int q = 0; q < nd; q++)
                    if (dmat[q][tid] == mat) cm = dcnt[q][tid];
            }
        }
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (cm > 0) {
            for (int b = 0; b < 8; b++) {
                const double om = 1.0 - (double)a.alpha[8 * mat + b];
                double dv = -(double)cm;
                for (int e = 0; e < cm - 1; e++) dv *= om;
                if (rescan) {
                    for (int j = 0; j < k; j++) {
                        const int32_t mt = mv.mat_off + mv.plane_mat[row[2 + j]];
                        if (mt != mat) dv *= 1.0 - (double)a.alpha[8 * mt + b];
                    }
                } else {
                    for (int q = 0; q < nd; q++) {
                        const int32_t mt = dmat[q][tid];
                        if (mt == mat) continue;
                        const double oq = 1.0 - (double)a.alpha[8 * mt + b];
                        for (int e = 0; e < dcnt[q][tid]; e++) dv *= oq;
                    }
                }
                v[b] = base[b] * dv;
            }
        }
        if (__ballot(cm > 0) != 0ull) {
            for (int b = 0; b < 8; b++) {
                double sum = v[b];
                for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
                if (lane == 0) red[wave][b] = sum;
            }
        } else if (lane < 8) {
            red[wave][lane] = 0.0;
        }
        __syncthreads();
        if (tid < 8) {
            double sum = 0.0;
            for (int w = 0; w < kAdjThreads / kWave; w++) sum += red[w][tid];
            partial[((int64_t)blockIdx.x * n_mat + mat) * 8 + tid] = sum;
        }
        __syncthreads();
    }
}

// grad[t] = sum over the used blocks of partial[block][t]: one wavefront per
// entry t, lane l summing blocks l, l + 64, ... in order, then a butterfly of
// lane exchanges (a fixed order: bitwise reproducible).
__global__ void k_adjoint_final(const double* __restrict__ partial, int nblocks, int32_t n_mat, const int64_t* n_is,
                                int64_t is_cap, float* __restrict__ grad) {
    const int t = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave);
    const int lane = threadIdx.x & (kWave - 1);
    if (t >= n_mat * 8) return;   // whole wavefronts leave together
    int64_t n = *n_is;
    if (n > is_cap) n = is_cap;
    const int used = (int)((n + kAdjThreads - 1) / kAdjThreads);
    double s = 0.0;
    for (int b = lane; b < used && b < nblocks; b += kWave) s += partial[(int64_t)b * n_mat * 8 + t];
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) grad[t] = (float)s;
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }
// grid-stride kernels: enough workgroups to fill the chip, no more
inline unsigned nblk_gs(int64_t n) {
    int64_t b = (n + 255) / 256;
    const int64_t cap = (int64_t)device_sm_count() * 8;
    if (b > cap) b = cap;
    return (unsigned)(b > 0 ? b : 1);
}

int check_is_args(const rt_scene* s, const int32_t* is_key, const int32_t* is_count, const double* is_dist,
                  const int64_t* n_is, int64_t is_cap, int32_t R, int64_t n_rays, int32_t n_rcv, const float* alpha,
                  const float* beta, float c, float fs, int64_t L) {
    RT_CHECK(s && n_is && alpha && beta, RT_EINVAL, "null argument");
    RT_CHECK(s->valid, RT_EINVAL, "the scene's last rebuild failed");
    RT_CHECK(is_cap >= 0 && (is_cap == 0 || (is_key && is_count && is_dist)), RT_EINVAL, "null image-source table");
    RT_CHECK(is_cap < ((int64_t)1 << 31), RT_EINVAL, "is_cap must be < 2^31");
    RT_CHECK(R >= 0 && R < 4096, RT_EINVAL, "max_reflections out of range");
    RT_CHECK(n_rays >= 1, RT_EINVAL, "n_rays must be >= 1");
    RT_CHECK(n_rcv >= 1 && n_rcv <= kMaxRcv, RT_EINVAL, "n_rcv must be in [1, %d]", kMaxRcv);
    RT_CHECK(c > 0.f && fs > 0.f, RT_EINVAL, "c and fs must be positive");
    RT_CHECK(L >= 1 && L <= ((int64_t)1 << 30), RT_EINVAL, "L out of range");
    return RT_OK;
}

IsArgs make_is_args(const rt_scene* s, const int32_t* is_key, const int32_t* is_count, const double* is_dist,
                    const int64_t* n_is, int64_t is_cap, int32_t R, int64_t n_rays, int32_t n_rcv, const float* alpha,
                    const float* beta, float c, float fs, int64_t L) {
    IsArgs a;
    a.key = is_key;
    a.count = is_count;
    a.dist = is_dist;
    a.n_is = n_is;
    a.is_cap = is_cap;
    a.R1 = R + 1;
    a.n_rays = n_rays;
    a.n_rcv = n_rcv;
    a.alpha = alpha;
    a.beta = beta;
    a.plane_mat = s->plane_mat;
    a.n_tri = s->n_tri;
    a.c = c;
    a.fs = fs;
    a.L = L;
    a.invalid = (uint64_t)n_rcv * (uint64_t)L;
    a.rcv_job = nullptr;
    a.jobs = nullptr;
    a.scenes = nullptr;
    return a;
}

constexpr int kMaxDevices = 64;

// Raises the dynamic-LDS limit of the given kernels on the current device, once
// per device (the attribute belongs to each device's copy of the code object).
// false, with the error message set, when a HIP call fails.
bool raise_lds_limit(bool* done, std::initializer_list<const void*> kernels, int bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && dev >= 0 && dev < kMaxDevices && done[dev]) return true;
    for (const void* k : kernels) {
        if (e != hipSuccess) break;
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    }
    if (e != hipSuccess) {
        set_error("rt_assemble_ir: raising the LDS limit to %d bytes failed: %s", bytes, hipGetErrorString(e));
        return false;
    }
    if (dev >= 0 && dev < kMaxDevices) done[dev] = true;
    return true;
}

}  // namespace

}  // namespace rtac

using namespace rtac;

namespace rtac {
namespace {
int assemble_common(const rt_scene* scene, const rt_batch* bt, const int32_t* is_key, const int32_t* is_count,
                    const double* is_dist, const int64_t* n_is, int64_t is_cap, int32_t max_reflections,
                    int64_t n_rays, int32_t n_rcv, const float* alpha, const float* beta, float c, float fs,
                    int64_t L, const float* fir, int32_t K, float* band_energy, float* hist, float* band_ir,
                    float* ir, void* stream) {
    int rc = check_is_args(scene, is_key, is_count, is_dist, n_is, is_cap, max_reflections, n_rays, bt ? 1 : n_rcv,
                           alpha, beta, c, fs, L);
    if (rc) {
        set_error("rt_assemble_ir: %s", rt_last_error());
        return rc;
    }
    RT_CHECK(fir && K >= 1 && (K & 1) == 1 && K <= 16383, RT_EINVAL, "rt_assemble_ir: K must be odd in [1, 16383]");
    RT_CHECK(band_energy && hist && band_ir && ir, RT_EINVAL, "rt_assemble_ir: null output");
    RT_CHECK((int64_t)n_rcv * L * 8 < ((int64_t)1 << 62), RT_EINVAL, "rt_assemble_ir: output too large");
    hipStream_t st = (hipStream_t)stream;
    rt_scene* s = const_cast<rt_scene*>(scene);
    Workspace& ws = s->ws;
    const int64_t cap = is_cap > 0 ? is_cap : 1;
    if (ws.asm_energy.ensure(sizeof(double) * 8 * cap) || ws.sort_keys[0].ensure(8 * cap) ||
        ws.sort_keys[1].ensure(8 * cap) || ws.sort_vals[0].ensure(4 * cap) || ws.sort_vals[1].ensure(4 * cap))
        return RT_ENOMEM;
    IsArgs a = make_is_args(scene, is_key, is_count, is_dist, n_is, is_cap, max_reflections, n_rays, n_rcv, alpha,
                            beta, c, fs, L);
    if (bt) {
        a.rcv_job = bt->rcv_job;
        a.jobs = bt->jobs;
        a.scenes = bt->scenes;
    }
    double* E = ws.asm_energy.as<double>();
    uint64_t* k0 = ws.sort_keys[0].as<uint64_t>();
    uint64_t* k1 = ws.sort_keys[1].as<uint64_t>();
    uint32_t* v0 = ws.sort_vals[0].as<uint32_t>();
    uint32_t* v1 = ws.sort_vals[1].as<uint32_t>();
    hipLaunchKernelGGL(k_is_energy, dim3(nblk_gs(cap)), dim3(256), 0, st, a, E, k0);
    // sort by (receiver, bin); the invalid key n_rcv * L lands last
    int bits = 8;
    while (bits < 64 && (a.invalid >> bits) != 0) bits += 8;
    int which = 0;
    rc = radix_sort_pairs(ws, k0, v0, k1, v1, cap, n_is, 0, bits, st, &which, true);
    if (rc) return rc;
    const int64_t hn = (int64_t)n_rcv * 8 * L;
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk(hn)), dim3(256), 0, st, hist, hn, 0.f);
    hipLaunchKernelGGL(k_bin_sum, dim3(nblk_gs(cap)), dim3(256), 0, st, a, which ? k1 : k0, which ? v1 : v0, E, hist);
    {
        const int64_t n_sig = (int64_t)n_rcv * 8;
        if (ws.band_partial.ensure(sizeof(double) * (size_t)n_sig * kBandChunks)) return RT_ENOMEM;
        double* part = ws.band_partial.as<double>();
        hipLaunchKernelGGL(k_band_partial, dim3(kBandChunks, (unsigned)n_sig), dim3(256), 0, st, hist, L, part);
        hipLaunchKernelGGL(k_band_final, dim3((unsigned)((n_sig + 255) / 256)), dim3(256), 0, st, part, n_sig,
                           band_energy);
    }
    if (K >= kFirFftMinK && K <= kFftN / 2) {
        // long filters: overlap-save FFT convolution
        if (ws.fir_twiddle.ensure(sizeof(float2) * kFftN) || ws.fir_spec.ensure(sizeof(float2) * 8 * kFftN))
            return RT_ENOMEM;
        const size_t fshm = sizeof(float2) * kFftN;
        static bool fft_attr_set[kMaxDevices] = {};
        if (!raise_lds_limit(fft_attr_set, {(const void*)k_fir_spectrum, (const void*)k_fir_fft}, (int)fshm))
            return RT_EHIP;
        float2* tw = ws.fir_twiddle.as<float2>();
        float2* spec = ws.fir_spec.as<float2>();
        // the twiddle table is a constant: computed once per workspace buffer, outside stream
        // capture (a captured launch only runs when the graph is replayed)
        if (ws.fir_twiddle_done != (const void*)tw) {
            hipLaunchKernelGGL(k_fft_twiddles, dim3(kFftN / 256), dim3(256), 0, st, tw);
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
                ws.fir_twiddle_done = tw;
        }
        hipLaunchKernelGGL(k_fir_spectrum, dim3(8), dim3(kFftThreads), fshm, st, fir, K, tw, spec);
        const int64_t B = kFftN - K + 1;
        const int64_t n_seg = (L + B - 1) / B;
        dim3 fgrid((unsigned)((n_seg + 1) / 2), (unsigned)(n_rcv * 8));
        hipLaunchKernelGGL(k_fir_fft, fgrid, dim3(kFftThreads), fshm, st, hist, spec, tw, K, L, band_ir);
    } else {
        const int Kpad = K + 112;
        const int Smax = (K + 15 + 15 + 3) / 4;
        const int W = kFirOut + 4 * Smax + 16;
        const size_t shm = sizeof(float) * ((size_t)Kpad + (size_t)((W >> 4) + 2) * 20);
        RT_CHECK(shm <= 160 * 1024, RT_EINVAL, "rt_assemble_ir: FIR taps too long for LDS");
        static bool attr_set[kMaxDevices] = {};
        if (!raise_lds_limit(attr_set, {(const void*)k_fir_mfma}, 160 * 1024)) return RT_EHIP;
        dim3 grid((unsigned)((L + kFirOut - 1) / kFirOut), (unsigned)(n_rcv * 8));
        hipLaunchKernelGGL(k_fir_mfma, grid, dim3(256), shm, st, hist, fir, K, L, band_ir);
    }
    hipLaunchKernelGGL(k_sum_bands, dim3(nblk((int64_t)n_rcv * L)), dim3(256), 0, st, band_ir, L, n_rcv, ir);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
}  // namespace
}  // namespace rtac

extern "C" int rt_assemble_ir(const rt_scene* scene, const int32_t* is_key, const int32_t* is_count,
                              const double* is_dist, const int64_t* n_is, int64_t is_cap, int32_t max_reflections,
                              int64_t n_rays, int32_t n_rcv, const float* alpha, const float* beta, float c, float fs,
                              int64_t L, const float* fir, int32_t K, float* band_energy, float* hist, float* band_ir,
                              float* ir, void* stream) {
    CallStream call_stream((hipStream_t)stream);
    return assemble_common(scene, nullptr, is_key, is_count, is_dist, n_is, is_cap, max_reflections, n_rays, n_rcv,
                           alpha, beta, c, fs, L, fir, K, band_energy, hist, band_ir, ir, stream);
}

extern "C" int rt_assemble_batch(rt_batch* b, const int32_t* is_key, const int32_t* is_count, const double* is_dist,
                                 const int64_t* n_is, int64_t is_cap, int32_t max_reflections, const float* alpha,
                                 const float* beta, float c, float fs, int64_t L, const float* fir, int32_t K,
                                 float* band_energy, float* hist, float* band_ir, float* ir, void* stream) {
    CallStream call_stream((hipStream_t)stream);
    RT_CHECK(b, RT_EINVAL, "rt_assemble_batch: null batch");
    return assemble_common(b->ws_owner, b, is_key, is_count, is_dist, n_is, is_cap, max_reflections, b->n_rays,
                           b->n_rcv, alpha, beta, c, fs, L, fir, K, band_energy, hist, band_ir, ir, stream);
}

namespace rtac {
namespace {
int adjoint_common(const rt_scene* scene, const rt_batch* bt, const int32_t* is_key, const int32_t* is_count,
                   const double* is_dist, const int64_t* n_is, int64_t is_cap, int32_t max_reflections,
                   int64_t n_rays, int32_t n_rcv, const float* alpha, int32_t n_mat, const float* beta, float c,
                   float fs, int64_t L, const float* grad_band_energy, float* grad_alpha, void* stream) {
    int rc = check_is_args(scene, is_key, is_count, is_dist, n_is, is_cap, max_reflections, n_rays, bt ? 1 : n_rcv,
                           alpha, beta, c, fs, L);
    if (rc) {
        set_error("rt_band_energy_adjoint: %s", rt_last_error());
        return rc;
    }
    RT_CHECK(grad_band_energy && grad_alpha, RT_EINVAL, "rt_band_energy_adjoint: null gradient buffer");
    RT_CHECK(n_mat >= (bt ? bt->n_mat : scene->n_mat) && n_mat <= 4096, RT_EINVAL,
             "rt_band_energy_adjoint: n_mat must cover the materials (%d)", bt ? bt->n_mat : scene->n_mat);
    hipStream_t st = (hipStream_t)stream;
    rt_scene* s = const_cast<rt_scene*>(scene);
    const int64_t cap = is_cap > 0 ? is_cap : 1;
    const int nb = (int)nblk(cap, kAdjThreads);
    if (s->ws.asm_partial.ensure(sizeof(double) * (size_t)nb * n_mat * 8)) return RT_ENOMEM;
    IsArgs a = make_is_args(scene, is_key, is_count, is_dist, n_is, is_cap, max_reflections, n_rays, n_rcv, alpha,
                            beta, c, fs, L);
    if (bt) {
        a.rcv_job = bt->rcv_job;
        a.jobs = bt->jobs;
        a.scenes = bt->scenes;
    }
    double* part = s->ws.asm_partial.as<double>();
    hipLaunchKernelGGL(k_adjoint_partial, dim3(nb), dim3(kAdjThreads), 0, st, a, n_mat, grad_band_energy, part);
    hipLaunchKernelGGL(k_adjoint_final, dim3(nblk((int64_t)n_mat * 8 * kWave)), dim3(256), 0, st, part, nb, n_mat,
                       n_is, is_cap, grad_alpha);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
}  // namespace
}  // namespace rtac

extern "C" int rt_band_energy_adjoint(const rt_scene* scene, const int32_t* is_key, const int32_t* is_count,
                                      const double* is_dist, const int64_t* n_is, int64_t is_cap,
                                      int32_t max_reflections, int64_t n_rays, int32_t n_rcv, const float* alpha,
                                      int32_t n_mat, const float* beta, float c, float fs, int64_t L,
                                      const float* grad_band_energy, float* grad_alpha, void* stream) {
    CallStream call_stream((hipStream_t)stream);
    return adjoint_common(scene, nullptr, is_key, is_count, is_dist, n_is, is_cap, max_reflections, n_rays, n_rcv,
                          alpha, n_mat, beta, c, fs, L, grad_band_energy, grad_alpha, stream);
}

extern "C" int rt_adjoint_batch(rt_batch* b, const int32_t* is_key, const int32_t* is_count, const double* is_dist,
                                const int64_t* n_is, int64_t is_cap, int32_t max_reflections, const float* alpha,
                                const float* beta, float c, float fs, int64_t L, const float* grad_band_energy,
                                float* grad_alpha, void* stream) {
    CallStream call_stream((hipStream_t)stream);
    RT_CHECK(b, RT_EINVAL, "rt_adjoint_batch: null batch");
    return adjoint_common(b->ws_owner, b, is_key, is_count, is_dist, n_is, is_cap, max_reflections, b->n_rays,
                          b->n_rcv, alpha, b->n_mat, beta, c, fs, L, grad_band_energy, grad_alpha, stream);
}
