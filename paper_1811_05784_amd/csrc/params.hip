// Room-acoustic parameters from the per-band energy histogram of an impulse
// response: the perceptive factors the paper tabulates for the Orange theater
// (EDT, T30, SPL, C80, D50, Ts; Table 3), defined as in room acoustics
// practice (ISO 3382-1) on the histogram H[s] of energy per bin of 1/fs:
// origin s0 = first bin with energy in any band of the receiver; Schroeder
// curve EDC(s) = sum_{s' >= s} H[s'] in dB re EDC(s0), up to the last bin with
// energy; EDT and T30 = -60 / slope of the least-squares lines over
// 0..-10 dB and -5..-35 dB; C80, D50 with windows of floor(0.08 fs + 1/2)
// and floor(0.05 fs + 1/2) bins; Ts the energy centroid time; SPL = 10 log10 of the
// received energy re the emitted energy.
//
// The histogram is read twice, in chunks of kChunk bins spread over the whole
// chip (a receiver's 8 bands x L bins would otherwise sit on a few compute
// units): pass 1 sums every chunk; a small per-band step turns the chunk sums
// into the origin, the total and the chunk prefix of the Schroeder curve;
// pass 2 scans each chunk from its prefix and accumulates the regression
// sums; a last step reduces them.  FP64 sums, each in a fixed order.
#include "common.h"

#include <cmath>
#include <mutex>

namespace rtac {
namespace {

constexpr int kPT = 256;                   // threads per chunk workgroup
constexpr int kPW = kPT / kWave;
constexpr int kPItems = 16;                // bins per thread
constexpr int64_t kChunk = (int64_t)kPT * kPItems;
constexpr int kNSum = 11;                  // regression sums (2 x 5) + lowest dB
constexpr double kRatio36 = 2.5118864315095795e-4;   // 10^-3.6: a bin this far down is below -36 dB

struct ChunkSums {
    double h, sh;            // sum H, sum s H (global bin index s)
    int64_t first, last;     // first / last bin with energy (L / -1: none)
};

struct BandInfo {
    int64_t s0, last;        // origin (L: the receiver has no energy), last bin with energy in the band
    double tot, e50, e80, shift;   // total, first n50 / n80 bins from s0, sum (s - s0) H
};

__device__ inline double wave_sum(double v) {
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum of each of N values over the workgroup: wave butterflies, then the
// wave totals in wave order.
template <int N>
__device__ inline void block_sum(double (&v)[N], double (*red)[kPW]) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int k = 0; k < N; k++) v[k] = wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < N; k++) red[k][w] = v[k];
    __syncthreads();
    for (int k = 0; k < N; k++) {
        double t = 0.0;
        for (int j = 0; j < kPW; j++) t += red[k][j];
        v[k] = t;
    }
    __syncthreads();
}

__device__ inline int64_t wave_min_i64(int64_t v) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

__device__ inline int64_t block_min_i64(int64_t v, int64_t* red) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    v = wave_min_i64(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    int64_t m = red[0];
    for (int j = 1; j < kPW; j++) m = red[j] < m ? red[j] : m;
    __syncthreads();
    return m;
}

// pass 1: one workgroup per (receiver, band, chunk)
__global__ void __launch_bounds__(kPT) k_rp_chunks(const float* __restrict__ hist, int64_t L, int64_t nc,
                                                   ChunkSums* __restrict__ cs) {
    __shared__ double red[2][kPW];
    __shared__ int64_t red_i[kPW];
    const int64_t g = blockIdx.x;                 // (m * 8 + b) * nc + c
    const int64_t c = g % nc, mb = g / nc;
    const float* h = hist + mb * L;
    const int64_t lo = c * kChunk, hi = lo + kChunk < L ? lo + kChunk : L;
    double acc[2] = {0.0, 0.0};
    int64_t first = L, last = -1;
    for (int64_t s = lo + threadIdx.x; s < hi; s += kPT) {
        const double v = (double)h[s];
        acc[0] += v;
        acc[1] += (double)s * v;
        if (v > 0.0) {
            first = s < first ? s : first;
            last = s;
        }
    }
    block_sum(acc, red);
    first = block_min_i64(first, red_i);
    last = -block_min_i64(-last, red_i);
    if (threadIdx.x == 0) cs[g] = ChunkSums{acc[0], acc[1], first, last};
}

// Sum of H over [lo, hi) of one band by one wavefront (fixed order).
__device__ inline double wave_range_sum(const float* h, int64_t lo, int64_t hi) {
    double v = 0.0;
    for (int64_t s = lo + (threadIdx.x & (kWave - 1)); s < hi; s += kWave) v += (double)h[s];
    return wave_sum(v);
}

// per band: one wavefront per (receiver, band)
__global__ void __launch_bounds__(kWave) k_rp_band(const float* __restrict__ hist, int64_t L, int64_t nc,
                                                   int64_t n50, int64_t n80, const ChunkSums* __restrict__ cs,
                                                   double* __restrict__ prefix, BandInfo* __restrict__ bi) {
    const int lane = threadIdx.x;
    const int64_t mb = blockIdx.x, m = mb >> 3;
    // origin over the 8 bands of the receiver
    int64_t s0 = L;
    for (int64_t i = lane; i < 8 * nc; i += kWave) {
        const int64_t f = cs[m * 8 * nc + i].first;
        s0 = f < s0 ? f : s0;
    }
    s0 = wave_min_i64(s0);
    // chunk prefix of the band (exclusive, in chunk order) and its last bin
    const ChunkSums* c = cs + mb * nc;
    double* pre = prefix + mb * nc;
    double run = 0.0, sh = 0.0;
    int64_t last = -1;
    for (int64_t base = 0; base < nc; base += kWave) {
        const int64_t i = base + lane;
        const double v = i < nc ? c[i].h : 0.0;
        double incl = v;
        for (int off = 1; off < kWave; off <<= 1) {
            const double x = __shfl_up(incl, off);
            if (lane >= off) incl += x;
        }
        if (i < nc) {
            pre[i] = run + (incl - v);
            sh += c[i].sh;
            last = c[i].last > last ? c[i].last : last;
        }
        run += __shfl(incl, kWave - 1);
    }
    sh = wave_sum(sh);
    last = -wave_min_i64(-last);
    const double tot = run;
    // early windows: every bin before s0 is empty, so E[s0, s0 + n) = sum H[0, s0 + n)
    double e[2] = {0.0, 0.0};
    const int64_t ends[2] = {s0 + n50, s0 + n80};
    for (int k = 0; k < 2; k++) {
        const int64_t end = ends[k] < L ? ends[k] : L;
        if (s0 >= L || end <= 0) continue;
        const int64_t ce = (end - 1) / kChunk;            // chunk holding the last bin of the window
        e[k] = pre[ce] + wave_range_sum(hist + mb * L, ce * kChunk, end);
    }
    if (lane == 0) bi[mb] = BandInfo{s0, last, tot, e[0], e[1], sh - (double)s0 * tot};
}

// pass 2: Schroeder curve of one chunk from its prefix; regression sums
__global__ void __launch_bounds__(kPT) k_rp_edc(const float* __restrict__ hist, int64_t L, int64_t nc, double fs,
                                                const double* __restrict__ prefix, const BandInfo* __restrict__ bi,
                                                double* __restrict__ part) {
    __shared__ double red[kNSum][kPW];
    __shared__ double wtot[kPW];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    const int64_t g = blockIdx.x;
    const int64_t c = g % nc, mb = g / nc;
    const BandInfo B = bi[mb];
    double rs[kNSum] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, INFINITY};   // EDT n,sx,sy,sxy,sxx; T30 ...; min dB
    const int64_t lo = c * kChunk;
    double* out = part + g * kNSum;
    if (B.s0 >= L || !(B.tot > 0.0) || lo > B.last || lo + kChunk <= B.s0) {
        if (t < kNSum) out[t] = rs[t];
        return;
    }
    const float* h = hist + mb * L;
    const int64_t i0 = lo + (int64_t)t * kPItems;
    double v[kPItems], own = 0.0;
    for (int j = 0; j < kPItems; j++) {
        v[j] = (i0 + j < L) ? (double)h[i0 + j] : 0.0;
        own += v[j];
    }
    double incl = own;
    for (int off = 1; off < kWave; off <<= 1) {
        const double x = __shfl_up(incl, off);
        if (lane >= off) incl += x;
    }
    if (lane == kWave - 1) wtot[w] = incl;
    __syncthreads();
    double before = prefix[g];
    for (int j = 0; j < w; j++) before += wtot[j];
    before += incl - own;
    for (int j = 0; j < kPItems; j++) {
        const int64_t s = i0 + j;
        if (s >= B.s0 && s <= B.last) {
            const double edc = B.tot - before;
            const double ratio = edc / B.tot;
            if (!(ratio >= kRatio36)) {
                // below -36 dB: outside both windows; only `lowest dB <= -35` matters
                rs[10] = fmin(rs[10], -1000.0);
                before += v[j];
                continue;
            }
            const double db = 10.0 * log10(ratio);
            const double x = (double)(s - B.s0) / fs;
            if (db < rs[10]) rs[10] = db;
            if (db <= 0.0 && db >= -10.0) {
                rs[0] += 1.0;
                rs[1] += x;
                rs[2] += db;
                rs[3] += x * db;
                rs[4] += x * x;
            }
            if (db <= -5.0 && db >= -35.0) {
                rs[5] += 1.0;
                rs[6] += x;
                rs[7] += db;
                rs[8] += x * db;
                rs[9] += x * x;
            }
        }
        before += v[j];
    }
    double low = rs[10];
    for (int off = kWave / 2; off > 0; off >>= 1) low = fmin(low, __shfl_xor(low, off));
    double sums[10];
    for (int k = 0; k < 10; k++) sums[k] = rs[k];
    if (lane == 0) red[10][w] = low;
    block_sum(sums, red);   // its first barrier also publishes red[10]
    if (t == 0) {
        for (int k = 0; k < 10; k++) out[k] = sums[k];
        double m = red[10][0];
        for (int j = 1; j < kPW; j++) m = fmin(m, red[10][j]);
        out[10] = m;
    }
}

__device__ inline double slope_of(double n, double sx, double sy, double sxy, double sxx) {
    const double den = n * sxx - sx * sx;
    if (n < 2.0 || !(den > 0.0)) return NAN;
    return (n * sxy - sx * sy) / den;
}

// final: one wavefront per (receiver, band) reduces the chunk sums in chunk order
__global__ void __launch_bounds__(kWave) k_rp_final(int64_t L, int64_t nc, double fs, const BandInfo* __restrict__ bi,
                                                    const double* __restrict__ part, double* __restrict__ params) {
    const int lane = threadIdx.x;
    const int64_t mb = blockIdx.x;
    const BandInfo B = bi[mb];
    double* o = params + mb * 6;
    if (B.s0 >= L || !(B.tot > 0.0)) {
        if (lane < 6) o[lane] = NAN;
        return;
    }
    double acc = lane < 10 ? 0.0 : INFINITY;
    if (lane < kNSum)
        for (int64_t c = 0; c < nc; c++) {
            const double x = part[(mb * nc + c) * kNSum + lane];
            acc = lane < 10 ? acc + x : fmin(acc, x);
        }
    double s[kNSum];
    for (int k = 0; k < kNSum; k++) s[k] = __shfl(acc, k);
    if (lane == 0) {
        const double se = slope_of(s[0], s[1], s[2], s[3], s[4]);
        const double st = slope_of(s[5], s[6], s[7], s[8], s[9]);
        const double low = s[10];
        o[0] = low <= -10.0 ? -60.0 / se : NAN;
        o[1] = low <= -35.0 ? -60.0 / st : NAN;
        const double late = B.tot - B.e80;
        o[2] = late > 0.0 ? 10.0 * log10(B.e80 / late) : NAN;
        o[3] = B.e50 / B.tot;
        o[4] = B.shift / fs / B.tot;
        o[5] = 10.0 * log10(B.tot);
    }
}

}  // namespace
}  // namespace rtac

using namespace rtac;

namespace rtac {
namespace {

// Scratch of one call: chunk sums, chunk prefixes, band facts, pass-2 sums.
struct RpScratch {
    size_t b_cs, b_pre, b_bi, b_part;
    size_t total() const { return b_cs + b_pre + b_bi + b_part; }
};

RpScratch rp_scratch_size(int64_t nb, int64_t nc) {
    RpScratch s;
    s.b_cs = sizeof(ChunkSums) * nb * nc;
    s.b_pre = sizeof(double) * nb * nc;
    s.b_bi = sizeof(BandInfo) * nb;
    s.b_part = sizeof(double) * kNSum * nb * nc;
    return s;
}

int rp_check(const float* hist, int32_t n_rcv, int64_t L, float fs, double* params, const char* who) {
    RT_CHECK(n_rcv >= 0 && L >= 1 && fs > 0.f, RT_EINVAL, "%s: bad sizes", who);
    RT_CHECK(n_rcv == 0 || (hist && params), RT_EINVAL, "%s: null argument", who);
    const int64_t nc = (L + kChunk - 1) / kChunk;
    RT_CHECK((int64_t)n_rcv * 8 * nc < ((int64_t)1 << 31), RT_EINVAL, "%s: histogram too large", who);
    return RT_OK;
}

// The four passes on a scratch area of rp_scratch_size(n_rcv * 8, chunks) bytes.
void rp_launch(const float* hist, int32_t n_rcv, int64_t L, float fs, double* params, char* ws, hipStream_t st) {
    const int64_t nb = (int64_t)n_rcv * 8;
    const int64_t nc = (L + kChunk - 1) / kChunk;
    const int64_t n80 = (int64_t)std::floor(0.08 * (double)fs + 0.5);
    const int64_t n50 = (int64_t)std::floor(0.05 * (double)fs + 0.5);
    const RpScratch sz = rp_scratch_size(nb, nc);
    ChunkSums* cs = reinterpret_cast<ChunkSums*>(ws);
    double* pre = reinterpret_cast<double*>(ws + sz.b_cs);
    BandInfo* bi = reinterpret_cast<BandInfo*>(ws + sz.b_cs + sz.b_pre);
    double* part = reinterpret_cast<double*>(ws + sz.b_cs + sz.b_pre + sz.b_bi);
    // every scratch element is written before it is read within the call
    hipLaunchKernelGGL(k_rp_chunks, dim3((unsigned)(nb * nc)), dim3(kPT), 0, st, hist, L, nc, cs);
    hipLaunchKernelGGL(k_rp_band, dim3((unsigned)nb), dim3(kWave), 0, st, hist, L, nc, n50, n80, cs, pre, bi);
    hipLaunchKernelGGL(k_rp_edc, dim3((unsigned)(nb * nc)), dim3(kPT), 0, st, hist, L, nc, (double)fs, pre, bi, part);
    hipLaunchKernelGGL(k_rp_final, dim3((unsigned)nb), dim3(kWave), 0, st, L, nc, (double)fs, bi, part, params);
}

// Fixed scratch of rt_room_params_noalloc: one copy per GPU, held until the
// process ends.  Host code reaches it only through the per-device address
// returned by hipGetSymbolAddress (the symbol itself is a host-side stand-in).
constexpr size_t kRpScratchMax = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kRpScratchMax];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch`, looked up once per device (with
// that device current: the caller's).
int rp_scratch_ptr(char** out) {
    int dev = 0;
    RT_HIP(hipGetDevice(&dev));
    RT_CHECK(dev >= 0 && dev < kMaxDevices, RT_EINVAL, "rt_room_params_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        RT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        RT_CHECK(p != nullptr, RT_EHIP, "rt_room_params_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return RT_OK;
}

}  // namespace
}  // namespace rtac

using namespace rtac;

extern "C" int rt_room_params(const float* hist, int32_t n_rcv, int64_t L, float fs, double* params, void* stream) {
    if (int rc = rp_check(hist, n_rcv, L, fs, params, "rt_room_params")) return rc;
    if (n_rcv == 0) return RT_OK;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = rp_scratch_size((int64_t)n_rcv * 8, (L + kChunk - 1) / kChunk).total();
    char* ws = nullptr;
    RT_HIP(hipMallocAsync((void**)&ws, bytes, st));
    rp_launch(hist, n_rcv, L, fs, params, ws, st);
    const hipError_t le = hipGetLastError();
    RT_HIP(hipFreeAsync(ws, st));
    RT_HIP(le);
    return RT_OK;
}

extern "C" int rt_room_params_noalloc(const float* hist, int32_t n_rcv, int64_t L, float fs, double* params,
                                      void* stream) {
    if (int rc = rp_check(hist, n_rcv, L, fs, params, "rt_room_params_noalloc")) return rc;
    const size_t bytes = rp_scratch_size((int64_t)n_rcv * 8, (L + kChunk - 1) / kChunk).total();
    RT_CHECK(bytes <= kRpScratchMax, RT_ECAPACITY,
             "rt_room_params_noalloc: %d receivers x %lld bins need %zu bytes of scratch, above the fixed %zu",
             n_rcv, (long long)L, bytes, kRpScratchMax);
    if (n_rcv == 0) return RT_OK;
    char* ws = nullptr;
    if (int rc = rp_scratch_ptr(&ws)) return rc;
    rp_launch(hist, n_rcv, L, fs, params, ws, (hipStream_t)stream);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
