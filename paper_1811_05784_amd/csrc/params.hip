// Room-acoustic parameters from the per-band energy histogram of an impulse
// response: the perceptive factors the paper tabulates for the Orange theater
// (EDT, T30, SPL, C80, D50, Ts; Table 3), defined as in room acoustics
// practice (ISO 3382-1) on the histogram H[s] of energy per bin of 1/fs:
// origin s0 = first bin with energy in any band of the receiver; Schroeder
// curve EDC(s) = sum_{s' >= s} H[s'] in dB re EDC(s0), up to the last bin with
// energy; EDT and T30 = -60 / slope of the least-squares lines over
// 0..-10 dB and -5..-35 dB; C80, D50 with windows of floor(0.08 fs + 1/2)
// and floor(0.05 fs + 1/2) bins; Ts the energy centroid time; SPL = 10 log10 of the
// received energy re the emitted energy.  FP64 sums in a fixed order.
#include "common.h"

#include <cmath>

namespace rtac {
namespace {

constexpr int kPT = 256;   // threads per workgroup (one workgroup per receiver)
constexpr int kPItems = 8;

template <int N>
__device__ inline void block_sum(double (&v)[N], double (*red)[kPT]) {
    const int t = threadIdx.x;
    for (int k = 0; k < N; k++) red[k][t] = v[k];
    __syncthreads();
    for (int off = kPT / 2; off > 0; off >>= 1) {
        if (t < off)
            for (int k = 0; k < N; k++) red[k][t] += red[k][t + off];
        __syncthreads();
    }
    for (int k = 0; k < N; k++) v[k] = red[k][0];
    __syncthreads();
}

__device__ inline double slope_of(double n, double sx, double sy, double sxy, double sxx) {
    const double den = n * sxx - sx * sx;
    if (n < 2.0 || !(den > 0.0)) return NAN;
    return (n * sxy - sx * sy) / den;
}

__global__ void __launch_bounds__(kPT) k_room_params(const float* __restrict__ hist, int64_t L, double fs, int64_t n80,
                                                     int64_t n50, double* __restrict__ out) {
    __shared__ double red[12][kPT];
    __shared__ int64_t s_min[kPT], s_max[kPT];
    __shared__ double scan_s[kPT];
    const int t = threadIdx.x;
    const int m = blockIdx.x;
    const float* hm = hist + (int64_t)m * 8 * L;
    double* om = out + (int64_t)m * 8 * 6;
    // origin: first bin with energy in any band
    int64_t first = L;
    for (int64_t s = t; s < L; s += kPT) {
        bool any = false;
        for (int b = 0; b < 8; b++) any |= hm[(int64_t)b * L + s] > 0.f;
        if (any) {
            first = s;
            break;
        }
    }
    s_min[t] = first;
    __syncthreads();
    for (int off = kPT / 2; off > 0; off >>= 1) {
        if (t < off && s_min[t + off] < s_min[t]) s_min[t] = s_min[t + off];
        __syncthreads();
    }
    const int64_t s0 = s_min[0];
    __syncthreads();
    for (int b = 0; b < 8; b++) {
        const float* h = hm + (int64_t)b * L;
        if (s0 >= L) {
            if (t < 6) om[b * 6 + t] = NAN;
            continue;
        }
        // pass 1: totals, early windows, centroid numerator, last bin with energy
        double acc[4] = {0.0, 0.0, 0.0, 0.0};   // tot, sum (s - s0) H, E50, E80
        int64_t last = -1;
        for (int64_t s = s0 + t; s < L; s += kPT) {
            const double v = (double)h[s];
            const int64_t k = s - s0;
            acc[0] += v;
            acc[1] += (double)k * v;
            if (k < n50) acc[2] += v;
            if (k < n80) acc[3] += v;
            if (v > 0.0) last = s;
        }
        block_sum(acc, red);
        s_max[t] = last;
        __syncthreads();
        for (int off = kPT / 2; off > 0; off >>= 1) {
            if (t < off && s_max[t + off] > s_max[t]) s_max[t] = s_max[t + off];
            __syncthreads();
        }
        const int64_t s_last = s_max[0];
        __syncthreads();
        const double tot = acc[0];
        // pass 2: Schroeder curve over [s0, s_last], regression sums of both windows
        double rs[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, INFINITY};   // EDT n,sx,sy,sxy,sxx; T30 ...; min dB
        double carry = 0.0;   // energy of the bins before the current chunk
        if (tot > 0.0) {
            for (int64_t base = s0; base <= s_last; base += (int64_t)kPT * kPItems) {
                const int64_t i0 = base + (int64_t)t * kPItems;
                double v[kPItems], own = 0.0;
                for (int j = 0; j < kPItems; j++) {
                    v[j] = (i0 + j <= s_last) ? (double)h[i0 + j] : 0.0;
                    own += v[j];
                }
                // exclusive scan of the thread totals (fixed order: Hillis-Steele in LDS)
                scan_s[t] = own;
                __syncthreads();
                for (int off = 1; off < kPT; off <<= 1) {
                    const double x = t >= off ? scan_s[t - off] : 0.0;
                    __syncthreads();
                    scan_s[t] += x;
                    __syncthreads();
                }
                double before = carry + scan_s[t] - own;
                const double chunk = scan_s[kPT - 1];
                __syncthreads();
                for (int j = 0; j < kPItems; j++) {
                    const int64_t s = i0 + j;
                    if (s <= s_last) {
                        const double edc = tot - before;
                        const double db = 10.0 * log10(edc / tot);
                        const double x = (double)(s - s0) / fs;
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
                carry += chunk;
            }
        }
        // reduce the regression sums (min of the dB values separately)
        double sums[10];
        for (int k = 0; k < 10; k++) sums[k] = rs[k];
        block_sum(sums, red);
        red[0][t] = rs[10];
        __syncthreads();
        for (int off = kPT / 2; off > 0; off >>= 1) {
            if (t < off && red[0][t + off] < red[0][t]) red[0][t] = red[0][t + off];
            __syncthreads();
        }
        const double low = red[0][0];
        __syncthreads();
        if (t == 0) {
            double* o = om + b * 6;
            if (!(tot > 0.0)) {
                for (int k = 0; k < 6; k++) o[k] = NAN;
            } else {
                const double se = slope_of(sums[0], sums[1], sums[2], sums[3], sums[4]);
                const double st = slope_of(sums[5], sums[6], sums[7], sums[8], sums[9]);
                o[0] = low <= -10.0 ? -60.0 / se : NAN;
                o[1] = low <= -35.0 ? -60.0 / st : NAN;
                const double late = tot - acc[3];
                o[2] = late > 0.0 ? 10.0 * log10(acc[3] / late) : NAN;
                o[3] = acc[2] / tot;
                o[4] = acc[1] / fs / tot;
                o[5] = 10.0 * log10(tot);
            }
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace rtac

using namespace rtac;

extern "C" int rt_room_params(const float* hist, int32_t n_rcv, int64_t L, float fs, double* params, void* stream) {
    RT_CHECK(n_rcv >= 0 && L >= 1 && fs > 0.f, RT_EINVAL, "rt_room_params: bad sizes");
    RT_CHECK(n_rcv == 0 || (hist && params), RT_EINVAL, "rt_room_params: null argument");
    if (n_rcv == 0) return RT_OK;
    const int64_t n80 = (int64_t)std::floor(0.08 * (double)fs + 0.5);
    const int64_t n50 = (int64_t)std::floor(0.05 * (double)fs + 0.5);
    hipLaunchKernelGGL(k_room_params, dim3((unsigned)n_rcv), dim3(kPT), 0, (hipStream_t)stream, hist, L, (double)fs,
                       n80, n50, params);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
