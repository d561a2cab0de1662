// Stable LSD radix sort of (uint64 key, uint32 value) pairs and an exclusive
// scan, both able to read the element count from device memory so that a
// producer kernel's count never has to come back to the host.
//
// Radix sort: 8-bit digits; per pass (1) per-tile digit histograms, (2) one
// workgroup per digit scans that digit's row of tile counts and records the
// row total, (3) each tile scans the 256 row totals into digit bases, ranks
// its keys stably (wave ballots on the 8 digit bits give each lane its peers,
// per-wave counts are combined in LDS in wave order) and scatters.
#include "common.h"

namespace rtac {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 4;
constexpr int kTile = kThreads * kItems;   // 1024 keys per workgroup
constexpr int kWaves = kThreads / kWave;

__device__ inline int64_t count_of(const int64_t* n_dev, int64_t cap) {
    if (!n_dev) return cap;
    int64_t n = *n_dev;
    return n < 0 ? 0 : (n > cap ? cap : n);
}

// Tiles holding at least one of the n keys; tables are laid out digit-major
// over these tiles only: hist[d * used + tile].
__device__ inline int used_tiles(int64_t n) { return (int)((n + kTile - 1) / kTile); }

__global__ void __launch_bounds__(kThreads) k_digit_hist(const uint64_t* __restrict__ keys, int64_t cap,
                                                          const int64_t* n_dev, int shift, uint32_t dmask,
                                                          uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    const int64_t n = count_of(n_dev, cap);
    const int used = used_tiles(n);
    if ((int)blockIdx.x >= used) return;
    h[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int i = 0; i < kItems; i++) {
        int64_t idx = base + (int64_t)i * kThreads + tid;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & dmask], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * used + blockIdx.x] = h[tid];
}

// In-place exclusive scan of a[0..len) by one workgroup of 1024 threads,
// 8192 elements per round: each thread scans 8 consecutive elements, waves
// scan their thread totals with lane shuffles, one wave scans the 16 wave
// totals (two barriers per round).
// len = len_mul * used_tiles(n) when n_dev is given, else len_fixed.
__global__ void __launch_bounds__(1024) k_scan_single(uint32_t* __restrict__ a, int64_t len_fixed,
                                                       const int64_t* n_dev, int64_t cap, int len_mul,
                                                       uint32_t* __restrict__ total) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t len = n_dev ? (int64_t)len_mul * used_tiles(count_of(n_dev, cap)) : len_fixed;
    uint32_t carry = 0;
    for (int64_t base = 0; base < len; base += 8192) {
        const int64_t i0 = base + 8 * (int64_t)tid;
        uint32_t v[8];
        uint32_t t = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            v[j] = i0 + j < len ? a[i0 + j] : 0u;
            t += v[j];
        }
        uint32_t incl = t;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t x = __shfl_up(incl, off);
            if (lane >= off) incl += x;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        if (wave == 0) {
            uint32_t w = lane < 16 ? wsum[lane] : 0u;
            uint32_t wi = w;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const uint32_t x = __shfl_up(wi, off);
                if (lane >= off) wi += x;
            }
            if (lane < 16) wsum[lane] = wi - w;   // exclusive wave offsets
            if (lane == 15) carry_s = wi;         // round total
        }
        __syncthreads();
        uint32_t run = carry + wsum[wave] + incl - t;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if (i0 + j < len) a[i0 + j] = run;
            run += v[j];
        }
        carry += carry_s;
        __syncthreads();
    }
    if (total && tid == 0) *total = carry;
}

// Row d of the digit-major table (tile counts of digit d) -> exclusive
// prefix over tiles, in place; rowtot[d] = the row's total.
__global__ void __launch_bounds__(kThreads) k_row_scan(uint32_t* __restrict__ hist, int64_t cap, const int64_t* n_dev,
                                                        uint32_t* __restrict__ rowtot) {
    __shared__ uint32_t wsum[kWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int used = used_tiles(count_of(n_dev, cap));
    uint32_t* row = hist + (int64_t)blockIdx.x * used;
    uint32_t carry = 0;
    for (int base = 0; base < used; base += kThreads * 4) {
        const int i0 = base + 4 * tid;
        uint32_t v[4], t = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            v[j] = i0 + j < used ? row[i0 + j] : 0u;
            t += v[j];
        }
        uint32_t incl = t;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t x = __shfl_up(incl, off);
            if (lane >= off) incl += x;
        }
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = 0, round = 0;
#pragma unroll
        for (int w = 0; w < kWaves; w++) {
            before += w < wave ? wsum[w] : 0u;
            round += wsum[w];
        }
        uint32_t run = carry + before + incl - t;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (i0 + j < used) row[i0 + j] = run;
            run += v[j];
        }
        carry += round;
        __syncthreads();
    }
    if (tid == 0) rowtot[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kThreads) k_rank_scatter(const uint64_t* __restrict__ kin,
                                                            const uint32_t* __restrict__ vin,
                                                            uint64_t* __restrict__ kout,
                                                            uint32_t* __restrict__ vout, int64_t cap,
                                                            const int64_t* n_dev, int shift, uint32_t dmask,
                                                            const uint32_t* __restrict__ offs,
                                                            const uint32_t* __restrict__ rowtot) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t wtot[kWaves];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const int64_t n = count_of(n_dev, cap);
    const int64_t base = (int64_t)blockIdx.x * kTile;
    if (base >= n) return;   // whole workgroup leaves together
    {
        // digit bases: exclusive scan of the 256 row totals
        const uint32_t t = rowtot[tid];
        uint32_t incl = t;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t x = __shfl_up(incl, off);
            if (lane >= off) incl += x;
        }
        if (lane == kWave - 1) wtot[wave] = incl;
        __syncthreads();
        uint32_t before = 0;
#pragma unroll
        for (int w = 0; w < kWaves; w++) before += w < wave ? wtot[w] : 0u;
        run[tid] = offs[(int64_t)tid * used_tiles(n) + blockIdx.x] + before + incl - t;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = 0; i < kItems; i++) {
        const int64_t idx = base + (int64_t)i * kThreads + tid;
        const bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0ull;
        uint32_t val = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
        uint32_t d = (uint32_t)(key >> shift) & dmask;
#pragma unroll
        for (int w = 0; w < kWaves; w++) wcnt[w][tid] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bal = __ballot(on);
            peers &= on ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t r = run[tid];
#pragma unroll
            for (int w = 0; w < kWaves; w++) {
                uint32_t c = wcnt[w][tid];
                wcnt[w][tid] = r;
                r += c;
            }
            run[tid] = r;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = wcnt[wave][d] + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
    }
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(kScanThreads) k_block_sums(const uint32_t* __restrict__ in, int64_t cap,
                                                              const int64_t* n_dev, uint32_t* __restrict__ sums) {
    __shared__ uint32_t red[kScanThreads];
    const int64_t n = count_of(n_dev, cap);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; i++)
        if (base + i < n) s += in[base + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kScanThreads) k_block_scan(const uint32_t* __restrict__ in, int64_t cap,
                                                              const int64_t* n_dev,
                                                              const uint32_t* __restrict__ block_offs,
                                                              const uint32_t* __restrict__ total,
                                                              uint32_t* __restrict__ out) {
    __shared__ uint32_t sc[kScanThreads];
    const int64_t n = count_of(n_dev, cap);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; i++) {
        v[i] = base + i < n ? in[base + i] : 0u;
        s += v[i];
    }
    sc[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint32_t t = (int)threadIdx.x >= off ? sc[threadIdx.x - off] : 0u;
        __syncthreads();
        sc[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t r = block_offs[blockIdx.x] + (threadIdx.x ? sc[threadIdx.x - 1] : 0u);
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = r;
        r += v[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total;
}

}  // namespace

int radix_sort_pairs(Workspace& ws, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t cap,
                     const int64_t* n_dev, int begin_bit, int end_bit, hipStream_t st, int* out_index,
                     bool iota_values) {
    *out_index = 0;
    if (cap <= 0) return RT_OK;
    RT_CHECK(begin_bit >= 0 && end_bit <= 64, RT_EINVAL, "radix sort: bits [%d, %d) out of range", begin_bit,
             end_bit);
    const int nblocks = (int)((cap + kTile - 1) / kTile);
    const int64_t hlen = (int64_t)256 * nblocks;
    if (ws.sort_hist.ensure(sizeof(uint32_t) * (size_t)(hlen + 256))) return RT_ENOMEM;
    uint32_t* hist = ws.sort_hist.as<uint32_t>();
    uint32_t* rowtot = hist + hlen;
    uint64_t* kin = k0;
    uint32_t* vin = v0;
    uint64_t* kout = k1;
    uint32_t* vout = v1;
    int cur = 0;
    bool first = true;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        // the last digit ends at end_bit
        const uint32_t dmask = end_bit - shift >= 8 ? 255u : (1u << (end_bit - shift)) - 1u;
        hipLaunchKernelGGL(k_digit_hist, dim3(nblocks), dim3(kThreads), 0, st, kin, cap, n_dev, shift, dmask, hist);
        hipLaunchKernelGGL(k_row_scan, dim3(256), dim3(kThreads), 0, st, hist, cap, n_dev, rowtot);
        hipLaunchKernelGGL(k_rank_scatter, dim3(nblocks), dim3(kThreads), 0, st, kin,
                           first && iota_values ? (const uint32_t*)nullptr : vin, kout, vout, cap, n_dev,
                           shift, dmask, hist, rowtot);
        first = false;
        std::swap(kin, kout);
        std::swap(vin, vout);
        cur ^= 1;
    }
    RT_HIP(hipGetLastError());
    *out_index = cur;
    return RT_OK;
}

int exclusive_scan_u32(Workspace& ws, const uint32_t* in, uint32_t* out, int64_t cap, const int64_t* n_dev,
                       hipStream_t st) {
    const int nblocks = (int)((cap + kScanTile - 1) / kScanTile);
    const int nb = nblocks > 0 ? nblocks : 1;
    if (ws.scan_tmp.ensure(sizeof(uint32_t) * (size_t)(nb + 1))) return RT_ENOMEM;
    uint32_t* sums = ws.scan_tmp.as<uint32_t>();
    hipLaunchKernelGGL(k_block_sums, dim3(nb), dim3(kScanThreads), 0, st, in, cap, n_dev, sums);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, sums, (int64_t)nb, (const int64_t*)nullptr,
                       (int64_t)0, 0, sums + nb);
    hipLaunchKernelGGL(k_block_scan, dim3(nb), dim3(kScanThreads), 0, st, in, cap, n_dev, sums, sums + nb, out);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rtac

extern "C" int rt_debug_radix_sort(uint64_t* keys, uint32_t* order, int64_t cap, const int64_t* n_dev,
                                   int32_t begin_bit, int32_t end_bit, void* stream) {
    using namespace rtac;
    RT_CHECK(keys && order, RT_EINVAL, "rt_debug_radix_sort: null keys or order");
    RT_CHECK(cap >= 0 && cap < ((int64_t)1 << 32), RT_EINVAL, "rt_debug_radix_sort: cap out of range");
    RT_CHECK(begin_bit >= 0 && begin_bit < end_bit && end_bit <= 64, RT_EINVAL,
             "rt_debug_radix_sort: bits [%d, %d) out of range", begin_bit, end_bit);
    if (cap == 0) return RT_OK;
    hipStream_t st = (hipStream_t)stream;
    CallStream call_stream(st);
    Workspace ws;
    Buf k1, v0;
    int rc = RT_OK;
    if (k1.ensure(sizeof(uint64_t) * (size_t)cap) || v0.ensure(sizeof(uint32_t) * (size_t)cap)) {
        rc = RT_ENOMEM;
    } else {
        int which = 0;
        rc = radix_sort_pairs(ws, keys, v0.as<uint32_t>(), k1.as<uint64_t>(), order, cap, n_dev, begin_bit, end_bit,
                              st, &which, true);
        if (rc == RT_OK && which == 0) {
            // the result is in (keys, v0): the order goes to `order`
            if (hipMemcpyAsync(order, v0.p, sizeof(uint32_t) * (size_t)cap, hipMemcpyDeviceToDevice, st) !=
                hipSuccess) {
                set_error("rt_debug_radix_sort: copy failed");
                rc = RT_EHIP;
            }
        } else if (rc == RT_OK) {
            // the result is in (k1, order): the keys go back to `keys`
            if (hipMemcpyAsync(keys, k1.p, sizeof(uint64_t) * (size_t)cap, hipMemcpyDeviceToDevice, st) !=
                hipSuccess) {
                set_error("rt_debug_radix_sort: copy failed");
                rc = RT_EHIP;
            }
        }
    }
    k1.release();
    v0.release();
    ws.release_all();
    return rc;
}

