// Image sources from detected rays (rt_collect_image_sources).
//
// A detected ray, pushed back along its last direction, lands on a point
// image source; all rays with the same reflection sequence land on the same
// one and the receiver counts n of them (section "Image-sources").  The key
// of a detection (ray, k, m) is (m, k, plane ids hit on segments 0..k-1).
// Keys are hashed (64-bit mix), the low 48 bits sorted (stable radix sort,
// six 8-bit passes), and split into groups wherever the hash changes or a
// full comparison of the sequences differs.  Equal 48-bit hashes of
// different keys (about n^2 / 2^49: 1e-3 for 10^6 distinct keys) are
// resolved by a per-run insertion sort on the full key, so grouping is exact
// at any hash width; a wide hash keeps those runs, and the single thread that
// re-sorts each of them, away from heavily detected keys.  Each
// group's position is the source mirrored through its planes in order (FP64).
#include "common.h"

namespace rtac {

namespace {

int g_hash_bits = 48;   // sorted hash width (keys are compared in full); the test hook lowers it

__device__ inline uint64_t mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

struct CollectArgs {
    const int32_t* hit_seq;
    const int32_t* det;
    const int64_t* n_det;
    int64_t det_cap;
    int64_t n_rays;
    int32_t R1;
    int32_t n_rcv;
    const int32_t* tri_plane;
    int64_t n_tri;
    // batched calls: global receiver row -> job -> scene
    const int32_t* rcv_job;
    const DevJob* jobs;
    const DevScene* scenes;
};

__device__ inline int64_t det_count(const CollectArgs& a) {
    int64_t n = *a.n_det;
    if (n < 0) n = 0;
    return n > a.det_cap ? a.det_cap : n;
}

// Detections are validated here; an invalid row gets k = -1 (key of its own).
__device__ inline bool det_row(const CollectArgs& a, int64_t i, int32_t& ray, int32_t& k, int32_t& m) {
    ray = a.det[3 * i];
    k = a.det[3 * i + 1];
    m = a.det[3 * i + 2];
    return ray >= 0 && ray < a.n_rays && k >= 0 && k < a.R1 && m >= 0 && m < a.n_rcv;
}

// Plane id of the triangle ending segment j of the ray, in the scene of
// receiver row m (batched calls) or of the call.
__device__ inline int32_t plane_at(const CollectArgs& a, int32_t m, int32_t ray, int32_t j) {
    const int32_t t = a.hit_seq[(int64_t)ray * a.R1 + j];
    if (a.rcv_job) {
        const DevScene& sc = a.scenes[a.jobs[a.rcv_job[m]].scene];
        return (t >= 0 && t < sc.n_tri) ? sc.tri_plane[t] : -1;
    }
    return (t >= 0 && t < a.n_tri) ? a.tri_plane[t] : -1;
}

// The triangle-to-plane table of receiver row m's scene.
__device__ inline void scene_planes(const CollectArgs& a, int32_t m, const int32_t*& tp, int32_t& nt) {
    if (a.rcv_job) {
        const DevScene& sc = a.scenes[a.jobs[a.rcv_job[m]].scene];
        tp = sc.tri_plane;
        nt = sc.n_tri;
    } else {
        tp = a.tri_plane;
        nt = a.n_tri;
    }
}

// Plane ids of hits j0 .. j0 + C - 1 of a ray (-1 past k or for an invalid
// triangle), every load of the chunk in flight together.
template <int C>
__device__ inline void planes_of(const CollectArgs& a, const int32_t* tp, int32_t nt, int32_t ray, int32_t j0,
                                 int32_t k, int32_t (&p)[C]) {
    int32_t t[C];
#pragma unroll
    for (int q = 0; q < C; q++) t[q] = j0 + q < k ? a.hit_seq[(int64_t)ray * a.R1 + j0 + q] : -1;
#pragma unroll
    for (int q = 0; q < C; q++) p[q] = (t[q] >= 0 && t[q] < nt) ? tp[t[q]] : -1;
}

__global__ void k_hash(CollectArgs a, uint64_t mask, uint64_t* __restrict__ hash, uint32_t* __restrict__ err) {
    const int64_t n = det_count(a);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t ray, k, m;
        if (!det_row(a, i, ray, k, m)) {
            atomicOr(err, 1u);
            hash[i] = mask;   // invalid rows sort together at the end
            continue;
        }
        uint64_t h = mix64(0x9E3779B97F4A7C15ull ^ ((uint64_t)(uint32_t)m << 32 | (uint32_t)k));
        const int32_t* tp;
        int32_t nt;
        scene_planes(a, m, tp, nt);
        for (int j0 = 0; j0 < k; j0 += 8) {
            int32_t p[8];
            planes_of<8>(a, tp, nt, ray, j0, k, p);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                if (j0 + q < k) {
                    if (p[q] < 0) atomicOr(err, 2u);
                    h = mix64(h + 0x632BE59BD9B4E019ull * (uint64_t)(uint32_t)(p[q] + 1));
                }
            }
        }
        hash[i] = h & mask;
    }
}

// Lexicographic comparison of two detections' keys: <0, 0, >0.
__device__ inline int key_cmp(const CollectArgs& a, uint32_t x, uint32_t y) {
    int32_t rx, kx, mx, ry, ky, my;
    const bool vx = det_row(a, x, rx, kx, mx), vy = det_row(a, y, ry, ky, my);
    if (!vx || !vy) return vx == vy ? 0 : (vx ? -1 : 1);
    if (mx != my) return mx < my ? -1 : 1;
    if (kx != ky) return kx < ky ? -1 : 1;
    for (int j = 0; j < kx; j++) {
        const int32_t px = plane_at(a, mx, rx, j), py = plane_at(a, my, ry, j);
        if (px != py) return px < py ? -1 : 1;
    }
    return 0;
}

__global__ void k_heads(CollectArgs a, const uint64_t* __restrict__ hash, const uint32_t* __restrict__ idx,
                        uint32_t* __restrict__ head, uint32_t* __restrict__ flags) {
    const int64_t n = det_count(a);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = 1;
        if (i > 0 && hash[i] == hash[i - 1]) {
            h = key_cmp(a, idx[i], idx[i - 1]) != 0;
            if (h) atomicOr(flags, 4u);   // equal hashes, different keys
        }
        head[i] = h;
    }
}

// First row of the sorted hash array [lo, hi) not below h / above h.
__device__ inline int64_t lower_row(const uint64_t* hash, int64_t lo, int64_t hi, uint64_t h) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (hash[mid] < h) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ inline int64_t upper_row(const uint64_t* hash, int64_t lo, int64_t hi, uint64_t h) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (hash[mid] <= h) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Runs of equal hash holding different keys: a row whose hash equals the
// previous one but whose key differs marks the first row of its run (bit 1
// of head; the run start is found by binary search in the sorted hashes).
// Does nothing unless a collision was seen.
__global__ void k_mark_mixed(CollectArgs a, const uint64_t* __restrict__ hash, uint32_t* __restrict__ head,
                             const uint32_t* __restrict__ flags) {
    if (!(*flags & 4u)) return;
    const int64_t n = det_count(a);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (i == 0 || !(head[i] & 1u) || hash[i] != hash[i - 1]) continue;
        atomicOr(&head[lower_row(hash, 0, i, hash[i])], 2u);
    }
}

// One thread per marked run: sort the run by full key (stable) and recompute
// its group heads.  Unmarked runs, however long, are not touched.
__global__ void k_fix_collisions(CollectArgs a, const uint64_t* __restrict__ hash, uint32_t* __restrict__ idx,
                                 uint32_t* __restrict__ head, const uint32_t* __restrict__ flags) {
    if (!(*flags & 4u)) return;
    const int64_t n = det_count(a);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!(head[i] & 2u)) continue;
        const int64_t e = upper_row(hash, i + 1, n, hash[i]);
        for (int64_t j = i + 1; j < e; j++) {   // stable insertion sort by key
            const uint32_t v = idx[j];
            int64_t q = j - 1;
            while (q >= i && key_cmp(a, idx[q], v) > 0) {
                idx[q + 1] = idx[q];
                q--;
            }
            idx[q + 1] = v;
        }
        head[i] = 1;
        for (int64_t j = i + 1; j < e; j++) head[j] = key_cmp(a, idx[j], idx[j - 1]) != 0;
    }
}

__global__ void k_head_pos(CollectArgs a, const uint32_t* __restrict__ head, const uint32_t* __restrict__ group,
                           uint32_t* __restrict__ hpos, int64_t* __restrict__ n_is) {
    const int64_t n = det_count(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t total = n > 0 ? (int64_t)group[n] : 0;
        *n_is = total;
        hpos[total] = (uint32_t)n;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (head[i]) hpos[group[i]] = (uint32_t)i;
}

// Every entry of the first n_is rows (R + 2 entries each) set to -1 with
// contiguous stores; k_emit then writes only the (receiver, k, planes) prefix.
__global__ void k_pad_rows(int32_t* __restrict__ is_key, int64_t row_len, const int64_t* __restrict__ n_is,
                           int64_t is_cap) {
    const int64_t ng = *n_is < is_cap ? *n_is : is_cap;
    const int64_t total = ng * row_len;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        is_key[i] = -1;
}

struct EmitArgs {
    const double* pn;
    const double* pp;
    double src[3];
    const float* rcv;
    int32_t* is_key;
    int32_t* is_count;
    double* is_pos;
    double* is_dist;
    int64_t is_cap;
};

__device__ void emit_one(const CollectArgs& a, const EmitArgs& e, const uint32_t* __restrict__ idx,
                         const uint32_t* __restrict__ hpos, int64_t g);

__global__ void k_emit(CollectArgs a, EmitArgs e, const uint32_t* __restrict__ idx, const uint32_t* __restrict__ hpos,
                       const int64_t* __restrict__ n_is) {
    const int64_t ng = *n_is < e.is_cap ? *n_is : e.is_cap;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += (int64_t)gridDim.x * blockDim.x)
        emit_one(a, e, idx, hpos, g);
}

__device__ void emit_one(const CollectArgs& a, const EmitArgs& e, const uint32_t* __restrict__ idx,
                         const uint32_t* __restrict__ hpos, int64_t g) {
    const uint32_t p0 = hpos[g], p1 = hpos[g + 1];
    const uint32_t d = idx[p0];
    int32_t ray, k, m;
    int32_t* row = e.is_key + g * (int64_t)(a.R1 + 1);
    if (!det_row(a, d, ray, k, m)) {
        e.is_count[g] = (int32_t)(p1 - p0);   // the row stays -1 (k_pad_rows)
        e.is_pos[3 * g] = e.is_pos[3 * g + 1] = e.is_pos[3 * g + 2] = 0.0;
        e.is_dist[g] = __longlong_as_double(0x7FF8000000000000ll);
        return;
    }
    row[0] = m;
    row[1] = k;
    double x = e.src[0], y = e.src[1], z = e.src[2];
    const double* pn = e.pn;
    const double* pp = e.pp;
    if (a.rcv_job) {
        const DevJob& jb = a.jobs[a.rcv_job[m]];
        x = jb.src[0];
        y = jb.src[1];
        z = jb.src[2];
        pn = a.scenes[jb.scene].plane_n;
        pp = a.scenes[jb.scene].plane_p;
    }
    const int32_t* tp;
    int32_t nt;
    scene_planes(a, m, tp, nt);
    for (int j0 = 0; j0 < k; j0 += 4) {
        // plane ids, normals and points of four hits fetched together, then mirrored in order
        int32_t p[4];
        planes_of<4>(a, tp, nt, ray, j0, k, p);
        double n[4][3], o[4][3];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const bool ok = p[q] >= 0;
            for (int c = 0; c < 3; c++) {
                n[q][c] = ok ? pn[3 * (int64_t)p[q] + c] : 0.0;
                o[q][c] = ok ? pp[3 * (int64_t)p[q] + c] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (j0 + q < k) {
                row[2 + j0 + q] = p[q];
                if (p[q] >= 0) {
                    const double nx = n[q][0], ny = n[q][1], nz = n[q][2];
                    const double h = (x - o[q][0]) * nx + (y - o[q][1]) * ny + (z - o[q][2]) * nz;
                    x -= 2.0 * h * nx;
                    y -= 2.0 * h * ny;
                    z -= 2.0 * h * nz;
                }
            }
        }
    }
    // entries 2 + k .. R + 1 keep the -1 written by k_pad_rows
    e.is_count[g] = (int32_t)(p1 - p0);
    e.is_pos[3 * g] = x;
    e.is_pos[3 * g + 1] = y;
    e.is_pos[3 * g + 2] = z;
    const double dx = x - (double)e.rcv[4 * m], dy = y - (double)e.rcv[4 * m + 1], dz = z - (double)e.rcv[4 * m + 2];
    e.is_dist[g] = sqrt(dx * dx + dy * dy + dz * dz);
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// grid-stride kernels: enough workgroups to fill the chip, no more
inline unsigned nblk(int64_t n) {
    int64_t b = (n + 255) / 256;
    const int64_t cap = (int64_t)device_sm_count() * 8;
    if (b > cap) b = cap;
    return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

}  // namespace rtac

using namespace rtac;

extern "C" int rt_debug_set_hash_bits(int bits) {
    RT_CHECK(bits >= 1 && bits <= 64, RT_EINVAL, "rt_debug_set_hash_bits: bits must be in [1, 64]");
    g_hash_bits = bits;
    return RT_OK;
}

namespace rtac {
namespace {
int collect_common(rt_scene* s, const rt_batch* b, const float* src_host, const float* rcv, int32_t n_rcv,
                   const int32_t* hit_seq, int64_t n_rays, int32_t max_reflections, const int32_t* det,
                   int64_t det_cap, const int64_t* n_det, int32_t* is_key, int32_t* is_count, double* is_pos,
                   double* is_dist, int64_t is_cap, int64_t* n_is, void* stream) {
    CallStream call_stream((hipStream_t)stream);
    RT_CHECK(s && src_host && n_det && n_is, RT_EINVAL, "rt_collect_image_sources: null argument");
    RT_CHECK(s->valid, RT_EINVAL, "rt_collect_image_sources: the scene's last rebuild failed");
    RT_CHECK(max_reflections >= 0 && max_reflections < 4096, RT_EINVAL,
             "rt_collect_image_sources: max_reflections out of range");
    RT_CHECK(n_rcv >= 1 && (b || n_rcv <= kMaxRcv) && rcv, RT_EINVAL, "rt_collect_image_sources: bad receivers");
    RT_CHECK(det_cap >= 0 && (det_cap == 0 || (det && hit_seq)), RT_EINVAL,
             "rt_collect_image_sources: det/hit_seq is NULL");
    RT_CHECK(det_cap < ((int64_t)1 << 31), RT_EINVAL, "rt_collect_image_sources: det_cap must be < 2^31");
    RT_CHECK(is_cap >= 0 && (is_cap == 0 || (is_key && is_count && is_pos && is_dist)), RT_EINVAL,
             "rt_collect_image_sources: null output");
    hipStream_t st = (hipStream_t)stream;
    Workspace& ws = s->ws;
    const int64_t cap = det_cap > 0 ? det_cap : 1;
    if (ws.sort_keys[0].ensure(8 * cap) || ws.sort_keys[1].ensure(8 * cap) || ws.sort_vals[0].ensure(4 * cap) ||
        ws.sort_vals[1].ensure(4 * cap) || ws.is_flags.ensure(4 * (cap + 1)) || ws.is_group.ensure(4 * (cap + 1)) ||
        ws.is_idx.ensure(4 * (cap + 2)) || ws.coll_err.ensure(16))
        return RT_ENOMEM;
    CollectArgs a;
    a.hit_seq = hit_seq;
    a.det = det;
    a.n_det = n_det;
    a.det_cap = det_cap;
    a.n_rays = n_rays;
    a.R1 = max_reflections + 1;
    a.n_rcv = n_rcv;
    a.tri_plane = s->tri_plane;
    a.n_tri = s->n_tri;
    a.rcv_job = b ? b->rcv_job : nullptr;
    a.jobs = b ? b->jobs : nullptr;
    a.scenes = b ? b->scenes : nullptr;
    uint32_t* err = ws.coll_err.as<uint32_t>();
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, err, 4);
    const uint64_t mask = g_hash_bits >= 64 ? ~0ull : ((1ull << g_hash_bits) - 1ull);
    uint64_t* h0 = ws.sort_keys[0].as<uint64_t>();
    uint64_t* h1 = ws.sort_keys[1].as<uint64_t>();
    uint32_t* v0 = ws.sort_vals[0].as<uint32_t>();
    uint32_t* v1 = ws.sort_vals[1].as<uint32_t>();
    hipLaunchKernelGGL(k_hash, dim3(nblk(cap)), dim3(256), 0, st, a, mask, h0, err);
    int which = 0;
    const int bits = g_hash_bits >= 64 ? 64 : ((g_hash_bits + 7) / 8) * 8;
    int rc = radix_sort_pairs(ws, h0, v0, h1, v1, cap, n_det, 0, bits, st, &which, true);
    if (rc) return rc;
    uint64_t* hs = which ? h1 : h0;
    uint32_t* ix = which ? v1 : v0;
    uint32_t* head = ws.is_flags.as<uint32_t>();
    uint32_t* group = ws.is_group.as<uint32_t>();
    uint32_t* hpos = ws.is_idx.as<uint32_t>();
    hipLaunchKernelGGL(k_heads, dim3(nblk(cap)), dim3(256), 0, st, a, hs, ix, head, err);
    hipLaunchKernelGGL(k_mark_mixed, dim3(nblk(cap)), dim3(256), 0, st, a, hs, head, err);
    hipLaunchKernelGGL(k_fix_collisions, dim3(nblk(cap)), dim3(256), 0, st, a, hs, ix, head, err);
    rc = exclusive_scan_u32(ws, head, group, cap, n_det, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_head_pos, dim3(nblk(cap)), dim3(256), 0, st, a, head, group, hpos, n_is);
    EmitArgs e;
    e.pn = s->plane_n;
    e.pp = s->plane_p;
    e.src[0] = src_host[0];
    e.src[1] = src_host[1];
    e.src[2] = src_host[2];
    e.rcv = rcv;
    e.is_key = is_key;
    e.is_count = is_count;
    e.is_pos = is_pos;
    e.is_dist = is_dist;
    e.is_cap = is_cap;
    hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)(device_sm_count() * 8)), dim3(256), 0, st, is_key,
                       (int64_t)(a.R1 + 1), n_is, is_cap);
    hipLaunchKernelGGL(k_emit, dim3(nblk(cap)), dim3(256), 0, st, a, e, ix, hpos, n_is);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
}  // namespace
}  // namespace rtac

extern "C" int rt_collect_image_sources(const rt_scene* scene, const float* src_host, const float* rcv, int32_t n_rcv,
                                        const int32_t* hit_seq, int64_t n_rays, int32_t max_reflections,
                                        const int32_t* det, int64_t det_cap, const int64_t* n_det, int32_t* is_key,
                                        int32_t* is_count, double* is_pos, double* is_dist, int64_t is_cap,
                                        int64_t* n_is, void* stream) {
    return collect_common(const_cast<rt_scene*>(scene), nullptr, src_host, rcv, n_rcv, hit_seq, n_rays,
                          max_reflections, det, det_cap, n_det, is_key, is_count, is_pos, is_dist, is_cap, n_is,
                          stream);
}

extern "C" int rt_collect_batch(rt_batch* b, const float* rcv, const int32_t* hit_seq, int32_t max_reflections,
                                const int32_t* det, int64_t det_cap, const int64_t* n_det, int32_t* is_key,
                                int32_t* is_count, double* is_pos, double* is_dist, int64_t is_cap, int64_t* n_is,
                                void* stream) {
    RT_CHECK(b, RT_EINVAL, "rt_collect_batch: null batch");
    const float zero[3] = {0.f, 0.f, 0.f};
    return collect_common(b->ws_owner, b, zero, rcv, b->n_rcv, hit_seq, b->n_rays, max_reflections, det, det_cap,
                          n_det, is_key, is_count, is_pos, is_dist, is_cap, n_is, stream);
}
