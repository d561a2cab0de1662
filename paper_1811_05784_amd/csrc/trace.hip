// Ray generation and specular ray propagation (rt_fibonacci_directions,
// rt_trace_rays).
//
// One persistent kernel runs every segment of every ray.  Each lane of a
// 64-wide wavefront owns one ray and keeps its whole state in registers:
// after a reflection it starts the next segment's nearest-hit query at once,
// and when its ray stops it takes a new ray from a global pool (one atomic
// per wavefront for all idle lanes).  Nothing round-trips to the host between
// bounces and no ray state is stored between segments (the register spills
// of the tightest register budget aside).
//
// Nearest hit (section "Standard algorithm": 0 <= lambda, mu, lambda + mu <= 1,
// delta > 0 minimal) walks the 4-wide tree with an ordered short stack (16
// entries per lane in LDS, spilling to a per-lane global area), a
// conservative slab test for the child boxes (Williams et al.'s test, which
// the paper uses to sort rays into daughter boxes) and the watertight FP32
// ray/triangle test of Woop, Benthin and Wald (2013): shared edges are never
// missed, and exact ties among the triangles a query tests go to the lowest
// triangle id (a box whose FP32 entry distance rounds just above a tie can be
// culled once its twin is found).  Lanes whose query is
// finished wait until enough of the wavefront is finished, then shade
// together: the chosen triangle's plane crossing, receiver tests and the
// reflection are evaluated in FP64 and rounded once to FP32.
//
// Once every ray has been handed out, the launch ends with the longest
// bounce chains, often one or two per wavefront.  A wavefront left with a
// single query in flight then searches it with all 64 lanes (two queries:
// 32 lanes each), breadth first over a frontier of tree nodes in LDS, which
// takes about as many steps as the tree is deep instead of one node per step
// (same nearest hit).  A wavefront shades its finished queries in groups to
// spread the FP64 shading over many lanes; with reflections the group size is
// a share of the lanes still working (16 of 64 by default), so that once the
// pool is empty and the wavefront holds only the rays it already has, no chain
// waits for the slowest query beside it (single-segment queries end at their
// shading, so there the group stays fixed).
#include "common.h"

namespace rtac {

namespace {

constexpr int kBlock = 256;
// LDS stack entries per lane (template parameter kRing of the trace kernel):
// 8, 16 (default) or 32; the ring spills to a per-lane global area in chunks.
constexpr int kRingDefault = 16;
constexpr int kSpillChunk = 8;

enum : int { kIdle = 0, kQuery = 1, kDone = 2 };

// A box is skipped only when its FP32 entry distance exceeds the nearest hit
// found so far by more than 16 units in the last place (at least 2^-20
// relative).  Each slab distance (b - o) / u is within 3 FP32 roundings
// (relative) of the exact one, which is never beyond the distance of a hit
// inside the box; so whenever the watertight distance of that hit is within
// 13 roundings of its exact value (all but near-grazing hits), a triangle
// whose FP32 distance equals the best one is always tested, whatever the
// search order, and exact ties go to the lowest triangle id.  t >= 0; +inf
// stays +inf.  (An integer add, so a wave-uniform bound stays scalar.)
__device__ inline float widen(float t) { return __uint_as_float(min(__float_as_uint(t) + 16u, 0x7F800000u)); }

enum : unsigned long long { kErrStack = 1ull, kErrNode = 2ull, kErrSteps = 4ull, kErrQueue = 8ull };

struct TraceArgs {
    const Node4* nodes;
    const float4* tri;
    const double* plane_n;
    const double* plane_p;
    int32_t n_nodes;
    int32_t n_ref;                  // triangle records (leaf ranges index them)
    float src[3];
    const float* origins;
    const float* dirs;
    const int32_t* start_plane;
    const float* start_len;
    int64_t n_rays;
    const float* rcv;
    int32_t n_rcv;
    int32_t R;
    float max_len;
    int32_t record;
    const int32_t* record_rows;     // NULL: ray i records into row i; else row record_rows[i] (< 0: none)
    int32_t* hit_seq;
    int32_t* det;
    int64_t det_cap;
    unsigned long long* counters;   // [0] n_det [1] queries [2] escapes [3] error
    unsigned long long* pool;       // [0] next ray
    unsigned long long* pool_xcd;   // NULL, or 8 counters 16 words apart: next ray of each eighth of the pool
    float* states;
    int32_t* spill;
    int32_t spill_per_lane;
    int32_t fetch_thr;
    int32_t shade_thr;
    int32_t scale_shade;            // nonzero: shade_thr applies to a full wavefront, scaled by its working lanes
    int32_t max_steps;
    const uint32_t* order;          // pool index -> ray id (NULL: identity)
    unsigned long long* stats;      // NULL or [4]
    // continuation rounds: rays still in flight when the pool is empty and a
    // wavefront is mostly idle are written to q_out and finished by the next
    // launch, which takes its rays from q_in instead of the source
    const int4* q_in;
    const unsigned long long* q_in_count;
    int4* q_out;
    unsigned long long* q_out_count;
    int64_t q_cap;                  // entries of q_in / q_out
    int32_t spill_thr;
    int32_t suspend_k;              // > 0: a ray about to start segment >= suspend_k goes to q_out
    int32_t beam_n;                 // > 0: range limit of the discrete model with beams of >= beam_n rays
    int32_t coop;                   // nonzero: a wavefront left with one query searches it with all lanes
    // batched calls: rays of many jobs (source + receivers in one scene)
    const DevJob* jobs;
    const DevScene* scenes;
    int32_t n_jobs;
};

// queued ray: (ray, k, last plane, -) (o.x, o.y, o.z, L low word) (u.x, u.y, u.z, L high word)
constexpr int kQueueInts = 12;

constexpr int kXcd = 8;             // accelerator complexes (own L2 each); workgroup b runs on b % 8
constexpr int kPoolWords = 32 + 16 * kXcd;

__global__ void k_trace_reset(unsigned long long* counters, unsigned long long* pool, unsigned long long* stats) {
    if (threadIdx.x < 4) counters[threadIdx.x] = 0ull;
    if (stats && threadIdx.x < 4) stats[threadIdx.x] = 0ull;
    // pool counters and queue lengths of every round, then the per-XCD counters
    for (int i = threadIdx.x; i < kPoolWords; i += blockDim.x) pool[i] = 0ull;
}

struct Ray {
    float ox, oy, oz, ux, uy, uz;
    float ix, iy, iz;      // reciprocal direction for the slab test
    float sx, sy, sz;      // shear constants of the watertight test
    int kx, ky, kz;
};

// Number of set bits of m in the lanes below this one.
__device__ inline uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline float pick(float a, float b, float c, int k) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ inline void setup_ray(Ray& r) {
    const float ax = fabsf(r.ux), ay = fabsf(r.uy), az = fabsf(r.uz);
    int kz = ax >= ay ? (ax >= az ? 0 : 2) : (ay >= az ? 1 : 2);
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    const float dz = pick(r.ux, r.uy, r.uz, kz);
    if (dz < 0.f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r.kx = kx;
    r.ky = ky;
    r.kz = kz;
    r.sx = pick(r.ux, r.uy, r.uz, kx) / dz;
    r.sy = pick(r.ux, r.uy, r.uz, ky) / dz;
    r.sz = 1.0f / dz;
    const float tiny = 1e-20f;
    r.ix = 1.0f / (fabsf(r.ux) > tiny ? r.ux : copysignf(tiny, r.ux));
    r.iy = 1.0f / (fabsf(r.uy) > tiny ? r.uy : copysignf(tiny, r.uy));
    r.iz = 1.0f / (fabsf(r.uz) > tiny ? r.uz : copysignf(tiny, r.uz));
}

// Watertight ray/triangle test.  Edge functions are evaluated without
// contraction so that a shared edge gives exactly opposite values for the
// two triangles that share it; zero values are re-evaluated in FP64.
// Returns t > 0 on a hit, else -1.
__device__ inline float watertight(const Ray& r, float4 v0, float4 v1, float4 v2) {
#pragma clang fp contract(off)
    const float a0 = v0.x - r.ox, a1 = v0.y - r.oy, a2 = v0.z - r.oz;
    const float b0 = v1.x - r.ox, b1 = v1.y - r.oy, b2 = v1.z - r.oz;
    const float c0 = v2.x - r.ox, c1 = v2.y - r.oy, c2 = v2.z - r.oz;
    const float Akx = pick(a0, a1, a2, r.kx), Aky = pick(a0, a1, a2, r.ky), Akz = pick(a0, a1, a2, r.kz);
    const float Bkx = pick(b0, b1, b2, r.kx), Bky = pick(b0, b1, b2, r.ky), Bkz = pick(b0, b1, b2, r.kz);
    const float Ckx = pick(c0, c1, c2, r.kx), Cky = pick(c0, c1, c2, r.ky), Ckz = pick(c0, c1, c2, r.kz);
    const float Ax = Akx - r.sx * Akz, Ay = Aky - r.sy * Akz;
    const float Bx = Bkx - r.sx * Bkz, By = Bky - r.sy * Bkz;
    const float Cx = Ckx - r.sx * Ckz, Cy = Cky - r.sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.f || V == 0.f || W == 0.f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return -1.f;
    float det = U + V + W;
    if (det == 0.f) return -1.f;
    const float Az = r.sz * Akz, Bz = r.sz * Bkz, Cz = r.sz * Ckz;
    float T = U * Az + V * Bz + W * Cz;
    if (det < 0.f) {
        det = -det;
        T = -T;
    }
    if (!(T > 0.f)) return -1.f;
    return T / det;
}

struct Stack {
    int base, cnt, gsp;
};

// The lane's spill area is spill_all + (block * kBlock + tid) * spill_n, formed
// only on the (rare) spill and refill paths so that no register holds it.
template <int kRing>
__device__ inline bool stack_push(Stack& s, int32_t* lds, int32_t* spill_all, int spill_n, int tid, int32_t item) {
    if (s.cnt == kRing) {
        if (s.gsp + kSpillChunk > spill_n) return false;
        int32_t* spill = spill_all + ((int64_t)blockIdx.x * kBlock + tid) * spill_n;
        for (int i = 0; i < kSpillChunk; i++) spill[s.gsp + i] = lds[((s.base + i) & (kRing - 1)) * kBlock + tid];
        s.gsp += kSpillChunk;
        s.base = (s.base + kSpillChunk) & (kRing - 1);
        s.cnt -= kSpillChunk;
    }
    lds[((s.base + s.cnt) & (kRing - 1)) * kBlock + tid] = item;
    s.cnt++;
    return true;
}

// Returns false when the stack is empty.
template <int kRing>
__device__ inline bool stack_pop(Stack& s, int32_t* lds, const int32_t* spill_all, int spill_n, int tid,
                                 int32_t& item) {
    if (s.cnt == 0) {
        if (s.gsp == 0) return false;
        const int32_t* spill = spill_all + ((int64_t)blockIdx.x * kBlock + tid) * spill_n;
        const int h = s.gsp < kSpillChunk ? s.gsp : kSpillChunk;
        s.gsp -= h;
        s.base = (s.base - h) & (kRing - 1);
        for (int i = 0; i < h; i++) lds[((s.base + i) & (kRing - 1)) * kBlock + tid] = spill[s.gsp + i];
        s.cnt = h;
    }
    s.cnt--;
    item = lds[((s.base + s.cnt) & (kRing - 1)) * kBlock + tid];
    return true;
}

// Range of the discrete model (eq. 13): with receiver radius r and N rays
// emitted, a beam of at least n rays is measurable up to d = (r / 2) sqrt(N / n).
// FP64, rounded once to FP32 (the precision of the travelled-length limit).
__device__ inline float beam_range(double r, int64_t n_rays, int32_t n) {
    return (float)(0.5 * r * sqrt((double)n_rays / (double)n));
}

__device__ inline void cswap(float& ta, int32_t& ra, float& tb, int32_t& rb) {
    if (tb < ta) {
        float t = ta;
        ta = tb;
        tb = t;
        int32_t q = ra;
        ra = rb;
        rb = q;
    }
}

// Minimum of v over each group of G lanes (G = 64: the wavefront; 32: its
// halves; 16: its rows; 8: half rows), in every lane of the group.  For 16 and
// more lanes: an inclusive min-scan
// within rows of 16 lanes by row shifts of 1, 2, 4, 8, then the broadcasts of
// lane 15 (to rows 1 and 3) and, for the whole wavefront, of lane 31 (to rows
// 2 and 3), all data-parallel moves between lanes; the group's last lane
// holds the minimum.  Every lane of the wavefront must be active.
__device__ inline uint32_t group_umin(uint32_t v, int G) {
    constexpr int kId = -1;   // 0xFFFFFFFF: the identity of an unsigned minimum
    auto take = [](uint32_t a, int b) { return a < (uint32_t)b ? a : (uint32_t)b; };
    if (G == 8) {
        // butterfly within each 8-lane half row: swap neighbours, swap pairs
        // (quad permutations), then mirror the half row; every lane ends with the minimum
        v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
        v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
        v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x141, 0xF, 0xF, false));   // row_half_mirror
        return v;
    }
    v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x111, 0xF, 0xF, false));   // row_shr:1
    v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x112, 0xF, 0xF, false));   // row_shr:2
    v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x114, 0xF, 0xF, false));   // row_shr:4
    v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x118, 0xF, 0xF, false));   // row_shr:8
    if (G == 16) {
        const int row = (int)((threadIdx.x & (kWave - 1)) >> 4);
        const uint32_t m0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
        const uint32_t m1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
        const uint32_t m2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
        const uint32_t m3 = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
        return row == 0 ? m0 : row == 1 ? m1 : row == 2 ? m2 : m3;
    }
    v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x142, 0xA, 0xF, false));   // row_bcast:15
    if (G == kWave) {
        v = take(v, __builtin_amdgcn_update_dpp(kId, (int)v, 0x143, 0xC, 0xF, false));   // row_bcast:31
        return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    }
    const uint32_t m0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    const uint32_t m1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    return (threadIdx.x & (kWave - 1)) < 32 ? m0 : m1;
}

// Nearest hit of one query by a group of G lanes (G = 64: the whole
// wavefront; 32: one half; 16: one row; lanes li = 0..G-1 from lane gbase;
// an inactive group has no query and idles), breadth first
// over a frontier kept in the group's columns of the LDS stack area (refs in
// the first half of the kRing slots, entry distances in the second: kRing/2 G
// entries).  Each step every
// lane of the group takes one frontier item, the most recent first: an inner
// node is slab-tested and every child whose box is hit joins the frontier
// (far children first, so the nearest are taken next); a leaf has its
// triangles tested.  So a step makes one dependent memory access per lane.
// The group keeps the nearest hit, (t, id) lexicographic: exact ties go to the
// lowest triangle id and the result is the per-lane walk's.  bt, bid, bj come
// in as the owner's best so far and leave as the group's result (the same in
// every lane of the group).  Returns false, for that group only, when its
// frontier would overflow or it meets a reference out of range, and for all
// groups when the step bound is reached; the owner then walks the query from
// the root, bounded by the best hit found so far.
template <int kRing>
__device__ inline bool coop_search(const Ray& q, int32_t qlp, float& bt, int32_t& bid, int32_t& bj, int32_t* plane_slot,
                                   int32_t* base_col,
                                   int li, int gbase, int G, bool active, const Node4* nodes, const float4* tri,
                                   int32_t n_nodes, int32_t n_tri, int32_t max_steps) {
    const int lg = 31 - __builtin_clz((unsigned)G);   // G is 8, 16, 32 or 64, the same in every lane
    const int kCap = (kRing / 2) << lg;
    int32_t* fref = base_col;
    float* ft = reinterpret_cast<float*>(base_col + (kRing / 2) * kBlock);
    auto fat = [lg, G](int k) { return (k >> lg) * kBlock + (k & (G - 1)); };
    int nf = active ? 1 : 0;   // a group without a query stays idle
    if (active && li == 0) {
        fref[0] = 0;
        ft[0] = 0.f;
    }
    bool ok = true;
    int csteps = 0;
    while (__ballot(nf > 0) != 0ull) {
        if (++csteps > max_steps) {
            ok = false;
            break;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // two tree levels per step: a frontier item takes four lanes.  For an
        // inner node, lane s slab-tests the node's child s and expands a hit
        // child in the same step (a child node's four boxes, or a leaf child's
        // triangles); a leaf item is tested by its first lane
        const int kItems = G >> 2;
        const int take = nf < kItems ? nf : kItems;
        const int base = nf - take;   // the most recent entries, deepest first
        const int slot = li & 3;
        int32_t parent = kEmpty;
        float pt = INFINITY;
        if ((li >> 2) < take) {
            parent = fref[fat(base + (li >> 2))];
            pt = ft[fat(base + (li >> 2))];
        }
        nf = base;
        const float tlim = widen(bt);
        bool bad = parent != kEmpty && parent >= n_nodes;
        int32_t item = kEmpty;   // what this lane expands
        float it = INFINITY;
        if (parent != kEmpty && !bad && pt <= tlim) {
            if (parent >= 0) {
                // child `slot` of the node: its box (one float of each of the
                // node's six bound vectors) and its reference
                const float* nb = reinterpret_cast<const float*>(nodes + parent);
                const float LX = nb[slot], HX = nb[4 + slot], LY = nb[8 + slot], HY = nb[12 + slot];
                const float LZ = nb[16 + slot], HZ = nb[20 + slot];
                const int32_t CH = reinterpret_cast<const int32_t*>(nb)[24 + slot];
                const float t0x = (LX - q.ox) * q.ix, t1x = (HX - q.ox) * q.ix;
                const float t0y = (LY - q.oy) * q.iy, t1y = (HY - q.oy) * q.iy;
                const float t0z = (LZ - q.oz) * q.iz, t1z = (HZ - q.oz) * q.iz;
                const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.f));
                float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));
                tmax *= 1.00000036f;
                if (CH != kEmpty && tmin <= tmax && tmin <= tlim) {
                    item = CH;
                    it = tmin;
                }
            } else if (slot == 0) {
                item = parent;
                it = pt;
            }
        }
        if (item != kEmpty && item >= n_nodes) bad = true;
        float tn[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
        int32_t rf[4] = {kEmpty, kEmpty, kEmpty, kEmpty};
        float lt = bt;
        int32_t lid = bid, lj = bj, lp = 0;
        const bool live = item != kEmpty && !bad && it <= tlim;
        int32_t first = 0, ntri = 0;
        if (live && item < 0) {
            first = leaf_first(item);
            ntri = leaf_count(item);
            if (ntri == 0 || first + ntri > n_tri) bad = true;
        }
        const bool is_node = live && item >= 0;
        const bool is_leaf = live && item < 0 && !bad;
        // one memory phase per step: an inner node's boxes and children and a
        // leaf's first triangle are loaded together, so a step whose lanes hold
        // both kinds waits on memory once
        const float4* src = is_node ? reinterpret_cast<const float4*>(nodes + item) : tri + 3 * (int64_t)first;
        float4 d0, d1, d2, d3, d4, d5, d6;
        if (is_node || is_leaf) {
            d0 = src[0];
            d1 = src[1];
            d2 = src[2];
        }
        if (is_node) {
            d3 = src[3];
            d4 = src[4];
            d5 = src[5];
            d6 = src[6];
        }
        if (is_node) {
            const int32_t c0 = __float_as_int(d6.x), c1 = __float_as_int(d6.y), c2 = __float_as_int(d6.z),
                          c3 = __float_as_int(d6.w);
#define RT_SLAB(S, LX, HX, LY, HY, LZ, HZ, CH)                                          \
    {                                                                                    \
        const float t0x = (LX - q.ox) * q.ix, t1x = (HX - q.ox) * q.ix;                  \
        const float t0y = (LY - q.oy) * q.iy, t1y = (HY - q.oy) * q.iy;                  \
        const float t0z = (LZ - q.oz) * q.iz, t1z = (HZ - q.oz) * q.iz;                  \
        const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)),               \
                                 fmaxf(fminf(t0z, t1z), 0.f));                           \
        float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));    \
        tmax *= 1.00000036f;                                                             \
        const bool h = (CH != kEmpty) && tmin <= tmax && tmin <= tlim;                   \
        tn[S] = h ? tmin : INFINITY;                                                     \
        rf[S] = h ? CH : kEmpty;                                                         \
    }
            RT_SLAB(0, d0.x, d1.x, d2.x, d3.x, d4.x, d5.x, c0)
            RT_SLAB(1, d0.y, d1.y, d2.y, d3.y, d4.y, d5.y, c1)
            RT_SLAB(2, d0.z, d1.z, d2.z, d3.z, d4.z, d5.z, c2)
            RT_SLAB(3, d0.w, d1.w, d2.w, d3.w, d4.w, d5.w, c3)
#undef RT_SLAB
        } else if (is_leaf) {
            for (int i = 0; i < ntri; i++) {
                const int32_t j = first + i;
                float4 v0 = d0, v1 = d1, v2 = d2;
                if (i > 0) {
                    v0 = tri[3 * j];
                    v1 = tri[3 * j + 1];
                    v2 = tri[3 * j + 2];
                }
                // the plane left by the ray is excluded in the acceptance test, not by
                // a branch before it, so the record's loads are issued together
                const float t = watertight(q, v0, v1, v2);
                const int32_t id = __float_as_int(v1.w);
                if (__float_as_int(v0.w) != qlp && t > 0.f && (t < lt || (t == lt && id < lid))) {
                    lt = t;
                    lid = id;
                    lj = j;
                    lp = __float_as_int(v0.w);
                }
            }
        }
        // nearest hit of the group: (t, id) lexicographic minimum (t >= 0, so its
        // bits order like its values), then the record of the first lane holding
        // it; only in steps where some lane found a nearer hit (lanes only ever
        // improve on the group's best, so otherwise it stands)
        const int lane = (int)(threadIdx.x & (kWave - 1));
        const uint64_t gmask = G == kWave ? ~0ull : (((1ull << (G & 63)) - 1ull) << gbase);
        const bool improved = lt != bt || lid != bid;
        if (__ballot(improved) != 0ull) {
            const uint32_t tbits = __float_as_uint(lt);
            const uint32_t tmin = group_umin(tbits, G);
            const uint32_t idmin = group_umin(tbits == tmin ? (uint32_t)lid : 0xFFFFFFFFu, G);
            const uint64_t holder = __ballot(tbits == tmin && (uint32_t)lid == idmin) & gmask;
            const int src_lane = __ffsll((long long)holder) - 1;   // the group's first lane holding the minimum
            bt = __uint_as_float(tmin);
            bid = (int32_t)idmin;
            bj = __shfl(lj, src_lane);
            // the holder records the hit's plane id in the owner's slot
            if (lane == src_lane && improved) *plane_slot = lp;
        }
        // children that can still hold a nearer or equal hit join the frontier;
        // each lane's offset counts the children of the group's lanes below it
        const float tkeep = widen(bt);
        int cnt = 0;
#pragma unroll
        for (int sl = 0; sl < 4; sl++) cnt += (rf[sl] != kEmpty && tn[sl] <= tkeep) ? 1 : 0;
        const uint64_t c1 = __ballot(cnt & 1) & gmask, c2 = __ballot(cnt & 2) & gmask, c4 = __ballot(cnt & 4) & gmask;
        const uint64_t below = lane ? (~0ull >> (kWave - lane)) : 0ull;
        const int excl = __popcll(c1 & below) + 2 * __popcll(c2 & below) + 4 * __popcll(c4 & below);
        const int total = __popcll(c1) + 2 * __popcll(c2) + 4 * __popcll(c4);
        // a group whose frontier would overflow, or that met a reference out of
        // range, stops (its owner falls back); the others go on
        if ((__ballot(bad) & gmask) != 0ull || nf + total > kCap) {
            ok = false;
            nf = 0;
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int at = nf + excl;
        // far children first, so that the nearest are taken next
#pragma unroll
        for (int sl = 3; sl >= 0; sl--) {
            if (rf[sl] != kEmpty && tn[sl] <= tkeep) {
                fref[fat(at)] = rf[sl];
                ft[fat(at)] = tn[sl];
                at++;
            }
        }
        nf += total;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return ok;
}

template <int kWavesPerEU, bool kBatch, int kRing, bool kStats>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWavesPerEU, 8)))
k_trace(TraceArgs a) {
    __shared__ int32_t lds_stack[kRing * kBlock];
    __shared__ double rcv_s[kMaxRcv][4];
    // travelled length of each lane's ray, FP64 across all its segments (kept
    // out of the registers of the node loop, which never reads it)
    __shared__ double len_s[kBlock];
    // plane id of each lane's nearest hit so far (read when the query is shaded)
    __shared__ int32_t hitp_s[kBlock];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    if (!kBatch && tid < a.n_rcv * 4) rcv_s[tid >> 2][tid & 3] = (double)a.rcv[tid];
    __syncthreads();
    // scene seen by this lane's ray (uniform unless batched)
    const Node4* nodes = a.nodes;
    const float4* tri = a.tri;
    const double* pl_n = a.plane_n;
    const double* pl_p = a.plane_p;
    int32_t n_nodes = a.n_nodes, n_tri = a.n_ref, rcv_off = 0, n_rcv = a.n_rcv;
    // travelled length at which a ray stops (+inf: no limit)
    float lim = a.max_len > 0.f ? a.max_len : INFINITY;
    if (!kBatch && a.beam_n > 0) {
        double r_max = 0.0;
        for (int m = 0; m < a.n_rcv; m++) r_max = fmax(r_max, rcv_s[m][3]);
        lim = fminf(lim, beam_range(r_max, a.n_rays, a.beam_n));
    }

    const int R1 = a.R + 1;

    int status = kIdle;
    int32_t ray = 0;
    int k = 0;
    len_s[tid] = 0.0;
    hitp_s[tid] = -1;
    int32_t last_plane = -1;
    Ray r;
    r.ox = r.oy = r.oz = r.ux = r.uy = r.uz = 0.f;
    setup_ray(r);
    int32_t cur = 0;
    Stack st{0, 0, 0};
    float best_t = INFINITY;
    int32_t best_j = -1, best_id = 0x7FFFFFFF;
    int32_t steps = 0;
    uint32_t n_query = 0, n_escape = 0;   // wave totals (the same in every lane)
    uint32_t st_nodes = 0, st_leaves = 0, st_tris = 0, st_spill = 0;
    constexpr bool want_stats = kStats;
    unsigned long long pool_n = a.q_in ? *a.q_in_count : (unsigned long long)a.n_rays;
    if (a.q_in && pool_n > (unsigned long long)a.q_cap) pool_n = (unsigned long long)a.q_cap;
    bool pool_empty = pool_n == 0;
    // XCD-local ray pools: the (direction-sorted) pool is cut into eighths and
    // a workgroup first takes rays from the eighth of its own XCD, so each L2
    // sees one cone of directions; it then helps the others
    const bool by_xcd = a.pool_xcd != nullptr && !a.q_in;
    const int home = (int)(blockIdx.x % kXcd);
    uint32_t seg_done = 0;

    for (;;) {
        // ---- refill idle lanes from the ray pool -----------------------------
        const uint64_t idle = __ballot(status == kIdle);
        const int n_idle = __popcll(idle);
        if (!pool_empty && n_idle > 0 && (n_idle >= a.fetch_thr || n_idle == kWave)) {
            const int leader = __ffsll((long long)idle) - 1;
            unsigned long long base = 0, hi = pool_n;   // this refill may take pool positions [base, hi)
            if (by_xcd) {
                if (lane == leader) {
                    base = ~0ull;
                    for (int t = 0; t < kXcd; t++) {
                        const int sg = (home + t) % kXcd;
                        if ((seg_done >> sg) & 1u) continue;
                        const unsigned long long lo = pool_n * (unsigned long long)sg / kXcd;
                        const unsigned long long shi = pool_n * (unsigned long long)(sg + 1) / kXcd;
                        const unsigned long long b = lo + atomicAdd(a.pool_xcd + 16 * sg, (unsigned long long)n_idle);
                        if (b < shi) {
                            base = b;
                            hi = shi;
                            break;
                        }
                        seg_done |= 1u << sg;
                    }
                }
                base = __shfl(base, leader);
                hi = __shfl(hi, leader);
                seg_done = __shfl(seg_done, leader);
                if (base == ~0ull) pool_empty = true;
            } else {
                if (lane == leader) base = atomicAdd(a.pool, (unsigned long long)n_idle);
                base = __shfl(base, leader);
                if (base + (unsigned long long)n_idle >= pool_n) pool_empty = true;
            }
            if (status == kIdle && base != ~0ull) {
                const unsigned long long my = base + (unsigned long long)lanes_below(idle);
                if (my < hi) {
                    if (kBatch && !a.q_in) {
                        const int64_t g = a.order ? (int64_t)a.order[my] : (int64_t)my;
                        const DevJob& jb = a.jobs[job_of_ray(a.jobs, a.n_jobs, g)];
                        float d[3];
                        fibonacci_dir(g - jb.ray_off, jb.n_rays, d);
                        ray = (int32_t)g;
                        r.ox = jb.src[0];
                        r.oy = jb.src[1];
                        r.oz = jb.src[2];
                        r.ux = d[0];
                        r.uy = d[1];
                        r.uz = d[2];
                        len_s[tid] = 0.0;
                        last_plane = -1;
                        k = 0;
                    } else if (a.q_in) {
                        const int4 e0 = a.q_in[3 * my], e1 = a.q_in[3 * my + 1], e2 = a.q_in[3 * my + 2];
                        ray = e0.x;
                        k = e0.y;
                        last_plane = e0.z;
                        r.ox = __int_as_float(e1.x);
                        r.oy = __int_as_float(e1.y);
                        r.oz = __int_as_float(e1.z);
                        len_s[tid] = __hiloint2double(e2.w, e1.w);
                        r.ux = __int_as_float(e2.x);
                        r.uy = __int_as_float(e2.y);
                        r.uz = __int_as_float(e2.z);
                    } else {
                        ray = a.order ? (int32_t)a.order[my] : (int32_t)my;
                        if (a.origins) {
                            r.ox = a.origins[3 * ray];
                            r.oy = a.origins[3 * ray + 1];
                            r.oz = a.origins[3 * ray + 2];
                        } else {
                            r.ox = a.src[0];
                            r.oy = a.src[1];
                            r.oz = a.src[2];
                        }
                        r.ux = a.dirs[3 * ray];
                        r.uy = a.dirs[3 * ray + 1];
                        r.uz = a.dirs[3 * ray + 2];
                        len_s[tid] = a.start_len ? (double)a.start_len[ray] : 0.0;
                        last_plane = a.start_plane ? a.start_plane[ray] : -1;
                        k = 0;
                    }
                    if (kBatch) {
                        const DevJob& jb = a.jobs[job_of_ray(a.jobs, a.n_jobs, ray)];
                        const DevScene& sc = a.scenes[jb.scene];
                        nodes = sc.nodes;
                        tri = sc.tri;
                        pl_n = sc.plane_n;
                        pl_p = sc.plane_p;
                        n_nodes = sc.n_nodes;
                        n_tri = sc.n_ref;
                        rcv_off = jb.rcv_off;
                        n_rcv = jb.n_rcv;
                        lim = jb.max_len > 0.f ? jb.max_len : INFINITY;
                        if (a.beam_n > 0) {
                            double r_max = 0.0;
                            for (int m = 0; m < n_rcv; m++)
                                r_max = fmax(r_max, (double)a.rcv[4 * (int64_t)(rcv_off + m) + 3]);
                            lim = fminf(lim, beam_range(r_max, jb.n_rays, a.beam_n));
                        }
                    }
                    setup_ray(r);
                    cur = 0;
                    st = Stack{0, 0, 0};
                    best_t = INFINITY;
                    best_j = -1;
                    best_id = 0x7FFFFFFF;
                    steps = 0;
                    status = kQuery;
                    if (r.ux == 0.f && r.uy == 0.f && r.uz == 0.f) status = kDone;   // degenerate: escapes
                }
            }
        }
        // ---- hand a mostly idle wavefront's rays to the next launch ----------
        if (pool_empty && a.q_out) {
            const uint64_t act = __ballot(status != kIdle);
            if (__popcll(act) <= a.spill_thr && __ballot(status == kDone) == 0ull) {
                const int n_act = __popcll(act);
                if (n_act > 0) {
                    const int leader = __ffsll((long long)act) - 1;
                    unsigned long long base = 0;
                    if (lane == leader) base = atomicAdd(a.q_out_count, (unsigned long long)n_act);
                    base = __shfl(base, leader);
                    if (status != kIdle) {
                        // the current segment restarts from its input state
                        const unsigned long long pos = base + (unsigned long long)lanes_below(act);
                        int4* q = a.q_out + 3 * pos;
                        q[0] = make_int4((int)ray, k, last_plane, 0);
                        const double lq = len_s[tid];
                        q[1] = make_int4(__float_as_int(r.ox), __float_as_int(r.oy), __float_as_int(r.oz),
                                         __double2loint(lq));
                        q[2] = make_int4(__float_as_int(r.ux), __float_as_int(r.uy), __float_as_int(r.uz),
                                         __double2hiint(lq));
                        status = kIdle;
                    }
                }
                break;
            }
        }
        if (__ballot(status != kIdle) == 0ull) {
            if (pool_empty) break;
            continue;
        }

        // ---- one to eight queries left in the wavefront: search them with every lane
        // (coop_search: breadth first over a frontier in the wavefront's LDS
        // stack area; the owners' own stacks are dropped, the other lanes' are
        // empty): one query takes all 64 lanes, two take 32 each, three or four
        // take 16 each, five to eight take 8 each, so a query takes about half
        // the tree depth in steps instead of one node per step; the result is
        // the owner's own walk's.
        if (!kBatch && a.coop && pool_empty) {
            const uint64_t act = __ballot(status == kQuery);
            const int n_act = __popcll(act);
            if (n_act >= 1 && n_act <= 8 && __ballot(status == kDone) == 0ull) {
                const int G = n_act == 1 ? 64 : (n_act == 2 ? 32 : (n_act <= 4 ? 16 : 8));
                const int g = lane / G;                       // this lane's group
                // owner of group g: the g-th query lane (groups beyond n_act stay idle)
                uint64_t rest = act;
                for (int i = 0; i < g && rest; i++) rest &= rest - 1;
                const bool has_query = rest != 0ull;
                const int mo = has_query ? __ffsll((long long)rest) - 1 : lane;
                Ray q;
                q.ox = __shfl(r.ox, mo);
                q.oy = __shfl(r.oy, mo);
                q.oz = __shfl(r.oz, mo);
                q.ux = __shfl(r.ux, mo);
                q.uy = __shfl(r.uy, mo);
                q.uz = __shfl(r.uz, mo);
                setup_ray(q);
                const int32_t qlp = __shfl(last_plane, mo);
                float bt = __shfl(best_t, mo);
                int32_t bid = __shfl(best_id, mo), bj = __shfl(best_j, mo);
                bool ok;
                int32_t* col = lds_stack + (tid - lane) + G * g;
                ok = coop_search<kRing>(q, qlp, bt, bid, bj, hitp_s + (tid - lane) + mo, col, lane & (G - 1), G * g, G,
                                        has_query, nodes, tri, n_nodes, n_tri, a.max_steps);
                // each owner takes its group's result (from the group's first lane)
                const int my_g = (int)lanes_below(act);   // an owner's group
                const int from = (status == kQuery ? my_g : 0) * G;
                const float rbt = __shfl(bt, from);
                const int32_t rbid = __shfl(bid, from), rbj = __shfl(bj, from);
                const bool rok = __shfl((int)ok, from) != 0;   // the group's outcome, not the owner lane's own
                if (status == kQuery) {
                    best_t = rbt;
                    best_id = rbid;
                    best_j = rbj;
                    st = Stack{0, 0, 0};
                    if (rok) {
                        status = kDone;
                    } else {
                        cur = 0;   // fall back: the owner's own walk from the root, bounded by the hit so far
                        steps = 0;
                    }
                }
            }
        }

        // ---- traverse until enough lanes have finished their query -----------
        // With reflections the shade threshold is a share of the working lanes
        // (lanes only go from query to done in this loop, so it is fixed here):
        // a full wavefront shades its finished queries in groups, one that has
        // run out of rays still shades as soon as that share is done.
        int shade_at = a.shade_thr;
        if (a.scale_shade) {
            const int working = __popcll(__ballot(status != kIdle));
            shade_at = max(1, (shade_at * working + kWave - 1) / kWave);
        }
        for (;;) {
            const uint64_t q = __ballot(status == kQuery);
            if (q == 0ull) break;
            if (__popcll(__ballot(status == kDone)) >= shade_at) break;
            if (status != kQuery) continue;
            bool have = true;
            if (++steps > a.max_steps) {
                atomicOr(&a.counters[3], kErrSteps);
                best_j = -1;
                status = kDone;
                continue;
            }
            // A step visits the lane's inner node, if it holds one: its four
            // children are slab-tested, the nearest inner child is descended
            // into, the nearest leaf child is tested in this same step and every
            // other hit child (inner or leaf) is pushed far to near.  A lane
            // holding a leaf taken from the stack tests it.  So each step runs
            // the triangle test at most once per lane: the wavefront executes
            // it once, not once per child slot.
            if (cur >= n_nodes) {
                atomicOr(&a.counters[3], kErrNode);
                best_j = -1;
                status = kDone;
                continue;
            }
            int32_t leaf = kEmpty;
            int32_t touch = 0;
            bool ok = true;
            if (cur >= 0) {
                if (want_stats) st_nodes++;
                const float4* np = reinterpret_cast<const float4*>(nodes + cur);
                const float4 lx = np[0], hx = np[1], ly = np[2], hy = np[3], lz = np[4], hz = np[5];
                const int4 ch = reinterpret_cast<const int4*>(np)[6];
                // once the pool is empty: touch the node on top of the stack along
                // with this one, so that a later pop finds it in the cache
                if (pool_empty && st.cnt > 0) {
                    const int32_t top = lds_stack[((st.base + st.cnt - 1) & (kRing - 1)) * kBlock + tid];
                    if (top >= 0 && top < n_nodes) touch = reinterpret_cast<const int32_t*>(nodes + top)[0];
                }
                const float tlim = widen(best_t);
                float tn[4];
                int32_t rf[4];
#define RT_SLAB(S, LX, HX, LY, HY, LZ, HZ, CH)                                          \
    {                                                                                    \
        const float t0x = (LX - r.ox) * r.ix, t1x = (HX - r.ox) * r.ix;                  \
        const float t0y = (LY - r.oy) * r.iy, t1y = (HY - r.oy) * r.iy;                  \
        const float t0z = (LZ - r.oz) * r.iz, t1z = (HZ - r.oz) * r.iz;                  \
        const float tmin = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)),               \
                                 fmaxf(fminf(t0z, t1z), 0.f));                           \
        float tmax = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z));    \
        tmax *= 1.00000036f;                                                             \
        const bool h = (CH != kEmpty) && tmin <= tmax && tmin <= tlim;                   \
        tn[S] = h ? tmin : INFINITY;                                                     \
        rf[S] = CH;                                                                      \
    }
                RT_SLAB(0, lx.x, hx.x, ly.x, hy.x, lz.x, hz.x, ch.x)
                RT_SLAB(1, lx.y, hx.y, ly.y, hy.y, lz.y, hz.y, ch.y)
                RT_SLAB(2, lx.z, hx.z, ly.z, hy.z, lz.z, hz.z, ch.z)
                RT_SLAB(3, lx.w, hx.w, ly.w, hy.w, lz.w, hz.w, ch.w)
#undef RT_SLAB
                cswap(tn[0], rf[0], tn[1], rf[1]);
                cswap(tn[2], rf[2], tn[3], rf[3]);
                cswap(tn[0], rf[0], tn[2], rf[2]);
                cswap(tn[1], rf[1], tn[3], rf[3]);
                cswap(tn[1], rf[1], tn[2], rf[2]);
                // slots of the nearest inner and the nearest leaf child that are hit
                int ii = -1, li = -1;
#pragma unroll
                for (int sl = 3; sl >= 0; sl--) {
                    if (tn[sl] < INFINITY) {
                        if (rf[sl] >= 0) ii = sl;
                        else li = sl;
                    }
                }
                if (want_stats) {
                    int np_ = 0;
#pragma unroll
                    for (int sl = 0; sl < 4; sl++) np_ += (tn[sl] < INFINITY && sl != ii && sl != li) ? 1 : 0;
                    if (st.cnt + np_ > kRing) st_spill++;
                }
#pragma unroll
                for (int sl = 3; sl >= 0; sl--)
                    if (tn[sl] < INFINITY && sl != ii && sl != li)
                        ok &= stack_push<kRing>(st, lds_stack, a.spill, a.spill_per_lane, tid, rf[sl]);
                leaf = li == 0 ? rf[0] : li == 1 ? rf[1] : li == 2 ? rf[2] : li == 3 ? rf[3] : kEmpty;
                cur = ii == 0 ? rf[0] : ii == 1 ? rf[1] : ii == 2 ? rf[2] : ii == 3 ? rf[3] : kEmpty;
            } else {
                leaf = cur;   // a leaf taken from the stack
                cur = kEmpty;
            }
            if (!ok) {
                atomicOr(&a.counters[3], kErrStack);
                best_j = -1;
                status = kDone;
                continue;
            }
            if (leaf != kEmpty) {
                const int32_t first = leaf_first(leaf), cnt = leaf_count(leaf);
                if (want_stats) {
                    st_leaves++;
                    st_tris += (uint32_t)cnt;
                }
                if (first + cnt > n_tri) {
                    atomicOr(&a.counters[3], kErrNode);
                    best_j = -1;
                    status = kDone;
                    continue;
                }
                for (int i = 0; i < cnt; i++) {
                    const int32_t j = first + i;
                    const float4 v0 = tri[3 * j], v1 = tri[3 * j + 1], v2 = tri[3 * j + 2];
                    // the plane left by the ray is excluded in the acceptance test, not
                    // by a branch before it, so the record's loads are issued together
                    const float t = watertight(r, v0, v1, v2);
                    const int32_t id = __float_as_int(v1.w);
                    if (__float_as_int(v0.w) != last_plane && t > 0.f &&
                        (t < best_t || (t == best_t && id < best_id))) {
                        best_t = t;
                        best_j = j;
                        hitp_s[tid] = __float_as_int(v0.w);
                        best_id = id;
                    }
                }
            }
            if (cur == kEmpty) have = stack_pop<kRing>(st, lds_stack, a.spill, a.spill_per_lane, tid, cur);
            if (!have) status = kDone;
            asm volatile("" ::"v"(touch));   // keeps the touch load
        }

        // ---- shade the finished queries (FP64), record, reflect ---------------
        const bool shading = status == kDone;
        n_query += (uint32_t)__popcll(__ballot(shading));
        n_escape += (uint32_t)__popcll(__ballot(shading && best_j < 0));
        uint32_t dm = 0;
        double dl = INFINITY;
        int32_t hit_id = -1, hit_plane = -1;
        const double ox = r.ox, oy = r.oy, oz = r.oz, ux = r.ux, uy = r.uy, uz = r.uz;
        const double uu = ux * ux + uy * uy + uz * uz;
        if (shading) {
            if (best_j >= 0) {
                // plane crossing of the chosen triangle in FP64 from its plane (unit
                // normal and point of the plane id's representative)
                hit_plane = hitp_s[tid];
                hit_id = best_id;
                const double* pn = pl_n + 3 * (int64_t)hit_plane;
                const double* pp = pl_p + 3 * (int64_t)hit_plane;
                const double nx = pn[0], ny = pn[1], nz = pn[2];
                const double num = (pp[0] - ox) * nx + (pp[1] - oy) * ny + (pp[2] - oz) * nz;
                const double den = ux * nx + uy * ny + uz * nz;
                dl = num / den;
                if (!(dl > 0.0)) dl = 0.0;
            }
            if (uu > 0.0) {
                const float inv_uuf = 1.0f / (r.ux * r.ux + r.uy * r.uy + r.uz * r.uz);
                double inv_uu = 0.0;   // FP64 1/|u|^2, computed for the first receiver past the screen
                for (int m = 0; m < n_rcv; m++) {
                    double cx, cy, cz, cr;
                    if (kBatch) {
                        const float* q = a.rcv + 4 * (int64_t)(rcv_off + m);
                        cx = q[0];
                        cy = q[1];
                        cz = q[2];
                        cr = q[3];
                    } else {
                        cx = rcv_s[m][0];
                        cy = rcv_s[m][1];
                        cz = rcv_s[m][2];
                        cr = rcv_s[m][3];
                    }
                    {
                        // FP32 screen.  The squared distance of the centre from the ray's
                        // line bounds the segment's from below; computed in FP32 from the
                        // FP32 inputs it is within about 30 units of 2^-24 |w|^2 of the
                        // exact value (w = centre - origin), so a line that clears the
                        // sphere by 64 such units misses it in the FP64 test too
                        const float wxf = (float)cx - r.ox, wyf = (float)cy - r.oy, wzf = (float)cz - r.oz;
                        const float af = wxf * wxf + wyf * wyf + wzf * wzf;
                        const float bf = wxf * r.ux + wyf * r.uy + wzf * r.uz;
                        const float crf = (float)cr;
                        if (af - bf * bf * inv_uuf > crf * crf + 0x1p-18f * af) continue;
                    }
                    if (inv_uu == 0.0) inv_uu = 1.0 / uu;
                    const double wx = cx - ox, wy = cy - oy, wz = cz - oz;
                    double ts = (wx * ux + wy * uy + wz * uz) * inv_uu;
                    if (ts < 0.0) ts = 0.0;
                    if (ts > dl) ts = dl;
                    const double qx = ox + ts * ux - cx;
                    const double qy = oy + ts * uy - cy;
                    const double qz = oz + ts * uz - cz;
                    if (qx * qx + qy * qy + qz * qz <= cr * cr) dm |= 1u << m;
                }
            }
        }
        // wave-wide append of detections: one atomic per wavefront (detections
        // are rare, so the scan runs only when some lane has one)
        if (__ballot(dm != 0u) != 0ull) {
            const int c = __popc(dm);
            int incl = c;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int t = __shfl_up(incl, off);
                if (lane >= off) incl += t;
            }
            const int total = __shfl(incl, kWave - 1);
            if (total > 0) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(&a.counters[0], (unsigned long long)total);
                base = __shfl(base, 0);
                unsigned long long pos = base + (unsigned long long)(incl - c);
                uint32_t bits = dm;
                while (bits) {
                    const int m = __ffs(bits) - 1;
                    bits &= bits - 1;
                    if (pos < (unsigned long long)a.det_cap) {
                        int32_t* d = a.det + 3 * pos;
                        d[0] = (int32_t)ray;
                        d[1] = k;
                        d[2] = rcv_off + m;
                    }
                    pos++;
                }
            }
        }
        bool susp = false;
        if (shading) {
            int32_t* hs = a.hit_seq + (int64_t)ray * R1;
            hs[k] = hit_id;
            const double Lc = len_s[tid];
            const int64_t srow = a.record ? (a.record_rows ? (int64_t)a.record_rows[ray] : (int64_t)ray) : -1;
            if (srow >= 0) {
                float* sp = a.states + (srow * (R1 + 1) + k) * 8;
                sp[0] = r.ox;
                sp[1] = r.oy;
                sp[2] = r.oz;
                sp[3] = r.ux;
                sp[4] = r.uy;
                sp[5] = r.uz;
                sp[6] = (float)Lc;
                sp[7] = __int_as_float(last_plane);
            }
            bool stop = true;
            if (hit_id >= 0) {
                const double nx = pl_n[3 * (int64_t)hit_plane], ny = pl_n[3 * (int64_t)hit_plane + 1],
                             nz = pl_n[3 * (int64_t)hit_plane + 2];
                const double udn = ux * nx + uy * ny + uz * nz;
                const double Ln = Lc + dl * sqrt(uu);
                r.ox = (float)(ox + dl * ux);
                r.oy = (float)(oy + dl * uy);
                r.oz = (float)(oz + dl * uz);
                r.ux = (float)(ux - 2.0 * udn * nx);
                r.uy = (float)(uy - 2.0 * udn * ny);
                r.uz = (float)(uz - 2.0 * udn * nz);
                len_s[tid] = Ln;
                last_plane = hit_plane;
                stop = (k == a.R) || Ln >= (double)lim;
                if (srow >= 0) {
                    float* sp = a.states + (srow * (R1 + 1) + k + 1) * 8;
                    sp[0] = r.ox;
                    sp[1] = r.oy;
                    sp[2] = r.oz;
                    sp[3] = r.ux;
                    sp[4] = r.uy;
                    sp[5] = r.uz;
                    sp[6] = (float)Ln;
                    sp[7] = __int_as_float(last_plane);
                }
            }
            if (stop) {
                status = kIdle;   // rest of the row keeps the -1 written by k_fill_rows
            } else if (a.suspend_k > 0 && a.q_out && k + 1 >= a.suspend_k) {
                // long chains: finish them in the next launch, all started together
                k++;
                susp = true;
                status = kIdle;
            } else {
                k++;
                setup_ray(r);
                cur = 0;
                st = Stack{0, 0, 0};
                best_t = INFINITY;
                best_j = -1;
                best_id = 0x7FFFFFFF;
                steps = 0;
                status = kQuery;
            }
        }
        if (a.suspend_k > 0 && a.q_out) {
            const uint64_t sm = __ballot(susp);
            if (sm) {
                const int leader = __ffsll((long long)sm) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(a.q_out_count, (unsigned long long)__popcll(sm));
                base = __shfl(base, leader);
                if (susp) {
                    const unsigned long long pos = base + (unsigned long long)lanes_below(sm);
                    if (pos < (unsigned long long)a.q_cap) {
                        int4* q = a.q_out + 3 * pos;
                        q[0] = make_int4((int)ray, k, last_plane, 0);
                        const double lq = len_s[tid];
                        q[1] = make_int4(__float_as_int(r.ox), __float_as_int(r.oy), __float_as_int(r.oz),
                                         __double2loint(lq));
                        q[2] = make_int4(__float_as_int(r.ux), __float_as_int(r.uy), __float_as_int(r.uz),
                                         __double2hiint(lq));
                    } else {
                        atomicOr(&a.counters[3], kErrQueue);
                    }
                }
            }
        }
    }
    // per-wave totals
    for (int off = kWave / 2; off > 0; off >>= 1) {
        if (want_stats) {
            st_nodes += __shfl_down(st_nodes, off);
            st_leaves += __shfl_down(st_leaves, off);
            st_tris += __shfl_down(st_tris, off);
            st_spill += __shfl_down(st_spill, off);
        }
    }
    if (lane == 0) {
        if (n_query) atomicAdd(&a.counters[1], (unsigned long long)n_query);
        if (n_escape) atomicAdd(&a.counters[2], (unsigned long long)n_escape);
        if (want_stats) {
            atomicAdd(&a.stats[0], (unsigned long long)st_nodes);
            atomicAdd(&a.stats[1], (unsigned long long)st_leaves);
            atomicAdd(&a.stats[2], (unsigned long long)st_tris);
            atomicAdd(&a.stats[3], (unsigned long long)st_spill);
        }
    }
}

// Sort key of a ray: Morton code of its direction's octahedral map (8 bits
// per axis) in the low 16 bits and, for per-ray origins, the Morton code of
// the origin in the scene box (10 bits per axis) above it.
__device__ inline uint32_t spread16(uint32_t x) {
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}
__device__ inline uint64_t spread10(uint64_t x) {
    x &= 0x3FFull;
    x = (x | (x << 16)) & 0x30000FFull;
    x = (x | (x << 8)) & 0x300F00Full;
    x = (x | (x << 4)) & 0x30C30C3ull;
    x = (x | (x << 2)) & 0x9249249ull;
    return x;
}

__global__ void k_ray_keys(const float* __restrict__ dirs, const float* __restrict__ origins, int64_t n,
                           float bx0, float by0, float bz0, float inv_ext, uint64_t* __restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = dirs[3 * i], y = dirs[3 * i + 1], z = dirs[3 * i + 2];
    const float s = fabsf(x) + fabsf(y) + fabsf(z);
    float u = 0.f, v = 0.f;
    if (s > 0.f) {
        x /= s;
        y /= s;
        z /= s;
        if (z < 0.f) {
            const float ox = (1.f - fabsf(y)) * (x >= 0.f ? 1.f : -1.f);
            const float oy = (1.f - fabsf(x)) * (y >= 0.f ? 1.f : -1.f);
            x = ox;
            y = oy;
        }
        u = fminf(fmaxf((x + 1.f) * 0.5f, 0.f), 1.f);
        v = fminf(fmaxf((y + 1.f) * 0.5f, 0.f), 1.f);
    }
    const uint32_t qu = (uint32_t)(u * 255.f), qv = (uint32_t)(v * 255.f);
    uint64_t k = (uint64_t)(spread16(qu) | (spread16(qv) << 1));
    if (origins) {
        const float ox = fminf(fmaxf((origins[3 * i] - bx0) * inv_ext, 0.f), 1.f);
        const float oy = fminf(fmaxf((origins[3 * i + 1] - by0) * inv_ext, 0.f), 1.f);
        const float oz = fminf(fmaxf((origins[3 * i + 2] - bz0) * inv_ext, 0.f), 1.f);
        const uint64_t m = (spread10((uint64_t)(ox * 1023.f)) << 2) | (spread10((uint64_t)(oy * 1023.f)) << 1) |
                           spread10((uint64_t)(oz * 1023.f));
        k |= m << 16;
    }
    key[i] = k;
}

// hit_seq <- -1 with 16-byte stores (rows are then written only where hit).
// The -1 fill of the hit rows streams past the caches (non-temporal stores), so
// that the tree and triangle records the trace is about to read stay in L2 and
// the Infinity Cache (a million rows of 61 entries are larger than both).
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
__global__ void k_fill_rows(int32_t* __restrict__ p, int64_t n) {
    const int64_t n4 = n >> 2;
    v4i32* q = reinterpret_cast<v4i32*>(p);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const v4i32 m1 = {-1, -1, -1, -1};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(m1, q + i);
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = -1;
}

__global__ void k_fill_rows_scalar(int32_t* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = -1;
}

// Fibonacci sphere: z_i = 1 - (2i+1)/n, phi_i = i pi (3 - sqrt5) mod 2 pi.
__global__ void k_fibonacci(int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    fibonacci_dir(i, n, out + 3 * i);
}

template <bool kBatch, int kRing>
void launch_trace_ring(int occ, unsigned nblk, hipStream_t st, const TraceArgs& a) {
    if (a.stats) {   // traversal counts: the 4-wave instance that keeps them
        hipLaunchKernelGGL((k_trace<4, kBatch, kRing, true>), dim3(nblk), dim3(kBlock), 0, st, a);
        return;
    }
    switch (occ) {
        case 8: hipLaunchKernelGGL((k_trace<8, kBatch, kRing, false>), dim3(nblk), dim3(kBlock), 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_trace<6, kBatch, kRing, false>), dim3(nblk), dim3(kBlock), 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_trace<5, kBatch, kRing, false>), dim3(nblk), dim3(kBlock), 0, st, a); break;
        default: hipLaunchKernelGGL((k_trace<4, kBatch, kRing, false>), dim3(nblk), dim3(kBlock), 0, st, a); break;
    }
}

template <bool kBatch>
void launch_trace_batch(int occ, int ring, unsigned nblk, hipStream_t st, const TraceArgs& a) {
    switch (ring) {
        case 8: launch_trace_ring<kBatch, 8>(occ, nblk, st, a); break;
        case 32: launch_trace_ring<kBatch, 32>(occ, nblk, st, a); break;
        default: launch_trace_ring<kBatch, kRingDefault>(occ, nblk, st, a); break;
    }
}

void launch_trace(int occ, int ring, bool batch, unsigned nblk, hipStream_t st, const TraceArgs& a) {
    if (batch) launch_trace_batch<true>(occ, ring, nblk, st, a);
    else launch_trace_batch<false>(occ, ring, nblk, st, a);
}

}  // namespace

}  // namespace rtac

using namespace rtac;

extern "C" int rt_fibonacci_directions(int64_t n, float* dirs, void* stream) {
    RT_CHECK(n >= 0, RT_EINVAL, "rt_fibonacci_directions: n < 0");
    if (n == 0) return RT_OK;
    RT_CHECK(dirs != nullptr, RT_EINVAL, "rt_fibonacci_directions: dirs is NULL");
    hipLaunchKernelGGL(k_fibonacci, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, dirs);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

namespace rtac {
namespace {

// Shared host part of the single-scene and batched traces: ray order, row
// fill, launches.  `ws` is the scene whose workspace holds the scratch.
int run_trace(rt_scene* ws, TraceArgs& a, const rt_trace_params* p, int depth, int64_t max_steps, int64_t n_rays,
              int32_t* hit_seq, const float* dirs, const float* origins, const float* bounds, hipStream_t st) {
    // 4 waves per SIMD by default: the 128-register budget of the kernel spills nothing.  A fifth
    // wavefront (96 registers, spills around the shading) raises the busy-phase rate of closed rooms a
    // little (the 100k-triangle box: 3 %) but slows the drain of an open scene's long bounce chains
    // (the theater: 9 %); the batched instance keeps a per-lane scene view and spills in its node loop
    // at 96 registers (5 and 6 waves are 42 % and 67 % slower on the 8-room batch).
    const int wps = p->waves_per_simd;
    const int occ = (wps == 4 || wps == 5 || wps == 6 || wps == 8) ? wps : 4;
    const int bpc = p->blocks_per_cu > 0 ? p->blocks_per_cu : occ;
    const int ring = p->stack_depth > 0 ? p->stack_depth : kRingDefault;
    int64_t nblk = (int64_t)device_sm_count() * bpc;
    const int64_t need = (n_rays + kBlock - 1) / kBlock;
    if (nblk > need) nblk = need;
    if (nblk < 1) nblk = 1;
    const int spill_n = ((3 * (depth + 1) + 2 * kSpillChunk) / kSpillChunk + 1) * kSpillChunk;
    if (ws->ws.stack_spill.ensure(sizeof(int32_t) * (size_t)nblk * kBlock * spill_n)) return RT_ENOMEM;
    a.spill = ws->ws.stack_spill.as<int32_t>();
    a.spill_per_lane = spill_n;
    a.fetch_thr = p->fetch_threshold > 0 ? p->fetch_threshold : 16;
    // shading batches: with one segment per ray a lane stops after it, so larger batches only save
    // shading rounds; with several, finished lanes should not wait long for the next segment
    a.shade_thr = p->shade_threshold > 0 ? p->shade_threshold : (p->max_reflections == 0 ? 48 : 16);
    a.scale_shade = p->max_reflections > 0 ? 1 : 0;
    a.max_steps = max_steps > 0x7FFFFFFF ? 0x7FFFFFFF : (int32_t)max_steps;
    a.order = nullptr;
    a.stats = (unsigned long long*)p->stats;
    if (!p->keep_order && n_rays > 1 && dirs) {
        Workspace& w = ws->ws;
        if (w.sort_keys[0].ensure(8 * n_rays) || w.sort_keys[1].ensure(8 * n_rays) ||
            w.sort_vals[0].ensure(4 * n_rays) || w.sort_vals[1].ensure(4 * n_rays))
            return RT_ENOMEM;
        float ext = 0.f;
        for (int c = 0; c < 3; c++) ext = fmaxf(ext, bounds[3 + c] - bounds[c]);
        hipLaunchKernelGGL(k_ray_keys, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, st, dirs, origins,
                           n_rays, bounds[0], bounds[1], bounds[2], ext > 0.f ? 1.f / ext : 0.f,
                           w.sort_keys[0].as<uint64_t>());
        int which = 0;
        int rc = radix_sort_pairs(w, w.sort_keys[0].as<uint64_t>(), w.sort_vals[0].as<uint32_t>(),
                                  w.sort_keys[1].as<uint64_t>(), w.sort_vals[1].as<uint32_t>(), n_rays, nullptr, 0,
                                  origins ? 48 : 16, st, &which, true);
        if (rc) return rc;
        a.order = which ? w.sort_vals[1].as<uint32_t>() : w.sort_vals[0].as<uint32_t>();
    }
    {
        const int64_t cells = n_rays * (int64_t)(p->max_reflections + 1);
        int64_t fb = (cells / 4 + 255) / 256;
        const int64_t fcap = (int64_t)device_sm_count() * 16;
        if (fb > fcap) fb = fcap;
        if (fb < 1) fb = 1;
        if (((uintptr_t)hit_seq & 15u) == 0) {
            hipLaunchKernelGGL(k_fill_rows, dim3((unsigned)fb), dim3(256), 0, st, hit_seq, cells);
        } else {
            hipLaunchKernelGGL(k_fill_rows_scalar, dim3((unsigned)fb), dim3(256), 0, st, hit_seq, cells);
        }
    }
    // continuation rounds: launch rd takes the rays left over by launch rd-1;
    // every launch hands over at most one ray per lane, so a queue of one
    // entry per lane of the grid never overflows.  With suspension, launch 0
    // traces every ray up to segment suspend_after - 1 and queues the rays
    // that go on (at most all of them); launch 1 finishes those together.
    const bool suspend = p->suspend_after > 0 && p->suspend_after <= p->max_reflections;
    const int rounds = suspend ? 2 : (p->rounds > 0 ? (p->rounds < 16 ? p->rounds : 16) : 1);
    const int64_t lanes = nblk * kBlock;
    const int64_t qcap = suspend ? (n_rays > lanes ? n_rays : lanes) : lanes;
    if (ws->ws.generic[0].ensure(sizeof(int32_t) * kQueueInts * (size_t)qcap * 2)) return RT_ENOMEM;
    int4* qbuf[2] = {ws->ws.generic[0].as<int4>(), ws->ws.generic[0].as<int4>() + 3 * qcap};
    a.q_cap = qcap;
    const int32_t spill_thr = p->spill_threshold > 0 ? p->spill_threshold : 24;
    unsigned long long* pool = a.pool;
    if (p->kernel_event_start) RT_HIP(hipEventRecord((hipEvent_t)p->kernel_event_start, st));
    for (int rd = 0; rd < rounds; rd++) {
        a.pool = pool + rd;
        a.pool_xcd = rd == 0 && p->xcd_pools >= 0 ? pool + 32 : nullptr;
        a.q_in = rd == 0 ? nullptr : qbuf[(rd - 1) & 1];
        a.q_in_count = rd == 0 ? nullptr : pool + 16 + (rd - 1);
        a.q_out = rd + 1 < rounds ? qbuf[rd & 1] : nullptr;
        a.q_out_count = pool + 16 + rd;
        a.suspend_k = suspend && rd == 0 ? p->suspend_after : 0;
        a.spill_thr = suspend ? 0 : spill_thr;
        if (rd > 0) a.order = nullptr;
        launch_trace(occ, ring, a.jobs != nullptr, (unsigned)nblk, st, a);
    }
    RT_HIP(hipGetLastError());
    if (p->kernel_event_stop) RT_HIP(hipEventRecord((hipEvent_t)p->kernel_event_stop, st));
    return RT_OK;
}

int check_params(const rt_trace_params* p) {
    RT_CHECK(p, RT_EINVAL, "null params");
    RT_CHECK(p->max_reflections >= 0 && p->max_reflections < 4096, RT_EINVAL,
             "max_reflections must be in [0, 4096)");
    RT_CHECK(p->suspend_after >= 0, RT_EINVAL, "suspend_after must be >= 0");
    RT_CHECK(p->min_beam_rays >= 0, RT_EINVAL, "min_beam_rays must be >= 0");
    RT_CHECK(p->xcd_pools >= -1 && p->xcd_pools <= 0, RT_EINVAL, "xcd_pools must be 0 or -1");
    RT_CHECK(p->coop_queries >= -1 && p->coop_queries <= 0, RT_EINVAL, "coop_queries must be 0 or -1");
    RT_CHECK(p->stack_depth == 0 || p->stack_depth == 8 || p->stack_depth == 16 || p->stack_depth == 32, RT_EINVAL,
             "stack_depth must be 0 (default 16), 8, 16 or 32");
    return RT_OK;
}

}  // namespace
}  // namespace rtac

extern "C" int rt_trace_rays(const rt_scene* scene, const float* src_host, const float* origins, const float* dirs,
                             const int32_t* start_plane, const float* start_len, int64_t n_rays, const float* rcv,
                             int32_t n_rcv, const rt_trace_params* p, int32_t* hit_seq, int32_t* det, int64_t det_cap,
                             int64_t* counters, float* states, void* stream) {
    CallStream call_stream((hipStream_t)stream);
    RT_CHECK(scene && p, RT_EINVAL, "rt_trace_rays: null scene or params");
    RT_CHECK(scene->valid, RT_EINVAL, "rt_trace_rays: the scene's last rebuild failed");
    RT_CHECK(n_rays >= 0 && n_rays < ((int64_t)1 << 31), RT_EINVAL, "rt_trace_rays: n_rays out of range");
    if (check_params(p)) return RT_EINVAL;
    RT_CHECK(n_rcv >= 0 && n_rcv <= kMaxRcv, RT_EINVAL, "rt_trace_rays: n_rcv must be in [0, %d]", kMaxRcv);
    RT_CHECK(n_rcv == 0 || rcv, RT_EINVAL, "rt_trace_rays: rcv is NULL");
    RT_CHECK(counters, RT_EINVAL, "rt_trace_rays: counters is NULL");
    RT_CHECK(det_cap >= 0 && (det_cap == 0 || det), RT_EINVAL, "rt_trace_rays: det is NULL");
    RT_CHECK(!p->record_states || states, RT_EINVAL, "rt_trace_rays: record_states needs states");
    RT_CHECK(origins || src_host, RT_EINVAL, "rt_trace_rays: need src_host or origins");
    RT_CHECK(n_rays == 0 || (dirs && hit_seq), RT_EINVAL, "rt_trace_rays: dirs/hit_seq is NULL");
    hipStream_t st = (hipStream_t)stream;
    rt_scene* s = const_cast<rt_scene*>(scene);
    if (s->ws.trace_pool.ensure(kPoolWords * sizeof(unsigned long long))) return RT_ENOMEM;
    unsigned long long* pool = s->ws.trace_pool.as<unsigned long long>();
    hipLaunchKernelGGL(k_trace_reset, dim3(1), dim3(64), 0, st, (unsigned long long*)counters, pool,
                       (unsigned long long*)p->stats);
    if (n_rays == 0) {
        RT_HIP(hipGetLastError());
        return RT_OK;
    }
    TraceArgs a{};
    a.nodes = s->nodes;
    a.tri = s->tri_rec;
    a.plane_n = s->plane_n;
    a.plane_p = s->plane_p;
    a.n_nodes = s->n_nodes;
    a.n_ref = (int32_t)s->n_ref;
    a.src[0] = src_host ? src_host[0] : 0.f;
    a.src[1] = src_host ? src_host[1] : 0.f;
    a.src[2] = src_host ? src_host[2] : 0.f;
    a.origins = origins;
    a.dirs = dirs;
    a.start_plane = start_plane;
    a.start_len = start_len;
    a.n_rays = n_rays;
    a.rcv = rcv;
    a.n_rcv = n_rcv;
    a.R = p->max_reflections;
    a.max_len = p->max_path_length;
    a.beam_n = p->min_beam_rays;
    // the statistics count the per-lane traversal only: requesting them turns
    // the cooperative search off, so that every step of every query is counted
    a.coop = p->coop_queries >= 0 && !p->stats ? 1 : 0;
    a.record = p->record_states ? 1 : 0;
    a.record_rows = p->record_rows;
    a.hit_seq = hit_seq;
    a.det = det;
    a.det_cap = det_cap;
    a.counters = (unsigned long long*)counters;
    a.pool = pool;
    a.states = states;
    a.jobs = nullptr;
    a.scenes = nullptr;
    a.n_jobs = 0;
    return run_trace(s, a, p, s->depth, 8 * ((int64_t)s->n_nodes + s->n_ref) + 4096, n_rays, hit_seq, dirs,
                     origins, s->bounds, st);
}

// ---------------------------------------------------------------------------
// batches of jobs over several scenes
// ---------------------------------------------------------------------------

extern "C" int rt_batch_create(const rt_scene* const* scenes, int32_t n_scenes, const rt_job* jobs, int32_t n_jobs,
                               void* stream, rt_batch** out) {
    RT_CHECK(out, RT_EINVAL, "rt_batch_create: out is NULL");
    *out = nullptr;
    RT_CHECK(scenes && jobs && n_scenes >= 1 && n_jobs >= 1, RT_EINVAL, "rt_batch_create: empty batch");
    std::vector<DevScene> hs(n_scenes);
    int32_t mat_off = 0;
    for (int i = 0; i < n_scenes; i++) {
        const rt_scene* s = scenes[i];
        RT_CHECK(s, RT_EINVAL, "rt_batch_create: scene %d is NULL", i);
        RT_CHECK(s->valid, RT_EINVAL, "rt_batch_create: scene %d: its last rebuild failed", i);
        hs[i] = DevScene{s->nodes, s->tri_rec, s->plane_n, s->plane_p, s->plane_mat, s->tri_plane, s->n_nodes,
                         (int32_t)s->n_tri, mat_off, s->n_mat, (int32_t)s->n_ref, 0};
        mat_off += s->n_mat;
    }
    std::vector<DevJob> hj(n_jobs);
    int64_t ray_off = 0;
    int32_t rcv_off = 0;
    std::vector<int32_t> rcv_job;
    for (int j = 0; j < n_jobs; j++) {
        const rt_job& jb = jobs[j];
        RT_CHECK(jb.scene >= 0 && jb.scene < n_scenes, RT_EINVAL, "rt_batch_create: job %d: bad scene", j);
        RT_CHECK(jb.n_rcv >= 1 && jb.n_rcv <= kMaxRcv, RT_EINVAL, "rt_batch_create: job %d: n_rcv in [1, %d]", j,
                 kMaxRcv);
        RT_CHECK(jb.n_rays >= 1, RT_EINVAL, "rt_batch_create: job %d: n_rays < 1", j);
        hj[j] = DevJob{ray_off, jb.n_rays, {jb.src[0], jb.src[1], jb.src[2]}, jb.max_path_length, jb.scene, rcv_off,
                       jb.n_rcv, 0};
        ray_off += jb.n_rays;
        for (int m = 0; m < jb.n_rcv; m++) rcv_job.push_back(j);
        rcv_off += jb.n_rcv;
    }
    RT_CHECK(ray_off < ((int64_t)1 << 31), RT_EINVAL, "rt_batch_create: more than 2^31 rays");
    rt_batch* b = new rt_batch();
    b->n_scenes = n_scenes;
    b->n_jobs = n_jobs;
    b->n_rcv = rcv_off;
    b->n_mat = mat_off;
    b->n_rays = ray_off;
    b->ws_owner = const_cast<rt_scene*>(scenes[0]);
    int depth = 0;
    int64_t steps = 0;
    for (int i = 0; i < n_scenes; i++) {
        depth = depth > scenes[i]->depth ? depth : scenes[i]->depth;
        const int64_t ms = 8 * ((int64_t)scenes[i]->n_nodes + scenes[i]->n_ref) + 4096;
        steps = steps > ms ? steps : ms;
    }
    b->max_depth = depth;
    b->max_steps = steps;
    b->scenes = (DevScene*)dcache_alloc(sizeof(DevScene) * n_scenes);
    b->jobs = (DevJob*)dcache_alloc(sizeof(DevJob) * n_jobs);
    b->rcv_job = (int32_t*)dcache_alloc(sizeof(int32_t) * rcv_off);
    if (!b->scenes || !b->jobs || !b->rcv_job) {
        rt_batch_destroy(b);
        set_error("rt_batch_create: out of device memory");
        return RT_ENOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(b->scenes, hs.data(), sizeof(DevScene) * n_scenes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->jobs, hj.data(), sizeof(DevJob) * n_jobs, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->rcv_job, rcv_job.data(), sizeof(int32_t) * rcv_off, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        rt_batch_destroy(b);
        set_error("rt_batch_create: upload failed");
        return RT_EHIP;
    }
    RT_HIP(hipGetDevice(&b->device));
    *out = b;
    return RT_OK;
}

extern "C" int rt_batch_destroy(rt_batch* b) {
    if (!b) return RT_OK;
    (void)hipDeviceSynchronize();
    dcache_free(b->scenes);
    dcache_free(b->jobs);
    dcache_free(b->rcv_job);
    delete b;
    return RT_OK;
}

extern "C" int rt_batch_info(const rt_batch* b, int64_t* info_host) {
    RT_CHECK(b && info_host, RT_EINVAL, "rt_batch_info: null argument");
    info_host[0] = b->n_jobs;
    info_host[1] = b->n_rays;
    info_host[2] = b->n_rcv;
    info_host[3] = b->n_mat;
    return RT_OK;
}

extern "C" int rt_trace_batch(rt_batch* b, const float* rcv, const rt_trace_params* p, int32_t* hit_seq, int32_t* det,
                              int64_t det_cap, int64_t* counters, float* states, void* stream) {
    CallStream call_stream((hipStream_t)stream);
    RT_CHECK(b && rcv && hit_seq && counters, RT_EINVAL, "rt_trace_batch: null argument");
    if (check_params(p)) return RT_EINVAL;
    RT_CHECK(!p->record_states || states, RT_EINVAL, "rt_trace_batch: record_states needs states");
    RT_CHECK(det_cap >= 0 && (det_cap == 0 || det), RT_EINVAL, "rt_trace_batch: det is NULL");
    hipStream_t st = (hipStream_t)stream;
    rt_scene* s = b->ws_owner;
    if (s->ws.trace_pool.ensure(kPoolWords * sizeof(unsigned long long))) return RT_ENOMEM;
    unsigned long long* pool = s->ws.trace_pool.as<unsigned long long>();
    hipLaunchKernelGGL(k_trace_reset, dim3(1), dim3(64), 0, st, (unsigned long long*)counters, pool,
                       (unsigned long long*)p->stats);
    TraceArgs a{};
    a.n_rays = b->n_rays;
    a.rcv = rcv;
    a.R = p->max_reflections;
    a.beam_n = p->min_beam_rays;
    a.coop = p->coop_queries >= 0 && !p->stats ? 1 : 0;
    a.record = p->record_states ? 1 : 0;
    a.record_rows = p->record_rows;
    a.states = states;
    a.hit_seq = hit_seq;
    a.det = det;
    a.det_cap = det_cap;
    a.counters = (unsigned long long*)counters;
    a.pool = pool;
    a.jobs = b->jobs;
    a.scenes = b->scenes;
    a.n_jobs = b->n_jobs;
    float bounds[6] = {0, 0, 0, 1, 1, 1};
    return run_trace(s, a, p, b->max_depth, b->max_steps, b->n_rays, hit_seq, nullptr, nullptr, bounds, st);
}
