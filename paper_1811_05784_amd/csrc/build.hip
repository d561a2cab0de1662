// Scene ingest and acceleration tree (rt_build_tree, rt_rebuild_tree).
//
// The paper builds its tree once per mesh: a mother box holding every
// element is split into two daughter boxes, recursively, down to one element
// per leaf (section "Tree-base acceleration").  Here the splits come from the
// Morton order of the triangle centroids: a binary radix tree (one leaf per
// triangle, every inner node separating one Morton prefix) built in one
// parallel pass, boxes refitted bottom-up, then every other level folded so
// that traversal sees a 4-wide tree with 128-byte nodes (one cache line per
// node on gfx950).  Subtrees of at most `leaf_size` triangles become leaves.
//
// Before the tree is built, thin triangles are cut into references (early
// split clipping, Ernst and Greiner 2007): a triangle whose bounding box has
// a surface above kEscTau times twice the triangle's area (a flat right
// triangle in an axis plane has 2) is cut into k slabs along the longest side
// of its box, and each reference carries the
// box of its piece only.  Fans of sliver triangles (a ring mesh around its
// centre) otherwise give hundreds of overlapping boxes around one point, and
// a query through that point tests every one of them.  A triangle may thus
// sit in several leaves; nearest hits do not change (the same triangle is
// tested again at the same distance).
//
// Everything per reference that traversal and shading need is re-laid out in
// tree order (48 B per reference) so a leaf is a contiguous range.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace rtac {

namespace {

enum : uint32_t {
    kErrIndex = 1u,
    kErrNonFinite = 2u,
    kErrZeroArea = 4u,
    kErrPlaneRange = 8u,
    kErrMaterial = 16u,
    kErrNotCoplanar = 32u,
    kErrMixedMaterial = 64u,
};

__device__ inline uint32_t ford(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float funord(uint32_t u) {
    uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    return __builtin_bit_cast(float, b);
}

// Per workgroup: part[14 b + 0..5] = vertex box (min xyz ordered, max xyz
// ordered), [6..11] = centroid box, [12] = error bits, [13] = max material;
// k_prep_reduce folds the workgroups' values (no contended global atomics).
__global__ void __launch_bounds__(256) k_tri_prep(const float* __restrict__ vtx, int64_t nv,
                                                  const int3* __restrict__ tri, int64_t nt,
                                                  const int32_t* __restrict__ material,
                                                  const int32_t* __restrict__ plane_id, float* __restrict__ tri_box,
                                                  float* __restrict__ centroid, uint32_t* __restrict__ part,
                                                  int32_t* __restrict__ prep) {
    __shared__ uint32_t sb[12];
    __shared__ uint32_t s_err, s_mat;
    const int tid = threadIdx.x;
    if (tid < 12) sb[tid] = (tid % 6) < 3 ? 0xFFFFFFFFu : 0u;
    if (tid == 0) {
        s_err = 0;
        s_mat = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
    // this lane's contribution to the 12 bounds (identity when it has none)
    uint32_t bl[12];
    for (int k = 0; k < 12; k++) bl[k] = (k % 6) < 3 ? 0xFFFFFFFFu : 0u;
    uint32_t mat_l = 0;
    bool plane_ok = false;   // valid triangle whose plane id may vote for the representative
    if (i < nt) {
        const int3 t = tri[i];
        uint32_t err = 0;
        if (t.x < 0 || t.y < 0 || t.z < 0 || t.x >= nv || t.y >= nv || t.z >= nv) err |= kErrIndex;
        const int32_t p = plane_id ? plane_id[i] : (int32_t)i;
        if (p < 0 || p >= nt) err |= kErrPlaneRange;
        const int32_t m = material[i];
        if (m < 0) err |= kErrMaterial;
        float v[3][3];
        if (!err) {
            const int idx[3] = {t.x, t.y, t.z};
            bool finite = true;
            for (int a = 0; a < 3; a++)
                for (int c = 0; c < 3; c++) {
                    v[a][c] = vtx[3 * (int64_t)idx[a] + c];
                    finite &= isfinite(v[a][c]);
                }
            if (!finite) err |= kErrNonFinite;
        }
        if (!err) {
            double e1[3], e2[3];
            for (int c = 0; c < 3; c++) {
                e1[c] = (double)v[1][c] - (double)v[0][c];
                e2[c] = (double)v[2][c] - (double)v[0][c];
            }
            const double cx = e1[1] * e2[2] - e1[2] * e2[1];
            const double cy = e1[2] * e2[0] - e1[0] * e2[2];
            const double cz = e1[0] * e2[1] - e1[1] * e2[0];
            if (cx == 0.0 && cy == 0.0 && cz == 0.0) err |= kErrZeroArea;
            mat_l = (uint32_t)m;
            plane_ok = true;
            for (int c = 0; c < 3; c++) {
                const float lo = fminf(v[0][c], fminf(v[1][c], v[2][c]));
                const float hi = fmaxf(v[0][c], fmaxf(v[1][c], v[2][c]));
                tri_box[6 * i + c] = lo;
                tri_box[6 * i + 3 + c] = hi;
                const float cen = (v[0][c] + v[1][c] + v[2][c]) * (1.0f / 3.0f);
                centroid[3 * i + c] = cen;
                bl[c] = ford(lo);
                bl[3 + c] = ford(hi);
                bl[6 + c] = ford(cen);
                bl[9 + c] = ford(cen);
            }
        } else {
            for (int c = 0; c < 3; c++) {
                tri_box[6 * i + c] = 0.f;
                tri_box[6 * i + 3 + c] = 0.f;
                centroid[3 * i + c] = 0.f;
            }
        }
        if (err) atomicOr(&s_err, err);
    }
    // plane representative = lowest triangle index of each plane id: only the
    // first lane of a run of equal ids in a wavefront (the lowest index of the
    // run) competes, and only while it can still lower the stored value
    {
        const int32_t pid = (i < nt && plane_ok) ? (plane_id ? plane_id[i] : (int32_t)i) : -1;
        const int32_t prev = __shfl_up(pid, 1);
        const bool first_of_run = (tid & (kWave - 1)) == 0 || prev != pid;
        if (pid >= 0 && first_of_run && (int32_t)i < prep[pid]) atomicMin(&prep[pid], (int32_t)i);
    }
    // wave reductions, then one LDS atomic per wave and bound
    for (int off = kWave / 2; off > 0; off >>= 1) {
        for (int k = 0; k < 12; k++) {
            const uint32_t o = __shfl_down(bl[k], off);
            bl[k] = (k % 6) < 3 ? (o < bl[k] ? o : bl[k]) : (o > bl[k] ? o : bl[k]);
        }
        const uint32_t om = __shfl_down(mat_l, off);
        mat_l = om > mat_l ? om : mat_l;
    }
    if ((tid & (kWave - 1)) == 0) {
        for (int k = 0; k < 12; k++) {
            if ((k % 6) < 3) atomicMin(&sb[k], bl[k]);
            else atomicMax(&sb[k], bl[k]);
        }
        atomicMax(&s_mat, mat_l);
    }
    __syncthreads();
    uint32_t* pb = part + 14 * (int64_t)blockIdx.x;
    if (tid < 12) pb[tid] = sb[tid];
    if (tid == 12) pb[12] = s_err;
    if (tid == 13) pb[13] = s_mat;
}

// bounds[0..11] and info[0..1] from the per-workgroup values of k_tri_prep
// (one workgroup; min / max / or in a fixed order).
__global__ void __launch_bounds__(256) k_prep_reduce(const uint32_t* __restrict__ part, int64_t nb,
                                                     uint32_t* __restrict__ bounds, uint32_t* __restrict__ info) {
    __shared__ uint32_t red[14][256 / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
    uint32_t v[14];
    for (int k = 0; k < 14; k++) v[k] = (k < 12 && (k % 6) < 3) ? 0xFFFFFFFFu : 0u;
    for (int64_t b = tid; b < nb; b += 256)
        for (int k = 0; k < 14; k++) {
            const uint32_t x = part[14 * b + k];
            v[k] = k == 12 ? (v[k] | x) : ((k < 12 && (k % 6) < 3) ? (x < v[k] ? x : v[k]) : (x > v[k] ? x : v[k]));
        }
    for (int off = kWave / 2; off > 0; off >>= 1)
        for (int k = 0; k < 14; k++) {
            const uint32_t x = __shfl_down(v[k], off);
            v[k] = k == 12 ? (v[k] | x) : ((k < 12 && (k % 6) < 3) ? (x < v[k] ? x : v[k]) : (x > v[k] ? x : v[k]));
        }
    if (lane == 0)
        for (int k = 0; k < 14; k++) red[k][w] = v[k];
    __syncthreads();
    if (tid < 14) {
        uint32_t r = red[tid][0];
        for (int j = 1; j < 256 / kWave; j++) {
            const uint32_t x = red[tid][j];
            r = tid == 12 ? (r | x) : ((tid < 12 && (tid % 6) < 3) ? (x < r ? x : r) : (x > r ? x : r));
        }
        if (tid < 12) bounds[tid] = r;
        else info[tid - 12] = r;
    }
}

// Plane table (FP64) from each plane id's representative (lowest index).
__global__ void k_plane_table(const float* __restrict__ vtx, const int3* __restrict__ tri, int64_t nt,
                              const int32_t* __restrict__ material, const int32_t* __restrict__ prep,
                              double* __restrict__ pn, double* __restrict__ pp, int32_t* __restrict__ pmat) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nt) return;
    const int32_t r = prep[p];
    if (r == INT32_MAX) {
        for (int c = 0; c < 3; c++) pn[3 * p + c] = pp[3 * p + c] = __longlong_as_double(0x7FF8000000000000ll);
        pmat[p] = -1;
        return;
    }
    const int3 t = tri[r];   // r passed validation in k_tri_prep
    double a[3], b[3], cc[3];
    for (int c = 0; c < 3; c++) {
        a[c] = vtx[3 * (int64_t)t.x + c];
        b[c] = vtx[3 * (int64_t)t.y + c];
        cc[c] = vtx[3 * (int64_t)t.z + c];
    }
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {cc[0] - a[0], cc[1] - a[1], cc[2] - a[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int c = 0; c < 3; c++) {
        pn[3 * p + c] = n[c] / len;
        pp[3 * p + c] = a[c];
    }
    pmat[p] = material[r];
}

// Members of a plane group lie in the representative's plane (1e-9 D, D the
// bounding-box diagonal) and share its material.  Also records the plane id
// of every triangle.  Triangles that failed validation are skipped.
__global__ void k_coplanar(const float* __restrict__ vtx, int64_t nv, const int3* __restrict__ tri, int64_t nt,
                           const int32_t* __restrict__ material, const int32_t* __restrict__ plane_id,
                           const double* __restrict__ pn, const double* __restrict__ pp,
                           const int32_t* __restrict__ pmat, const uint32_t* __restrict__ bounds,
                           int32_t* __restrict__ tri_plane, uint32_t* __restrict__ info) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    const int32_t p = plane_id ? plane_id[i] : (int32_t)i;
    const int3 t = tri[i];
    const bool ok = p >= 0 && p < nt && t.x >= 0 && t.y >= 0 && t.z >= 0 && t.x < nv && t.y < nv && t.z < nv;
    tri_plane[i] = ok ? p : 0;
    if (!ok) return;
    double d2 = 0.0;
    for (int c = 0; c < 3; c++) {
        const double e = (double)funord(bounds[3 + c]) - (double)funord(bounds[c]);
        d2 += e * e;
    }
    const double tol = 1e-9 * sqrt(d2);
    if (material[i] != pmat[p]) atomicOr(&info[0], kErrMixedMaterial);
    const int idx[3] = {t.x, t.y, t.z};
    for (int a = 0; a < 3; a++) {
        double d = 0;
        for (int c = 0; c < 3; c++) d += ((double)vtx[3 * (int64_t)idx[a] + c] - pp[3 * p + c]) * pn[3 * p + c];
        if (!(fabs(d) <= tol)) atomicOr(&info[0], kErrNotCoplanar);
    }
}

__device__ inline uint64_t spread21(uint64_t x) {
    x &= 0x1FFFFFull;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// 30-bit Morton code of the centre of a reference's box, quantised to 2^10
// cells per axis on a cube spanning the scene box (equal cells on every axis;
// equal codes are ordered by reference index).  Box centres split sliver
// triangles' boxes better than triangle centroids do (fewer node visits per
// query on the theater and the jittered box).  Ten bits per axis sort in four 8-bit passes;
// on the workloads here (436k-triangle theater, 2^20-triangle tetrahedron,
// lattice rooms up to 177k triangles) the trees trace as fast as with 16
// bits per axis and six passes.  A small dense object in a large empty box
// would share codes more often: equal codes split by index, which is correct
// but gives looser boxes.
constexpr int kMortonBits = 10;
constexpr float kMortonMax = (float)((1 << kMortonBits) - 1);
__global__ void k_morton(const float* __restrict__ ref_box, int64_t nr, const uint32_t* __restrict__ bounds,
                         uint64_t* __restrict__ code) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    float lo[3], ext = 0.f;
    for (int c = 0; c < 3; c++) {
        lo[c] = funord(bounds[c]);
        ext = fmaxf(ext, funord(bounds[3 + c]) - lo[c]);
    }
    const float scale = ext > 0.f ? kMortonMax / ext : 0.f;
    uint64_t q[3];
    for (int c = 0; c < 3; c++) {
        const float centre = 0.5f * (ref_box[6 * i + c] + ref_box[6 * i + 3 + c]);
        float f = (centre - lo[c]) * scale;
        f = fminf(fmaxf(f, 0.f), kMortonMax);
        q[c] = (uint64_t)f;
    }
    code[i] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
}

// ---------------------------------------------------------------------------
// early split clipping
// ---------------------------------------------------------------------------
constexpr double kEscTau = 16.0;  // box surface / (2 x triangle area) above which a triangle is cut
constexpr int kEscMax = 64;       // most references per triangle

// The triangle's vertices in FP64, or false when its indices or coordinates
// are invalid (reported by the validation; it then gets one reference).
__device__ inline bool esc_vertices(const float* __restrict__ vtx, int64_t nv, const int3* __restrict__ tri,
                                    int64_t t, double (&p)[3][3]) {
    const int3 v = tri[t];
    if (v.x < 0 || v.y < 0 || v.z < 0 || v.x >= nv || v.y >= nv || v.z >= nv) return false;
    const int idx[3] = {v.x, v.y, v.z};
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            const float f = vtx[3 * (int64_t)idx[a] + c];
            if (!isfinite(f)) return false;
            p[a][c] = (double)f;
        }
    return true;
}

// Number of slabs for the triangle and the axis they cut (its box's longest).
__device__ inline int esc_slabs(const double (&p)[3][3], int& ax, double& lo, double& ext) {
    double e[3], l[3];
    for (int c = 0; c < 3; c++) {
        l[c] = fmin(p[0][c], fmin(p[1][c], p[2][c]));
        e[c] = fmax(p[0][c], fmax(p[1][c], p[2][c])) - l[c];
    }
    ax = e[0] >= e[1] ? (e[0] >= e[2] ? 0 : 2) : (e[1] >= e[2] ? 1 : 2);
    lo = l[ax];
    ext = e[ax];
    double a[3], b[3];
    for (int c = 0; c < 3; c++) {
        a[c] = p[1][c] - p[0][c];
        b[c] = p[2][c] - p[0][c];
    }
    const double nx = a[1] * b[2] - a[2] * b[1], ny = a[2] * b[0] - a[0] * b[2], nz = a[0] * b[1] - a[1] * b[0];
    const double two_area = sqrt(nx * nx + ny * ny + nz * nz);
    const double box_area = 2.0 * (e[0] * e[1] + e[1] * e[2] + e[0] * e[2]);
    if (!(two_area > 0.0) || !(ext > 0.0) || box_area <= kEscTau * two_area) return 1;
    const double k = ceil(box_area / (kEscTau * two_area));
    return k >= (double)kEscMax ? kEscMax : (int)k;
}

// One side of an axis-aligned plane (Sutherland-Hodgman): the vertices of
// polygon `in` with coordinate `ax` >= v (keep_lo false) or <= v (true), at
// most `cap` of them.  The decisions compare exact coordinates (original
// vertices, or v itself for points on an earlier cut parallel to this one),
// so a convex input gains at most one vertex.
__device__ inline int esc_clip(const double (*in)[3], int n, int ax, double v, bool keep_lo, double (*out)[3],
                               int cap) {
    int m = 0;
    for (int i = 0; i < n; i++) {
        const double* a = in[i];
        const double* b = in[i + 1 < n ? i + 1 : 0];
        const bool ia = keep_lo ? a[ax] <= v : a[ax] >= v;
        const bool ib = keep_lo ? b[ax] <= v : b[ax] >= v;
        if (ia && m < cap) {
            for (int c = 0; c < 3; c++) out[m][c] = a[c];
            m++;
        }
        if (ia != ib && m < cap) {
            const double t = (v - a[ax]) / (b[ax] - a[ax]);
            for (int c = 0; c < 3; c++) out[m][c] = a[c] + t * (b[c] - a[c]);
            out[m][ax] = v;
            m++;
        }
    }
    return m;
}

__device__ inline float round_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}
__device__ inline float round_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

__global__ void k_esc_count(const float* __restrict__ vtx, int64_t nv, const int3* __restrict__ tri, int64_t nt,
                            uint32_t* __restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    double p[3][3];
    int ax;
    double lo, ext;
    cnt[t] = esc_vertices(vtx, nv, tri, t, p) ? (uint32_t)esc_slabs(p, ax, lo, ext) : 1u;
}

// Triangle of every reference: t at off[t] .. off[t+1] - 1.
__global__ void k_esc_owner(int64_t nt, const uint32_t* __restrict__ off, uint32_t* __restrict__ ref_tri) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    for (uint32_t r = off[t]; r < off[t + 1]; r++) ref_tri[r] = (uint32_t)t;
}

// Reference r: piece i of triangle t = ref_tri[r] (one thread per reference,
// so triangles cut into many pieces do not hold up a wavefront).  An unsplit triangle keeps its FP32 box
// (tri_box, from the validated mesh);
// piece i of k is the triangle clipped to slab i of its box's longest side
// (FP64), its box rounded outward to FP32 and widened by `margin` (8 units in
// the last place of the scene's extent: the FP32 watertight test decides hits
// within a few such units of an edge, and a cut adds box faces that the
// triangle's own box did not have).
__global__ void k_esc_emit(const float* __restrict__ vtx, int64_t nv, const int3* __restrict__ tri, int64_t nt,
                           const uint32_t* __restrict__ off, int64_t nr, const uint32_t* __restrict__ bounds,
                           const uint32_t* __restrict__ ref_tri, const float* __restrict__ tri_box,
                           float* __restrict__ ref_box) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const int64_t t = ref_tri[r];
    if (t >= nt) return;
    const int i = (int)(r - (int64_t)off[t]);
    const int k = (int)(off[t + 1] - off[t]);
    if (k == 1) {
        for (int c = 0; c < 6; c++) ref_box[6 * r + c] = tri_box[6 * t + c];
        return;
    }
    double p[3][3];
    if (!esc_vertices(vtx, nv, tri, t, p)) {
        for (int c = 0; c < 6; c++) ref_box[6 * r + c] = 0.f;
        return;
    }
    int ax;
    double lo, ext;
    esc_slabs(p, ax, lo, ext);
    double scene = 0.0;
    for (int c = 0; c < 3; c++) scene = fmax(scene, (double)funord(bounds[3 + c]) - (double)funord(bounds[c]));
    const double margin = scene * 0x1p-20;
    double q1[4][3], q2[5][3];
    int m = 3;
    const double(*cur)[3] = p;
    if (i > 0) {
        m = esc_clip(cur, m, ax, lo + ext * (double)i / (double)k, false, q1, 4);
        cur = q1;
    }
    if (i + 1 < k) {
        m = esc_clip(cur, m, ax, lo + ext * (double)(i + 1) / (double)k, true, q2, 5);
        cur = q2;
    }
    double bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int j = 0; j < m; j++)
        for (int c = 0; c < 3; c++) {
            bl[c] = fmin(bl[c], cur[j][c]);
            bh[c] = fmax(bh[c], cur[j][c]);
        }
    for (int c = 0; c < 3; c++) {
        ref_box[6 * r + c] = m > 0 ? round_down(bl[c] - margin) : INFINITY;
        ref_box[6 * r + 3 + c] = m > 0 ? round_up(bh[c] + margin) : -INFINITY;
    }
}

__device__ inline int prefix_len(const uint64_t* __restrict__ k, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    const uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((uint32_t)(i ^ j));
    return __clzll(a ^ b);
}

// Binary radix tree over sorted codes (one inner node per adjacent pair):
// node i covers [first, last]; its split is where the common prefix ends.
// Children: >= 0 inner node, < 0 leaf ~j.  parent arrays: -1 for the root.
__global__ void k_radix_tree(const uint64_t* __restrict__ k, int64_t n, int2* __restrict__ kids,
                             int2* __restrict__ range, int32_t* __restrict__ parent_in,
                             int32_t* __restrict__ parent_leaf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (prefix_len(k, n, i, i + 1) - prefix_len(k, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = prefix_len(k, n, i, i - d);
    int64_t lmax = 2;
    while (prefix_len(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(k, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = prefix_len(k, n, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(k, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int64_t g = i + s * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t lc, rc;
    if (lo == g) {
        lc = ~(int32_t)g;
        parent_leaf[g] = (int32_t)i;
    } else {
        lc = (int32_t)g;
        parent_in[g] = (int32_t)i;
    }
    if (hi == g + 1) {
        rc = ~(int32_t)(g + 1);
        parent_leaf[g + 1] = (int32_t)i;
    } else {
        rc = (int32_t)(g + 1);
        parent_in[g + 1] = (int32_t)i;
    }
    kids[i] = make_int2(lc, rc);
    range[i] = make_int2((int32_t)lo, (int32_t)hi);
    if (i == 0) parent_in[0] = -1;
}

// Boxes of inner nodes.  Every inner node of the radix tree covers a range
// [first, last] of the Morton-ordered triangles, so its box is a range union:
// a segment tree over the ordered triangle boxes (level l entry i covers
// triangles [i 2^l, (i+1) 2^l)) answers it with O(log M) reads and no atomics.
struct SegBox {
    float4 lo, hi;
};

struct SegLevels {
    const SegBox* lvl[32];
    int n_levels;
};

// Level l of the segment tree has ceil(n / 2^l) entries; entry i covers
// entries 2i and 2i+1 (if present) of level l-1.
struct SegOut {
    SegBox* lvl[32];
    int n_levels;
};

__device__ inline void seg_merge(float (&a)[6], const float* b) {
    for (int c = 0; c < 3; c++) {
        a[c] = fminf(a[c], b[c]);
        a[3 + c] = fmaxf(a[3 + c], b[3 + c]);
    }
}
__device__ inline void seg_put(SegBox* dst, const float (&a)[6]) {
    *dst = SegBox{make_float4(a[0], a[1], a[2], 0.f), make_float4(a[3], a[4], a[5], 0.f)};
}

// Levels 0..kSegBlockLevels of the segment tree for 2^kSegBlockLevels
// consecutive leaves per workgroup (1024 threads): every entry of those levels
// depends on that range only, so each level is formed in LDS after one barrier.
constexpr int kSegBlockLevels = 11;
constexpr int kSegBlockLeaves = 1 << kSegBlockLevels;
__global__ __launch_bounds__(1024) void k_seg_block(int64_t n, const uint32_t* __restrict__ order,
                                                   const float* __restrict__ tri_box, SegOut seg) {
    __shared__ float sb[1024][6];
    const int t = threadIdx.x;
    const int64_t b = blockIdx.x;
    float a[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    bool have = false;
    for (int q = 0; q < 2; q++) {
        const int64_t j = b * kSegBlockLeaves + 2 * t + q;
        if (j < n) {
            const float* tb = tri_box + 6 * (int64_t)order[j];
            float e[6];
            for (int c = 0; c < 6; c++) e[c] = tb[c];
            seg_put(seg.lvl[0] + j, e);
            seg_merge(a, e);
            have = true;
        }
    }
    if (seg.n_levels > 1 && have) seg_put(seg.lvl[1] + (b * (kSegBlockLeaves / 2) + t), a);
    for (int c = 0; c < 6; c++) sb[t][c] = a[c];
    for (int l = 2; l <= kSegBlockLevels && l < seg.n_levels; l++) {
        __syncthreads();
        const int cnt = kSegBlockLeaves >> l;
        const int64_t wl = (n + ((int64_t)1 << l) - 1) >> l;
        const int64_t wp = (n + ((int64_t)1 << (l - 1)) - 1) >> (l - 1);
        bool ok = false;
        float e[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        if (t < cnt) {
            const int64_t gi = b * cnt + t;
            if (gi < wl) {
                seg_merge(e, sb[2 * t]);
                if (2 * gi + 1 < wp) seg_merge(e, sb[2 * t + 1]);
                seg_put(seg.lvl[l] + gi, e);
                ok = true;
            }
        }
        __syncthreads();
        if (ok)
            for (int c = 0; c < 6; c++) sb[t][c] = e[c];
    }
}

// Levels above kSegBlockLevels: one workgroup, a barrier between levels.
__global__ __launch_bounds__(1024) void k_seg_top(int64_t n, SegOut seg) {
    const int t = threadIdx.x;
    for (int l = kSegBlockLevels + 1; l < seg.n_levels; l++) {
        const int64_t wl = (n + ((int64_t)1 << l) - 1) >> l;
        const int64_t wp = (n + ((int64_t)1 << (l - 1)) - 1) >> (l - 1);
        for (int64_t i = t; i < wl; i += blockDim.x) {
            const SegBox c0 = seg.lvl[l - 1][2 * i];
            float e[6] = {c0.lo.x, c0.lo.y, c0.lo.z, c0.hi.x, c0.hi.y, c0.hi.z};
            if (2 * i + 1 < wp) {
                const SegBox c1 = seg.lvl[l - 1][2 * i + 1];
                const float f[6] = {c1.lo.x, c1.lo.y, c1.lo.z, c1.hi.x, c1.hi.y, c1.hi.z};
                seg_merge(e, f);
            }
            seg_put(seg.lvl[l] + i, e);
        }
        __threadfence_block();
        __syncthreads();
    }
}

__global__ void k_node_boxes(int64_t n_in, const int2* __restrict__ range,
                             SegLevels seg, float* __restrict__ box_in) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_in) return;
    const int2 fl = range[i];
    int64_t l = fl.x, r = (int64_t)fl.y + 1;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int lv = 0; l < r && lv < seg.n_levels; lv++) {
        if (l & 1) {
            const SegBox b = seg.lvl[lv][l++];
            lo[0] = fminf(lo[0], b.lo.x); lo[1] = fminf(lo[1], b.lo.y); lo[2] = fminf(lo[2], b.lo.z);
            hi[0] = fmaxf(hi[0], b.hi.x); hi[1] = fmaxf(hi[1], b.hi.y); hi[2] = fmaxf(hi[2], b.hi.z);
        }
        if (r & 1) {
            const SegBox b = seg.lvl[lv][--r];
            lo[0] = fminf(lo[0], b.lo.x); lo[1] = fminf(lo[1], b.lo.y); lo[2] = fminf(lo[2], b.lo.z);
            hi[0] = fmaxf(hi[0], b.hi.x); hi[1] = fmaxf(hi[1], b.hi.y); hi[2] = fmaxf(hi[2], b.hi.z);
        }
        l >>= 1;
        r >>= 1;
    }
    for (int a = 0; a < 3; a++) {
        box_in[6 * i + a] = lo[a];
        box_in[6 * i + 3 + a] = hi[a];
    }
}

__device__ inline int32_t node_size(const int2* range, int32_t c) {
    if (c < 0) return 1;
    const int2 fl = range[c];
    return fl.y - fl.x + 1;
}

// Inner nodes above the leaf-cluster level at even depth become 4-wide nodes.
__global__ void k_flag4(int64_t n_in, const int2* __restrict__ range,
                        const int32_t* __restrict__ parent_in, int32_t leaf_size, uint32_t* __restrict__ flag,
                        int32_t* __restrict__ depth_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_in) return;
    int depth = 0;
    for (int32_t p = parent_in[i]; p >= 0 && depth < 4096; p = parent_in[p]) depth++;
    depth_out[i] = depth;
    const int32_t size = node_size(range, (int32_t)i);
    flag[i] = (size > leaf_size && (depth & 1) == 0) ? 1u : 0u;
}

// Writes the 4-wide node of flagged binary node i; returns its depth level.
// Its slots are the two children, each replaced by its own two children when
// it is an inner node larger than a leaf: with eA, eB those two choices the
// slot refs have closed forms, so every slot's loads can be in flight at once.
__device__ inline uint32_t emit4_one(int64_t i, const int2* __restrict__ kids, const int2* __restrict__ range,
                                     const uint32_t* __restrict__ index, const int32_t* __restrict__ depth_in,
                                     const float* __restrict__ box_in, const float* __restrict__ tri_box,
                                     const uint32_t* __restrict__ order, int32_t leaf_size, Node4* __restrict__ nodes) {
    const int2 cc = kids[i];
    const int32_t c0 = cc.x, c1 = cc.y;
    const bool eA = c0 >= 0 && node_size(range, c0) > leaf_size;
    const bool eB = c1 >= 0 && node_size(range, c1) > leaf_size;
    const int2 ka = eA ? kids[c0] : make_int2(c0, 0);
    const int2 kb = eB ? kids[c1] : make_int2(c1, 0);
    const int32_t a0 = ka.x, a1 = ka.y;
    const int32_t b0 = kb.x, b1 = kb.y;
    int32_t ref[4];
    bool use[4];
    ref[0] = a0;
    use[0] = true;
    ref[1] = eA ? a1 : b0;
    use[1] = true;
    ref[2] = eA ? b0 : b1;
    use[2] = eA || eB;
    ref[3] = b1;
    use[3] = eA && eB;
    Node4 nd;
#pragma unroll
    for (int sl = 0; sl < 4; sl++) {
        float bx[6];
        int32_t child = kEmpty;
        if (use[sl]) {
            const int32_t c = ref[sl];
            // a box is 6 floats at a multiple of 24 bytes: three 8-byte loads
            const float2* b = c < 0 ? reinterpret_cast<const float2*>(tri_box + 6 * (int64_t)order[~c])
                                    : reinterpret_cast<const float2*>(box_in + 6 * (int64_t)c);
            for (int q = 0; q < 3; q++) {
                const float2 v = b[q];
                bx[2 * q] = v.x;
                bx[2 * q + 1] = v.y;
            }
            if (c < 0) {
                child = leaf_ref(~c, 1);
            } else {
                const int2 fl = range[c];
                const int32_t sz = fl.y - fl.x + 1;
                child = sz <= leaf_size ? leaf_ref(fl.x, sz) : (int32_t)index[c];
            }
        } else {
            bx[0] = bx[1] = bx[2] = INFINITY;
            bx[3] = bx[4] = bx[5] = -INFINITY;
        }
        nd.lox[sl] = bx[0];
        nd.loy[sl] = bx[1];
        nd.loz[sl] = bx[2];
        nd.hix[sl] = bx[3];
        nd.hiy[sl] = bx[4];
        nd.hiz[sl] = bx[5];
        nd.child[sl] = child;
        nd.pad[sl] = 0;
    }
    nodes[index[i]] = nd;
    return (uint32_t)(depth_in[i] / 2 + 1);
}

// Flagged binary nodes, listed in the order of their 4-wide node index.
__global__ void k_list4(int64_t n_in, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ index,
                        int32_t* __restrict__ list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_in && flag[i]) list[index[i]] = (int32_t)i;
}

// One thread per 4-wide node (the count index[n_in] is read on the device).
__global__ void k_emit4(int64_t n_in, const int2* __restrict__ kids, const int2* __restrict__ range,
                        const int32_t* __restrict__ list, const uint32_t* __restrict__ index,
                        const int32_t* __restrict__ depth_in, const float* __restrict__ box_in,
                        const float* __restrict__ tri_box, const uint32_t* __restrict__ order, int32_t leaf_size,
                        Node4* __restrict__ nodes, uint32_t* __restrict__ info) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = (int64_t)index[n_in];
    uint32_t d = 0;
    if (j < n4)
        d = emit4_one(list[j], kids, range, index, depth_in, box_in, tri_box, order, leaf_size, nodes);
    // tree depth: one atomic per wavefront
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const uint32_t o = __shfl_down(d, off);
        d = o > d ? o : d;
    }
    if ((threadIdx.x & (kWave - 1)) == 0 && d) atomicMax(&info[2], d);
}

// Root made of a single leaf (the whole mesh fits one leaf).
__global__ void k_single_leaf_root(const uint32_t* __restrict__ bounds, int32_t count, Node4* __restrict__ nodes) {
    Node4 nd;
    for (int s = 0; s < 4; s++) {
        nd.lox[s] = nd.loy[s] = nd.loz[s] = INFINITY;
        nd.hix[s] = nd.hiy[s] = nd.hiz[s] = -INFINITY;
        nd.child[s] = kEmpty;
        nd.pad[s] = 0;
    }
    nd.lox[0] = funord(bounds[0]);
    nd.loy[0] = funord(bounds[1]);
    nd.loz[0] = funord(bounds[2]);
    nd.hix[0] = funord(bounds[3]);
    nd.hiy[0] = funord(bounds[4]);
    nd.hiz[0] = funord(bounds[5]);
    nd.child[0] = leaf_ref(0, count);
    nodes[0] = nd;
}

__global__ void k_tri_records(const float* __restrict__ vtx, int64_t nv, const int3* __restrict__ tri, int64_t nr,
                              const int32_t* __restrict__ material, const int32_t* __restrict__ tri_plane,
                              const uint32_t* __restrict__ order, const uint32_t* __restrict__ ref_tri,
                              float4* __restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nr) return;
    const uint32_t t = ref_tri[order[j]];
    const int3 v = tri[t];
    if (v.x < 0 || v.y < 0 || v.z < 0 || v.x >= nv || v.y >= nv || v.z >= nv) return;   // reported already
    const int idx[3] = {v.x, v.y, v.z};
    const int32_t w[3] = {tri_plane[t], (int32_t)t, material[t]};
    for (int a = 0; a < 3; a++) {
        const float* p = vtx + 3 * (int64_t)idx[a];
        rec[3 * j + a] = make_float4(p[0], p[1], p[2], __int_as_float(w[a]));
    }
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst) { *dst = *src; }

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_init_bounds(uint32_t* b, uint32_t* info) {
    const int t = threadIdx.x;
    if (t < 12) b[t] = (t % 6) < 3 ? 0xFFFFFFFFu : 0u;
    if (t < 8) info[t] = 0;
}

inline int blocks(int64_t n, int t = 256) { return (int)((n + t - 1) / t); }

const char* err_text(uint32_t e) {
    if (e & kErrIndex) return "vertex index out of range";
    if (e & kErrPlaneRange) return "plane id out of range [0, n_tri)";
    if (e & kErrMaterial) return "negative material index";
    if (e & kErrNonFinite) return "non-finite vertex coordinate";
    if (e & kErrZeroArea) return "zero-area triangle";
    if (e & kErrNotCoplanar) return "plane group member not in its representative's plane";
    if (e & kErrMixedMaterial) return "plane group members with different materials";
    return "invalid mesh";
}

// Device memory of one build: the scene's own arrays and its temporaries are
// growable buffers of the scene, so a rebuild of a scene of the same size (or
// smaller) allocates nothing.  A buffer that must grow returns its old block
// fenced on the build's stream (work queued earlier may still read it).
struct BuildMem {
    rt_scene* s;
    size_t next = 0;
    template <class T>
    T* keep(Buf& b, size_t count) {
        return b.ensure(sizeof(T) * (count ? count : 1)) ? nullptr : b.as<T>();
    }
    template <class T>
    T* get(size_t count) {
        if (next == s->tmp.size()) s->tmp.emplace_back();
        return keep<T>(s->tmp[next++], count);
    }
};

// Builds (fresh) or rebuilds the scene `s` on stream `st`.  On failure the
// caller destroys a fresh scene; a rebuilt one is left marked invalid.
// Host-side argument checks of a build (before any device call).
int check_build_args(const char* who, const float* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                     const int32_t* material, const rt_build_params* params) {
    RT_CHECK(vtx && tri && material, RT_EINVAL, "%s: null input array", who);
    RT_CHECK(n_tri >= 1 && n_vtx >= 3, RT_EINVAL, "%s: need n_tri >= 1 and n_vtx >= 3", who);
    RT_CHECK(n_tri < kMaxTris, RT_EINVAL, "%s: n_tri must be < 2^27", who);
    const int leaf = params ? params->leaf_size : 1;
    RT_CHECK(leaf >= 1 && leaf <= kMaxLeaf, RT_EINVAL, "%s: leaf_size must be in [1, %d]", who, kMaxLeaf);
    return RT_OK;
}

int build_scene(rt_scene* s, const char* who, const float* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                const int32_t* material, const int32_t* plane_id, const rt_build_params* params, hipStream_t st) {
    s->valid = false;
    const int leaf = params ? params->leaf_size : 1;
    const int64_t nt = n_tri;
    BuildMem tmp{s};
    s->n_tri = nt;
    s->n_vtx = n_vtx;
    s->leaf_size = leaf;
    s->exact = true;
    s->plane_n = tmp.keep<double>(s->m_plane_n, 3 * nt);
    s->plane_p = tmp.keep<double>(s->m_plane_p, 3 * nt);
    s->plane_mat = tmp.keep<int32_t>(s->m_plane_mat, nt);
    s->tri_plane = tmp.keep<int32_t>(s->m_tri_plane, nt);
    float* tri_box = tmp.get<float>(6 * nt);
    float* cen = tmp.get<float>(3 * nt);
    uint32_t* bounds = tmp.get<uint32_t>(12);
    // [0] errors [1] max material [2] depth [3] 4-wide nodes [4] references; kept with the scene
    uint32_t* info = tmp.keep<uint32_t>(s->m_info, 8);
    s->info_dev = info;
    uint32_t* prep_part = tmp.get<uint32_t>(14 * (int64_t)blocks(nt));
    int32_t* prep = tmp.get<int32_t>(nt);
    uint32_t* ref_cnt = tmp.get<uint32_t>(nt);
    uint32_t* ref_off = tmp.get<uint32_t>(nt + 1);
    if (!s->plane_n || !s->plane_p || !s->plane_mat || !s->tri_plane || !tri_box || !cen || !bounds || !info ||
        !prep_part || !prep || !ref_cnt || !ref_off) {
        set_error("%s: out of device memory", who);
        return RT_ENOMEM;
    }
    hipLaunchKernelGGL(k_init_bounds, dim3(1), dim3(64), 0, st, bounds, info);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(nt)), dim3(256), 0, st, prep, nt, INT32_MAX);
    hipLaunchKernelGGL(k_tri_prep, dim3(blocks(nt)), dim3(256), 0, st, vtx, n_vtx, (const int3*)tri, nt, material,
                       plane_id, tri_box, cen, prep_part, prep);
    hipLaunchKernelGGL(k_prep_reduce, dim3(1), dim3(256), 0, st, prep_part, (int64_t)blocks(nt), bounds, info);
    hipLaunchKernelGGL(k_plane_table, dim3(blocks(nt)), dim3(256), 0, st, vtx, (const int3*)tri, nt, material, prep,
                       s->plane_n, s->plane_p, s->plane_mat);
    hipLaunchKernelGGL(k_coplanar, dim3(blocks(nt)), dim3(256), 0, st, vtx, n_vtx, (const int3*)tri, nt, material,
                       plane_id, s->plane_n, s->plane_p, s->plane_mat, bounds, s->tri_plane, info);
    // references: slab counts per triangle, their offsets, then the total
    hipLaunchKernelGGL(k_esc_count, dim3(blocks(nt)), dim3(256), 0, st, vtx, n_vtx, (const int3*)tri, nt, ref_cnt);
    int rc = exclusive_scan_u32(s->ws, ref_cnt, ref_off, nt, nullptr, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, st, ref_off + nt, info + 4);
    RT_HIP(hipGetLastError());
    // the one wait of the build: the reference count sizes the per-reference
    // arrays; the scene box and the largest material are final by now
    uint32_t h_info[5], h_bounds[12];
    RT_HIP(hipMemcpyAsync(h_info, info, sizeof(h_info), hipMemcpyDeviceToHost, st));
    RT_HIP(hipMemcpyAsync(h_bounds, bounds, sizeof(h_bounds), hipMemcpyDeviceToHost, st));
    RT_HIP(hipStreamSynchronize(st));
    if (h_info[0]) {
        set_error("%s: %s", who, err_text(h_info[0]));
        const bool degen = (h_info[0] & (kErrNonFinite | kErrZeroArea)) &&
                           !(h_info[0] & (kErrIndex | kErrPlaneRange | kErrMaterial));
        return degen ? RT_EDEGENERATE : RT_EINVAL;
    }
    const int64_t nr = h_info[4];
    RT_CHECK(nr >= nt && nr < kMaxTris, RT_EINVAL, "%s: %lld references (at most 2^27)", who, (long long)nr);
    const int64_t n_in = nr - 1;
    const bool single = n_in == 0 || nr <= leaf;
    // upper bound of 4-wide nodes: inner binary nodes (one per adjacent pair)
    const int64_t node_cap = single ? 1 : n_in;
    s->n_ref = nr;
    s->tri_rec = tmp.keep<float4>(s->m_tri_rec, 3 * nr);
    s->nodes = tmp.keep<Node4>(s->m_nodes, node_cap);
    float* ref_box = tmp.get<float>(6 * nr);
    uint32_t* ref_tri = tmp.get<uint32_t>(nr);
    uint64_t* codes0 = tmp.get<uint64_t>(nr);
    uint64_t* codes1 = tmp.get<uint64_t>(nr);
    uint32_t* ord0 = tmp.get<uint32_t>(nr);
    uint32_t* ord1 = tmp.get<uint32_t>(nr);
    if (!s->tri_rec || !s->nodes || !ref_box || !ref_tri || !codes0 || !codes1 || !ord0 || !ord1) {
        set_error("%s: out of device memory", who);
        return RT_ENOMEM;
    }
    hipLaunchKernelGGL(k_esc_owner, dim3(blocks(nt)), dim3(256), 0, st, nt, ref_off, ref_tri);
    hipLaunchKernelGGL(k_esc_emit, dim3(blocks(nr)), dim3(256), 0, st, vtx, n_vtx, (const int3*)tri, nt, ref_off, nr,
                       bounds, ref_tri, tri_box, ref_box);
    hipLaunchKernelGGL(k_morton, dim3(blocks(nr)), dim3(256), 0, st, ref_box, nr, bounds, codes0);
    int which = 0;
    rc = radix_sort_pairs(s->ws, codes0, ord0, codes1, ord1, nr, nullptr, 0, 3 * kMortonBits, st, &which, true);
    if (rc) return rc;
    uint64_t* codes = which ? codes1 : codes0;
    uint32_t* order = which ? ord1 : ord0;
    uint32_t* n4_dev = info + 3;
    if (single) {
        hipLaunchKernelGGL(k_single_leaf_root, dim3(1), dim3(1), 0, st, bounds, (int32_t)nr, s->nodes);
    } else {
        int2* kids = tmp.get<int2>(n_in);    // (left, right) child refs; ~leaf for a leaf child
        int2* range = tmp.get<int2>(n_in);   // (first, last) reference covered
        int32_t* par_in = tmp.get<int32_t>(n_in);
        int32_t* par_leaf = tmp.get<int32_t>(nr);
        int32_t* depth = tmp.get<int32_t>(n_in);
        float* box_in = tmp.get<float>(6 * n_in);
        uint32_t* flag = tmp.get<uint32_t>(n_in);
        uint32_t* index = tmp.get<uint32_t>(n_in + 1);
        int32_t* list4 = tmp.get<int32_t>(n_in);
        if (!kids || !range || !par_in || !par_leaf || !depth || !box_in || !flag ||
            !index || !list4) {
            set_error("%s: out of device memory", who);
            return RT_ENOMEM;
        }
        hipLaunchKernelGGL(k_radix_tree, dim3(blocks(n_in)), dim3(256), 0, st, codes, nr, kids, range,
                           par_in, par_leaf);
        // segment tree over the ordered reference boxes, then one range query per inner node
        SegLevels seg;
        seg.n_levels = 0;
        int64_t total = 0;
        for (int64_t w = nr;; w = (w + 1) / 2) {
            total += w;
            seg.n_levels++;
            if (w == 1 || seg.n_levels == 32) break;
        }
        SegBox* segbuf = tmp.get<SegBox>(total);
        if (!segbuf) {
            set_error("%s: out of device memory", who);
            return RT_ENOMEM;
        }
        {
            SegOut segw;
            segw.n_levels = seg.n_levels;
            int64_t off = 0;
            for (int lv = 0; lv < seg.n_levels; lv++) {
                segw.lvl[lv] = segbuf + off;
                seg.lvl[lv] = segbuf + off;
                off += (nr + ((int64_t)1 << lv) - 1) >> lv;
            }
            hipLaunchKernelGGL(k_seg_block, dim3((unsigned)((nr + kSegBlockLeaves - 1) / kSegBlockLeaves)), dim3(1024),
                               0, st, nr, order, ref_box, segw);
            if (seg.n_levels > kSegBlockLevels + 1)
                hipLaunchKernelGGL(k_seg_top, dim3(1), dim3(1024), 0, st, nr, segw);
        }
        hipLaunchKernelGGL(k_node_boxes, dim3(blocks(n_in)), dim3(256), 0, st, n_in, range, seg, box_in);
        hipLaunchKernelGGL(k_flag4, dim3(blocks(n_in)), dim3(256), 0, st, n_in, range, par_in, leaf, flag,
                           depth);
        rc = exclusive_scan_u32(s->ws, flag, index, n_in, nullptr, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_list4, dim3(blocks(n_in)), dim3(256), 0, st, n_in, flag, index, list4);
        hipLaunchKernelGGL(k_emit4, dim3(blocks(n_in)), dim3(256), 0, st, n_in, kids, range, list4,
                           index, depth, box_in, ref_box, order, leaf, s->nodes, info);
        hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, st, index + n_in, n4_dev);
    }
    hipLaunchKernelGGL(k_tri_records, dim3(blocks(nr)), dim3(256), 0, st, vtx, n_vtx, (const int3*)tri, nr, material,
                       s->tri_plane, order, ref_tri, s->tri_rec);
    RT_HIP(hipGetLastError());
    // No wait at the end: the node count and depth stay on the device until
    // rt_scene_info asks for them (the trace sizes its stack spill area from a
    // bound on the depth and checks node references against the capacity), and
    // the temporaries are released once the build is known to have finished.
    s->n_mat = (int32_t)h_info[1] + 1;
    double d2 = 0;
    for (int c = 0; c < 3; c++) {
        s->bounds[c] = funord(h_bounds[c]);
        s->bounds[3 + c] = funord(h_bounds[3 + c]);
        const double e = (double)s->bounds[3 + c] - (double)s->bounds[c];
        d2 += e * e;
    }
    s->diag = std::sqrt(d2);
    if (single) {
        s->n_nodes = 1;
        s->depth = 1;
    } else {
        // a root-to-leaf path of the binary tree fixes one more bit of the
        // (30-bit Morton code, reference index) key per level
        int bits = 1;
        while (bits < 40 && ((int64_t)1 << bits) < nr) bits++;
        s->n_nodes = (int32_t)node_cap;
        s->depth = (30 + bits + 1) / 2 + 2;
        s->exact = false;
    }
    if (!s->built) RT_HIP(hipEventCreateWithFlags(&s->built, hipEventDisableTiming));
    RT_HIP(hipEventRecord(s->built, st));
    s->valid = true;
    return RT_OK;
}

}  // namespace

}  // namespace rtac

using namespace rtac;

extern "C" int rt_build_tree(const float* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                             const int32_t* material, const int32_t* plane_id, const rt_build_params* params,
                             void* stream, rt_scene** out_scene) {
    RT_CHECK(out_scene != nullptr, RT_EINVAL, "rt_build_tree: out_scene is NULL");
    *out_scene = nullptr;
    if (check_build_args("rt_build_tree", vtx, n_vtx, tri, n_tri, material, params)) return RT_EINVAL;
    CallStream call_stream((hipStream_t)stream);
    rt_scene* s = new rt_scene();
    int rc = hipGetDevice(&s->device) == hipSuccess ? RT_OK : RT_EHIP;
    if (rc) set_error("rt_build_tree: hipGetDevice failed");
    if (!rc)
        rc = build_scene(s, "rt_build_tree", vtx, n_vtx, tri, n_tri, material, plane_id, params,
                         (hipStream_t)stream);
    if (rc) {
        rt_scene_destroy(s);
        return rc;
    }
    *out_scene = s;
    return RT_OK;
}

extern "C" int rt_rebuild_tree(rt_scene* scene, const float* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                               const int32_t* material, const int32_t* plane_id, const rt_build_params* params,
                               void* stream) {
    RT_CHECK(scene != nullptr, RT_EINVAL, "rt_rebuild_tree: null scene");
    if (check_build_args("rt_rebuild_tree", vtx, n_vtx, tri, n_tri, material, params)) {
        scene->valid = false;
        return RT_EINVAL;
    }
    int dev = -1;
    RT_HIP(hipGetDevice(&dev));
    RT_CHECK(dev == scene->device, RT_EINVAL, "rt_rebuild_tree: scene lives on device %d, current device is %d",
             scene->device, dev);
    CallStream call_stream((hipStream_t)stream);
    return build_scene(scene, "rt_rebuild_tree", vtx, n_vtx, tri, n_tri, material, plane_id, params,
                       (hipStream_t)stream);
}
