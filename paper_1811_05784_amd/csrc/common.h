// Internal declarations shared by the librtac translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rtac.h"

namespace rtac {

void set_error(const char* fmt, ...);

#define RT_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::rtac::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                              __FILE__, __LINE__);                                        \
            return RT_EHIP;                                                               \
        }                                                                                 \
    } while (0)

#define RT_CHECK(cond, code, ...)             \
    do {                                      \
        if (!(cond)) {                        \
            ::rtac::set_error(__VA_ARGS__);   \
            return (code);                    \
        }                                     \
    } while (0)

constexpr int kWave = 64;
constexpr int kMaxRcv = 32;
constexpr int kMaxLeaf = 8;

// 4-wide tree node: child boxes as SoA (96 B) + child references (32 B).
// child[i] >= 0: inner node index; child[i] < 0: leaf, see leaf_ref();
// cnt unused slot: child = kEmpty and an inverted (empty) box.
struct __attribute__((aligned(128))) Node4 {
    float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
    int32_t child[4];
    int32_t pad[4];
};
static_assert(sizeof(Node4) == 128, "node size");

constexpr int32_t kEmpty = (int32_t)0x80000000u;   // count field 0 => empty slot
__host__ __device__ inline int32_t leaf_ref(int32_t first, int32_t count) {
    return (int32_t)(0x80000000u | ((uint32_t)count << 27) | (uint32_t)first);
}
__host__ __device__ inline int32_t leaf_first(int32_t ref) { return (int32_t)((uint32_t)ref & 0x07FFFFFFu); }
__host__ __device__ inline int32_t leaf_count(int32_t ref) { return (int32_t)(((uint32_t)ref >> 27) & 0xFu); }
constexpr int64_t kMaxTris = (int64_t)1 << 27;

// Growable device scratch owned by a scene.
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    int ensure(size_t n);
    void release();
    template <class T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

struct Workspace {
    Buf sort_keys[2], sort_vals[2], sort_hist, scan_tmp;
    Buf stack_spill, trace_pool;
    Buf is_hash, is_idx, is_flags, is_group, coll_err;
    Buf asm_key, asm_idx, asm_energy, asm_partial, asm_pressure, fir_twiddle, fir_spec, band_partial;
    const void* fir_twiddle_done = nullptr;   // fir_twiddle's address once its table has been computed
    Buf generic[4];
    void release_all();
};

// Device-side view of one scene and of one job (a source with its rays and
// receivers in one scene) for batched calls.
struct DevScene {
    const Node4* nodes;
    const float4* tri;
    const double* plane_n;
    const double* plane_p;
    const int32_t* plane_mat;
    const int32_t* tri_plane;
    int32_t n_nodes;
    int32_t n_tri;
    int32_t mat_off;   // first row of this scene's materials in a batch absorption table
    int32_t n_mat;
    int32_t n_ref;     // triangle records (references) in tree order
    int32_t pad;
};

struct DevJob {
    int64_t ray_off;   // first global ray id
    int64_t n_rays;
    float src[3];
    float max_len;
    int32_t scene;
    int32_t rcv_off;   // first global receiver row
    int32_t n_rcv;
    int32_t pad;
};

// Fibonacci sphere direction i of n: z = 1 - (2i+1)/n, phi = i pi (3 - sqrt5)
// mod 2 pi, FP64 without contraction, rounded once.
__device__ inline void fibonacci_dir(int64_t i, int64_t n, float* out) {
#pragma clang fp contract(off)
    const double pi = 3.14159265358979323846;
    const double golden = pi * (3.0 - sqrt(5.0));
    const double two_pi = 2.0 * pi;
    const double z = 1.0 - (double)(2 * i + 1) / (double)n;
    const double phi = fmod((double)i * golden, two_pi);
    const double zz = z * z;
    const double rho = sqrt(1.0 - zz);
    const double x = rho * cos(phi);
    const double y = rho * sin(phi);
    out[0] = (float)x;
    out[1] = (float)y;
    out[2] = (float)z;
}

// Job of a global ray id (jobs hold contiguous ray ranges, ray_off ascending).
__device__ inline int32_t job_of_ray(const DevJob* jobs, int32_t n_jobs, int64_t g) {
    int32_t lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (jobs[mid].ray_off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace rtac

struct rt_batch {
    int device = 0;
    int32_t n_scenes = 0, n_jobs = 0, n_rcv = 0, n_mat = 0;
    int64_t n_rays = 0;
    rtac::DevScene* scenes = nullptr;   // device
    rtac::DevJob* jobs = nullptr;       // device
    int32_t* rcv_job = nullptr;         // device, [n_rcv]
    rt_scene* ws_owner = nullptr;       // scene whose workspace the batch uses
    int32_t max_depth = 0;
    int64_t max_steps = 0;
};

struct rt_scene {
    int device = 0;
    int64_t n_tri = 0;
    int64_t n_ref = 0;          // references (triangle records in tree order; >= n_tri)
    int64_t n_vtx = 0;
    int32_t n_mat = 0;
    int32_t leaf_size = 1;
    int32_t n_nodes = 0;        // 4-wide nodes; until `exact`, the allocated capacity
    int32_t depth = 0;          // 4-wide tree depth (levels of inner nodes); until `exact`, a bound
    bool exact = true;          // n_nodes and depth read back from the device
    bool valid = false;         // a build has succeeded (a failed rebuild clears it)
    uint32_t* info_dev = nullptr;   // build counters on the device ([2] depth, [3] 4-wide nodes)
    hipEvent_t built = nullptr;     // recorded after the build's last kernel
    // device memory of the build, kept so that a rebuild reuses it: the
    // scene's arrays below, and the temporaries (released by rt_scene_info
    // once the build has finished, taken again by the next rebuild)
    rtac::Buf m_nodes, m_tri_rec, m_plane_n, m_plane_p, m_plane_mat, m_tri_plane, m_info;
    std::vector<rtac::Buf> tmp;
    double diag = 0.0;
    float bounds[6] = {0, 0, 0, 0, 0, 0};
    // device arrays
    rtac::Node4* nodes = nullptr;   // [n_nodes]
    float4* tri_rec = nullptr;      // [n_ref * 3] one record per reference, in tree (Morton) order:
                                    // (v0, plane id) (v1, triangle id) (v2, material) as int bits in w
    double* plane_n = nullptr;      // [n_tri * 3] unit normal per plane id (representative)
    double* plane_p = nullptr;      // [n_tri * 3] first vertex of the representative
    int32_t* plane_mat = nullptr;   // [n_tri] material of each plane id (-1 unused)
    int32_t* tri_plane = nullptr;   // [n_tri] plane id per original triangle id
    rtac::Workspace ws;
};

namespace rtac {

// ---------------------------------------------------------------------------
// sorting and scanning primitives (sort.hip)
// ---------------------------------------------------------------------------

// Stable LSD radix sort of (uint64 key, uint32 value) pairs over bits
// [begin_bit, end_bit).  n_dev (device) overrides n when non-null (the
// count is read on the device, buffers are sized for `cap`).  Result ends in
// keys[out]/vals[out] where out is returned (0 or 1).  iota_values: the
// input values are taken to be 0, 1, 2, ... (vals0 is then only scratch).
int radix_sort_pairs(Workspace& ws, uint64_t* keys0, uint32_t* vals0, uint64_t* keys1, uint32_t* vals1,
                     int64_t cap, const int64_t* n_dev, int begin_bit, int end_bit, hipStream_t st,
                     int* out_index, bool iota_values = false);

// Exclusive scan of uint32 flags[0..cap) into out[0..cap]; out[n] = total.
int exclusive_scan_u32(Workspace& ws, const uint32_t* in, uint32_t* out, int64_t cap, const int64_t* n_dev,
                       hipStream_t st);

int device_sm_count();

// Process-wide caching device allocator (per device, best fit within 2x):
// repeated scene builds and scratch growth reuse freed blocks instead of
// calling hipMalloc/hipFree again.  A block freed inside a call that works on
// a stream (see CallStream) is held back until an event recorded on that
// stream at the free has completed, so work already queued there can still
// read it while other streams allocate; a block freed outside such a call
// (after a synchronisation) is reusable at once.
void* dcache_alloc(size_t bytes);
void dcache_free(void* p);

// Marks the stream of the entry point running on this thread for the
// lifetime of the object (frees made meanwhile are fenced on it).
struct CallStream {
    explicit CallStream(hipStream_t s);
    ~CallStream();
    CallStream(const CallStream&) = delete;
    CallStream& operator=(const CallStream&) = delete;
    hipStream_t prev;
    bool had;
};

}  // namespace rtac
