// Error reporting, scratch buffers, scene lifetime and small host queries.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>

#include "common.h"

namespace rtac {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

namespace {
struct Cache {
    std::mutex mu;
    std::map<void*, std::pair<int, size_t>> live;          // ptr -> (device, bytes)
    std::multimap<std::pair<int, size_t>, void*> free_;    // (device, bytes) -> ptr
};
Cache& cache() {
    static Cache* c = new Cache();   // never destroyed: freed blocks live until exit
    return *c;
}
}  // namespace

void* dcache_alloc(size_t bytes) {
    if (bytes == 0) bytes = 1;
    bytes = (bytes + 255) & ~(size_t)255;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    Cache& c = cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.free_.lower_bound({dev, bytes});
        if (it != c.free_.end() && it->first.first == dev && it->first.second <= 2 * bytes) {
            void* p = it->second;
            c.live[p] = it->first;
            c.free_.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        // give cached blocks back to the runtime and retry once
        std::lock_guard<std::mutex> g(c.mu);
        for (auto it = c.free_.begin(); it != c.free_.end();) {
            if (it->first.first == dev) {
                (void)hipFree(it->second);
                it = c.free_.erase(it);
            } else {
                ++it;
            }
        }
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of %zu bytes failed", bytes);
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> g(c.mu);
    c.live[p] = {dev, bytes};
    return p;
}

void dcache_free(void* p) {
    if (!p) return;
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    c.free_.insert({it->second, p});
    c.live.erase(it);
}

int Buf::ensure(size_t n) {
    if (n <= bytes && p) return 0;
    dcache_free(p);
    p = nullptr;
    bytes = 0;
    size_t want = n < 256 ? 256 : n;
    p = dcache_alloc(want);
    if (!p) return 1;
    bytes = want;
    return 0;
}

void Buf::release() {
    dcache_free(p);
    p = nullptr;
    bytes = 0;
}

void Workspace::release_all() {
    for (auto* b : {&sort_keys[0], &sort_keys[1], &sort_vals[0], &sort_vals[1], &sort_hist, &scan_tmp,
                    &stack_spill, &trace_pool, &is_hash, &is_idx, &is_flags, &is_group, &coll_err, &asm_key,
                    &asm_idx, &asm_energy, &asm_partial, &asm_pressure, &fir_twiddle, &fir_spec, &band_partial,
                    &generic[0], &generic[1], &generic[2], &generic[3]})
        b->release();
    fir_twiddle_done = nullptr;
}

int device_sm_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

}  // namespace rtac

extern "C" const char* rt_last_error(void) { return rtac::g_err; }

extern "C" const char* rt_version(void) { return "librtac 0.1 (gfx950)"; }

extern "C" int rt_scene_destroy(rt_scene* s) {
    if (!s) return RT_OK;
    (void)hipDeviceSynchronize();
    for (void* p : s->pending) rtac::dcache_free(p);
    s->pending.clear();
    rtac::dcache_free(s->info_dev);
    if (s->built) (void)hipEventDestroy(s->built);
    rtac::dcache_free(s->nodes);
    rtac::dcache_free(s->tri_rec);
    rtac::dcache_free(s->plane_n);
    rtac::dcache_free(s->plane_p);
    rtac::dcache_free(s->plane_mat);
    rtac::dcache_free(s->tri_plane);
    s->ws.release_all();
    delete s;
    return RT_OK;
}

extern "C" int rt_scene_info(const rt_scene* cs, int64_t* info, double* diag) {
    RT_CHECK(cs != nullptr, RT_EINVAL, "rt_scene_info: null scene");
    rt_scene* s = const_cast<rt_scene*>(cs);
    if (info && !s->exact) {
        // the first query waits for the build and reads the node count and depth
        uint32_t h[4];
        RT_HIP(hipEventSynchronize(s->built));
        RT_HIP(hipMemcpy(h, s->info_dev, sizeof(h), hipMemcpyDeviceToHost));
        RT_CHECK(h[3] >= 1 && (int64_t)h[3] <= s->n_nodes && (int32_t)h[2] <= s->depth, RT_EHIP,
                 "rt_scene_info: inconsistent tree");
        s->n_nodes = (int32_t)h[3];
        s->depth = (int32_t)h[2];
        s->exact = true;
        for (void* p : s->pending) rtac::dcache_free(p);
        s->pending.clear();
    }
    if (info) {
        info[0] = s->n_tri;
        info[1] = s->n_mat;
        info[2] = s->n_nodes;
        info[3] = s->depth;
        info[4] = s->leaf_size;
        info[5] = s->n_ref;
    }
    if (diag) diag[0] = s->diag;
    return RT_OK;
}
