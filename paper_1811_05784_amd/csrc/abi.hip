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
struct Held {
    hipEvent_t ev;   // recorded on the freeing call's stream
    int ev_dev;      // the device the event belongs to
    std::pair<int, size_t> key;
    void* p;
};
struct Cache {
    std::mutex mu;
    std::map<void*, std::pair<int, size_t>> live;          // ptr -> (device, bytes)
    std::multimap<std::pair<int, size_t>, void*> free_;    // (device, bytes) -> ptr
    std::vector<Held> held;                                 // freed, waiting for their event
    std::vector<std::pair<int, hipEvent_t>> spare;          // (device, completed event) for reuse
};
Cache& cache() {
    static Cache* c = new Cache();   // never destroyed: freed blocks live until exit
    return *c;
}
thread_local hipStream_t t_stream = nullptr;
thread_local bool t_has_stream = false;

// Whether the calling entry point's stream is being captured into a graph
// (no event is recorded or queried then).
bool call_stream_capturing() {
    if (!t_has_stream) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(t_stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return true;   // unknown: treat as capturing (free at once, query nothing)
    }
    return cs != hipStreamCaptureStatusNone;
}

// Moves held blocks whose event has completed to the free lists (lock held).
void release_completed(Cache& c) {
    bool queried_busy = false;
    for (size_t i = 0; i < c.held.size();) {
        const hipError_t q = hipEventQuery(c.held[i].ev);
        if (q == hipSuccess) {
            c.free_.insert({c.held[i].key, c.held[i].p});
            c.spare.push_back({c.held[i].ev_dev, c.held[i].ev});
            c.held[i] = c.held.back();
            c.held.pop_back();
        } else {
            queried_busy = true;
            i++;
        }
    }
    if (queried_busy) (void)hipGetLastError();   // "not ready" is no error of the caller's
}
}  // namespace

CallStream::CallStream(hipStream_t s) : prev(t_stream), had(t_has_stream) {
    t_stream = s;
    t_has_stream = true;
}

CallStream::~CallStream() {
    t_stream = prev;
    t_has_stream = had;
}

void* dcache_alloc(size_t bytes) {
    if (bytes == 0) bytes = 1;
    bytes = (bytes + 255) & ~(size_t)255;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    Cache& c = cache();
    {
        std::lock_guard<std::mutex> g(c.mu);
        if (!c.held.empty() && !call_stream_capturing()) release_completed(c);
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
        if (!call_stream_capturing()) release_completed(c);
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
    const std::pair<int, size_t> key = it->second;
    c.live.erase(it);
    // fence the block on the calling stream (not while it is being captured
    // into a graph: there the caller keeps its buffers alive)
    if (t_has_stream && !call_stream_capturing()) {
        // an event of the current device (the calling stream's)
        int cur = 0;
        (void)hipGetDevice(&cur);
        hipEvent_t ev = nullptr;
        for (size_t i = 0; i < c.spare.size(); i++) {
            if (c.spare[i].first == cur) {
                ev = c.spare[i].second;
                c.spare[i] = c.spare.back();
                c.spare.pop_back();
                break;
            }
        }
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            ev = nullptr;
        }
        if (ev && hipEventRecord(ev, t_stream) == hipSuccess) {
            c.held.push_back({ev, cur, key, p});
            return;
        }
        if (ev) {
            (void)hipGetLastError();   // the record failed: the block is free at once
            c.spare.push_back({cur, ev});
        }
    }
    c.free_.insert({key, p});
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
    for (rtac::Buf& b : s->tmp) b.release();
    for (rtac::Buf* b : {&s->m_nodes, &s->m_tri_rec, &s->m_plane_n, &s->m_plane_p, &s->m_plane_mat, &s->m_tri_plane,
                         &s->m_info})
        b->release();
    if (s->built) (void)hipEventDestroy(s->built);
    s->ws.release_all();
    delete s;
    return RT_OK;
}

extern "C" int rt_scene_info(const rt_scene* cs, int64_t* info, double* diag) {
    RT_CHECK(cs != nullptr, RT_EINVAL, "rt_scene_info: null scene");
    RT_CHECK(cs->valid, RT_EINVAL, "rt_scene_info: the scene's last rebuild failed");
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
        // the build has finished: its temporaries go back to the cache (a
        // rebuild takes them again)
        for (rtac::Buf& b : s->tmp) b.release();
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
