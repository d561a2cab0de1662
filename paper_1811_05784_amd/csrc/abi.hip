// Error reporting, scratch buffers, scene lifetime and small host queries.
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace rtac {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int Buf::ensure(size_t n) {
    if (n <= bytes && p) return 0;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    size_t want = n < 256 ? 256 : n;
    if (hipMalloc(&p, want) != hipSuccess) {
        p = nullptr;
        set_error("hipMalloc of %zu bytes failed", want);
        return 1;
    }
    bytes = want;
    return 0;
}

void Buf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

void Workspace::release_all() {
    for (auto* b : {&sort_keys[0], &sort_keys[1], &sort_vals[0], &sort_vals[1], &sort_hist, &scan_tmp,
                    &stack_spill, &trace_pool, &is_hash, &is_idx, &is_flags, &is_group, &coll_err, &asm_key,
                    &asm_idx, &asm_energy, &asm_partial, &asm_pressure, &generic[0], &generic[1], &generic[2],
                    &generic[3]})
        b->release();
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
    (void)hipFree(s->nodes);
    (void)hipFree(s->tri_rec);
    (void)hipFree(s->plane_n);
    (void)hipFree(s->plane_p);
    (void)hipFree(s->plane_mat);
    (void)hipFree(s->tri_plane);
    s->ws.release_all();
    delete s;
    return RT_OK;
}

extern "C" int rt_scene_info(const rt_scene* s, int64_t* info, double* diag) {
    RT_CHECK(s != nullptr, RT_EINVAL, "rt_scene_info: null scene");
    if (info) {
        info[0] = s->n_tri;
        info[1] = s->n_mat;
        info[2] = s->n_nodes;
        info[3] = s->depth;
        info[4] = s->leaf_size;
    }
    if (diag) diag[0] = s->diag;
    return RT_OK;
}
