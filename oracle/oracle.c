/*
 * oracle.c -- plain, slow FP64 CPU oracle of the ray-tracing part of the
 * hybrid ray-tracing / image-source method of Aussal & Gueguen (2018).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library; both read the same input arrays.
 *
 * What it computes (section "Implementation", "Standard algorithm"):
 *   - nearest hit by brute force over every triangle (no tree): the ray
 *     a + delta*u meets the triangle b + lambda*v + mu*w with 0 <= lambda,
 *     0 <= mu, lambda + mu <= 1, delta > 0, and delta minimal; solved with the
 *     Moller-Trumbore formulation the paper names;
 *   - receiver detection against the sphere (x - x_m)^2 = r^2 (segment vs
 *     closed ball; the sphere is transparent);
 *   - specular reflection u_r = (u.T)T - (u.n)n = u - 2(u.n)n (eq. "u_r",
 *     section "Presence of an obstacle");
 *   - the propagation loop: reflect, stop after R reflections, past a path
 *     length, or when a ray in open air hits nothing;
 *   - the Fibonacci sphere directions used for an omnidirectional source
 *     (section "Discrete model");
 *   - image-source positions: the source mirrored through the reflecting
 *     planes in order (section "Image-sources").
 *
 * Readings where the paper is silent:
 *   - the triangle of the last reflection's plane is excluded from the next
 *     search (a ray leaving a plane cannot meet it again), instead of an
 *     epsilon offset; every other candidate needs delta > 0 strictly;
 *   - exact ties in delta go to the lowest triangle index;
 *   - each plane id's representative is its lowest-index triangle; its unit
 *     normal and first vertex define the plane used for reflection and for
 *     image-source mirroring.
 *
 * Flags: a query is flagged when an FP32 implementation could legitimately
 * decide differently (near an edge, near miss, tie, tiny delta, grazing,
 * receiver near tangent, path length near the stop).  eps is relative to the
 * scene bounding-box diagonal D for distances.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846
#define OR_FLAG_EDGE 1u
#define OR_FLAG_NEAR_MISS 2u
#define OR_FLAG_TIE 4u
#define OR_FLAG_TINY 8u
#define OR_FLAG_GRAZING 16u
#define OR_FLAG_TANGENT 32u
#define OR_FLAG_LENGTH 64u

typedef struct {
    double v0[3], v1[3], v2[3];
    double e1[3], e2[3];
    double lo[3], hi[3];
    int plane;
} otri;

typedef struct {
    int64_t nt;
    otri* t;
    double* pn;     /* [nt*3] unit normal of each plane id's representative */
    double* pp;     /* [nt*3] first vertex of the representative            */
    int* prep;      /* [nt] representative triangle of plane id, -1 unused  */
    double diag;    /* bounding-box diagonal D                              */
} or_scene;

static void sub3(const double* a, const double* b, double* o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------------ */
/* scene                                                                     */
/* ------------------------------------------------------------------------ */

or_scene* or_scene_new(const float* vtx, int64_t nv, const int32_t* tri, int64_t nt, const int32_t* plane_id) {
    or_scene* s = (or_scene*)calloc(1, sizeof(or_scene));
    s->nt = nt;
    s->t = (otri*)malloc(sizeof(otri) * (size_t)(nt > 0 ? nt : 1));
    s->pn = (double*)calloc((size_t)(nt > 0 ? nt : 1) * 3, sizeof(double));
    s->pp = (double*)calloc((size_t)(nt > 0 ? nt : 1) * 3, sizeof(double));
    s->prep = (int*)malloc(sizeof(int) * (size_t)(nt > 0 ? nt : 1));
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t v = 0; v < nv; v++)
        for (int a = 0; a < 3; a++) {
            double x = (double)vtx[3 * v + a];
            if (x < blo[a]) blo[a] = x;
            if (x > bhi[a]) bhi[a] = x;
        }
    double d[3];
    sub3(bhi, blo, d);
    s->diag = nv > 0 ? sqrt(dot3(d, d)) : 0.0;
    for (int64_t i = 0; i < nt; i++) s->prep[i] = -1;
    for (int64_t i = 0; i < nt; i++) {
        otri* t = &s->t[i];
        for (int a = 0; a < 3; a++) {
            t->v0[a] = (double)vtx[3 * tri[3 * i + 0] + a];
            t->v1[a] = (double)vtx[3 * tri[3 * i + 1] + a];
            t->v2[a] = (double)vtx[3 * tri[3 * i + 2] + a];
        }
        sub3(t->v1, t->v0, t->e1);
        sub3(t->v2, t->v0, t->e2);
        for (int a = 0; a < 3; a++) {
            t->lo[a] = fmin(t->v0[a], fmin(t->v1[a], t->v2[a]));
            t->hi[a] = fmax(t->v0[a], fmax(t->v1[a], t->v2[a]));
        }
        t->plane = plane_id ? plane_id[i] : (int)i;
        int p = t->plane;
        if (s->prep[p] < 0 || s->prep[p] > i) s->prep[p] = (int)i;
    }
    for (int64_t p = 0; p < nt; p++) {
        if (s->prep[p] < 0) continue;
        otri* t = &s->t[s->prep[p]];
        double n[3];
        cross3(t->e1, t->e2, n);
        double len = sqrt(dot3(n, n));
        for (int a = 0; a < 3; a++) {
            s->pn[3 * p + a] = n[a] / len;
            s->pp[3 * p + a] = t->v0[a];
        }
    }
    return s;
}

void or_scene_free(or_scene* s) {
    if (!s) return;
    free(s->t);
    free(s->pn);
    free(s->pp);
    free(s->prep);
    free(s);
}

double or_scene_diag(const or_scene* s) { return s->diag; }

/* plane table export: normals and points of each plane id (NaN if unused) */
void or_scene_planes(const or_scene* s, double* normals, double* points) {
    for (int64_t p = 0; p < s->nt; p++)
        for (int a = 0; a < 3; a++) {
            normals[3 * p + a] = s->prep[p] < 0 ? NAN : s->pn[3 * p + a];
            points[3 * p + a] = s->prep[p] < 0 ? NAN : s->pp[3 * p + a];
        }
}

/* ------------------------------------------------------------------------ */
/* Fibonacci sphere directions (omnidirectional source)                      */
/* ------------------------------------------------------------------------ */

/* z_i = 1 - (2i+1)/N, phi_i = i * pi(3 - sqrt5) mod 2pi,
 * u_i = (sqrt(1 - z^2) cos phi, sqrt(1 - z^2) sin phi, z), FP64, rounded once. */
void or_fibonacci(int64_t n, float* out) {
    const double golden = OR_PI * (3.0 - sqrt(5.0));
    const double two_pi = 2.0 * OR_PI;
    for (int64_t i = 0; i < n; i++) {
        double z = 1.0 - (double)(2 * i + 1) / (double)n;
        double phi = fmod((double)i * golden, two_pi);
        double zz = z * z;
        double rho = sqrt(1.0 - zz);
        double c = cos(phi), s = sin(phi);
        double x = rho * c;
        double y = rho * s;
        out[3 * i + 0] = (float)x;
        out[3 * i + 1] = (float)y;
        out[3 * i + 2] = (float)z;
    }
}

/* ------------------------------------------------------------------------ */
/* geometry primitives                                                       */
/* ------------------------------------------------------------------------ */

/* Moller-Trumbore: returns 0 if the ray is parallel to the plane (det == 0),
 * else 1 with the plane crossing delta and barycentrics lambda (along e1) and
 * mu (along e2).  Inside-ness is decided by the caller. */
static int mt(const otri* t, const double* o, const double* u, double* delta, double* lam, double* mu) {
    double pv[3], tv[3], qv[3];
    cross3(u, t->e2, pv);
    double det = dot3(t->e1, pv);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    sub3(o, t->v0, tv);
    *lam = dot3(tv, pv) * inv;
    cross3(tv, t->e1, qv);
    *mu = dot3(u, qv) * inv;
    *delta = dot3(t->e2, qv) * inv;
    return 1;
}

static double seg_dist2(const double* p, const double* a, const double* b) {
    double ab[3], ap[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    double den = dot3(ab, ab);
    double s = den > 0 ? dot3(ap, ab) / den : 0.0;
    if (s < 0) s = 0;
    if (s > 1) s = 1;
    double q[3] = {a[0] + s * ab[0] - p[0], a[1] + s * ab[1] - p[1], a[2] + s * ab[2] - p[2]};
    return dot3(q, q);
}

/* distance from p to the nearest edge (segment) of t */
static double edge_dist(const otri* t, const double* p) {
    double d = seg_dist2(p, t->v0, t->v1);
    double d2 = seg_dist2(p, t->v1, t->v2);
    double d3 = seg_dist2(p, t->v2, t->v0);
    if (d2 < d) d = d2;
    if (d3 < d) d = d3;
    return sqrt(d);
}

/* distance from a point of the triangle's plane to the closed triangle:
 * 0 inside, else the distance to the nearest edge. */
static double tri_dist(const otri* t, const double* p, double lam, double mu) {
    if (lam >= 0 && mu >= 0 && lam + mu <= 1) return 0.0;
    return edge_dist(t, p);
}

/* ------------------------------------------------------------------------ */
/* one query                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int hit;          /* triangle index, -1 on escape */
    double delta;     /* hit distance (INFINITY on escape) */
    uint32_t det;     /* receiver bit mask */
    uint32_t flags;
    double next[7];   /* o', u', L' (valid when hit >= 0) */
} qres;

static void query(const or_scene* s, const double* o, const double* u, int last_plane, double L,
                  const float* rcv, int n_rcv, double max_len, double eps, int want_flags, qres* r,
                  int64_t* tests) {
    int best = -1;
    double bd = INFINITY;
    for (int64_t j = 0; j < s->nt; j++) {
        const otri* t = &s->t[j];
        if (t->plane == last_plane) continue;
        double d, la, mu;
        if (!mt(t, o, u, &d, &la, &mu)) continue;
        if (la >= 0 && mu >= 0 && la + mu <= 1 && d > 0 && d < bd) {
            bd = d;
            best = (int)j;
        }
    }
    *tests += s->nt;
    r->hit = best;
    r->delta = bd;
    r->flags = 0;
    double tol = eps * s->diag;
    double un2 = dot3(u, u), un = sqrt(un2);
    if (want_flags) {
        for (int64_t j = 0; j < s->nt; j++) {
            const otri* t = &s->t[j];
            if (t->plane == last_plane) continue;
            double d, la, mu;
            if (!mt(t, o, u, &d, &la, &mu)) continue;
            if (d < -tol || d > bd + tol) continue;
            double p[3] = {o[0] + d * u[0], o[1] + d * u[1], o[2] + d * u[2]};
            int near_box = 1;
            for (int a = 0; a < 3; a++)
                if (p[a] < t->lo[a] - tol || p[a] > t->hi[a] + tol) near_box = 0;
            if (!near_box) continue;
            double dist = tri_dist(t, p, la, mu);
            if (dist > tol) continue;
            if ((int)j != best) {
                if (best >= 0 && fabs(d - bd) * un <= tol) r->flags |= OR_FLAG_TIE;
                /* another triangle passing within tol of the ray is a near miss;
                   in front of the chosen hit also at distance 0, where the
                   closed-triangle test rejected it only by the rounding of
                   lambda and mu (a ray through a shared edge or vertex) */
                if (d > 0 && (dist > 0 || d < bd)) r->flags |= OR_FLAG_NEAR_MISS;
            }
            if (fabs(d) * un <= tol) r->flags |= OR_FLAG_TINY;
        }
        if (best >= 0) {
            const otri* t = &s->t[best];
            double p[3] = {o[0] + bd * u[0], o[1] + bd * u[1], o[2] + bd * u[2]};
            if (edge_dist(t, p) <= tol) r->flags |= OR_FLAG_EDGE;
            double n[3];
            cross3(t->e1, t->e2, n);
            double c = fabs(dot3(u, n)) / (un * sqrt(dot3(n, n)));
            if (c <= eps) r->flags |= OR_FLAG_GRAZING;
        }
    }
    /* receiver spheres: closest point of the segment [0, delta_hit] */
    r->det = 0;
    for (int m = 0; m < n_rcv; m++) {
        double xm[3] = {rcv[4 * m + 0], rcv[4 * m + 1], rcv[4 * m + 2]};
        double rad = rcv[4 * m + 3];
        double w[3];
        sub3(xm, o, w);
        double ts = dot3(w, u) / un2;
        if (ts < 0) ts = 0;
        if (ts > bd) ts = bd;
        double q[3] = {o[0] + ts * u[0] - xm[0], o[1] + ts * u[1] - xm[1], o[2] + ts * u[2] - xm[2]};
        double d2 = dot3(q, q);
        if (d2 <= rad * rad) r->det |= 1u << m;
        if (want_flags && fabs(sqrt(d2) - rad) <= tol) r->flags |= OR_FLAG_TANGENT;
    }
    if (best >= 0) {
        const double* n = &s->pn[3 * s->t[best].plane];
        double un_dot = dot3(u, n);
        for (int a = 0; a < 3; a++) {
            r->next[a] = o[a] + bd * u[a];
            r->next[3 + a] = u[a] - 2.0 * un_dot * n[a];
        }
        r->next[6] = L + bd * un;
        if (want_flags && max_len > 0 && fabs(r->next[6] - max_len) <= tol) r->flags |= OR_FLAG_LENGTH;
    }
}

/* ------------------------------------------------------------------------ */
/* thread pool over items                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    atomic_llong next;
    int64_t n;
    int64_t chunk;
    void (*fn)(void* ctx, int64_t i, int64_t* tests);
    void* ctx;
    atomic_llong tests;
} pool_t;

static void* pool_worker(void* arg) {
    pool_t* p = (pool_t*)arg;
    int64_t tests = 0;
    for (;;) {
        int64_t b = atomic_fetch_add(&p->next, p->chunk);
        if (b >= p->n) break;
        int64_t e = b + p->chunk < p->n ? b + p->chunk : p->n;
        for (int64_t i = b; i < e; i++) p->fn(p->ctx, i, &tests);
    }
    atomic_fetch_add(&p->tests, tests);
    return NULL;
}

static int64_t run_pool(int64_t n, int nthreads, int64_t chunk, void (*fn)(void*, int64_t, int64_t*), void* ctx) {
    pool_t p;
    atomic_init(&p.next, 0);
    atomic_init(&p.tests, 0);
    p.n = n;
    p.chunk = chunk;
    p.fn = fn;
    p.ctx = ctx;
    if (nthreads < 1) nthreads = 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, pool_worker, &p);
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    free(th);
    return (int64_t)atomic_load(&p.tests);
}

/* ------------------------------------------------------------------------ */
/* batch of independent queries from given FP32 states                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    const or_scene* s;
    const float *o, *u, *L;
    const int32_t* last_plane;
    const float* rcv;
    int n_rcv;
    double max_len, eps;
    int want_flags;
    int32_t* hit;
    double* delta;
    uint32_t* det;
    double* next;
    uint32_t* flags;
} qb_ctx;

static void qb_item(void* vc, int64_t i, int64_t* tests) {
    qb_ctx* c = (qb_ctx*)vc;
    double o[3] = {c->o[3 * i], c->o[3 * i + 1], c->o[3 * i + 2]};
    double u[3] = {c->u[3 * i], c->u[3 * i + 1], c->u[3 * i + 2]};
    double L = c->L ? (double)c->L[i] : 0.0;
    int lp = c->last_plane ? c->last_plane[i] : -1;
    qres r;
    query(c->s, o, u, lp, L, c->rcv, c->n_rcv, c->max_len, c->eps, c->want_flags, &r, tests);
    c->hit[i] = r.hit;
    if (c->delta) c->delta[i] = r.delta;
    if (c->det) c->det[i] = r.det;
    if (c->flags) c->flags[i] = r.flags;
    if (c->next)
        for (int a = 0; a < 7; a++) c->next[7 * i + a] = r.hit >= 0 ? r.next[a] : NAN;
}

int64_t or_query_batch(const or_scene* s, const float* o, const float* u, const int32_t* last_plane,
                       const float* L, int64_t nq, const float* rcv, int n_rcv, double max_len, double eps,
                       int want_flags, int nthreads, int32_t* hit, double* delta, uint32_t* det,
                       double* next, uint32_t* flags) {
    if (n_rcv > 32) return -1;
    qb_ctx c = {s, o, u, L, last_plane, rcv, n_rcv, max_len, eps, want_flags, hit, delta, det, next, flags};
    return run_pool(nq, nthreads, 4, qb_item, &c);
}

/* ------------------------------------------------------------------------ */
/* full trajectories from a point source                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const or_scene* s;
    const float* src;
    const float* dirs;
    const double* start;   /* [N, 8] per-ray start state (o, u, L, last plane) or NULL */
    const float* rcv;
    int n_rcv, R, want_flags;
    double max_len, eps;
    int32_t* hit_seq;   /* [N, R+1] */
    uint32_t* det;      /* [N, R+1] */
    uint32_t* flags;    /* [N, R+1] */
    double* states;     /* [N, R+2, 8] or NULL */
} tr_ctx;

static void tr_item(void* vc, int64_t i, int64_t* tests) {
    tr_ctx* c = (tr_ctx*)vc;
    const int R1 = c->R + 1;
    double o[3], u[3], L = 0.0;
    int lp = -1;
    if (c->start) {
        /* resumed ray: its state after an earlier call's last reflection */
        const double* st0 = &c->start[8 * i];
        for (int a = 0; a < 3; a++) {
            o[a] = st0[a];
            u[a] = st0[3 + a];
        }
        L = st0[6];
        lp = (int)st0[7];
    } else {
        for (int a = 0; a < 3; a++) {
            o[a] = c->src[a];
            u[a] = c->dirs[3 * i + a];
        }
    }
    for (int k = 0; k < R1; k++) {
        c->hit_seq[i * R1 + k] = -1;
        if (c->det) c->det[i * R1 + k] = 0;
        if (c->flags) c->flags[i * R1 + k] = 0;
    }
    if (c->states)
        for (int k = 0; k < (R1 + 1) * 8; k++) c->states[i * (R1 + 1) * 8 + k] = NAN;
    for (int k = 0; k < R1; k++) {
        if (c->states) {
            double* st = &c->states[(i * (R1 + 1) + k) * 8];
            st[0] = o[0]; st[1] = o[1]; st[2] = o[2];
            st[3] = u[0]; st[4] = u[1]; st[5] = u[2];
            st[6] = L; st[7] = lp;
        }
        qres r;
        query(c->s, o, u, lp, L, c->rcv, c->n_rcv, c->max_len, c->eps, c->want_flags, &r, tests);
        c->hit_seq[i * R1 + k] = r.hit;
        if (c->det) c->det[i * R1 + k] = r.det;
        if (c->flags) c->flags[i * R1 + k] = r.flags;
        if (r.hit < 0) break;                       /* open air: eliminated */
        for (int a = 0; a < 3; a++) {
            o[a] = r.next[a];
            u[a] = r.next[3 + a];
        }
        L = r.next[6];
        lp = c->s->t[r.hit].plane;
        if (c->states) {
            double* st = &c->states[(i * (R1 + 1) + k + 1) * 8];
            st[0] = o[0]; st[1] = o[1]; st[2] = o[2];
            st[3] = u[0]; st[4] = u[1]; st[5] = u[2];
            st[6] = L; st[7] = lp;
        }
        if (c->max_len > 0 && L >= c->max_len) break;
    }
}

int64_t or_trace(const or_scene* s, const float* src, const float* dirs, int64_t n_rays, const float* rcv,
                 int n_rcv, int R, double max_len, double eps, int want_flags, int nthreads, int32_t* hit_seq,
                 uint32_t* det, uint32_t* flags, double* states) {
    if (n_rcv > 32 || R < 0) return -1;
    tr_ctx c = {s, src, dirs, NULL, rcv, n_rcv, R, want_flags, max_len, eps, hit_seq, det, flags, states};
    return run_pool(n_rays, nthreads, 8, tr_item, &c);
}

/* The same propagation loop continued from per-ray FP64 states start[N, 8] =
 * (o, u, L, last plane), e.g. rows of an earlier call's `states` taken after
 * its last reflection: segment 0 of this call is the next segment of that ray. */
int64_t or_trace_from(const or_scene* s, const double* start, int64_t n_rays, const float* rcv, int n_rcv, int R,
                      double max_len, double eps, int want_flags, int nthreads, int32_t* hit_seq, uint32_t* det,
                      uint32_t* flags, double* states) {
    if (n_rcv > 32 || R < 0) return -1;
    tr_ctx c = {s, NULL, NULL, start, rcv, n_rcv, R, want_flags, max_len, eps, hit_seq, det, flags, states};
    return run_pool(n_rays, nthreads, 8, tr_item, &c);
}

/* ------------------------------------------------------------------------ */
/* image-source positions: mirror the source through the planes in order     */
/* ------------------------------------------------------------------------ */

/* planes: flat list of plane ids; offs[i]..offs[i+1] are image source i's
 * reflecting planes in hit order.  out[i] = mirrored source position. */
void or_image_positions(const or_scene* s, const float* src, const int32_t* planes, const int64_t* offs,
                        int64_t n, double* out) {
    for (int64_t i = 0; i < n; i++) {
        double x[3] = {src[0], src[1], src[2]};
        for (int64_t j = offs[i]; j < offs[i + 1]; j++) {
            const double* nn = &s->pn[3 * planes[j]];
            const double* p0 = &s->pp[3 * planes[j]];
            double w[3];
            sub3(x, p0, w);
            double h = dot3(w, nn);
            for (int a = 0; a < 3; a++) x[a] -= 2.0 * h * nn[a];
        }
        for (int a = 0; a < 3; a++) out[3 * i + a] = x[a];
    }
}

/* 'same'-mode direct FIR: y[n] = sum_j h[j] x[n + (K-1)/2 - j], zero outside. */
typedef struct {
    const double* x;
    const double* h;
    double* y;
    int64_t L;
    int K;
    int64_t nsig;
} fir_ctx;

static void fir_item(void* vc, int64_t i, int64_t* tests) {
    fir_ctx* c = (fir_ctx*)vc;
    int64_t sig = i / c->L, n = i % c->L;
    int b = (int)(sig % 8);
    const double* x = c->x + sig * c->L;
    const double* h = c->h + (int64_t)b * c->K;
    int64_t cen = (c->K - 1) / 2;
    double acc = 0.0;
    for (int j = 0; j < c->K; j++) {
        int64_t m = n + cen - j;
        if (m >= 0 && m < c->L) acc += h[j] * x[m];
    }
    c->y[i] = acc;
    (void)tests;
}

/* x, y: [nsig, L] with signal sig using band (sig % 8)'s taps h[8, K] */
void or_fir_same(const double* x, int64_t nsig, int64_t L, const double* h, int K, double* y, int nthreads) {
    fir_ctx c = {x, h, y, L, K, nsig};
    run_pool(nsig * L, nthreads, 256, fir_item, &c);
}
