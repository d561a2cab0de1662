/*
 * rtac.h -- C-ABI of librtac, a gfx950 (MI355X) implementation of the
 * data-parallel hot path of the hybrid ray-tracing / image-source room
 * acoustics method of Aussal & Gueguen, "Open-source platforms for fast room
 * acoustic simulations in complex structures" (2018).
 *
 * Conventions (every entry point):
 *   - Array pointers are DEVICE pointers (HIP global memory) unless the
 *     parameter name ends in _host.  Layouts are row-major, C-contiguous.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue kernels on it and return without waiting, except
 *     rt_build_tree and rt_rebuild_tree, which synchronise once to validate
 *     the mesh.
 *   - The caller owns every input and output buffer; the library owns the
 *     rt_scene object and the scratch memory attached to it.  Scratch grows
 *     on demand (hipMalloc outside any kernel) and is freed by
 *     rt_scene_destroy.  Calls sharing one scene must be ordered on one
 *     stream; different scenes may work on different streams at the same
 *     time (freed scratch is reused only once the freeing call's stream has
 *     passed the point of the free).
 *   - Return value: RT_OK (0) or a negative status; rt_last_error() gives a
 *     thread-local message.  No call throws or aborts.  Outputs that the
 *     device can only size after the fact (detections, image sources) are
 *     never written past their capacity: the required count is stored in the
 *     device counter instead and the caller re-runs with a larger buffer.
 *   - Integers are int32, counts int64.  Triangle ids, plane ids and ray ids
 *     are the caller's indices (original order).
 */
#ifndef RTAC_H
#define RTAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RT_OK = 0,
    RT_EINVAL = -1,      /* bad argument or invalid mesh                       */
    RT_ENOMEM = -2,      /* device allocation failed                           */
    RT_ECAPACITY = -3,   /* reported only by host-side size checks             */
    RT_EHIP = -4,        /* a HIP runtime call failed                          */
    RT_EDEGENERATE = -5  /* zero-area triangle or non-finite vertex            */
};

typedef struct rt_scene rt_scene;

/* Tree-build options.  leaf_size: largest number of triangles per leaf
 * (1 = one element per leaf, as in the paper's tree; at most 8). */
typedef struct {
    int32_t leaf_size;
} rt_build_params;

/*
 * rt_build_tree -- scene ingest and acceleration tree (section "Tree-base
 * acceleration": a mother box containing all elements is split recursively
 * into two daughter boxes down to leaves of one element; built once, in
 * O(M log M), before any ray is traced).
 *
 * The tree is a binary radix tree over the 30-bit Morton codes (10 bits
 * per axis) of the triangle centroids (each split separates the elements of
 * one Morton prefix: a spatial median split cycling through the axes),
 * collapsed into a 4-wide tree for traversal.  Nearest hits do not depend on
 * the tree.
 *
 *   vtx       [n_vtx, 3] float   vertex coordinates (m)
 *   tri       [n_tri, 3] int32   vertex indices of each flat triangle
 *   material  [n_tri]    int32   material index (>= 0) per triangle
 *   plane_id  [n_tri]    int32   coplanar group of each triangle, 0 <= id <
 *                                n_tri, or NULL (= triangle id).  The group's
 *                                representative is its lowest-index triangle;
 *                                its unit normal and first vertex define the
 *                                plane used for reflection and image sources.
 *                                Members must lie in that plane (1e-9 of the
 *                                bounding-box diagonal) and share its material.
 *   params    may be NULL (defaults).
 *   out_scene receives the scene handle (host pointer).
 * Errors: RT_EINVAL (index out of range, plane group not coplanar or of mixed
 * material, n_tri < 1), RT_EDEGENERATE (zero-area triangle, NaN/Inf vertex),
 * RT_ENOMEM, RT_EHIP.  Synchronises `stream` once (validation and the
 * reference count, which sizes the per-reference arrays); the rest of the
 * build runs on after the call returns (the first rt_scene_info call waits for
 * it; the build's temporaries are kept until then, or until rt_scene_destroy).
 */
int rt_build_tree(const float* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                  const int32_t* material, const int32_t* plane_id, const rt_build_params* params,
                  void* stream, rt_scene** out_scene);

/*
 * rt_rebuild_tree -- the same build as rt_build_tree (same section, same
 * arguments and errors), into an existing scene: the tree, triangle records
 * and plane table are replaced by those of the new mesh, reusing the scene's
 * device memory (nothing is allocated when the mesh is no larger than the
 * one of an earlier build of this scene and rt_scene_info has not released
 * the temporaries since).  For a caller that re-runs the whole path per frame
 * or per job, e.g. one scene per stream with the jobs of several streams
 * overlapping on the GPU.
 *   scene   a scene from rt_build_tree on the current device.  Earlier calls
 *           that use it must be on `stream` (in stream order they finish
 *           before the rebuild overwrites what they read) or finished.
 *   others  as for rt_build_tree.
 * Batches made from the scene (rt_batch_create) hold its old sizes and
 * addresses: destroy and recreate them after a rebuild.  On any error the
 * scene is marked invalid (every call that takes it returns RT_EINVAL) until
 * a rebuild succeeds; rt_scene_destroy still frees it.
 */
int rt_rebuild_tree(rt_scene* scene, const float* vtx, int64_t n_vtx, const int32_t* tri, int64_t n_tri,
                    const int32_t* material, const int32_t* plane_id, const rt_build_params* params,
                    void* stream);

/* Frees the scene and its scratch (synchronises the device). */
int rt_scene_destroy(rt_scene* scene);

/* Host-side facts about a built scene: info_host[0] = n_tri, [1] = number of
 * materials (max material + 1), [2] = 4-wide tree nodes, [3] = tree depth,
 * [4] = leaf size, [5] = references (triangle records of the tree, >= n_tri:
 * thin triangles are cut into several); diag_host[0] = bounding-box
 * diagonal D (m).  With info_host, the first call waits for the build to
 * finish and reads the node count and depth from the device (RT_EHIP if they
 * are inconsistent); diag_host alone never waits. */
int rt_scene_info(const rt_scene* scene, int64_t* info_host, double* diag_host);

/*
 * rt_fibonacci_directions -- omnidirectional source sampling (section
 * "Discrete model": rays leave the source along a uniform sampling of the
 * unit sphere, e.g. by Fibonacci's rule, each with energy 4 pi / N).
 *   dirs [n, 3] float out:  z_i = 1 - (2i+1)/n,  phi_i = i pi (3 - sqrt 5) mod 2pi,
 *   u_i = (sqrt(1 - z_i^2) cos phi_i, sqrt(1 - z_i^2) sin phi_i, z_i), evaluated in
 *   FP64 and rounded once to FP32.
 */
int rt_fibonacci_directions(int64_t n, float* dirs, void* stream);

/*
 * rt_icosahedral_directions -- omnidirectional source sampled by icosahedron
 * subdivision (section "Discrete model", one of the uniform samplings named).
 *   f     frequency, 1 <= f <= 14000: each face is cut into f^2 triangles
 *   dirs  [10 f^2 + 2, 3] float out (device), unit directions:
 *         the icosahedron's vertices V_0..V_11 are the cyclic placements
 *         (0, a, b), (a, b, 0), (b, 0, a) of a = +-1, b = +-phi (phi the golden
 *         ratio; placements in that order, signs (-,-), (-,+), (+,-), (+,+));
 *         edges are the vertex pairs at distance 2 (a < b, lexicographic),
 *         faces the mutually adjacent triples (a < b < c, lexicographic).
 *         Rows: the 12 vertices; for each edge, (f-q) V_a + q V_b for
 *         q = 1..f-1; for each face, (f-i-j) V_a + i V_b + j V_c for i >= 1,
 *         j >= 1, i + j <= f-1, by i then j.  Each point p is divided by
 *         sqrt(x^2 + y^2 + z^2); FP64 without contraction, rounded once.
 * Every ray then carries energy 1/N with N = 10 f^2 + 2.
 */
int rt_icosahedral_directions(int32_t f, float* dirs, void* stream);

/*
 * rt_directional_directions -- directional source sampled non-uniformly
 * (section "Discrete model", footnote on directional sources): energy per
 * solid angle proportional to (1 + cos theta)^m about `axis` (directivity
 * factor m + 1 on the axis), every ray carrying the same energy 1/N, so the
 * pattern is the density of the rays.
 *   n          rays, 0 <= n < 2^31
 *   m          pattern exponent, finite, >= 0 (0: omnidirectional)
 *   axis_host  [3] float host, nonzero (normalised in FP64)
 *   dirs       [n, 3] float out (device)
 * Ray i: F = 1 - (2i+1)/(2n), z = 2 F^(1/(m+1)) - 1 (inverse of the
 * distribution ((1+z)/2)^(m+1) of cos theta), phi = i pi (3 - sqrt 5) mod
 * 2 pi, u = rho cos(phi) t1 + rho sin(phi) t2 + z axis with rho = sqrt(1 - z^2);
 * t1 = the part of h orthogonal to the axis, normalised (h = e_x, or e_y
 * when |axis_x| >= 0.9), t2 = axis x t1.  FP64, rounded once.
 * Errors: RT_EINVAL (n out of range, m negative or not finite, axis zero).
 */
int rt_directional_directions(int64_t n, double m, const float* axis_host, float* dirs, void* stream);

/* Trace options. */
typedef struct {
    int32_t max_reflections;   /* R >= 0: segments 0..R are traced (R reflections)           */
    float max_path_length;     /* > 0: a ray stops once its travelled length reaches it        */
    int32_t record_states;     /* nonzero: write each segment's input state to `states`        */
    int32_t fetch_threshold;   /* 0 = default; lanes idle before a wave fetches new rays       */
    int32_t shade_threshold;   /* 0 = default (16; 48 when max_reflections = 0); finished queries
                                  before a wave shades them.  With reflections this is for a full
                                  wave and scales with the lanes still working (at least 1)     */
    int32_t blocks_per_cu;     /* 0 = default; persistent workgroups per compute unit          */
    int32_t keep_order;        /* 0: rays are handed to wavefronts sorted by a Morton key of
                                  their direction (and origin) for coherence; 1: in index order */
    int64_t* stats;            /* NULL or device int64[4], overwritten: inner nodes visited,
                                  leaves visited, triangle tests, stack spills.  Counts the
                                  per-lane traversal, so a call with stats runs with
                                  coop_queries off and 4 waves per SIMD (same results)          */
    int32_t rounds;            /* 0 = default (1); kernel launches: once the ray pool is empty,
                                  a wavefront with few rays left hands them to the next launch  */
    int32_t spill_threshold;   /* 0 = default; most rays a wavefront may still hold to hand over */
    int32_t waves_per_simd;    /* 0 = default (4); register budget of the trace kernel: 4, 5, 6, 8 */
    void* kernel_event_start;  /* NULL or a hipEvent_t: recorded on `stream` just before the first
                                  traversal-kernel launch (after ray ordering and output fill)  */
    void* kernel_event_stop;   /* NULL or a hipEvent_t: recorded just after the last one        */
    int32_t suspend_after;     /* 0 = off; S in [1, R]: two launches, the first traces segments
                                  0..S-1 of every ray and queues the rays that continue, the second
                                  finishes them all together (long bounce chains start at once).
                                  Results are identical; overrides `rounds`                     */
    int32_t min_beam_rays;     /* 0 = off; n >= 1: the range of the discrete model (eq. 13): a ray
                                  stops once its travelled length reaches (r / 2) sqrt(N / n), r =
                                  the largest receiver radius and N = the rays of the call (of the
                                  job, in a batch); FP64, rounded to FP32.  Combined with
                                  max_path_length by taking the smaller limit                     */
    int32_t xcd_pools;         /* 0 = default (on), -1 off: the ordered ray pool is cut into eighths,
                                  one per accelerator complex (each has its own L2), which
                                  workgroups drain first before helping the others             */
    int32_t coop_queries;      /* 0 = default (on), -1 off: once every ray has been handed out, a
                                  wavefront left with one to eight queries in flight searches
                                  them with all its lanes (64, 32, 16 or 8 per query), breadth
                                  first, two tree levels per step; same nearest hit            */
    const int32_t* record_rows; /* NULL: with record_states, ray i writes row i of `states`; else
                                  device int32[n_rays] (global ray ids in a batch): ray i writes
                                  row record_rows[i] (< 0: not recorded), so a few rays of a large
                                  launch can be recorded without changing the launch            */
    int32_t stack_depth;       /* 0 = default (16); 8, 16 or 32: LDS traversal-stack entries per lane
                                  (the stack spills to global memory beyond them; the cooperative
                                  search's frontier holds stack_depth / 2 entries per lane)     */
} rt_trace_params;

/*
 * rt_trace_rays -- specular ray propagation with receiver detection
 * (sections "Presence of an obstacle", "Standard algorithm" and "Tree-base
 * acceleration").  For each ray and each segment k = 0..R:
 *   - nearest hit: minimal delta > 0 of o + delta u over the triangles with
 *     0 <= lambda, mu and lambda + mu <= 1, skipping the plane of the previous
 *     reflection; exact FP32 ties go to the lowest triangle id (watertight
 *     FP32 ray/triangle test, 4-wide tree traversal; a box is culled only
 *     when its FP32 entry distance exceeds the best hit by more than 2^-20
 *     relative, so the rule holds whatever the search order, except for
 *     near-grazing hits whose FP32 distance is off by more than 13 roundings);
 *   - detection: receiver m is crossed when the segment [0, delta_hit]
 *     (unbounded on escape) comes within its radius of its centre (closed
 *     ball, FP64; the sphere is transparent);
 *   - reflection: u' = u - 2 (u.n) n with the plane's unit normal,
 *     o' = o + delta u, L' = L + delta |u| (FP64, rounded to FP32);
 *   - the ray stops after segment R, once L' >= max_path_length or the
 *     eq. 13 range (min_beam_rays), or when it hits nothing (open air:
 *     eliminated).
 *
 *   src_host    [3] float host  source; used when origins == NULL
 *   origins     [n_rays, 3] float or NULL  per-ray start point
 *   dirs        [n_rays, 3] float           start direction (not normalised by the library)
 *   start_plane [n_rays] int32 or NULL      plane excluded from segment 0 (-1 none)
 *   start_len   [n_rays] float or NULL      travelled length at the start (0)
 *   rcv         [n_rcv, 4] float            receiver spheres (x, y, z, r); n_rcv <= 32
 *   hit_seq     [n_rays, R+1] int32 out     triangle id ending segment k; -1 on escape
 *                                           and after the ray stopped
 *   det         [det_cap, 3] int32 out      detections (ray, k, receiver), any order
 *   counters    [4] int64 out (device)      [0] detections (may exceed det_cap: then
 *                                           only det_cap rows were written), [1] queries
 *                                           (ray-segments traced), [2] escapes,
 *                                           [3] device error word (0 = none)
 *   states      [n_rays, R+2, 8] float or NULL   when record_states: input state
 *                                           (o, u, L, last plane as int bits) of each
 *                                           segment, and after the last reflection
 *                                           (rows as selected by record_rows)
 * The travelled length is carried in FP64 from segment to segment (it is
 * rounded to FP32 only where it is recorded).
 * The counters are overwritten (not accumulated).
 */
int rt_trace_rays(const rt_scene* scene, const float* src_host, const float* origins, const float* dirs,
                  const int32_t* start_plane, const float* start_len, int64_t n_rays, const float* rcv,
                  int32_t n_rcv, const rt_trace_params* params, int32_t* hit_seq, int32_t* det,
                  int64_t det_cap, int64_t* counters, float* states, void* stream);

/*
 * rt_collect_image_sources -- image sources from detected rays (section
 * "Image-sources": rays reaching the receiver are retro-propagated and focus
 * on point image sources; each carries n rays).  Key of a detection
 * (ray, k, m): (m, k, plane ids of the ray's hits on segments 0..k-1).  Keys
 * are hashed, sorted and deduplicated with a full comparison; n = number of
 * detections per key.  Position: the source mirrored through the key's
 * planes in order (FP64); distance to the receiver centre (FP64).
 *
 *   src_host  [3] float host; hit_seq [n_rays, R+1]; det [det_cap, 3]
 *   n_det     device int64 (e.g. trace counters[0]); rows beyond min(n_det,
 *             det_cap) are ignored
 *   is_key    [is_cap, R+2] int32 out: (m, k, planes..., -1 padding)
 *   is_count  [is_cap] int32 out;  is_pos [is_cap, 3] double out;
 *   is_dist   [is_cap] double out; n_is: device int64 out (may exceed is_cap:
 *             then only is_cap rows were written).  Row order: deterministic
 *             (by key hash), not part of the contract.
 */
int rt_collect_image_sources(const rt_scene* scene, const float* src_host, const float* rcv, int32_t n_rcv,
                             const int32_t* hit_seq, int64_t n_rays, int32_t max_reflections,
                             const int32_t* det, int64_t det_cap, const int64_t* n_det, int32_t* is_key,
                             int32_t* is_count, double* is_pos, double* is_dist, int64_t is_cap,
                             int64_t* n_is, void* stream);

/*
 * rt_assemble_ir -- impulse response from the image sources (section
 * "Image-sources": E_s(f) = n/N exp(-beta(f) d_s) prod_j (1 - alpha_j(f));
 * arrival time d_s / c; pressure p = sqrt(E); FIR filters over 8 octave
 * bands, abstract).  Per receiver r and band b:
 *   hist[r,b,s]    = sum of E_s(b) over image sources with floor(d_s fs / c) = s < L
 *                    (FP64 sums in a fixed order, rounded to float)
 *   band_ir[r,b,:] = 'same' FIR of sqrt(hist[r,b,:]) with taps fir[b, :] (K odd):
 *                    y[n] = sum_j fir[b,j] p[n + (K-1)/2 - j]
 *   ir[r,:]        = sum_b band_ir[r,b,:];   band_energy[r,b] = sum_s hist[r,b,s]
 *   is_key/is_count/is_dist/n_is as written by rt_collect_image_sources;
 *   alpha [n_mat, 8] float; beta [8] float (1/m, energy); fir [8, K] float.
 *   Outputs: band_energy [n_rcv, 8], hist [n_rcv, 8, L], band_ir [n_rcv, 8, L],
 *   ir [n_rcv, L], all float.
 */
int rt_assemble_ir(const rt_scene* scene, const int32_t* is_key, const int32_t* is_count,
                   const double* is_dist, const int64_t* n_is, int64_t is_cap, int32_t max_reflections,
                   int64_t n_rays, int32_t n_rcv, const float* alpha, const float* beta, float c, float fs,
                   int64_t L, const float* fir, int32_t K, float* band_energy, float* hist, float* band_ir,
                   float* ir, void* stream);

/*
 * rt_band_energy_adjoint -- gradient of band energies with respect to the
 * per-material absorption (the energy of an image source is a polynomial in
 * alpha, eq. for E_s).  For an image source with c_m reflections on material m:
 *   dE_s(b)/dalpha[m,b] = -n/N e^{-beta_b d_s} c_m (1 - alpha[m,b])^(c_m - 1)
 *                         prod_{m' != m} (1 - alpha[m',b])^(c_m')
 * grad_alpha[m,b] = sum_r grad_band_energy[r,b] * sum_{s of r, bin < L} dE_s(b)/dalpha[m,b].
 *   grad_band_energy [n_rcv, 8] float; grad_alpha [n_mat, 8] float out
 *   (overwritten).  Deterministic (fixed-order FP64 reduction).
 */
int rt_band_energy_adjoint(const rt_scene* scene, const int32_t* is_key, const int32_t* is_count,
                           const double* is_dist, const int64_t* n_is, int64_t is_cap,
                           int32_t max_reflections, int64_t n_rays, int32_t n_rcv, const float* alpha,
                           int32_t n_mat, const float* beta, float c, float fs, int64_t L,
                           const float* grad_band_energy, float* grad_alpha, void* stream);

/*
 * Batches: many jobs -- a source with its own Fibonacci rays and receivers in
 * one of several scenes (rooms of uneven size) -- traced by one persistent
 * launch (each job follows the same definitions as
 * rt_trace_rays, rt_collect_image_sources, rt_assemble_ir and
 * rt_band_energy_adjoint).  Rays of job j are global ids ray_off_j ..
 * ray_off_j + n_rays_j - 1 (jobs in order), receivers of job j are global rows
 * rcv_off_j .. + n_rcv_j - 1, materials of scene i are global rows
 * mat_off_i .. + n_mat_i - 1 (scenes in order).  Directions are generated on
 * the device: ray i of a job with n rays takes Fibonacci direction i of n.
 */
typedef struct rt_batch rt_batch;

typedef struct {
    int32_t scene;             /* index into the scenes of rt_batch_create          */
    int32_t n_rcv;             /* receivers of this job, 1..32                      */
    int64_t n_rays;            /* rays of this job                                  */
    float src[3];              /* point source                                      */
    float max_path_length;     /* > 0: stop once travelled length reaches it        */
} rt_job;

/* Uploads the job and scene tables (synchronises `stream` once).  The scenes
 * must outlive the batch; the first scene's scratch is used by batch calls. */
int rt_batch_create(const rt_scene* const* scenes, int32_t n_scenes, const rt_job* jobs, int32_t n_jobs, void* stream,
                    rt_batch** out);
int rt_batch_destroy(rt_batch* batch);
/* info_host[0] = jobs, [1] = total rays, [2] = total receivers, [3] = total materials */
int rt_batch_info(const rt_batch* batch, int64_t* info_host);

/* One persistent launch over every ray of every job.  rcv [total_rcv, 4];
 * hit_seq [total_rays, R+1]; det rows are (global ray, k, global receiver);
 * counters as in rt_trace_rays; states as in rt_trace_rays, indexed by global
 * ray id (or by record_rows), NULL unless record_states. */
int rt_trace_batch(rt_batch* batch, const float* rcv, const rt_trace_params* params, int32_t* hit_seq, int32_t* det,
                   int64_t det_cap, int64_t* counters, float* states, void* stream);

/* Image sources of all jobs: keys start with the global receiver row; the
 * position mirrors the job's source in its scene's planes. */
int rt_collect_batch(rt_batch* batch, const float* rcv, const int32_t* hit_seq, int32_t max_reflections,
                     const int32_t* det, int64_t det_cap, const int64_t* n_det, int32_t* is_key, int32_t* is_count,
                     double* is_pos, double* is_dist, int64_t is_cap, int64_t* n_is, void* stream);

/* Impulse responses of all jobs: alpha [total_mat, 8]; E_s uses the job's ray
 * count; outputs indexed by global receiver row ([total_rcv, 8] etc.). */
int rt_assemble_batch(rt_batch* batch, const int32_t* is_key, const int32_t* is_count, const double* is_dist,
                      const int64_t* n_is, int64_t is_cap, int32_t max_reflections, const float* alpha,
                      const float* beta, float c, float fs, int64_t L, const float* fir, int32_t K,
                      float* band_energy, float* hist, float* band_ir, float* ir, void* stream);

/* Gradient of sum_r,b g[r,b] band_energy[r,b] w.r.t. alpha [total_mat, 8]. */
int rt_adjoint_batch(rt_batch* batch, const int32_t* is_key, const int32_t* is_count, const double* is_dist,
                     const int64_t* n_is, int64_t is_cap, int32_t max_reflections, const float* alpha,
                     const float* beta, float c, float fs, int64_t L, const float* grad_band_energy,
                     float* grad_alpha, void* stream);

/* ------------------------------------------------------------------------
 * Late-tail surrogate (an extension of the method, not in the paper).  The
 * paper notes that late image sources are reached by few rays (section
 * "Discrete model"), so the late response is the noisiest and costliest part
 * of a trace.  A ReLU multilayer perceptron maps the per-band energy
 * histogram of reflection orders 0..8 (features) to the per-band decay curve
 * of the full trace (Schroeder backward integration, dB re total).
 *
 * Network: widths w_0 .. w_L (each a multiple of 64 in [64, 4096], L <= 8);
 * hidden layers h_l = relu(W_l h_{l-1} + b_l), output y = W_L h_{L-1} + b_L.
 * Parameters are one flat vector, layer after layer: W_l [w_l, w_{l-1}]
 * row-major, then b_l [w_l].  theta (FP32 master copy) and theta_bf16 (its
 * round-to-nearest-even BF16 copy, read by the matrix-core kernels) share
 * that layout, as do the gradient and both Adam moments.  Products run on
 * the BF16 matrix cores with FP32 accumulation; activations are stored in
 * BF16.  A handle owns the activations of its last forward call and the
 * backward scratch; calls on one handle must be ordered on one stream.
 * ------------------------------------------------------------------------ */
typedef struct rt_mlp rt_mlp;

/* widths: host int32 [n_layers + 1]; max_batch: largest batch of any call. */
int rt_mlp_create(const int32_t* widths, int32_t n_layers, int64_t max_batch, rt_mlp** out);
int rt_mlp_destroy(rt_mlp* net);
/* info: host int64[4] = number of parameters, layers, max_batch, activation elements. */
int rt_mlp_info(const rt_mlp* net, int64_t* info);

/* y [batch, w_L] float = network(x [batch, w_0] bf16).  theta_f32 (may be
 * NULL): when given, biases are read from it in FP32, else from theta_bf16.
 * x and theta_bf16 must be 16-byte aligned.  Keeps the hidden activations
 * for rt_mlp_backward. */
int rt_mlp_forward(rt_mlp* net, const uint16_t* theta_bf16, const float* theta_f32, const uint16_t* x,
                   int64_t batch, float* y, void* stream);

/* Masked squared error S = sum m (y - t)^2 over [batch, w_L] (mask NULL: all
 * ones) and its gradient dS/dtheta into grad [n_params] float (overwritten,
 * not divided by sum m).  loss_terms: device double[2] out = (S, sum m); the
 * mean loss is S / sum m.  Must follow rt_mlp_forward on the same x and
 * batch (the batch is checked, x is not). */
int rt_mlp_backward(rt_mlp* net, const uint16_t* theta_bf16, const uint16_t* x, int64_t batch, const float* y,
                    const float* target, const float* mask, float* grad, double* loss_terms, void* stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected moments) at step >= 1 on
 * all n_params entries: g = grad / loss_terms[1] (g = grad when loss_terms
 * is NULL; 0 when the mask sum is 0), m = b1 m + (1 - b1) g, v = b2 v +
 * (1 - b2) g^2, theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * in FP32; theta_bf16 (may be NULL) receives the rounded copy. */
int rt_mlp_adam(int64_t n_params, float* theta, uint16_t* theta_bf16, const float* grad, float* m, float* v,
                const double* loss_terms, int32_t step, float lr, float beta1, float beta2, float eps,
                void* stream);

/* y [n] bf16 = round-to-nearest-even(x [n] float). */
int rt_to_bf16(const float* x, int64_t n, uint16_t* y, void* stream);

/* Surrogate features: x[i] = (max(10 log10 hist[i], floor_db) + offset_db) /
 * scale_db as BF16 (a bin with no energy gives floor_db). */
int rt_hist_features(const float* hist, int64_t n, float floor_db, float offset_db, float scale_db, uint16_t* x,
                     void* stream);

/* Energy decay curve per row of hist [rows, bins] (energy per time bin):
 * edc[r, s] = 10 log10(sum_{s' >= s} hist[r, s'] / sum_{s'} hist[r, s']),
 * FP64 sums, clamped below at floor_db (a row without energy is all floor). */
int rt_edc_db(const float* hist, int64_t rows, int32_t bins, float floor_db, float* edc, void* stream);

/*
 * rt_room_params -- perceptive factors from the per-band energy histogram of
 * an impulse response (the paper tabulates EDT, T30, SPL, C80, D50 and Ts for
 * its theater, Table 3; definitions as in room-acoustics practice, ISO 3382-1).
 *   hist   [n_rcv, 8, L] float: energy per time bin of width 1/fs (e.g. the
 *          `hist` output of rt_assemble_ir)
 *   params [n_rcv, 8, 6] double out: EDT (s), T30 (s), C80 (dB), D50
 *          (fraction), Ts (s), SPL (dB re the emitted energy)
 * Origin s0 = first bin with energy in any band of the receiver.  Schroeder
 * curve EDC(s) = sum_{s' >= s} H[s'] in dB re EDC(s0), up to the last bin with
 * energy.  EDT, T30 = -60 / slope of the least-squares line of EDC_dB against
 * (s - s0) / fs over 0..-10 dB and -5..-35 dB; NaN unless the curve reaches
 * -10 (-35) dB and 2 bins qualify.  C80 = 10 log10(E_early / E_late) with
 * floor(0.08 fs + 1/2) early bins (NaN without late energy); D50 = share of
 * the first floor(0.05 fs + 1/2) bins; Ts = energy-weighted mean of
 * (s - s0) / fs; SPL = 10 log10 sum H.  A band without energy gives NaN.
 */
int rt_room_params(const float* hist, int32_t n_rcv, int64_t L, float fs, double* params, void* stream);

/*
 * rt_room_params_noalloc -- rt_room_params for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * rt_room_params (bit for bit); no hipMalloc, hipFree or other allocating
 * call is made.  Its scratch (chunk sums, chunk prefixes, per-band facts and
 * regression sums: 128 bytes per (receiver, band, chunk of 4096 bins) plus 48
 * bytes per (receiver, band)) lives in a fixed 4 MiB device array, one copy
 * per GPU, held until the process ends; its address is looked up on the
 * first call on each device: up to 520,192 bins with 32 receivers, or
 * 2,093,056 bins with 8.  Larger requests return RT_ECAPACITY with a message
 * before any device call.
 * Every scratch element is written before it is read in a call, so nothing
 * needs clearing between calls.  All calls on one GPU share the array: calls
 * that overlap in time on that GPU (two streams, two threads) race and must
 * be serialised by the caller.
 */
int rt_room_params_noalloc(const float* hist, int32_t n_rcv, int64_t L, float fs, double* params, void* stream);

/* Test hook for the exact-grouping path of rt_collect_image_sources: keep
 * only the low `bits` bits (1..64, default 48) of the 64-bit key hash so that
 * distinct keys collide.  Process-wide; not thread-safe with concurrent
 * collect calls.  Grouping stays exact at any setting (full-key comparison);
 * only speed changes. */
int rt_debug_set_hash_bits(int bits);

/* Test hook for the library's internal radix sort (used by the tree build,
 * the ray order, the image-source collection and the IR assembly): sorts
 * keys[0, n) by bits [begin_bit, end_bit) of each key, stably, in place, and
 * writes to order[0, n) the position each key had before the sort.
 *   keys   [cap] uint64 in/out;  order [cap] uint32 out
 *   n_dev  device int64 count n (clamped to [0, cap]), or NULL for n = cap;
 *          keys[n, cap) and order[n, cap) are unspecified afterwards
 *   0 <= begin_bit < end_bit <= 64.
 * Allocates its scratch per call (fenced frees on `stream`).  Errors: RT_EINVAL,
 * RT_ENOMEM, RT_EHIP. */
int rt_debug_radix_sort(uint64_t* keys, uint32_t* order, int64_t cap, const int64_t* n_dev, int32_t begin_bit,
                        int32_t end_bit, void* stream);

/* Thread-local message describing the last non-OK status of this thread. */
const char* rt_last_error(void);

/* Library version string. */
const char* rt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RTAC_H */
