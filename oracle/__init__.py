"""FP64 CPU oracle of the hybrid ray-tracing / image-source method.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the GPU path; the two read the same seeded input arrays (``synth``).

Each function cites the part of the paper it follows:

* ``fibonacci``       -- omnidirectional source, unit-sphere sampling by
                         Fibonacci's rule (section "Discrete model").
* ``trace`` /
  ``trace_from`` /
  ``query_batch``     -- brute-force nearest hit over all triangles with the
                         parametric conditions 0 <= lambda, mu; lambda + mu <= 1;
                         delta > 0 minimal (section "Standard algorithm"),
                         receiver sphere (x - x_m)^2 = r^2, specular reflection
                         (eq. for u_r), elimination of rays leaving an open room.
* ``image_sources``   -- detected rays grouped by their reflection sequence;
                         each group is one point image source whose position is
                         the source mirrored through the planes in order, with
                         n = number of rays (section "Image-sources").
* ``is_energy``       -- E_s(f) = n/N exp(-beta(f) d_s) prod_j (1 - alpha_j(f))
                         (eq. for E_s with air absorption).
* ``assemble_ir``     -- arrival time d_s/c, energy histogram per band,
                         p = sqrt(E), FIR filtering over 8 octave bands, summed.
* ``band_energy_grad``-- analytic derivative of the band energies w.r.t. the
                         per-material absorption (E is a polynomial in alpha).
* ``icosahedral`` /
  ``directional``     -- source variants (section "Discrete model"): unit-sphere
                         sampling by icosahedron subdivision, and a directional
                         source sampled non-uniformly (footnote on directional
                         sources), every ray carrying the same energy.
* ``range_limit``     -- maximum range of the discrete model, d <= (r/2) sqrt(N/n)
                         (eq. 13); ``trace`` stops rays there through max_len
                         (section "Standard algorithm": rays propagate while the
                         travelled length satisfies it).

Parity unpinned: none of the functions above; each is pinned by the tests in
``tests/test_oracle_*.py`` against closed forms, exact rational arithmetic,
invariants or the paper's printed parameters.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLAG_EDGE, FLAG_NEAR_MISS, FLAG_TIE, FLAG_TINY, FLAG_GRAZING, FLAG_TANGENT, FLAG_LENGTH = (
    1, 2, 4, 8, 16, 32, 64)
DEFAULT_EPS = 1e-6


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.or_scene_new.restype = P
        L.or_scene_new.argtypes = [P, i64, P, i64, P]
        L.or_scene_free.argtypes = [P]
        L.or_scene_diag.restype = dbl
        L.or_scene_diag.argtypes = [P]
        L.or_scene_planes.argtypes = [P, P, P]
        L.or_fibonacci.argtypes = [i64, P]
        L.or_query_batch.restype = i64
        L.or_query_batch.argtypes = [P, P, P, P, P, i64, P, i32, dbl, dbl, i32, i32, P, P, P, P, P]
        L.or_trace.restype = i64
        L.or_trace.argtypes = [P, P, P, i64, P, i32, i32, dbl, dbl, i32, i32, P, P, P, P]
        L.or_trace_from.restype = i64
        L.or_trace_from.argtypes = [P, P, i64, P, i32, i32, dbl, dbl, i32, i32, P, P, P, P]
        L.or_image_positions.argtypes = [P, P, P, P, i64, P]
        L.or_fir_same.argtypes = [P, i64, i64, P, i32, P, i32]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def host_cpus() -> Dict[str, int]:
    """What the host offers this process: logical CPUs of the machine, CPUs in
    the process's affinity mask, and the thread share it is granted
    (OMP_NUM_THREADS when set, at most 16: the share of one GPU's host on a
    shared GPU node)."""
    total = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = total
    share = affinity
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        share = min(share, int(env))
    return {"cpu_count": total, "affinity": affinity, "threads": max(1, min(16, share))}


def default_threads() -> int:
    return host_cpus()["threads"]


class OracleScene:
    """FP64 copy of a mesh: per-triangle vertices and edges, plane table of
    representatives (lowest triangle index of each plane id)."""

    def __init__(self, vtx, tri, plane_id=None):
        self.vtx = np.ascontiguousarray(vtx, np.float32)
        self.tri = np.ascontiguousarray(tri, np.int32)
        self.plane_id = (np.arange(len(tri), dtype=np.int32) if plane_id is None
                         else np.ascontiguousarray(plane_id, np.int32))
        self._h = lib().or_scene_new(_p(self.vtx), len(self.vtx), _p(self.tri), len(self.tri),
                                     _p(self.plane_id))

    @classmethod
    def of(cls, scene) -> "OracleScene":
        return cls(scene.vtx, scene.tri, scene.plane_id)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_scene_free(self._h)
            self._h = None

    @property
    def diag(self) -> float:
        return float(lib().or_scene_diag(self._h))

    def planes(self) -> Tuple[np.ndarray, np.ndarray]:
        n = np.empty((len(self.tri), 3))
        p = np.empty((len(self.tri), 3))
        lib().or_scene_planes(self._h, _p(n), _p(p))
        return n, p


def range_limit(r: float, n_rays: int, n: int = 1) -> float:
    """Eq. 13: a beam of n >= 1 of the N emitted rays, crossing a receiver of
    radius r, is measurable up to d = (r/2) sqrt(N/n) (the small-angle count
    n/N ~ r^2 / (4 d^2) of eq. 12 solved for d).  FP64."""
    return 0.5 * float(r) * math.sqrt(float(n_rays) / float(n))


def icosahedron_vertices() -> np.ndarray:
    """The 12 vertices of the regular icosahedron (unnormalised, edge 2):
    the cyclic placements (0, a, b), (a, b, 0), (b, 0, a) of a = +-1,
    b = +-phi, phi the golden ratio; placements in that order, signs of
    (a, b) in the order (-,-), (-,+), (+,-), (+,+)."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    out = []
    for place in range(3):
        for sa in (-1.0, 1.0):
            for sb in (-1.0, 1.0):
                a, b = sa, sb * phi
                out.append([(0.0, a, b), (a, b, 0.0), (b, 0.0, a)][place])
    return np.array(out)


def icosahedral(f: int) -> np.ndarray:
    """[10 f^2 + 2, 3] FP32 unit directions: every face of the icosahedron
    cut into f^2 triangles, the grid points (f-i-j) A + i B + j C pushed to
    the unit sphere (FP64, rounded once).  Order: the 12 vertices; the f-1
    inner points of each edge (a < b, edges in lexicographic order), from a
    towards b; the inner points of each face (a < b < c, faces in
    lexicographic order), by i then j."""
    v = icosahedron_vertices()
    n = len(v)
    adj = [[float(((v[p] - v[q]) ** 2).sum()) < 4.5 for q in range(n)] for p in range(n)]
    edges = [(p, q) for p in range(n) for q in range(p + 1, n) if adj[p][q]]
    faces = [(p, q, r) for p in range(n) for q in range(p + 1, n) for r in range(q + 1, n)
             if adj[p][q] and adj[q][r] and adj[p][r]]
    assert len(edges) == 30 and len(faces) == 20
    pts = [v[p] for p in range(n)]
    for a, b in edges:
        for q in range(1, f):
            pts.append((f - q) * v[a] + q * v[b])
    for a, b, c in faces:
        for i in range(1, f - 1):
            for j in range(1, f - i):
                pts.append((f - i - j) * v[a] + i * v[b] + j * v[c])
    p = np.array(pts, dtype=np.float64).reshape(-1, 3)
    nrm = np.sqrt(p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1] + p[:, 2] * p[:, 2])
    return (p / nrm[:, None]).astype(np.float32)


def directional(n: int, m: float, axis) -> np.ndarray:
    """[n, 3] FP32 directions of a directional source whose radiated energy
    per solid angle is proportional to (1 + cos theta)^m about `axis`
    (m >= 0; m = 0 is omnidirectional).  Every ray carries energy 1/N, so
    the pattern is the density of the rays: the Fibonacci points with
    F_i = 1 - (2i+1)/(2n) and phi_i = i pi (3 - sqrt5) mod 2 pi, the polar
    coordinate warped by the inverse of the pattern's distribution function
    of cos theta, F(z) = ((1 + z)/2)^(m+1): z_i = 2 F_i^(1/(m+1)) - 1.  Local
    frame: t1 = the unit part of h orthogonal to the axis (h = e_x, or e_y
    when |axis_x| >= 0.9), t2 = axis x t1.  FP64, rounded once."""
    a = np.asarray(axis, np.float32).astype(np.float64)
    a = a / math.sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2])
    h = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = h - (h[0] * a[0] + h[1] * a[1] + h[2] * a[2]) * a
    t1 = t1 / math.sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2])
    t2 = np.array([a[1] * t1[2] - a[2] * t1[1], a[2] * t1[0] - a[0] * t1[2], a[0] * t1[1] - a[1] * t1[0]])
    out = np.empty((n, 3), np.float32)
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for i in range(n):
        F = 1.0 - (2 * i + 1) / (2.0 * n)
        z = 2.0 * F ** (1.0 / (m + 1.0)) - 1.0
        phi = math.fmod(i * golden, 2.0 * math.pi)
        rho = math.sqrt(max(0.0, 1.0 - z * z))
        x, y = rho * math.cos(phi), rho * math.sin(phi)
        out[i] = x * t1 + y * t2 + z * a
    return out


def directivity(m: float, cos_theta):
    """Energy per solid angle of the directional source relative to an
    omnidirectional one of the same power: (m+1) (1 + cos theta)^m / 2^m."""
    return (m + 1.0) * (1.0 + np.asarray(cos_theta, np.float64)) ** m / 2.0 ** m


def fibonacci(n: int) -> np.ndarray:
    """[n, 3] FP32 Fibonacci-sphere directions (FP64 formula, rounded once)."""
    out = np.empty((n, 3), np.float32)
    lib().or_fibonacci(n, _p(out))
    return out


def query_batch(sc: OracleScene, o, u, last_plane=None, L=None, rcv=None, max_len: float = 0.0,
                eps: float = DEFAULT_EPS, flags: bool = True, threads: int = 0) -> Dict[str, np.ndarray]:
    """Independent queries from given FP32 states: nearest hit, hit distance,
    receiver bit mask, next state (o', u', L') and flags."""
    o = np.ascontiguousarray(o, np.float32)
    u = np.ascontiguousarray(u, np.float32)
    n = len(o)
    lp = None if last_plane is None else np.ascontiguousarray(last_plane, np.int32)
    Lf = None if L is None else np.ascontiguousarray(L, np.float32)
    rcv = np.zeros((0, 4), np.float32) if rcv is None else np.ascontiguousarray(rcv, np.float32)
    hit = np.empty(n, np.int32)
    delta = np.empty(n)
    det = np.empty(n, np.uint32)
    nxt = np.empty((n, 7))
    fl = np.empty(n, np.uint32)
    tests = lib().or_query_batch(sc._h, _p(o), _p(u), _p(lp), _p(Lf), n, _p(rcv), len(rcv),
                                 float(max_len), float(eps), int(flags), threads or default_threads(),
                                 _p(hit), _p(delta), _p(det), _p(nxt), _p(fl))
    assert tests >= 0
    return dict(hit=hit, delta=delta, det=det, next=nxt, flags=fl, tests=tests)


def trace(sc: OracleScene, src, dirs, rcv, max_reflections: int, max_len: float = 0.0,
          eps: float = DEFAULT_EPS, flags: bool = True, states: bool = False,
          threads: int = 0) -> Dict[str, np.ndarray]:
    """FP64 trajectories of rays from a point source (one per direction).

    hit_seq[i, k] = triangle that ends segment k of ray i (-1 after the ray
    ended or when segment k escaped); det[i, k] = receivers crossed by
    segment k (bit mask); flags[i, k] = query flags; states[i, k] = FP64
    input state (o, u, L, last plane) of segment k."""
    src = np.ascontiguousarray(src, np.float32)
    dirs = np.ascontiguousarray(dirs, np.float32)
    rcv = np.ascontiguousarray(rcv, np.float32).reshape(-1, 4)
    n, R1 = len(dirs), max_reflections + 1
    hs = np.empty((n, R1), np.int32)
    det = np.empty((n, R1), np.uint32)
    fl = np.empty((n, R1), np.uint32)
    st = np.empty((n, R1 + 1, 8)) if states else None
    tests = lib().or_trace(sc._h, _p(src), _p(dirs), n, _p(rcv), len(rcv), max_reflections,
                           float(max_len), float(eps), int(flags), threads or default_threads(),
                           _p(hs), _p(det), _p(fl), _p(st))
    assert tests >= 0
    return dict(hit_seq=hs, det=det, flags=fl, states=st, tests=tests)


def trace_from(sc: OracleScene, start, rcv, max_reflections: int, max_len: float = 0.0,
               eps: float = DEFAULT_EPS, flags: bool = True, states: bool = False,
               threads: int = 0) -> Dict[str, np.ndarray]:
    """The propagation of ``trace`` continued from per-ray FP64 states
    start [N, 8] = (o, u, L, last plane), such as ``trace(states=True)``'s row
    after a reflection: segment 0 here is the ray's next segment (section
    "Standard algorithm": the iteration only carries the ray's position,
    direction and travelled length from one reflection to the next)."""
    start = np.ascontiguousarray(start, np.float64).reshape(-1, 8)
    rcv = np.ascontiguousarray(rcv, np.float32).reshape(-1, 4)
    n, R1 = len(start), max_reflections + 1
    hs = np.empty((n, R1), np.int32)
    det = np.empty((n, R1), np.uint32)
    fl = np.empty((n, R1), np.uint32)
    st = np.empty((n, R1 + 1, 8)) if states else None
    tests = lib().or_trace_from(sc._h, _p(start), n, _p(rcv), len(rcv), max_reflections, float(max_len),
                                float(eps), int(flags), threads or default_threads(), _p(hs), _p(det), _p(fl),
                                _p(st))
    assert tests >= 0
    return dict(hit_seq=hs, det=det, flags=fl, states=st, tests=tests)


def detections_from_bits(det_bits: np.ndarray) -> np.ndarray:
    """Bit masks [N, R+1] -> sorted (ray, k, receiver) int32 rows."""
    rows = []
    for m in range(32):
        r, k = np.nonzero((det_bits >> np.uint32(m)) & np.uint32(1))
        if len(r):
            rows.append(np.stack([r, k, np.full(len(r), m)], axis=1))
    if not rows:
        return np.zeros((0, 3), np.int32)
    d = np.concatenate(rows).astype(np.int32)
    return d[np.lexsort((d[:, 2], d[:, 1], d[:, 0]))]


# ----------------------------------------------------------------------------
# image sources and impulse response
# ----------------------------------------------------------------------------

def image_source_keys(plane_id, hit_seq, det) -> Dict[tuple, int]:
    """Group detections by key (receiver, k, plane ids of hits 1..k) -> count n."""
    out: Dict[tuple, int] = {}
    for ray, k, r in np.asarray(det):
        seq = tuple(int(plane_id[t]) for t in hit_seq[ray, :k])
        assert len(seq) == k and all(t >= 0 for t in hit_seq[ray, :k])
        key = (int(r), int(k)) + seq
        out[key] = out.get(key, 0) + 1
    return out


def image_sources(sc: OracleScene, src, rcv, keys: Dict[tuple, int]):
    """Canonical image-source table sorted by (receiver, k, plane sequence).

    Returns dict(keys=list of tuples, count int64 [n], pos f64 [n,3],
    dist f64 [n]); pos = source mirrored through the key's planes in order,
    dist = distance from the image source to the receiver centre."""
    ks = sorted(keys.keys())
    counts = np.array([keys[k] for k in ks], np.int64)
    flat = np.array([p for k in ks for p in k[2:]], np.int32)
    offs = np.zeros(len(ks) + 1, np.int64)
    offs[1:] = np.cumsum([len(k) - 2 for k in ks])
    pos = np.empty((len(ks), 3))
    src = np.ascontiguousarray(src, np.float32)
    if len(ks):
        lib().or_image_positions(sc._h, _p(src), _p(flat if len(flat) else np.zeros(1, np.int32)),
                                 _p(offs), len(ks), _p(pos))
    rcv = np.asarray(rcv, np.float64).reshape(-1, 4)
    r_idx = np.array([k[0] for k in ks], np.int64)
    dist = np.linalg.norm(pos - rcv[r_idx, :3], axis=1) if len(ks) else np.zeros(0)
    return dict(keys=ks, count=counts, pos=pos, dist=dist)


def key_materials(keys, material_of_plane) -> list:
    return [[int(material_of_plane[p]) for p in k[2:]] for k in keys]


def is_energy(table, n_rays: int, alpha, beta, material_of_plane) -> np.ndarray:
    """[n_is, 8] E_s(b) = n/N exp(-beta_b d_s) prod_j (1 - alpha[mat_j, b]) in FP64."""
    alpha = np.asarray(alpha, np.float64)
    beta = np.asarray(beta, np.float64)
    n = len(table["keys"])
    E = np.empty((n, 8))
    for i, k in enumerate(table["keys"]):
        prod = np.ones(8)
        for p in k[2:]:
            prod = prod * (1.0 - alpha[material_of_plane[p]])
        E[i] = table["count"][i] / n_rays * np.exp(-beta * table["dist"][i]) * prod
    return E


def arrival_bins(dist, c: float, fs: float) -> np.ndarray:
    """s = floor(d_s * fs / c) in FP64 (histogram bin of [s/fs, (s+1)/fs))."""
    return np.floor(np.asarray(dist, np.float64) * np.float64(fs) / np.float64(c)).astype(np.int64)


def fir_same(x: np.ndarray, taps: np.ndarray, threads: int = 0) -> np.ndarray:
    """x [..., 8, L] FP64 -> 'same'-mode FIR of each band with its own taps."""
    x = np.ascontiguousarray(x, np.float64)
    taps = np.ascontiguousarray(taps, np.float64)
    L = x.shape[-1]
    K = taps.shape[1]
    y = np.empty_like(x)
    nsig = x.size // L
    lib().or_fir_same(_p(x), nsig, L, _p(taps), K, _p(y), threads or default_threads())
    return y


def assemble_ir(table, n_rays: int, n_rcv: int, alpha, beta, material_of_plane, c: float,
                fs: float, L: int, taps) -> Dict[str, np.ndarray]:
    """Histogram H[r, b, s] of image-source energies by arrival bin, pressure
    p = sqrt(H), band IRs = FIR_b * p_b ('same'), IR = sum over bands, band
    energy = sum_s H.  All FP64."""
    E = is_energy(table, n_rays, alpha, beta, material_of_plane)
    s = arrival_bins(table["dist"], c, fs)
    r = np.array([k[0] for k in table["keys"]], np.int64)
    keep = (s >= 0) & (s < L)
    H = np.zeros((n_rcv, 8, L))
    for b in range(8):
        np.add.at(H[:, b, :], (r[keep], s[keep]), E[keep, b])
    p = np.sqrt(H)
    band_ir = fir_same(p, np.asarray(taps, np.float64))
    return dict(hist=H, band_ir=band_ir, ir=band_ir.sum(axis=1), band_energy=H.sum(axis=2),
                energy=E, bins=s)


def band_energy_grad(table, n_rays: int, n_rcv: int, n_mat: int, alpha, beta, material_of_plane,
                     c: float, fs: float, L: int, grad_band_energy) -> np.ndarray:
    """d(sum_{r,b} g[r,b] * band_energy[r,b]) / d alpha[m, b], FP64.

    For one image source with c_m reflections on material m,
    dE_s(b)/dalpha[m,b] = -n/N e^{-beta d} c_m (1-alpha[m,b])^(c_m - 1)
    prod_{m' != m} (1-alpha[m',b])^(c_m'); other bands do not depend on
    alpha[m, b].  Only sources whose arrival bin falls inside the IR count."""
    alpha = np.asarray(alpha, np.float64)
    beta = np.asarray(beta, np.float64)
    g = np.asarray(grad_band_energy, np.float64)
    out = np.zeros((n_mat, 8))
    s = arrival_bins(table["dist"], c, fs)
    for i, k in enumerate(table["keys"]):
        if not (0 <= s[i] < L):
            continue
        cnt: Dict[int, int] = {}
        for p in k[2:]:
            m = int(material_of_plane[p])
            cnt[m] = cnt.get(m, 0) + 1
        base = table["count"][i] / n_rays * np.exp(-beta * table["dist"][i])
        for m, cm in cnt.items():
            d = -cm * (1.0 - alpha[m]) ** (cm - 1)
            for m2, c2 in cnt.items():
                if m2 != m:
                    d = d * (1.0 - alpha[m2]) ** c2
            out[m] += g[k[0]] * base * d
    return out
