"""Small helpers shared by the tests (no method arithmetic)."""
import numpy as np


def ulp_diff(a, b):
    """Distance in FP32 units in the last place (same-sign finite values)."""
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, np.int64(-2 ** 31) - ia, ia)
    ib = np.where(ib < 0, np.int64(-2 ** 31) - ib, ib)
    return np.abs(ia - ib)


def material_of_plane(scene):
    m = np.full(scene.n_tri, -1, np.int64)
    for t in range(scene.n_tri - 1, -1, -1):
        m[scene.plane_id[t]] = scene.material[t]
    return m


def gpu_is_dict(isrc):
    key, cnt, pos, dist = [t.cpu().numpy() for t in isrc.valid()]
    out = {}
    for row, c, p, d in zip(key, cnt, pos, dist):
        k = tuple(int(v) for v in row[: 2 + row[1]])
        assert k not in out, "duplicate image-source row"
        out[k] = (int(c), p, float(d))
    return out


def synthetic_is_table(scene, n_is, max_reflections, n_rcv, seed, L, c, fs, n_rays):
    """Seeded image-source table: keys (receiver, k, plane ids of existing
    planes), counts, distances spread over the IR (with some beyond it)."""
    rng = np.random.default_rng(seed)
    planes = np.unique(scene.plane_id)
    keys, counts, dists = [], [], []
    tmax = L / fs
    for _ in range(n_is):
        r = int(rng.integers(0, n_rcv))
        k = int(rng.integers(0, max_reflections + 1))
        seq = tuple(int(p) for p in rng.choice(planes, size=k))
        keys.append((r, k) + seq)
        counts.append(int(rng.integers(1, 50)))
        dists.append(float(rng.uniform(0.0, max(1.05 * c * tmax, 1e-3))))
    # merge duplicates (keys must be unique)
    d = {}
    for k, n, x in zip(keys, counts, dists):
        if k not in d:
            d[k] = (n, x)
    ks = list(d.keys())
    tab = dict(keys=ks, count=np.array([d[k][0] for k in ks], np.int64), dist=np.array([d[k][1] for k in ks]))
    R2 = max_reflections + 2
    arr = -np.ones((len(ks), R2), np.int32)
    for i, k in enumerate(ks):
        arr[i, : len(k)] = k
    return tab, arr


def crossing_and_miss(o, u, v0, v1, v2):
    """FP64 plane crossing of rays o + t u with triangles (v0, v1, v2), row by
    row: t of the crossing (inf when u is parallel to the plane) and the
    distance from the crossing point to the closed triangle (0 inside).
    Plain geometry for checking a flagged query's GPU answer; no arithmetic
    of the method."""
    o, u, v0, v1, v2 = [np.asarray(a, np.float64).reshape(-1, 3) for a in (o, u, v0, v1, v2)]
    e1, e2 = v1 - v0, v2 - v0
    n = np.cross(e1, e2)
    den = np.einsum("ij,ij->i", u, n)
    num = np.einsum("ij,ij->i", v0 - o, n)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(den != 0.0, num / den, np.inf)
    p = o + np.where(np.isfinite(t), t, 0.0)[:, None] * u
    miss = np.zeros(len(o))
    for i in range(len(o)):
        if not np.isfinite(t[i]):
            miss[i] = np.inf
            continue
        miss[i] = _point_triangle_distance(p[i], v0[i], v1[i], v2[i])
    return t, miss


def _point_triangle_distance(p, a, b, c):
    """Distance from p (in the triangle's plane) to the closed triangle abc:
    0 when the barycentric coordinates are all >= 0, else the distance to the
    nearest of the three edge segments."""
    m = np.array([b - a, c - a]).T
    lam, mu = np.linalg.lstsq(m, p - a, rcond=None)[0]
    if lam >= 0 and mu >= 0 and lam + mu <= 1:
        return 0.0
    best = np.inf
    for s0, s1 in ((a, b), (b, c), (c, a)):
        d = s1 - s0
        w = np.clip(np.dot(p - s0, d) / np.dot(d, d), 0.0, 1.0)
        best = min(best, float(np.linalg.norm(p - (s0 + w * d))))
    return best


def _segment_distance(p, a, b):
    """Row-wise distance from points p to segments ab (arrays [n, 3])."""
    d = b - a
    den = np.einsum("ij,ij->i", d, d)
    w = np.clip(np.einsum("ij,ij->i", p - a, d) / np.where(den > 0, den, 1.0), 0.0, 1.0)
    return np.linalg.norm(p - (a + w[:, None] * d), axis=1)


def skips_only_at_boundaries(o, u, t_hit, vtx, tri, eps):
    """Whether the ray o + t u, answered by a hit at parameter t_hit (inf for
    an escape), passes every triangle it crosses before t_hit - eps / |u|
    within eps of that triangle's boundary: the answer then skipped only edge
    or vertex seams, a decision within rounding; a triangle crossed well
    inside before t_hit makes the answer wrong.  FP64 plain geometry over the
    whole mesh (plane crossing, barycentric inside test, distance to the three
    edge segments); no arithmetic of the method."""
    o = np.asarray(o, np.float64)
    u = np.asarray(u, np.float64)
    v0, v1, v2 = (np.asarray(vtx, np.float64)[np.asarray(tri)[:, k]] for k in range(3))
    e1, e2 = v1 - v0, v2 - v0
    n = np.cross(e1, e2)
    den = n @ u
    ok = den != 0.0
    t = np.full(len(n), np.inf)
    t[ok] = np.einsum("ij,ij->i", v0[ok] - o, n[ok]) / den[ok]
    lim = t_hit - eps / np.linalg.norm(u)
    cand = np.nonzero(ok & (t > 0) & (t < lim))[0]
    if len(cand) == 0:
        return True
    p = o + t[cand, None] * u
    # barycentric coordinates in the triangle's plane
    a, b, c = v0[cand], v1[cand], v2[cand]
    f1, f2, w = b - a, c - a, p - a
    d11, d12, d22 = (np.einsum("ij,ij->i", x, y) for x, y in ((f1, f1), (f1, f2), (f2, f2)))
    w1, w2 = np.einsum("ij,ij->i", w, f1), np.einsum("ij,ij->i", w, f2)
    det = d11 * d22 - d12 * d12
    lam = (d22 * w1 - d12 * w2) / det
    mu = (d11 * w2 - d12 * w1) / det
    inside = (lam >= 0) & (mu >= 0) & (lam + mu <= 1)
    if not inside.any():
        return True
    pi, ai, bi, ci = p[inside], a[inside], b[inside], c[inside]
    edge = np.minimum(np.minimum(_segment_distance(pi, ai, bi), _segment_distance(pi, bi, ci)),
                      _segment_distance(pi, ci, ai))
    return bool(np.all(edge <= eps))
