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
