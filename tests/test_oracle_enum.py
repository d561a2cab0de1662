"""Exhaustive image-source enumeration on tiny rooms (brute force, FP64).

Every reflection sequence up to order K is mirrored (section "Image-sources":
the source seen through the reflecting planes) and back-traced from the
receiver: the line from the image toward the receiver must cross each
reflecting plane inside that plane's polygon, in reverse order, with nothing
in between.  Sequences that stay valid for a bundle of points spread over the
receiver sphere (robustly visible) and whose solid-angle share is at least 5
rays must be found by the oracle's ray tracing, with the expected count; and
every sequence the oracle finds must back-trace close to valid.
"""
import itertools

import numpy as np
import pytest

import synth


def _groups(vtx, tri, plane):
    v = vtx.astype(np.float64)
    out = {}
    for t, p in enumerate(plane):
        out.setdefault(int(p), []).append(t)
    info = {}
    for p, ts in out.items():
        a, b, c = v[tri[ts[0]]]
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        # boundary edges of the coplanar group: used by exactly one member triangle
        cnt = {}
        for t in ts:
            for e in ((tri[t][0], tri[t][1]), (tri[t][1], tri[t][2]), (tri[t][2], tri[t][0])):
                k = tuple(sorted(e))
                cnt[k] = cnt.get(k, 0) + 1
        bnd = [(v[a_], v[b_]) for (a_, b_), c_ in cnt.items() if c_ == 1]
        info[p] = dict(n=n, p0=a, tris=[v[tri[t]] for t in ts], bnd=bnd)
    return info


def _mirror(x, g):
    return x - 2 * np.dot(x - g["p0"], g["n"]) * g["n"]


def _in_group(q, g, margin):
    """q in the group's polygon, at least `margin` from its boundary (margin may be < 0)."""
    inside = False
    for a, b, c in g["tris"]:
        e1, e2, w = b - a, c - a, q - a
        d00, d01, d11 = e1 @ e1, e1 @ e2, e2 @ e2
        d20, d21 = w @ e1, w @ e2
        den = d00 * d11 - d01 * d01
        l1 = (d11 * d20 - d01 * d21) / den
        l2 = (d00 * d21 - d01 * d20) / den
        if l1 >= -1e-12 and l2 >= -1e-12 and l1 + l2 <= 1 + 1e-12:
            inside = True
            break
    dmin = min(_seg_dist(q, a, b) for a, b in g["bnd"])
    if margin >= 0:
        return inside and dmin >= margin
    return inside or dmin <= -margin


def _seg_dist(p, a, b):
    ab = b - a
    s = np.clip((p - a) @ ab / (ab @ ab), 0, 1)
    return np.linalg.norm(a + s * ab - p)


def _blocked(a, b, vtx, tri, skip_planes, plane):
    v = vtx.astype(np.float64)
    d = b - a
    for t in range(len(tri)):
        if plane[t] in skip_planes:
            continue
        p0, p1, p2 = v[tri[t]]
        e1, e2 = p1 - p0, p2 - p0
        pv = np.cross(d, e2)
        det = e1 @ pv
        if abs(det) < 1e-14:
            continue
        tv = a - p0
        lam = tv @ pv / det
        qv = np.cross(tv, e1)
        mu = d @ qv / det
        s = e2 @ qv / det
        if lam >= 0 and mu >= 0 and lam + mu <= 1 and 1e-9 < s < 1 - 1e-9:
            return True
    return False


def back_trace(seq, src, P, G, vtx, tri, plane, margin):
    X = [np.asarray(src, np.float64)]
    for p in seq:
        X.append(_mirror(X[-1], G[p]))
    target = np.asarray(P, np.float64)
    nxt_plane = None
    for j in range(len(seq), 0, -1):
        g = G[seq[j - 1]]
        a, b = X[j], target
        den = (b - a) @ g["n"]
        if abs(den) < 1e-14:
            return False, X[-1]
        s = (g["p0"] - a) @ g["n"] / den
        if not (0 < s < 1):
            return False, X[-1]
        q = a + s * (b - a)
        if not _in_group(q, g, margin):
            return False, X[-1]
        if _blocked(q, target, vtx, tri, {seq[j - 1], nxt_plane}, plane):
            return False, X[-1]
        target, nxt_plane = q, seq[j - 1]
    if _blocked(np.asarray(src, np.float64), target, vtx, tri, {nxt_plane}, plane):
        return False, X[-1]
    return True, X[-1]


ROOMS = {
    "tetra": lambda: synth.tetra_room(4.0) + (np.array([1.2, 0.9, 0.7], np.float32),
                                             np.array([[2.6, 1.3, 0.9, 0.25]], np.float32)),
    "box": lambda: synth.box_mesh((5.0, 4.0, 3.0)) + (np.array([4.0, 2.0, 1.7], np.float32),
                                                     np.array([[2.0, 2.0, 1.7, 0.25]], np.float32)),
    "lroom": lambda: synth.lroom() + (np.array([1.5, 1.0, 1.4], np.float32),
                                      np.array([[1.2, 4.5, 1.5, 0.3]], np.float32)),
}


@pytest.mark.parametrize("room", sorted(ROOMS))
def test_exhaustive_image_sources(room, oracle_lib):
    vtx, tri, mat, plane, src, rcv = ROOMS[room]()
    K = 3
    N = 200_000
    sc = oracle_lib.OracleScene(vtx, tri, plane)
    dirs = oracle_lib.fibonacci(N)
    tr = oracle_lib.trace(sc, src, dirs, rcv, K, flags=False)
    det = oracle_lib.detections_from_bits(tr["det"])
    keys = oracle_lib.image_source_keys(plane, tr["hit_seq"], det)
    tab = oracle_lib.image_sources(sc, src, rcv, keys)
    G = _groups(vtx, tri, plane)
    planes = sorted(G)
    P = rcv[0, :3].astype(np.float64)
    r = float(rcv[0, 3])
    bundle = [P] + [P + r * s * e for e in np.eye(3) for s in (-1, 1)]
    found = {k[2:]: n for k, n in zip(tab["keys"], tab["count"])}
    must = 0
    for k in range(K + 1):
        for seq in itertools.product(planes, repeat=k):
            if any(seq[i] == seq[i + 1] for i in range(k - 1)):
                continue
            ok_all = True
            for pt in bundle:
                ok, X = back_trace(seq, src, pt, G, vtx, tri, plane, margin=0.2)
                ok_all &= ok
                if not ok_all:
                    break
            if not ok_all:
                continue
            d = np.linalg.norm(X - P)
            e = N * (1 - np.sqrt(1 - r * r / (d * d))) / 2
            if e < 5:
                continue
            must += 1
            n = found.get(tuple(seq), 0)
            assert abs(n - e) <= 3 * np.sqrt(e) + 2, (room, seq, n, e)
    assert must >= 4
    # soundness: each found sequence back-traces close to valid from the receiver
    for key, n, pos in zip(tab["keys"], tab["count"], tab["pos"]):
        seq = key[2:]
        ok, X = back_trace(seq, src, P, G, vtx, tri, plane, margin=-2 * r)
        assert np.allclose(X, pos, atol=1e-12)
        if n >= 3:
            assert ok or any(back_trace(seq, src, pt, G, vtx, tri, plane, margin=-2 * r)[0]
                             for pt in bundle[1:]), (room, seq, n)
