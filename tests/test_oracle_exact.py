"""Pins of the oracle's per-query geometry against exact rational arithmetic.

The nearest hit is defined by the parametric conditions of the section
"Standard algorithm" (0 <= lambda, 0 <= mu, lambda + mu <= 1, delta > 0,
delta minimal); the receiver test by the sphere's cartesian equation.  Here
both are recomputed with Python ``fractions`` from the exact FP32 inputs by a
different route (Gaussian elimination of the 3x3 system instead of the
Moller-Trumbore triple products), so a dropped term, a sign or a transposed
operand in the oracle fails.  Queries the oracle flags may differ; all others
must agree exactly.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.filterwarnings("ignore")


def _solve3(a, b):
    """Exact solution of the 3x3 system a x = b (Fractions), None if singular."""
    m = [list(a[i]) + [b[i]] for i in range(3)]
    for c in range(3):
        piv = next((r for r in range(c, 3) if m[r][c] != 0), None)
        if piv is None:
            return None
        m[c], m[piv] = m[piv], m[c]
        for r in range(3):
            if r != c and m[r][c] != 0:
                f = m[r][c] / m[c][c]
                m[r] = [m[r][k] - f * m[c][k] for k in range(4)]
    return [m[i][3] / m[i][i] for i in range(3)]


def exact_query(vtx, tri, plane, o, u, last_plane, rcv):
    """Exact nearest hit (lowest index on ties), exact delta, exact detections."""
    V = [[F(float(x)) for x in row] for row in vtx]
    O = [F(float(x)) for x in o]
    U = [F(float(x)) for x in u]
    best, bd = -1, None
    for j, (a, b, c) in enumerate(tri):
        if plane[j] == last_plane:
            continue
        e1 = [V[b][k] - V[a][k] for k in range(3)]
        e2 = [V[c][k] - V[a][k] for k in range(3)]
        A = [[e1[k], e2[k], -U[k]] for k in range(3)]
        rhs = [O[k] - V[a][k] for k in range(3)]
        s = _solve3(A, rhs)
        if s is None:
            continue
        lam, mu, d = s
        if lam >= 0 and mu >= 0 and lam + mu <= 1 and d > 0 and (bd is None or d < bd):
            best, bd = j, d
    det = 0
    uu = sum(x * x for x in U)
    for m, (x, y, z, r) in enumerate(rcv):
        W = [F(float(x)) - O[0], F(float(y)) - O[1], F(float(z)) - O[2]]
        ts = sum(W[k] * U[k] for k in range(3)) / uu
        ts = max(ts, F(0))
        if bd is not None:
            ts = min(ts, bd)
        q = [O[k] + ts * U[k] - (W[k] + O[k]) for k in range(3)]
        if sum(x * x for x in q) <= F(float(r)) ** 2:
            det |= 1 << m
    return best, bd, det


def _compare(oracle_lib, vtx, tri, plane, o, u, lp, rcv):
    sc = oracle_lib.OracleScene(vtx, tri, plane)
    res = oracle_lib.query_batch(sc, o, u, lp, None, rcv, flags=True)
    mism_unflagged = 0
    flagged = 0
    for i in range(len(o)):
        b, d, det = exact_query(vtx, tri, plane, o[i], u[i], lp[i], rcv)
        fl = int(res["flags"][i])
        flagged += fl != 0
        ok_hit = res["hit"][i] == b
        ok_det = res["det"][i] == det
        if ok_hit and b >= 0:
            ok_hit = abs(res["delta"][i] - float(d)) <= 1e-12 * (1 + float(d))
        if not (ok_hit and ok_det):
            if fl == 0:
                mism_unflagged += 1
    return mism_unflagged, flagged, res


def test_single_triangle_random_rays(oracle_lib):
    rng = np.random.default_rng(7)
    vtx = np.array([[0, 0, 0], [2, 0.1, 0], [0.3, 1.7, 0.2]], np.float32)
    tri = np.array([[0, 1, 2]], np.int32)
    n = 400
    o = np.concatenate([rng.uniform(-1, 3, (n, 2)), rng.uniform(0.5, 2, (n, 1))], 1).astype(np.float32)
    tgt = np.concatenate([rng.uniform(-0.5, 2.5, (n, 2)), np.zeros((n, 1))], 1)
    u = (tgt - o).astype(np.float32)
    rcv = np.array([[0.5, 0.5, 0.5, 0.4], [0.5, 0.5, -1.0, 0.6]], np.float32)   # 2nd behind
    bad, flagged, res = _compare(oracle_lib, vtx, tri, np.zeros(1, np.int32), o, u,
                                 np.full(n, -1, np.int32), rcv)
    assert bad == 0
    assert (res["hit"] == 0).sum() > 50 and (res["hit"] == -1).sum() > 50
    assert flagged < n // 20


def test_shared_edge_and_fan_exact_ties(oracle_lib):
    # two triangles sharing the edge (1,0,0)-(0,1,0), and a 6-triangle fan at (3,3,0)
    vtx = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]]
    tri = [[0, 1, 2], [1, 3, 2]]
    c = len(vtx)
    vtx.append([3, 3, 0])
    for k in range(6):
        a = 2 * np.pi * k / 6
        vtx.append([3 + np.cos(a), 3 + np.sin(a), 0])
    for k in range(6):
        tri.append([c, c + 1 + k, c + 1 + (k + 1) % 6])
    vtx = np.array(vtx, np.float32)
    tri = np.array(tri, np.int32)
    plane = np.arange(len(tri), dtype=np.int32)
    o = np.array([[0.5, 0.5, 1.0], [0.25, 0.75, 2.0], [3, 3, 1], [3.5, 3.0, 1.0], [0.5, 0.5, -1.0],
                  [0.2, 0.2, 1.0], [0.9, 0.9, 1.0]], np.float32)
    u = np.array([[0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, -1], [0, 0, 1], [0, 0, -1], [0, 0, -1]],
                 np.float32)
    bad, flagged, res = _compare(oracle_lib, vtx, tri, plane, o, u, np.full(len(o), -1, np.int32),
                                 np.zeros((0, 4), np.float32))
    assert bad == 0
    # exact ties on the shared edge / the fan centre go to the lowest index
    assert res["hit"][0] == 0 and res["hit"][2] == 2
    assert res["flags"][0] & oracle_lib.FLAG_EDGE and res["flags"][0] & oracle_lib.FLAG_TIE
    assert res["hit"][5] == 0 and res["hit"][6] == 1 and res["flags"][5] == 0 and res["flags"][6] == 0


def test_random_soup_with_plane_exclusion(oracle_lib):
    rng = np.random.default_rng(11)
    nt = 12
    vtx = rng.uniform(-2, 2, (3 * nt, 3)).astype(np.float32)
    tri = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
    plane = np.arange(nt, dtype=np.int32)
    plane[5] = 4            # share a plane id (exclusion is by id)
    n = 300
    o = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    u = synth.random_unit_dirs(rng, n)
    lp = rng.integers(-1, nt, size=n).astype(np.int32)
    rcv = np.array([[0, 0, 0, 0.5], [1.5, -1, 0.5, 0.3], [-3, 0, 0, 1.0]], np.float32)
    bad, flagged, res = _compare(oracle_lib, vtx, tri, plane, o, u, lp, rcv)
    assert bad == 0
    assert flagged < n // 10
    hits = res["hit"]
    assert np.all((hits < 0) | (plane[np.maximum(hits, 0)] != lp))


def test_reflection_invariants(oracle_lib):
    s = synth.tessellated_box_c2(jitter=True)
    sc = oracle_lib.OracleScene.of(s)
    o, u, lp, L = synth.surface_query_states(s, 200, seed=3, toward=(5.0, 3.5, 1.5))
    res = oracle_lib.query_batch(sc, o, u, lp, L, s.rcv)
    ok = res["hit"] >= 0
    # closed room; the 1 cm jitter can fold a few triangles over, so a ray that
    # leaves such a face on its "inner" side may exit through the fold
    assert ok.mean() > 0.97
    o, u, lp, L = o[ok], u[ok], lp[ok], L[ok]
    res = {k: (v[ok] if isinstance(v, np.ndarray) else v) for k, v in res.items()}
    nn, _ = sc.planes()
    n = nn[s.plane_id[res["hit"]]]
    u64 = u.astype(np.float64)
    un = res["next"][:, 3:6]
    # |u'| = |u| and u'.n = -u.n (specular law)
    assert np.allclose(np.linalg.norm(un, axis=1), np.linalg.norm(u64, axis=1), rtol=1e-14)
    assert np.allclose((un * n).sum(1), -(u64 * n).sum(1), atol=1e-14)
    # tangential part unchanged: u' - u is along n
    du = un - u64
    assert np.allclose(np.cross(du, n), 0, atol=1e-14)
    # next origin is the hit point on the hit triangle's plane; L grows by |delta u|
    v0 = s.vtx.astype(np.float64)[s.tri[res["hit"], 0]]
    assert np.allclose(((res["next"][:, :3] - v0) * n).sum(1), 0, atol=1e-12)
    step = np.linalg.norm(res["next"][:, :3] - o.astype(np.float64), axis=1)
    assert np.allclose(res["next"][:, 6], L.astype(np.float64) + step, rtol=1e-12)


def test_fibonacci_properties(oracle_lib):
    for n in (1, 2, 7, 1000, 100_000):
        d = oracle_lib.fibonacci(n).astype(np.float64)
        i = np.arange(n)
        # z spacing is the closed form 1 - (2i+1)/N (equal-area bands)
        assert np.allclose(d[:, 2], 1 - (2 * i + 1) / n, atol=6e-8)
        assert np.allclose(np.linalg.norm(d, axis=1), 1, atol=2e-7)
        if n >= 7:
            phi = np.arctan2(d[:, 1], d[:, 0])
            step = np.mod(np.diff(phi), 2 * np.pi)
            golden = np.pi * (3 - np.sqrt(5))
            rho = np.hypot(d[:-1, 0], d[:-1, 1])
            good = rho > 1e-3
            assert np.allclose(step[good], golden, atol=1e-4)
    # uniformity: the fraction of directions in a random cap ~ its area fraction
    d = oracle_lib.fibonacci(100_000).astype(np.float64)
    rng = np.random.default_rng(0)
    for axis in synth.random_unit_dirs(rng, 20).astype(np.float64):
        cosang = rng.uniform(-0.9, 0.9)
        frac = (d @ axis >= cosang).mean()
        assert abs(frac - (1 - cosang) / 2) < 2e-3


def test_fir_same_against_numpy_convolve(oracle_lib):
    rng = np.random.default_rng(1)
    x = rng.random((2, 8, 300))
    taps = rng.standard_normal((8, 41))
    y = oracle_lib.fir_same(x, taps)
    for r in range(2):
        for b in range(8):
            full = np.convolve(x[r, b], taps[b])
            assert np.allclose(y[r, b], full[20:20 + 300], rtol=1e-12, atol=1e-12)
    # identity filter returns the input
    assert np.array_equal(oracle_lib.fir_same(x, synth.delta_taps(5).astype(np.float64)), x)
