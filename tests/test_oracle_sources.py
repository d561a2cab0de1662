"""Pins of the source-variant oracles (section "Discrete model": uniform
unit-sphere sampling by icosahedron subdivision; the footnote's directional
source sampled non-uniformly).

* Icosahedral grid: frequency 1 is the icosahedron (5 neighbours at
  arccos(1/sqrt5)); frequency 2 is the set of the recursive midpoint
  icosphere of level 1 (built independently in ``synth``); every frequency
  gives 10 f^2 + 2 distinct unit points, symmetric under u -> -u, and a
  spherical 5-design (a union of orbits of the icosahedral rotation group,
  which has no invariant harmonics of degree 1-5): sum u = 0,
  sum u u^T = N/3 I and sum (u.a)^4 = N/5 for every unit a; the documented
  order puts edge points on their edge's great circle.
* Directional source: m = 0 about e_z is the Fibonacci set (the C oracle's);
  the distribution of cos theta follows ((1 + z)/2)^(m+1) to within 1/N; the
  azimuth is balanced; free-field ray counts at receivers around the source
  follow N D(theta) Omega_m / (4 pi) with D = (m+1)(1 + cos theta)^m / 2^m.
"""
import math

import numpy as np
import pytest

import synth


def test_icosahedral_frequency_one_is_the_icosahedron(oracle_lib):
    d = oracle_lib.icosahedral(1).astype(np.float64)
    assert d.shape == (12, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-7)
    c = d @ d.T
    for i in range(12):
        near = np.sort(np.arccos(np.clip(c[i], -1, 1)))[1:6]
        assert np.allclose(near, math.acos(1 / math.sqrt(5)), atol=1e-6)


def test_icosahedral_frequency_two_is_the_midpoint_icosphere(oracle_lib):
    d = oracle_lib.icosahedral(2).astype(np.float64)
    v, _ = synth.icosphere(1)
    v = v.astype(np.float64)
    assert len(d) == len(v) == 42
    dist = np.linalg.norm(d[:, None, :] - v[None, :, :], axis=2)
    assert dist.min(axis=1).max() < 1e-6 and dist.min(axis=0).max() < 1e-6


@pytest.mark.parametrize("f", [1, 2, 3, 5, 8, 13])
def test_icosahedral_grid_is_a_five_design(oracle_lib, f):
    d = oracle_lib.icosahedral(f).astype(np.float64)
    N = 10 * f * f + 2
    assert d.shape == (N, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-7)
    # distinct, and closed under u -> -u
    key = np.round(d * 1e5).astype(np.int64)
    assert len({tuple(k) for k in key}) == N
    far = np.linalg.norm(d[:, None, :] + d[None, :, :], axis=2).min(axis=1)
    assert far.max() < 1e-6
    tol = 1e-6 * N
    assert np.abs(d.sum(axis=0)).max() < tol
    assert np.abs(d.T @ d - N / 3 * np.eye(3)).max() < tol
    rng = np.random.default_rng(f)
    for a in synth.random_unit_dirs(rng, 5).astype(np.float64):
        a /= np.linalg.norm(a)
        assert abs(((d @ a) ** 4).sum() - N / 5) < 4 * tol
        assert abs(((d @ a) ** 3).sum()) < 4 * tol
    # the documented order: vertices, then edge points on their edge's great circle
    v = oracle_lib.icosahedron_vertices()
    vn = v / np.linalg.norm(v, axis=1, keepdims=True)
    assert np.allclose(d[:12], vn, atol=1e-7)
    edges = [(p, q) for p in range(12) for q in range(p + 1, 12) if ((v[p] - v[q]) ** 2).sum() < 4.5]
    assert len(edges) == 30
    for e, (p, q) in enumerate(edges):
        seg = d[12 + e * (f - 1): 12 + (e + 1) * (f - 1)]
        if len(seg):
            nrm = np.cross(vn[p], vn[q])
            assert np.abs(seg @ nrm).max() < 1e-6
            # from p towards q: the angle to p grows
            assert np.all(np.diff(seg @ vn[p]) < 0)


def test_directional_m0_is_fibonacci(oracle_lib):
    n = 5000
    a = oracle_lib.directional(n, 0.0, [0.0, 0.0, 1.0])
    b = oracle_lib.fibonacci(n)
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    assert np.abs(ia - ib).max() <= 2 or np.abs(a - b).max() < 1e-7


@pytest.mark.parametrize("m,axis", [(1.0, [0, 0, 1]), (2.0, [1, 2, -0.5]), (7.5, [0.95, 0.1, 0.0]),
                                    (0.5, [-1, 0, 0])])
def test_directional_density_follows_the_pattern(oracle_lib, m, axis):
    n = 20_000
    d = oracle_lib.directional(n, m, axis).astype(np.float64)
    a = np.asarray(axis, np.float32).astype(np.float64)
    a /= np.linalg.norm(a)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    z = np.sort(d @ a)
    cdf_emp = (np.arange(n) + 0.5) / n
    cdf = ((1 + z) / 2) ** (m + 1)
    assert np.abs(cdf - cdf_emp).max() < 1.0 / n + 1e-6
    # azimuth balanced about the axis
    perp = d - np.outer(d @ a, a)
    assert np.linalg.norm(perp.sum(axis=0)) < 0.02 * n ** 0.5 + 1e-3 * n
    # mean direction: E[cos theta] = (m + 1) / (m + 2) * 2 - 1 for F(z) = ((1+z)/2)^(m+1)
    assert abs((d @ a).mean() - (2 * (m + 1) / (m + 2) - 1)) < 2.0 / n


def test_directional_free_field_counts(oracle_lib):
    """n/N at a receiver of radius r at distance d and angle theta from the
    axis: D(theta) Omega_m / (4 pi) with the exact solid angle."""
    s = synth.open_scene_far_triangle()
    sc = oracle_lib.OracleScene.of(s)
    N, m, r, dist = 400_000, 2.0, 0.3, 10.0
    axis = np.array([0.6, 0.0, -0.8])
    th = np.radians([0.0, 30.0, 60.0, 90.0, 135.0])
    t1 = np.array([0.8, 0.0, 0.6])                      # unit, orthogonal to the axis
    cen = dist * (np.cos(th)[:, None] * axis + np.sin(th)[:, None] * t1)
    rcv = np.concatenate([cen, np.full((len(th), 1), r)], 1).astype(np.float32)
    dirs = oracle_lib.directional(N, m, axis)
    tr = oracle_lib.trace(sc, np.zeros(3, np.float32), dirs, rcv, 0, flags=False)
    counts = np.array([((tr["det"][:, 0] >> np.uint32(k)) & 1).sum() for k in range(len(th))])
    dd = np.linalg.norm(rcv[:, :3].astype(np.float64), axis=1)
    cos_t = (rcv[:, :3].astype(np.float64) @ axis) / dd
    expect = N * oracle_lib.directivity(m, cos_t) * (1 - np.sqrt(1 - r * r / (dd * dd))) / 2
    assert np.all(np.abs(counts - expect) <= 3 * np.sqrt(expect) + 2), (counts, expect)
    assert counts[0] > 2.5 * N * (1 - np.sqrt(1 - r * r / dist ** 2)) / 2       # on axis: Q = m + 1 = 3
