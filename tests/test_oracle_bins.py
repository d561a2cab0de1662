"""Pins of the oracle's arrival bins and air absorption (section
"Image-sources": an image source at distance d_s from the receiver arrives at
d_s / c and carries E_s(f) = n/N exp(-beta(f) d_s) prod_j (1 - alpha_j(f));
the impulse response is a histogram of those energies over time).

Every expected value here comes from geometry worked out in the test (exact
rational arithmetic where the distance is rational), not from the oracle's
own formulas:

* free field: a receiver placed at a chosen distance d on a coordinate axis
  receives its direct sound in bin floor(d fs / c), evaluated with
  ``fractions.Fraction``; distances one FP32 ulp below and above a bin edge
  land on either side of it;
* a table of distances at, just below and just above exactly representable
  bin edges (c = 256 m/s, fs = 32768 Hz: edges at s/128 m) and near the
  realistic edges s * 343 / 48000: each lands in its exact bin, the last
  kept bin is L - 1, a source at bin L is dropped;
* air absorption: with alpha = 0 the direct sound's band ratio is
  exp(-(beta_i - beta_j) d) with d from geometry; over a reflecting floor the
  first-order image source lies at the mirrored distance 5 m (a 3-4-5
  triangle), its energy per band relative to the direct sound is
  (n1 / n0) exp(-beta (5 - sqrt 17)) (1 - alpha) with n counted from the
  detections.  A dropped or doubled beta, the ray's own path length in place
  of the image-source distance, or a missing (1 - alpha) factor fails here.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth


def _floor_frac(x: Fraction) -> int:
    return x.numerator // x.denominator


def _exact_bin(d: float, c: float, fs: float) -> int:
    return _floor_frac(Fraction(d) * Fraction(fs) / Fraction(c))


def _f32_around(x: Fraction):
    """(largest FP32 below x, smallest FP32 at or above x)."""
    f = np.float32(float(x))
    while Fraction(float(f)) < x:
        f = np.nextafter(f, np.float32(np.inf))
    while Fraction(float(f)) >= x:
        f = np.nextafter(f, np.float32(-np.inf))
    lo = f
    hi = np.nextafter(lo, np.float32(np.inf))
    assert Fraction(float(lo)) < x <= Fraction(float(hi))
    return float(lo), float(hi)


def _f64_around(x: Fraction, rel: float):
    """FP64 values about rel * x below and above x (on the right sides)."""
    lo, hi = float(x) * (1 - rel), float(x) * (1 + rel)
    assert Fraction(lo) < x < Fraction(hi)
    return lo, hi


@pytest.fixture(scope="module")
def free_field(oracle_lib):
    """Source at the origin, receivers (r = 2 m) on the six half-axes at
    distances one FP32 ulp below / at-or-above three bin edges of
    c = 343 m/s, fs = 48 kHz; nothing but a far triangle in the scene."""
    c, fs = 343.0, 48000.0
    edges = [Fraction(343 * s, 48000) for s in (1000, 2800, 5000)]   # 7.15 m, 20.0 m, 35.7 m
    ds = []
    for e in edges:
        lo, hi = _f32_around(e)
        ds += [lo, hi]
    axes = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], np.float64)
    rcv = np.zeros((6, 4), np.float32)
    for m, (d, a) in enumerate(zip(ds, axes)):
        rcv[m, :3] = (a * d).astype(np.float32)
        rcv[m, 3] = 2.0
        assert float(np.linalg.norm(rcv[m, :3].astype(np.float64))) == d     # on an axis: exact
    s = synth.open_scene_far_triangle()
    src = np.zeros(3, np.float32)
    N = 200_000
    sc = oracle_lib.OracleScene.of(s)
    dirs = oracle_lib.fibonacci(N)
    tr = oracle_lib.trace(sc, src, dirs, rcv, 1, flags=False)
    det = oracle_lib.detections_from_bits(tr["det"])
    keys = oracle_lib.image_source_keys(s.plane_id, tr["hit_seq"], det)
    tab = oracle_lib.image_sources(sc, src, rcv, keys)
    return dict(s=s, rcv=rcv, ds=ds, edges=edges, N=N, det=det, tab=tab, c=c, fs=fs, src=src)


def test_free_field_direct_sound_lands_in_its_exact_bin(free_field, oracle_lib):
    ff = free_field
    s, tab, N, c, fs = ff["s"], ff["tab"], ff["N"], ff["c"], ff["fs"]
    L = 24_000
    out = oracle_lib.assemble_ir(tab, N, 6, np.zeros((1, 8)), np.zeros(8), np.zeros(1, np.int64), c, fs, L,
                                 synth.delta_taps(1))
    H = out["hist"]
    for m, d in enumerate(ff["ds"]):
        want = _exact_bin(d, c, fs)
        e = ff["edges"][m // 2]
        # one below, one at/above the edge: consecutive bins
        assert want == _floor_frac(e * Fraction(48000, 343)) - (1 if m % 2 == 0 else 0)
        n0 = int(((ff["det"][:, 2] == m) & (ff["det"][:, 1] == 0)).sum())
        assert n0 > 100                                   # the receiver is well resolved
        nz = np.nonzero(H[m, 0])[0]
        assert list(nz) == [want], (m, d, want, nz[:5])  # nothing else arrives within 0.5 s
        assert np.all(H[m, :, want] == n0 / N)           # beta = 0: the energy is n/N in every band


def test_bin_edges_exact_and_realistic(oracle_lib):
    """Distances at and around bin edges, straight into the histogram."""
    rows = []
    # c = 256 m/s, fs = 32768 Hz: bin s starts at exactly s / 128 m (dyadic, exact in FP64)
    c1, fs1, L1 = 256.0, 32768.0, 5000
    for s in (0, 1, 2, 127, 128, 999, 4096, L1 - 1, L1):
        e = Fraction(s, 128)
        cand = [float(e)]
        if s > 0:
            cand.append(float(np.nextafter(float(e), -np.inf)))
        cand.append(float(np.nextafter(float(e), np.inf)))
        rows += [(d, c1, fs1, L1) for d in cand]
    # realistic constants: 1e-9 relative either side of s * 343 / 48000
    c2, fs2, L2 = 343.0, 48000.0, 96_000
    for s in (1, 7, 48_000, 95_999, 96_000):
        lo, hi = _f64_around(Fraction(343 * s, 48000), 1e-9)
        rows += [(lo, c2, fs2, L2), (hi, c2, fs2, L2)]
    for c, fs, L in ((c1, fs1, L1), (c2, fs2, L2)):
        ds = [d for d, cc, ff, _ in rows if cc == c and ff == fs]
        want = [_exact_bin(d, c, fs) for d in ds]
        got = oracle_lib.arrival_bins(np.array(ds), c, fs)
        assert list(got) == want
        # the same distances as single-plane image sources of one receiver
        keys = [(0, 1, i) for i in range(len(ds))]
        tab = dict(keys=keys, count=np.ones(len(ds), np.int64), dist=np.array(ds))
        mop = np.zeros(len(ds), np.int64)
        out = oracle_lib.assemble_ir(tab, 1, 1, np.zeros((1, 8)), np.zeros(8), mop, c, fs, L,
                                     synth.delta_taps(1))
        expect = np.zeros(L)
        for w in want:
            if 0 <= w < L:
                expect[w] += 1.0
        assert np.array_equal(out["hist"][0, 3], expect)
        assert (np.array(want) == L).any() and (np.array(want) == L - 1).any()


def test_direct_sound_band_ratio_is_air_absorption(free_field, oracle_lib):
    """alpha = 0, ISO beta: E_i / E_j of the direct sound = exp(-(beta_i -
    beta_j) d), d the receiver's distance placed on its axis."""
    ff = free_field
    beta = synth.iso9613_beta().astype(np.float64)
    tab, N = ff["tab"], ff["N"]
    E = oracle_lib.is_energy(tab, N, np.zeros((1, 8)), beta, np.zeros(1, np.int64))
    for i, key in enumerate(tab["keys"]):
        if key[1] != 0:
            continue
        d = ff["ds"][key[0]]
        for b in range(1, 8):
            assert E[i, b] / E[i, 0] == pytest.approx(np.exp(-(beta[b] - beta[0]) * d), rel=1e-12)
        # the 8 kHz band loses 10 beta d / ln 10 dB over d
        db = 10 * np.log10(E[i, 7] / (tab["count"][i] / N))
        assert db == pytest.approx(-10.0 * beta[7] * d / np.log(10.0), rel=1e-12)


def test_reflected_image_source_distance_and_absorption(oracle_lib):
    """A large reflecting floor z = 0, source 2 m above it, receiver at
    (4, 0, 1): the direct path is sqrt 17 m long, the floor's image source
    (0, 0, -2) lies 5 m from the receiver.  Band energies relative to the
    direct sound follow from those two distances, the detected counts and the
    floor's absorption."""
    W = 1000.0
    vtx = np.array([[-W, -W, 0], [W, -W, 0], [W, W, 0], [-W, W, 0]], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    pid = np.zeros(2, np.int32)
    sc = oracle_lib.OracleScene(vtx, tri, pid)
    src = np.array([0, 0, 2], np.float32)
    rcv = np.array([[4, 0, 1, 0.5]], np.float32)
    N = 200_000
    tr = oracle_lib.trace(sc, src, oracle_lib.fibonacci(N), rcv, 1, flags=False)
    det = oracle_lib.detections_from_bits(tr["det"])
    keys = oracle_lib.image_source_keys(pid, tr["hit_seq"], det)
    assert set(keys) == {(0, 0), (0, 1, 0)}
    tab = oracle_lib.image_sources(sc, src, rcv, keys)
    i0, i1 = tab["keys"].index((0, 0)), tab["keys"].index((0, 1, 0))
    assert np.allclose(tab["pos"][i1], [0, 0, -2], atol=0, rtol=0)
    assert tab["dist"][i1] == 5.0 and tab["dist"][i0] == pytest.approx(np.sqrt(17.0), rel=1e-15)
    n0, n1 = keys[(0, 0)], keys[(0, 1, 0)]
    # solid-angle counts of a 0.5 m sphere at sqrt 17 m and at 5 m
    for n, d in ((n0, np.sqrt(17.0)), (n1, 5.0)):
        e = N * (1 - np.sqrt(1 - 0.25 / d ** 2)) / 2
        assert abs(n - e) <= 3 * np.sqrt(e) + 2
    alpha = np.array([[0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8]])
    beta = synth.iso9613_beta().astype(np.float64) * 100.0          # strong, so that the factor shows
    c, fs, L = 343.0, 48000.0, 2000
    out = oracle_lib.assemble_ir(tab, N, 1, alpha, beta, np.zeros(1, np.int64), c, fs, L, synth.delta_taps(1))
    s0 = _exact_bin(float(np.sqrt(17.0)), c, fs)
    s1 = _exact_bin(5.0, c, fs)
    assert s1 == 699 and s0 == _floor_frac(Fraction(np.sqrt(17.0)) * 48000 / 343)
    H = out["hist"][0]
    assert list(np.nonzero(H[0])[0]) == [s0, s1]
    ratio = H[:, s1] / H[:, s0]
    want = (n1 / n0) * np.exp(-beta * (5.0 - np.sqrt(17.0))) * (1 - alpha[0])
    assert np.allclose(ratio, want, rtol=1e-12, atol=0)
    assert np.allclose(H[:, s0], n0 / N * np.exp(-beta * np.sqrt(17.0)), rtol=1e-12, atol=0)
