"""GPU parity of image-source collection, impulse-response assembly and the
absorption adjoint against the FP64 oracle, on the same seeded inputs.

* Image sources from a seeded path table (hit sequences + detections with
  the structure of a trace): keys and counts must be identical (integer
  work); FP64 positions and distances within 1e-9 relative (different
  operation order).  The collision path (hash truncated to a few bits) must
  give the same table.
* Assembly from a seeded image-source table: per-band receiver energies within
  1e-4 relative; histogram bins within 1e-4 relative where the oracle's bin
  is >= 1e-9 of the band maximum; energies of the FIR-filtered band IRs
  (sum of squares, FP32 MFMA accumulation over K taps) within 1e-4 relative.
* Adjoint: FP64 reductions on both sides, rounded once to FP32: 1e-5 relative.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from tests._util import gpu_is_dict, material_of_plane, synthetic_is_table

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rt():
    import paper_1811_05784_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def c2(rt):
    s = synth.tessellated_box_c2(jitter=True)
    return s, rt.Scene.from_synth(s, device="cuda:0")


@pytest.fixture(scope="module")
def c1(rt):
    s = synth.shoebox_c1()
    return s, rt.Scene.from_synth(s, device="cuda:0")


def _check_is(oracle_lib, s, isrc, hs, det):
    g = gpu_is_dict(isrc)
    keys = oracle_lib.image_source_keys(s.plane_id, hs, det)
    assert set(g) == set(keys)
    assert all(g[k][0] == n for k, n in keys.items())
    tab = oracle_lib.image_sources(oracle_lib.OracleScene.of(s), s.src, s.rcv, keys)
    gp = np.array([g[k][1] for k in tab["keys"]])
    gd = np.array([g[k][2] for k in tab["keys"]])
    scale = np.abs(tab["pos"]).max() + 1.0
    assert np.abs(gp - tab["pos"]).max() <= 1e-9 * scale
    assert np.allclose(gd, tab["dist"], rtol=1e-9, atol=1e-9 * scale)
    return len(keys)


@pytest.mark.parametrize("n_rays,R,n_rcv", [(1, 0, 1), (5000, 20, 3), (200_000, 50, 3)])
def test_collect_parity_synthetic_paths(rt, oracle_lib, c2, n_rays, R, n_rcv):
    s, sc = c2
    s = synth.Scene(**{**s.__dict__, "rcv": s.rcv[:n_rcv]})
    hs, det = synth.synthetic_paths(s, n_rays, R, n_rcv, seed=n_rays + R)
    _say("collect synthetic", n_rays, R, len(det))
    isrc = rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=hs, det=det, max_reflections=R)
    n = _check_is(oracle_lib, s, isrc, hs, det)
    assert n == isrc.n_is()


def test_collect_collisions_resolved_exactly(rt, oracle_lib, c2):
    s, sc = c2
    hs, det = synth.synthetic_paths(s, 20_000, 10, 3, seed=3)
    ref = gpu_is_dict(rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=hs, det=det, max_reflections=10))
    lib = rt.load()
    try:
        for bits in (4, 13):
            assert lib.rt_debug_set_hash_bits(bits) == 0
            got = gpu_is_dict(rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=hs, det=det,
                                                       max_reflections=10))
            assert set(got) == set(ref) and all(got[k][0] == ref[k][0] for k in ref)
    finally:
        lib.rt_debug_set_hash_bits(32)
    _check_is(oracle_lib, s, rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=hs, det=det,
                                                      max_reflections=10), hs, det)


def test_collect_capacity_and_empty(rt, c2):
    s, sc = c2
    hs, det = synth.synthetic_paths(s, 3000, 8, 3, seed=9)
    small = rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=hs, det=det, max_reflections=8, is_cap=5,
                                     check_capacity=False)
    assert small.n_is() > 5
    full = rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=hs, det=det, max_reflections=8, is_cap=5)
    assert full.n_is() == small.n_is()
    empty = rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=hs, det=det[:0], max_reflections=8)
    assert empty.n_is() == 0


def _is_from_table(rt, sc, arr, tab, R):
    dev = "cuda:0"
    n = len(arr)
    return rt.ImageSources(key=torch.as_tensor(arr, device=dev),
                           count=torch.as_tensor(tab["count"].astype(np.int32), device=dev),
                           pos=torch.zeros((n, 3), dtype=torch.float64, device=dev),
                           dist=torch.as_tensor(tab["dist"], device=dev),
                           n_is_dev=torch.tensor([n], dtype=torch.int64, device=dev), max_reflections=R)


@pytest.mark.parametrize("n_is,R,n_rcv,L,K", [(1, 0, 1, 1, 1), (3000, 10, 2, 5000, 63), (40_000, 30, 3, 48_000, 4095),
                                             (20_000, 20, 8, 24_321, 1023), (5000, 12, 1, 1000, 1025),
                                             (30_000, 25, 5, 37_001, 8191), (2, 3, 2, 7, 2049)])
def test_assemble_parity(rt, oracle_lib, c2, n_is, R, n_rcv, L, K):
    """K >= 1024 takes the overlap-save FFT path (16384-point segments; one
    segment, several, and the longest filter), shorter filters the direct
    matrix-core path."""
    s, sc = c2
    n_rays = 1_000_000
    tab, arr = synthetic_is_table(s, n_is, R, n_rcv, seed=n_is + L, L=L, c=s.c, fs=s.fs, n_rays=n_rays)
    _say("assemble", len(arr), R, n_rcv, L, K)
    taps = synth.octave_fir_taps(K) if K > 1 else synth.delta_taps(1)
    isrc = _is_from_table(rt, sc, arr, tab, R)
    ir = rt.assemble_ir(sc, isrc, n_rays, n_rcv, s.alpha, s.beta, s.c, s.fs, L, taps)
    ref = oracle_lib.assemble_ir(tab, n_rays, n_rcv, s.alpha, s.beta, material_of_plane(s), s.c, s.fs, L, taps)
    be = ir.band_energy.cpu().numpy().astype(np.float64)
    assert np.allclose(be, ref["band_energy"], rtol=1e-4, atol=1e-30)
    H = ir.hist.cpu().numpy().astype(np.float64)
    Hr = ref["hist"]
    big = Hr >= 1e-9 * Hr.max(axis=2, keepdims=True)
    assert np.all(np.abs(H - Hr)[big] <= 1e-4 * Hr[big])
    assert np.all(H[~big] <= 1e-9 * Hr.max(axis=2, keepdims=True).repeat(L, 2)[~big] + 1e-30)
    eb = (ir.band_ir.cpu().numpy().astype(np.float64) ** 2).sum(-1)
    er = (ref["band_ir"] ** 2).sum(-1)
    assert np.allclose(eb, er, rtol=1e-4, atol=1e-30)
    irr = ir.ir.cpu().numpy().astype(np.float64)
    scale = np.abs(ref["ir"]).max()
    assert np.abs(irr - ref["ir"]).max() <= 1e-4 * scale


def test_assemble_delta_taps_is_sqrt_hist(rt, c2):
    s, sc = c2
    tab, arr = synthetic_is_table(s, 5000, 12, 3, seed=4, L=30_000, c=s.c, fs=s.fs, n_rays=100_000)
    isrc = _is_from_table(rt, sc, arr, tab, 12)
    ir = rt.assemble_ir(sc, isrc, 100_000, 3, s.alpha, s.beta, s.c, s.fs, 30_000, synth.delta_taps(1))
    assert torch.allclose(ir.band_ir, torch.sqrt(ir.hist), rtol=1e-6, atol=0)
    ir2 = rt.assemble_ir(sc, isrc, 100_000, 3, s.alpha, s.beta, s.c, s.fs, 30_000, synth.delta_taps(1))
    assert torch.equal(ir.hist, ir2.hist) and torch.equal(ir.band_ir, ir2.band_ir)   # deterministic


@pytest.mark.parametrize("alpha_kind", ["random", "ones"])
def test_adjoint_parity(rt, oracle_lib, c2, alpha_kind):
    s, sc = c2
    n_rays, R, n_rcv, L = 200_000, 15, 3, 20_000
    tab, arr = synthetic_is_table(s, 8000, R, n_rcv, seed=11, L=L, c=s.c, fs=s.fs, n_rays=n_rays)
    alpha = s.alpha.copy()
    if alpha_kind == "ones":
        alpha[::2, ::3] = 1.0
    g = np.random.default_rng(1).standard_normal((n_rcv, 8)).astype(np.float32)
    isrc = _is_from_table(rt, sc, arr, tab, R)
    got = rt.band_energy_adjoint(sc, isrc, n_rays, n_rcv, alpha, s.beta, s.c, s.fs, L, g).cpu().numpy()
    ref = oracle_lib.band_energy_grad(tab, n_rays, n_rcv, s.n_mat, alpha, s.beta, material_of_plane(s), s.c, s.fs,
                                      L, g)
    scale = np.abs(ref).max()
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-6 * scale)


def test_band_energy_autograd_and_finite_differences(rt, c1):
    s, sc = c1
    dirs = rt.fibonacci_directions(s.n_rays, device="cuda:0")
    tr = rt.trace_rays(sc, dirs, s.rcv, s.max_reflections, src=s.src, max_path_length=s.max_path_length)
    isrc = rt.collect_image_sources(sc, s.src, s.rcv, tr)
    alpha = torch.tensor(s.alpha, device="cuda:0", requires_grad=True)
    beta = torch.tensor(s.beta, device="cuda:0")
    e = rt.BandEnergy.apply(alpha, sc, isrc, s.n_rays, 1, beta, s.c, s.fs, s.ir_len)
    w = torch.arange(1, 9, dtype=torch.float32, device="cuda:0")
    (e * w).sum().backward()
    grad = alpha.grad.cpu().numpy().astype(np.float64)
    h = 1e-4
    fd = np.zeros_like(grad)
    with torch.no_grad():
        for m in range(s.n_mat):
            for b in range(8):
                ap = alpha.detach().clone()
                am = alpha.detach().clone()
                ap[m, b] += h
                am[m, b] -= h
                ep = rt.BandEnergy.apply(ap, sc, isrc, s.n_rays, 1, beta, s.c, s.fs, s.ir_len)
                em = rt.BandEnergy.apply(am, sc, isrc, s.n_rays, 1, beta, s.c, s.fs, s.ir_len)
                fd[m, b] = float(((ep - em) * w).sum()) / (2 * h)
    scale = np.abs(grad).max()
    assert scale > 0
    assert np.allclose(grad, fd, rtol=1e-2, atol=1e-2 * scale)


def _full_size_tables(rt, oracle_lib, s, sc, R, mpl, mirror_rows, seed):
    """Trace every ray of the configuration, collect and assemble, then check
    properties that hold at any size: counts add up to the detections, keys
    are distinct, the positions of `mirror_rows` seeded rows (all rows if
    None) are the source mirrored (FP64) through their keys' planes taken from
    the mesh, distances match positions, and the band energies are the sums
    over the table of n/N e^(-beta d) prod(1 - alpha) over the sources that
    arrive within the response (1e-4 relative).  Returns (n_is, n_det, max rel)."""
    N = s.n_rays
    dirs = rt.fibonacci_directions(N, device="cuda:0")
    tr = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl, det_cap=6 * N)
    isrc = rt.collect_image_sources(sc, s.src, s.rcv, tr)
    key, cnt, pos, dist = [t.cpu().numpy() for t in isrc.valid()]
    assert int(cnt.sum()) == int(tr.counters[0]) and len(key) > 10_000
    kk = key[:, 1].astype(np.int64)
    width = 2 + int(kk.max())
    trimmed = np.where(np.arange(width)[None, :] < (2 + kk)[:, None], key[:, :width], -2)
    assert len(np.unique(trimmed, axis=0)) == len(key)
    pn, pp = oracle_lib.OracleScene.of(s).planes()
    rcv = s.rcv.astype(np.float64)
    src = np.asarray(s.src, np.float64)
    scale = float(np.abs(pos).max())
    rows = np.arange(len(key)) if mirror_rows is None else \
        np.random.default_rng(seed).choice(len(key), mirror_rows, replace=False)
    for i in rows:
        r, p, d = key[i], pos[i], dist[i]
        m, k = int(r[0]), int(r[1])
        x = src.copy()
        for j in range(k):
            q = int(r[2 + j])
            x = x - 2.0 * np.dot(x - pp[q], pn[q]) * pn[q]
        assert np.abs(x - p).max() <= 1e-9 * scale
        assert abs(np.linalg.norm(p - rcv[m, :3]) - d) <= 1e-12 * max(d, 1.0)
    taps = synth.octave_fir_taps(4095)
    ir = rt.assemble_ir(sc, isrc, N, len(s.rcv), s.alpha, s.beta, s.c, s.fs, s.ir_len, taps)
    mop = material_of_plane(s)
    one_minus = np.vstack([1.0 - np.asarray(s.alpha, np.float64), np.ones((1, 8))])   # last row: no plane
    beta = np.asarray(s.beta, np.float64)
    want = np.zeros((len(s.rcv), 8))
    inside = np.floor(dist * s.fs / s.c) < s.ir_len
    for c0 in range(0, len(key), 50_000):
        sl = slice(c0, c0 + 50_000)
        pl = key[sl, 2:2 + R].astype(np.int64)
        live = np.arange(pl.shape[1])[None, :] < kk[sl, None]
        mat = np.where(live, mop[np.where(live, pl, 0)], len(one_minus) - 1)
        e = (cnt[sl] / N)[:, None] * np.exp(-beta[None, :] * dist[sl, None]) * one_minus[mat].prod(axis=1)
        e[~inside[sl]] = 0.0
        np.add.at(want, key[sl, 0], e)
    got = ir.band_energy.cpu().numpy().astype(np.float64)
    rel = float(np.max(np.abs(got - want) / np.maximum(want, 1e-30)))
    assert np.all(np.abs(got - want) <= 1e-4 * np.abs(want) + 1e-30)
    return len(key), int(cnt.sum()), rel


def test_theater_full_size_image_sources_and_bands(rt, oracle_lib):
    """The benchmarked trace (436,120 triangles, 10^6 rays, R = 60, 8
    receivers, 2 s response): every image-source row checked."""
    s = synth.theater_c3()
    sc = rt.Scene.from_synth(s, device="cuda:0")
    n_is, n_det, rel = _full_size_tables(rt, oracle_lib, s, sc, s.max_reflections, s.max_path_length, None, 0)
    _say("theater full size: %d image sources, %d detections, band energies max rel %.1e" % (n_is, n_det, rel))


def test_jittered_box_full_size_image_sources_and_bands(rt, oracle_lib, c2):
    """The 100k-triangle jittered box at full size (10^6 rays, R = 50, 3
    receivers, 1 s response, plane id = triangle id): 3,000 seeded rows
    mirrored, every row in the band energies."""
    s, sc = c2
    n_is, n_det, rel = _full_size_tables(rt, oracle_lib, s, sc, s.max_reflections, s.max_path_length, 3_000, 22)
    _say("jittered box full size: %d image sources, %d detections, band energies max rel %.1e" % (n_is, n_det, rel))
