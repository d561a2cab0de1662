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
        lib.rt_debug_set_hash_bits(48)
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


def _full_size_tables(rt, oracle_lib, s, sc, R, mpl):
    """Trace every ray of the configuration (the benchmarked launch), collect
    and assemble its image sources and response, and compare with the oracle
    computed from the GPU's own hit sequences and detections (section
    "Image-sources"): the oracle keys every detection, so keys and counts must
    be identical; it mirrors the source through each key's planes, so
    positions and distances must agree within 1e-9 (both FP64, different
    order); from that table it assembles the response (FP64 histogram, sqrt,
    direct 'same' FIR with the 4095 taps), so band energies, histogram bins
    (those >= 1e-9 of the band's largest) and FIR band energies must agree
    within 1e-4.  Returns (n_is, n_det, max rel of the band energies, of the
    FIR band energies)."""
    N = s.n_rays
    dirs = rt.fibonacci_directions(N, device="cuda:0")
    tr = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl, det_cap=6 * N)
    isrc = rt.collect_image_sources(sc, s.src, s.rcv, tr)
    g = gpu_is_dict(isrc)
    n_det = int(tr.counters[0])
    assert sum(v[0] for v in g.values()) == n_det and len(g) > 10_000
    hs = tr.hit_seq.cpu().numpy()
    det = tr.detections().cpu().numpy()
    _say("  %d detections, %d GPU image sources; keying on the CPU" % (n_det, len(g)))
    okeys = oracle_lib.image_source_keys(s.plane_id, hs, det)
    assert set(g) == set(okeys)
    assert all(g[k][0] == n for k, n in okeys.items())
    tab = oracle_lib.image_sources(oracle_lib.OracleScene.of(s), s.src, s.rcv, okeys)
    gp = np.array([g[k][1] for k in tab["keys"]])
    gd = np.array([g[k][2] for k in tab["keys"]])
    scale = float(np.abs(tab["pos"]).max())
    assert np.abs(gp - tab["pos"]).max() <= 1e-9 * scale
    assert np.all(np.abs(gd - tab["dist"]) <= 1e-9 * np.maximum(tab["dist"], 1.0))
    taps = synth.octave_fir_taps(4095)
    n_rcv = len(s.rcv)
    ir = rt.assemble_ir(sc, isrc, N, n_rcv, s.alpha, s.beta, s.c, s.fs, s.ir_len, taps)
    ref = oracle_lib.assemble_ir(tab, N, n_rcv, s.alpha, s.beta, material_of_plane(s), s.c, s.fs, s.ir_len, taps)
    be = ir.band_energy.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(be - ref["band_energy"]) <= 1e-4 * ref["band_energy"])
    H = ir.hist.cpu().numpy().astype(np.float64)
    big = ref["hist"] >= 1e-9 * ref["hist"].max(axis=2, keepdims=True)
    assert big.any() and np.all(np.abs(H - ref["hist"])[big] <= 1e-4 * ref["hist"][big])
    e_gpu = (ir.band_ir.cpu().numpy().astype(np.float64) ** 2).sum(-1)
    e_ref = (ref["band_ir"] ** 2).sum(-1)
    assert np.all(np.abs(e_gpu - e_ref) <= 1e-4 * e_ref)
    rel_b = float(np.max(np.abs(be - ref["band_energy"]) / ref["band_energy"]))
    rel_f = float(np.max(np.abs(e_gpu - e_ref) / e_ref))
    return len(g), n_det, rel_b, rel_f


def test_theater_full_size_image_sources_and_bands(rt, oracle_lib):
    """The benchmarked trace (436,120 triangles, 10^6 rays, R = 60, 8
    receivers, 2 s response at 48 kHz: L = 96,000, K = 4095): the whole
    image-source set and response against the oracle."""
    s = synth.theater_c3()
    sc = rt.Scene.from_synth(s, device="cuda:0")
    n_is, n_det, rb, rf = _full_size_tables(rt, oracle_lib, s, sc, s.max_reflections, s.max_path_length)
    _say("theater full size: %d image sources, %d detections; band energies max rel %.1e, FIR band energies "
         "(L = 96,000, K = 4095) max rel %.1e" % (n_is, n_det, rb, rf))


def test_jittered_box_full_size_image_sources_and_bands(rt, oracle_lib, c2):
    """The 100k-triangle jittered box at full size (10^6 rays, R = 50, 3
    receivers, 1 s response, plane id = triangle id): the whole image-source
    set and response against the oracle."""
    s, sc = c2
    n_is, n_det, rb, rf = _full_size_tables(rt, oracle_lib, s, sc, s.max_reflections, s.max_path_length)
    _say("jittered box full size: %d image sources, %d detections; band energies max rel %.1e, FIR band energies "
         "max rel %.1e" % (n_is, n_det, rb, rf))
