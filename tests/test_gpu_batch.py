"""Batched jobs over rooms of uneven size in one persistent launch, captured
in a HIP graph, with launch settings chosen by the autotuner.

The batched path must reproduce, job by job, what the single-scene path
computes (itself checked against the FP64 oracle): identical hit sequences
(each job's rays take Fibonacci direction i of n on the device), identical
detections and image-source keys and counts (receiver rows and material rows
offset per job / scene), equal energies and gradients (FP64 reductions in
another order: 1e-6 relative).  A graph replay must equal the eager run on
every replay, with eager work and synchronisations in between.
"""
import os
import sys

import numpy as np
import pytest
import torch

import synth
from tests._util import gpu_is_dict, material_of_plane

pytestmark = pytest.mark.gpu

R = 12
N_PAIR = 4000
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rt():
    import paper_1811_05784_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def setup(rt):
    rooms = synth.batched_rooms(n_rooms=4, pairs_per_room=2, rays_per_pair=N_PAIR, m_hi=20_000.0)
    scenes = [rt.Scene.from_synth(r, device=DEV) for r in rooms]
    jobs = []
    for i, r in enumerate(rooms):
        for p in range(len(r.src)):
            jobs.append(dict(scene=i, src=r.src[p], rcv=r.rcv[p:p + 1], n_rays=N_PAIR + 17 * p,
                             max_path_length=60.0))
    b = rt.Batch(scenes, jobs, device=DEV)
    return rooms, scenes, jobs, b


def _single(rt, scene, job):
    d = rt.fibonacci_directions(job["n_rays"], device=DEV)
    return rt.trace_rays(scene, d, job["rcv"], R, src=job["src"], max_path_length=job["max_path_length"])


def test_batch_trace_equals_single_scene(rt, setup):
    rooms, scenes, jobs, b = setup
    tr = rt.trace_batch(b, R)
    hs = tr.hit_seq.cpu().numpy()
    det = tr.detections().cpu().numpy()
    tot_q = 0
    for j, job in enumerate(jobs):
        one = _single(rt, scenes[job["scene"]], job)
        lo, hi = b.ray_off[j], b.ray_off[j + 1]
        assert np.array_equal(hs[lo:hi], one.hit_seq.cpu().numpy()), j
        dj = det[(det[:, 0] >= lo) & (det[:, 0] < hi)].copy()
        dj[:, 0] -= lo
        dj[:, 2] -= b.rcv_off[j]
        d1 = one.detections().cpu().numpy()
        assert np.array_equal(dj[np.lexsort(dj.T[::-1])], d1[np.lexsort(d1.T[::-1])]), j
        tot_q += int(one.counters[1])
    assert int(tr.counters[1]) == tot_q
    _say("batch: %d jobs, %d rays, %d queries, %d detections" % (b.n_jobs, b.n_rays, tot_q, len(det)))


def test_batch_collect_assemble_adjoint_equal_single(rt, setup):
    rooms, scenes, jobs, b = setup
    tr = rt.trace_batch(b, R)
    isb = rt.collect_batch(b, tr)
    gb = gpu_is_dict(isb)
    L, c, fs = 24_000, 343.0, 48_000.0
    taps = synth.octave_fir_taps(255)
    alpha = np.concatenate([r.alpha for r in rooms]).astype(np.float32)
    beta = rooms[0].beta
    irb = rt.assemble_batch(b, isb, alpha, beta, c, fs, L, taps)
    g = np.random.default_rng(0).standard_normal((b.n_rcv, 8)).astype(np.float32)
    gab = rt.adjoint_batch(b, isb, alpha, beta, c, fs, L, g).cpu().numpy()
    grad_ref = np.zeros_like(gab)
    for j, job in enumerate(jobs):
        sc = scenes[job["scene"]]
        one = _single(rt, sc, job)
        is1 = rt.collect_image_sources(sc, job["src"], job["rcv"], one)
        g1 = gpu_is_dict(is1)
        r0 = int(b.rcv_off[j])
        sub = {(k[0] - r0,) + k[1:]: v for k, v in gb.items() if r0 <= k[0] < r0 + 1}
        assert set(sub) == set(g1), j
        for k, (n, pos, d) in g1.items():
            assert sub[k][0] == n and np.allclose(sub[k][1], pos, rtol=0, atol=1e-9) and abs(sub[k][2] - d) < 1e-9
        room = rooms[job["scene"]]
        ir1 = rt.assemble_ir(sc, is1, job["n_rays"], 1, room.alpha, beta, c, fs, L, taps)
        assert np.allclose(irb.band_energy[r0:r0 + 1].cpu().numpy(), ir1.band_energy.cpu().numpy(), rtol=1e-6,
                           atol=0)
        assert np.allclose(irb.ir[r0:r0 + 1].cpu().numpy(), ir1.ir.cpu().numpy(), rtol=1e-5, atol=1e-12)
        ga1 = rt.band_energy_adjoint(sc, is1, job["n_rays"], 1, room.alpha, beta, c, fs, L, g[r0:r0 + 1])
        m0 = int(b.mat_off[job["scene"]])
        grad_ref[m0:m0 + sc.n_mat] += ga1.cpu().numpy().astype(np.float64)
    scale = np.abs(grad_ref).max()
    assert scale > 0
    assert np.allclose(gab, grad_ref, rtol=1e-5, atol=1e-6 * scale)


def test_batch_collect_assemble_adjoint_match_oracle(rt, oracle_lib, setup):
    """Batched image sources, responses and absorption gradient against the
    FP64 oracle, job by job, from the batched launch's own hit sequences and
    detections (sections "Image-sources" and the eq. for E_s): keys and counts
    identical, positions and distances within 1e-9, band energies, histogram
    bins and FIR band energies within 1e-4, the gradient (summed over the
    jobs of each room, per material row) within 1e-5."""
    rooms, scenes, jobs, b = setup
    tr = rt.trace_batch(b, R)
    isb = rt.collect_batch(b, tr)
    gb = gpu_is_dict(isb)
    L, c, fs = 24_000, 343.0, 48_000.0
    taps = synth.octave_fir_taps(255)
    alpha = np.concatenate([r.alpha for r in rooms]).astype(np.float32)
    beta = rooms[0].beta
    irb = rt.assemble_batch(b, isb, alpha, beta, c, fs, L, taps)
    g = np.random.default_rng(3).standard_normal((b.n_rcv, 8)).astype(np.float32)
    gab = rt.adjoint_batch(b, isb, alpha, beta, c, fs, L, g).cpu().numpy()
    hs = tr.hit_seq.cpu().numpy()
    det = tr.detections().cpu().numpy()
    band = irb.band_energy.cpu().numpy().astype(np.float64)
    hist = irb.hist.cpu().numpy().astype(np.float64)
    bir = irb.band_ir.cpu().numpy().astype(np.float64)
    grad_ref = np.zeros(gab.shape)
    n_keys = 0
    for j, job in enumerate(jobs):
        room = rooms[job["scene"]]
        lo, hi = b.ray_off[j], b.ray_off[j + 1]
        r0 = int(b.rcv_off[j])
        dj = det[(det[:, 0] >= lo) & (det[:, 0] < hi)].copy()
        dj[:, 0] -= lo
        dj[:, 2] -= r0
        okeys = oracle_lib.image_source_keys(room.plane_id, hs[lo:hi], dj)
        sub = {(k[0] - r0,) + k[1:]: v for k, v in gb.items() if k[0] == r0}
        assert set(sub) == set(okeys), j
        assert all(sub[k][0] == n for k, n in okeys.items()), j
        tab = oracle_lib.image_sources(oracle_lib.OracleScene.of(room), job["src"], job["rcv"], okeys)
        gp = np.array([sub[k][1] for k in tab["keys"]])
        gd = np.array([sub[k][2] for k in tab["keys"]])
        assert np.abs(gp - tab["pos"]).max() <= 1e-9 * max(1.0, float(np.abs(tab["pos"]).max())), j
        assert np.abs(gd - tab["dist"]).max() <= 1e-9 * max(1.0, float(tab["dist"].max())), j
        mop = material_of_plane(room)
        ref = oracle_lib.assemble_ir(tab, job["n_rays"], 1, room.alpha, beta, mop, c, fs, L, taps)
        assert np.all(np.abs(band[r0] - ref["band_energy"][0]) <= 1e-4 * ref["band_energy"][0]), j
        big = ref["hist"][0] >= 1e-9 * ref["hist"][0].max(axis=1, keepdims=True)
        assert np.all(np.abs(hist[r0] - ref["hist"][0])[big] <= 1e-4 * ref["hist"][0][big]), j
        e_ref = (ref["band_ir"][0] ** 2).sum(-1)
        assert np.all(np.abs((bir[r0] ** 2).sum(-1) - e_ref) <= 1e-4 * e_ref), j
        m0 = int(b.mat_off[job["scene"]])
        grad_ref[m0:m0 + room.n_mat] += oracle_lib.band_energy_grad(tab, job["n_rays"], 1, room.n_mat, room.alpha,
                                                                    beta, mop, c, fs, L, g[r0:r0 + 1])
        n_keys += len(okeys)
    scale = np.abs(grad_ref).max()
    assert scale > 0
    assert np.allclose(gab, grad_ref, rtol=1e-5, atol=1e-6 * scale)
    _say("batch vs oracle: %d jobs, %d image sources, gradient scale %.3e" % (len(jobs), n_keys, scale))


def test_graph_replay_matches_eager(rt, setup):
    rooms, scenes, jobs, b = setup
    L, c, fs = 24_000, 343.0, 48_000.0
    taps = torch.as_tensor(synth.octave_fir_taps(255), device=DEV)
    alpha = torch.as_tensor(np.concatenate([r.alpha for r in rooms]), device=DEV)
    beta = torch.as_tensor(rooms[0].beta, device=DEV)
    g = torch.ones((b.n_rcv, 8), dtype=torch.float32, device=DEV)
    # eager reference, and buffers sized for capture (no allocation inside the graph)
    tr = rt.trace_batch(b, R, det_cap=4 * b.n_rays)
    isb = rt.collect_batch(b, tr, is_cap=tr.det.shape[0])
    ir = rt.assemble_batch(b, isb, alpha, beta, c, fs, L, taps)
    ga = rt.adjoint_batch(b, isb, alpha, beta, c, fs, L, g)
    torch.cuda.synchronize()
    ref = [t.clone() for t in (tr.hit_seq, ir.band_energy, ir.ir, ga)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # warm-up on the capture stream (workspaces sized), then capture
        rt.trace_batch(b, R, out=tr, check_capacity=False)
        rt.collect_batch(b, tr, out=isb, check_capacity=False)
        rt.assemble_batch(b, isb, alpha, beta, c, fs, L, taps, out=ir)
        rt.adjoint_batch(b, isb, alpha, beta, c, fs, L, g, out=ga)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rt.trace_batch(b, R, out=tr, check_capacity=False)
        rt.collect_batch(b, tr, out=isb, check_capacity=False)
        rt.assemble_batch(b, isb, alpha, beta, c, fs, L, taps, out=ir)
        rt.adjoint_batch(b, isb, alpha, beta, c, fs, L, g, out=ga)
    for rep in range(3):
        for t in (tr.hit_seq, ir.band_energy, ir.ir, ga):
            t.zero_()
        _ = torch.randn(1000, device=DEV).sum()          # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(tr.hit_seq, ref[0]), rep
        assert torch.allclose(ir.band_energy, ref[1], rtol=1e-6, atol=0), rep
        assert torch.allclose(ir.ir, ref[2], rtol=1e-6, atol=1e-12), rep
        assert torch.allclose(ga, ref[3], rtol=1e-6, atol=1e-12), rep
    assert int(tr.counters[3]) == 0


def test_autotuner_picks_and_caches(rt, setup, tmp_path, monkeypatch):
    from paper_1811_05784_amd import autotune
    rooms, scenes, jobs, b = setup
    monkeypatch.setenv("RTAC_TUNE_CACHE", str(tmp_path / "tune.json"))
    space = {"waves_per_simd": [4], "blocks_per_cu": [0, 8], "fetch_threshold": [8, 16], "shade_threshold": [16],
             "stack_depth": [8, 16, 32]}
    out = rt.trace_batch(b, R, det_cap=4 * b.n_rays)
    calls = []

    def run(setting):
        calls.append(setting)
        rt.trace_batch(b, R, out=out, check_capacity=False, **setting)

    key = autotune.key_for(max(sc.n_tri for sc in scenes), b.n_rays)
    best = autotune.tune(run, key, space=space, repeats=1)
    assert best in autotune.candidates(space)
    n = len(calls)
    again = autotune.tune(run, key, space=space)
    assert again == best and len(calls) == n            # served from the cache
    # the chosen setting, and every stack depth, give the same result
    ref = rt.trace_batch(b, R).hit_seq
    got = rt.trace_batch(b, R, **best).hit_seq
    assert torch.equal(ref, got)
    for depth in (8, 32):
        assert torch.equal(ref, rt.trace_batch(b, R, stack_depth=depth).hit_seq), depth


def test_batch_suspension_unchanged(rt, setup):
    rooms, scenes, jobs, b = setup
    a = rt.trace_batch(b, R)
    s = rt.trace_batch(b, R, suspend_after=2)
    assert torch.equal(a.hit_seq, s.hit_seq) and torch.equal(a.counters[:3], s.counters[:3])
    da, ds = a.detections().cpu().numpy(), s.detections().cpu().numpy()
    assert np.array_equal(da[np.lexsort(da.T[::-1])], ds[np.lexsort(ds.T[::-1])])


def test_batch_eq13_range_equals_single(rt, setup):
    """min_beam_rays in a batch: each job stops its rays at the eq. 13 range
    of its own receivers and ray count, as the single-scene call does (which
    is checked against the oracle)."""
    rooms, scenes, jobs, b = setup
    tr = rt.trace_batch(b, R, min_beam_rays=2)
    full = rt.trace_batch(b, R)
    assert int(tr.counters[1]) < int(full.counters[1])       # the range shortens the paths
    hs = tr.hit_seq.cpu().numpy()
    det = tr.detections().cpu().numpy()
    for j, job in enumerate(jobs):
        d = rt.fibonacci_directions(job["n_rays"], device=DEV)
        one = rt.trace_rays(scenes[job["scene"]], d, job["rcv"], R, src=job["src"],
                            max_path_length=job["max_path_length"], min_beam_rays=2)
        lo, hi = b.ray_off[j], b.ray_off[j + 1]
        assert np.array_equal(hs[lo:hi], one.hit_seq.cpu().numpy()), j
        dj = det[(det[:, 0] >= lo) & (det[:, 0] < hi)].copy()
        dj[:, 0] -= lo
        dj[:, 2] -= b.rcv_off[j]
        d1 = one.detections().cpu().numpy()
        assert np.array_equal(dj[np.lexsort(dj.T[::-1])], d1[np.lexsort(d1.T[::-1])]), j


def test_rooms_full_size_sampled(rt, oracle_lib):
    """The benchmarked batch at full size: 8 rooms of 976-177,356 triangles,
    8 source/receiver pairs each, 2e5 rays per pair (1.28e7 rays), R = 50, in
    one persistent launch with the tuned settings.  In every room, 6 rays of
    one pair (seeded) are traced by the oracle from the same FP32 directions:
    each hit sequence equals the oracle's or first differs at a flagged query,
    detections equal on unflagged agreeing rays."""
    rooms = synth.batched_rooms(seed=4)
    R, T, c = rooms[0].max_reflections, rooms[0].ir_seconds, rooms[0].c
    scenes = [rt.Scene.from_synth(r, device=DEV) for r in rooms]
    jobs = []
    for i, r in enumerate(rooms):
        for p in range(len(r.src)):
            jobs.append(dict(scene=i, src=r.src[p], rcv=r.rcv[p:p + 1], n_rays=r.n_rays,
                             max_path_length=c * T + float(r.rcv[p, 3])))
    b = rt.Batch(scenes, jobs, device=DEV)
    tr = rt.trace_batch(b, R, det_cap=2 * b.n_rays, waves_per_simd=4, blocks_per_cu=8, fetch_threshold=16,
                        shade_threshold=16)
    det = tr.detections().cpu().numpy()
    rng = np.random.default_rng(404)
    checked = flagged = differing = 0
    for i, r in enumerate(rooms):
        j = i * len(r.src) + int(rng.integers(len(r.src)))
        job = jobs[j]
        lo = b.ray_off[j]
        idx = np.sort(rng.choice(job["n_rays"], 6, replace=False))
        dirs = rt.fibonacci_directions(job["n_rays"], device=DEV).cpu().numpy()[idx]
        ref = oracle_lib.trace(oracle_lib.OracleScene.of(r), job["src"], np.ascontiguousarray(dirs), job["rcv"], R,
                               max_len=job["max_path_length"])
        hs = tr.hit_seq[torch.as_tensor(lo + idx, device=DEV)].cpu().numpy()
        diff = (hs != ref["hit_seq"]).any(axis=1)
        for q in np.nonzero(diff)[0]:
            k = int(np.argmax(hs[q] != ref["hit_seq"][q]))
            assert ref["flags"][q, : k + 1].any(), "room %d job %d ray %d: unflagged divergence" % (i, j, idx[q])
        good = ~diff & ~ref["flags"].any(axis=1)
        sel = np.isin(det[:, 0], lo + idx)
        gbits = np.zeros((len(idx), R + 1), np.uint32)
        rows = np.searchsorted(lo + idx, det[sel, 0])
        rcv_local = det[sel, 2] - b.rcv_off[j]
        np.bitwise_or.at(gbits, (rows, det[sel, 1]), (np.uint32(1) << rcv_local.astype(np.uint32)))
        assert np.array_equal(gbits[good], ref["det"][good])
        checked += len(idx)
        flagged += int(ref["flags"].any(axis=1).sum())
        differing += int(diff.sum())
    _say("rooms full size: %d rays checked, %d differing (all at flagged queries), %d flagged, queries %d" % (
        checked, differing, flagged, int(tr.counters[1])))
