"""Stepwise replay of the benchmarked launches' own recorded states.

The launch the benchmark times (default settings, full size) is run again
with states recorded for a seeded subset of its rays (record_rows: only those
rays write states, so the launch itself is unchanged; its hit sequences and
detections are compared bit for bit with an unrecorded run).  Every query
those rays made is replayed by the FP64 oracle from the recorded FP32 state
and checked as described in tests/_replay.py; n_queries, n_flagged and
n_flagged_mismatch are printed.  Pass: no unflagged mismatch, every flagged
mismatch a valid answer.

* theater: 436,120 triangles, 10^6 rays, R = 60, 8 receivers: 500 seeded rays
  and the 40 longest chains;
* jittered box: 100,316 triangles, 10^6 rays, R = 50, 3 receivers: 2,000 rays;
* eight rooms of 976-177,356 triangles x 8 pairs, 2e5 rays each, R = 50, one
  batched launch with the tuned settings: 6 seeded rays of every pair.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from tests._replay import det_bits, replay

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rt():
    import paper_1811_05784_amd as m
    m.load()
    return m


def _sorted(d):
    return d[np.lexsort(d.T[::-1])]


def _check(out, tag):
    _say("%s replay: n_queries %d n_flagged %d n_flagged_mismatch %d problems %d" % (
        tag, out["n_queries"], out["n_flagged"], out["n_flagged_mismatch"], len(out["problems"])))
    for p in out["problems"][:20]:
        _say("  " + p)
    assert not out["problems"]


@pytest.mark.parametrize("name,n_random,n_long", [("c3", 500, 40), ("c2", 2000, 0)])
def test_replay_of_benchmarked_launch(rt, oracle_lib, name, n_random, n_long):
    s = synth.theater_c3() if name == "c3" else synth.tessellated_box_c2(jitter=True)
    _say("replay %s: %d triangles" % (name, s.n_tri))
    sc = rt.Scene.from_synth(s, device=DEV)
    N, R = s.n_rays, s.max_reflections
    dirs = rt.fibonacci_directions(N, device=DEV)
    rcv = torch.as_tensor(s.rcv, device=DEV)
    lim = float(np.float32(s.max_path_length))
    plain = rt.trace_rays(sc, dirs, rcv, R, src=s.src, max_path_length=s.max_path_length, det_cap=6 * N)
    hs_all = plain.hit_seq.cpu().numpy()
    lens = (hs_all >= 0).sum(axis=1)
    rng = np.random.default_rng(77 + n_random)
    pick = rng.choice(N, n_random, replace=False)
    if n_long:
        pick = np.concatenate([pick, np.argsort(-lens, kind="stable")[:n_long]])
    idx = np.unique(pick)
    rows = np.full(N, -1, np.int32)
    rows[idx] = np.arange(len(idx), dtype=np.int32)
    rec = rt.trace_rays(sc, dirs, rcv, R, src=s.src, max_path_length=s.max_path_length, det_cap=6 * N,
                        record_states=True, record_rows=rows)
    # recording a few rays leaves the launch's results unchanged
    assert torch.equal(rec.hit_seq, plain.hit_seq)
    assert torch.equal(rec.counters[:3], plain.counters[:3]) and int(rec.counters[3]) == 0
    assert np.array_equal(_sorted(rec.detections().cpu().numpy()), _sorted(plain.detections().cpu().numpy()))
    states = rec.states.cpu().numpy()
    hs = hs_all[idx]
    bits = det_bits(rec.detections().cpu().numpy(), {int(r): i for i, r in enumerate(idx)}, len(idx), R + 1)
    osc = oracle_lib.OracleScene.of(s)
    rcv_np = np.asarray(s.rcv, np.float32)
    out = replay(oracle_lib, osc, s.vtx, s.tri, states, hs, bits, lambda i: rcv_np,
                 np.full(len(idx), lim), R, s.diag())
    _check(out, "%s (%d rays, longest %d segments)" % (name, len(idx), int(lens[idx].max())))
    assert out["n_queries"] >= len(idx) and (n_long == 0 or lens[idx].max() >= 20)


def test_replay_of_benchmarked_batch(rt, oracle_lib):
    rooms = synth.batched_rooms(seed=4)
    R, T, c = rooms[0].max_reflections, rooms[0].ir_seconds, rooms[0].c
    scenes = [rt.Scene.from_synth(r, device=DEV) for r in rooms]
    jobs = []
    for i, r in enumerate(rooms):
        for p in range(len(r.src)):
            jobs.append(dict(scene=i, src=r.src[p], rcv=r.rcv[p:p + 1], n_rays=r.n_rays,
                             max_path_length=c * T + float(r.rcv[p, 3])))
    b = rt.Batch(scenes, jobs, device=DEV)
    tune = dict(waves_per_simd=4, blocks_per_cu=8, fetch_threshold=16, shade_threshold=16)
    plain = rt.trace_batch(b, R, det_cap=2 * b.n_rays, **tune)
    rng = np.random.default_rng(406)
    idx, job_of = [], []
    for j, job in enumerate(jobs):
        for q in np.sort(rng.choice(job["n_rays"], 6, replace=False)):
            idx.append(int(b.ray_off[j]) + int(q))
            job_of.append(j)
    idx = np.array(idx)
    job_of = np.array(job_of)
    rows = np.full(b.n_rays, -1, np.int32)
    rows[idx] = np.arange(len(idx), dtype=np.int32)
    rec = rt.trace_batch(b, R, det_cap=2 * b.n_rays, record_rows=torch.as_tensor(rows, device=DEV), **tune)
    assert torch.equal(rec.hit_seq, plain.hit_seq)
    assert torch.equal(rec.counters[:3], plain.counters[:3]) and int(rec.counters[3]) == 0
    assert np.array_equal(_sorted(rec.detections().cpu().numpy()), _sorted(plain.detections().cpu().numpy()))
    states = rec.states.cpu().numpy()
    hs = rec.hit_seq[torch.as_tensor(idx, device=DEV)].cpu().numpy()
    rcv_off = np.array([b.rcv_off[j] for j in job_of])
    bits = det_bits(rec.detections().cpu().numpy(), {int(r): i for i, r in enumerate(idx)}, len(idx), R + 1,
                    rcv_off=rcv_off)
    tot = dict(n_queries=0, n_flagged=0, n_flagged_mismatch=0, problems=[])
    for i, r in enumerate(rooms):
        sel = np.nonzero(np.array([jobs[j]["scene"] for j in job_of]) == i)[0]
        osc = oracle_lib.OracleScene.of(r)
        rcv_rows = {int(k): np.asarray(jobs[job_of[k]]["rcv"], np.float32) for k in sel}
        lim = np.array([float(np.float32(jobs[job_of[k]]["max_path_length"])) for k in sel])
        out = replay(oracle_lib, osc, r.vtx, r.tri, states[sel], hs[sel], bits[sel],
                     lambda q, sel=sel, rcv_rows=rcv_rows: rcv_rows[int(sel[q])], lim, R, r.diag())
        for key in ("n_queries", "n_flagged", "n_flagged_mismatch"):
            tot[key] += out[key]
        tot["problems"] += ["room %d: %s" % (i, p) for p in out["problems"]]
    _check(tot, "rooms batch (%d rays of %d pairs)" % (len(idx), len(jobs)))
    assert tot["n_queries"] >= len(idx)
