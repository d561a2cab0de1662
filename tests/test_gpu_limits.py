"""Sizes at the documented limits and just past them.

* 32 receivers (the most a call takes) on the shoebox: trajectories equal the
  oracle's or first differ at a query it flags, and all 32 detection bits of
  the agreeing rays are equal; 33 receivers are rejected.
* R = 4095 reflections (the largest accepted) in the paper's closed box:
  every ray runs all 4096 segments without escaping; the first 40 segments
  follow the oracle's trajectories (FP32 and FP64 paths drift apart over
  thousands of bounces, so later segments are checked for validity only);
  R = 4096 is rejected.
* Leaves of 8 triangles (the largest) against leaves of 1: the nearest hit
  does not depend on the tree, so hit sequences and detections are
  identical; a leaf size of 9 is rejected.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def rt():
    import paper_1811_05784_amd as m
    m.load()
    return m


def _first_divergences_flagged(hs, ref, upto):
    diff = (hs[:, :upto] != ref["hit_seq"][:, :upto]).any(axis=1)
    for i in np.nonzero(diff)[0]:
        k = int(np.argmax(hs[i, :upto] != ref["hit_seq"][i, :upto]))
        assert ref["flags"][i, : k + 1].any(), "unflagged divergence of ray %d at segment %d" % (i, k)
    return diff


def test_thirty_two_receivers(rt, oracle_lib):
    s = synth.shoebox_c1()
    rng = np.random.default_rng(32)
    lo = s.vtx.min(0) + 0.5
    hi = s.vtx.max(0) - 0.5
    rcv = np.concatenate([rng.uniform(lo, hi, size=(32, 3)), rng.uniform(0.2, 0.8, size=(32, 1))], 1)
    rcv = rcv.astype(np.float32)
    sc = rt.Scene.from_synth(s, device=DEV)
    N, R = 5000, 12
    dirs = oracle_lib.fibonacci(N)
    tr = rt.trace_rays(sc, dirs, rcv, R, src=s.src)
    ref = oracle_lib.trace(oracle_lib.OracleScene.of(s), s.src, dirs, rcv, R)
    hs = tr.hit_seq.cpu().numpy()
    diff = _first_divergences_flagged(hs, ref, R + 1)
    good = ~diff & ~ref["flags"].any(axis=1)
    det = tr.detections().cpu().numpy()
    assert det[:, 2].max() == 31
    gbits = np.zeros_like(ref["det"])
    np.bitwise_or.at(gbits, (det[:, 0], det[:, 1]), (np.uint32(1) << det[:, 2].astype(np.uint32)))
    assert np.array_equal(gbits[good], ref["det"][good]) and good.mean() > 0.98
    with pytest.raises(rt.RtError):
        rt.trace_rays(sc, dirs[:10], np.concatenate([rcv, rcv[:1]]), R, src=s.src)


def test_longest_chains(rt, oracle_lib):
    s = synth.paper_box(n_rays=256)
    sc = rt.Scene.from_synth(s, device=DEV)
    N, R = 256, 4095
    dirs = oracle_lib.fibonacci(N)
    tr = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src)
    hs = tr.hit_seq.cpu().numpy()
    assert hs.shape == (N, R + 1) and (hs >= 0).all() and (hs < s.n_tri).all()
    assert int(tr.counters[1]) == N * (R + 1) and int(tr.counters[2]) == 0 and int(tr.counters[3]) == 0
    ref = oracle_lib.trace(oracle_lib.OracleScene.of(s), s.src, dirs, s.rcv, 39)
    _first_divergences_flagged(hs, ref, 40)
    # consecutive hits lie on different walls (the plane just left is excluded)
    pid = s.plane_id[hs]
    assert (pid[:, 1:] != pid[:, :-1]).all()
    with pytest.raises(rt.RtError):
        rt.trace_rays(sc, dirs[:4], s.rcv, 4096, src=s.src)


def test_leaf_size_eight_equals_one(rt):
    s = synth.tessellated_box_c2(jitter=True)
    one = rt.Scene.from_synth(s, leaf_size=1, device=DEV)
    eight = rt.Scene.from_synth(s, leaf_size=8, device=DEV)
    assert eight.n_nodes < one.n_nodes
    dirs = rt.fibonacci_directions(50_000, device=DEV)
    a = rt.trace_rays(one, dirs, s.rcv, 20, src=s.src)
    b = rt.trace_rays(eight, dirs, s.rcv, 20, src=s.src)
    assert torch.equal(a.hit_seq, b.hit_seq) and torch.equal(a.counters[:3], b.counters[:3])
    da, db = a.detections().cpu().numpy(), b.detections().cpu().numpy()
    assert np.array_equal(da[np.lexsort(da.T[::-1])], db[np.lexsort(db.T[::-1])])
    with pytest.raises(rt.RtError):
        rt.Scene.from_synth(s, leaf_size=9, device=DEV)
