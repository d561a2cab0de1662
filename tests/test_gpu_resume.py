"""Checkpoint / resume on the GPU (section "Standard algorithm": from one
reflection to the next a ray carries only its position, direction, travelled
length and the plane it leaves).  One call traces R reflections with every
state recorded; a second call continues the rays still going after
reflection k from the recorded state after it (origins, dirs, start_plane,
start_len) with R - k reflections left.  Its hit sequences and detections must
equal the one-shot call's from segment k on, bit for bit.  The travelled length
is carried in FP64 inside a call but recorded in FP32, so with a path-length
limit a ray may stop one segment apart only where its length at the limit
lies within FP32 rounding of it (checked)."""
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


def _sorted(d):
    return d[np.lexsort(d.T[::-1])]


@pytest.mark.parametrize("name,n,R,k,mpl", [("c2", 50_000, 20, 5, 0.0), ("c3", 200_000, 60, 3, 0.0),
                                            ("c2", 50_000, 20, 7, 60.0), ("c1", 10_000, 20, 1, 0.0)])
def test_resume_equals_one_shot(rt, name, n, R, k, mpl):
    s = {"c1": synth.shoebox_c1, "c2": lambda: synth.tessellated_box_c2(jitter=True), "c3": synth.theater_c3}[name]()
    sc = rt.Scene.from_synth(s, device=DEV)
    dirs = rt.fibonacci_directions(n, device=DEV)
    one = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl, record_states=True, det_cap=8 * n)
    hs = one.hit_seq.cpu().numpy()
    st = one.states.cpu().numpy()
    lim = np.float32(mpl) if mpl > 0 else np.float32(np.inf)
    alive = (hs[:, k - 1] >= 0) & (st[:, k, 6] < lim)
    idx = np.nonzero(alive)[0]
    assert len(idx) > 100
    sk = st[idx, k]
    res = rt.trace_rays(sc, np.ascontiguousarray(sk[:, 3:6]), s.rcv, R - k, origins=np.ascontiguousarray(sk[:, 0:3]),
                        start_plane=sk[:, 7].copy().view(np.int32), start_len=np.ascontiguousarray(sk[:, 6]),
                        max_path_length=mpl, det_cap=8 * n)
    got = res.hit_seq.cpu().numpy()
    want = hs[idx, k:]
    d1 = one.detections().cpu().numpy()
    d1 = d1[d1[:, 1] >= k]
    pos = np.full(n, -1)
    pos[idx] = np.arange(len(idx))
    assert np.all(pos[d1[:, 0]] >= 0)
    d1 = np.stack([pos[d1[:, 0]], d1[:, 1] - k, d1[:, 2]], 1)
    d2 = res.detections().cpu().numpy()
    differ = np.nonzero((got != want).any(axis=1))[0]
    if mpl > 0:
        # only at the limit: one of the one-shot ray's recorded FP32 lengths
        # lies within rounding of the limit
        for i in differ:
            Ls = st[idx[i], k:, 6]
            near = np.abs(Ls.astype(np.float64) - float(lim)) <= 4 * float(np.spacing(lim))
            assert near.any(), i
        keep = np.setdiff1d(np.arange(len(idx)), differ)
        d1 = d1[np.isin(d1[:, 0], keep)]
        d2 = d2[np.isin(d2[:, 0], keep)]
        assert len(differ) <= 5
    else:
        assert len(differ) == 0
    assert np.array_equal(_sorted(d1), _sorted(d2))
    if name == "c3":
        assert (got[:, 0] >= 0).sum() > 0 and (got < 0).any()
