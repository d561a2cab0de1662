"""Checkpoint / resume of the oracle's propagation (section "Standard
algorithm": from one reflection to the next the iteration carries only the
ray's position, direction, travelled length and the plane it leaves).

Tracing R reflections in one call equals tracing k of them, then continuing
from the recorded state after reflection k: hit sequences, detections, flags
and states are bitwise equal, including rays that stop on the path-length
limit in the continued call.  A resume that forgets the plane the ray is
leaving (it would re-hit it at delta ~ 0), restarts the travelled length, or
lets rays that already stopped go on, fails here.
"""
import numpy as np
import pytest

import synth


def _continued(ref, k, max_len):
    """Rays whose segment k was traced by the one-shot call."""
    hs = ref["hit_seq"]
    alive = hs[:, k - 1] >= 0
    if max_len > 0:
        alive &= ref["states"][:, k, 6] < max_len
    return np.nonzero(alive)[0]


@pytest.mark.parametrize("name,k,max_len", [("c1", 1, 0.0), ("c1", 5, 0.0), ("c1", 9, 60.0),
                                            ("lroom", 4, 0.0), ("open", 1, 0.0)])
def test_resume_equals_one_shot(oracle_lib, name, k, max_len):
    if name == "c1":
        s = synth.shoebox_c1()
        vtx, tri, pid = s.vtx, s.tri, s.plane_id
        src, rcv, R, N = s.src, s.rcv, 12, 3000
    elif name == "lroom":
        vtx, tri, _, pid = synth.lroom()
        src = np.array([2.0, 1.5, 1.2], np.float32)
        rcv = np.array([[6.5, 1.0, 1.5, 0.4], [1.0, 5.0, 2.0, 0.3]], np.float32)
        R, N = 10, 2000
    else:   # open box: floor and two walls only, most rays escape after a few reflections
        s = synth.shoebox_c1()
        keep = np.isin(s.plane_id, np.unique(s.plane_id)[:3])
        vtx, tri = s.vtx, s.tri[keep]
        pid = np.searchsorted(np.nonzero(keep)[0], s.plane_id[keep]).astype(np.int32)
        src, rcv, R, N = s.src, s.rcv, 8, 3000
    sc = oracle_lib.OracleScene(vtx, tri, pid)
    dirs = oracle_lib.fibonacci(N)
    ref = oracle_lib.trace(sc, src, dirs, rcv, R, max_len=max_len, states=True)
    idx = _continued(ref, k, max_len)
    assert len(idx) > N // 4
    res = oracle_lib.trace_from(sc, ref["states"][idx, k], rcv, R - k, max_len=max_len, states=True)
    assert np.array_equal(res["hit_seq"], ref["hit_seq"][idx, k:])
    assert np.array_equal(res["det"], ref["det"][idx, k:])
    assert np.array_equal(res["flags"], ref["flags"][idx, k:])
    assert np.array_equal(res["states"], ref["states"][idx, k:], equal_nan=True)
    ended = (ref["hit_seq"][idx, -1] < 0).sum()
    if max_len > 0:
        # some continued rays end on the length limit, not on R
        L_end = np.nanmax(ref["states"][idx, :, 6], axis=1)
        assert (L_end >= max_len).sum() > 10
    if name == "open":
        assert ended > len(idx) // 2                    # most continued rays escape
    # segments 0..k-1 of those rays are untouched by the resume
    assert np.all(ref["hit_seq"][idx, :k] >= 0)
