"""GPU parity of the source variants (rt_icosahedral_directions,
rt_directional_directions) with the FP64 oracle, and ray propagation from
them.

Both sides evaluate the documented FP64 formula without contraction and
round once; the icosahedral grid uses only correctly rounded operations in
the same order, so the rows are bit-equal.  The directional source also
calls cos, sin and pow, where the device library and the host's may differ
by one FP64 ulp: rows within 1 FP32 ulp, nearly all bit-equal."""
import sys

import numpy as np
import pytest
import torch

import synth
from tests._util import ulp_diff

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


@pytest.mark.parametrize("f", [1, 2, 3, 17, 64, 100])
def test_icosahedral_matches_oracle(rt, oracle_lib, f):
    g = rt.icosahedral_directions(f, device=DEV).cpu().numpy()
    o = oracle_lib.icosahedral(f)
    _say("icosahedral f=%d rows=%d" % (f, len(g)))
    assert g.shape == o.shape == (10 * f * f + 2, 3)
    assert np.array_equal(g, o)


@pytest.mark.parametrize("n,m,axis", [(1, 0.0, [0, 0, 1]), (7, 3.0, [0, 1, 0]), (10_000, 0.0, [0, 0, 1]),
                                      (50_001, 1.0, [1, 2, -0.5]), (65_536, 2.5, [0.95, 0.1, 0.0]),
                                      (100_003, 8.0, [-1, 0, 0])])
def test_directional_matches_oracle(rt, oracle_lib, n, m, axis):
    g = rt.directional_directions(n, m, axis, device=DEV).cpu().numpy()
    o = oracle_lib.directional(n, m, axis)
    d = ulp_diff(g, o)
    _say("directional n=%d m=%g: max ulp %d, equal %.6f" % (n, m, int(d.max()), float((d == 0).mean())))
    assert d.max() <= 1 and (d == 0).mean() > 0.999


def test_source_variant_errors(rt):
    with pytest.raises(rt.RtError):
        rt.icosahedral_directions(0, device=DEV)
    with pytest.raises(rt.RtError):
        rt.directional_directions(10, -1.0, [0, 0, 1], device=DEV)
    with pytest.raises(rt.RtError):
        rt.directional_directions(10, 1.0, [0, 0, 0], device=DEV)
    with pytest.raises(rt.RtError):
        rt.directional_directions(10, float("nan"), [0, 0, 1], device=DEV)
    assert rt.directional_directions(0, 1.0, [0, 0, 1], device=DEV).shape == (0, 3)


@pytest.mark.parametrize("kind", ["icosahedral", "directional"])
def test_trajectories_from_source_variants_match_oracle(rt, oracle_lib, kind):
    """The shoebox traced from each variant's directions (the oracle's own
    rows): hit sequences equal the oracle's or first differ at a flagged
    query; detections equal on the agreeing, unflagged rays."""
    s = synth.shoebox_c1()
    sc = rt.Scene.from_synth(s, device=DEV)
    if kind == "icosahedral":
        dirs = oracle_lib.icosahedral(31)                     # 9,612 rays
    else:
        dirs = oracle_lib.directional(10_000, 2.0, s.rcv[0, :3] - s.src)
    R = s.max_reflections
    tr = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=s.max_path_length)
    hs = tr.hit_seq.cpu().numpy()
    ref = oracle_lib.trace(oracle_lib.OracleScene.of(s), s.src, dirs, s.rcv, R, max_len=s.max_path_length)
    diff = (hs != ref["hit_seq"]).any(axis=1)
    for i in np.nonzero(diff)[0]:
        k = int(np.argmax(hs[i] != ref["hit_seq"][i]))
        assert ref["flags"][i, : k + 1].any(), "unflagged divergence, ray %d" % i
    good = ~diff & ~ref["flags"].any(axis=1)
    det = tr.detections().cpu().numpy()
    gbits = np.zeros_like(ref["det"])
    np.bitwise_or.at(gbits, (det[:, 0], det[:, 1]), (np.uint32(1) << det[:, 2].astype(np.uint32)))
    assert np.array_equal(gbits[good], ref["det"][good])
    assert good.mean() > 0.98
    _say("%s: rays %d, detections %d, differing %d" % (kind, len(hs), len(det), int(diff.sum())))
