"""GPU parity of ray generation and ray propagation against the FP64 oracle.

* Fibonacci directions: FP64 on both sides, rounded once; the two libms may
  differ by one FP64 ulp in cos/sin, so FP32 results agree to <= 1 ulp.
* One-segment queries from seeded states (on-surface origins excluding their
  own plane, interior origins): the nearest-hit triangle must equal the
  oracle's unless the oracle flags the query, and then the GPU's triangle must
  be crossed within eps D of it and not beyond the oracle's hit by more than
  eps D (an escape only with an edge or near-miss flag); the detections must
  equal the oracle's unless the oracle flags a near-tangent receiver or the
  hit changed; the next state
  (o', u', L') is FP64 rounded once on the GPU, so it is within 1 FP32 ulp of
  the oracle's FP64 value (plus the FP32 rounding of sub-ulp differences in
  delta: a tolerance of 2 ulp of the coordinate magnitude, relative 1e-9 of
  the step for values near zero).
* Full trajectories on the 12-triangle shoebox from the same FP32 directions:
  every ray's hit sequence equals the oracle's, or first differs at a query
  the oracle flags.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from tests._util import crossing_and_miss, gpu_is_dict, skips_only_at_boundaries, ulp_diff

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
def scenes(rt):
    out = {}
    for name, mk in [("c1", synth.shoebox_c1), ("c2", lambda: synth.tessellated_box_c2(jitter=True)),
                     ("c2flat", lambda: synth.tessellated_box_c2(jitter=False)), ("c3", synth.theater_c3)]:
        s = mk()
        out[name] = (s, rt.Scene.from_synth(s, device="cuda:0"))
    return out


@pytest.mark.parametrize("n", [1, 7, 1000, 65_537, 1_000_000])
def test_fibonacci_matches_oracle(rt, oracle_lib, n):
    _say("fibonacci n=%d" % n)
    g = rt.fibonacci_directions(n, device="cuda:0").cpu().numpy()
    o = oracle_lib.fibonacci(n)
    d = ulp_diff(g, o)
    assert d.max() <= 1
    assert (d == 0).mean() > 0.9999


def test_build_tree_reports(rt, scenes):
    for name, (s, sc) in scenes.items():
        _say("scene", name, sc.n_tri, sc.n_ref, sc.n_nodes, sc.depth, sc.n_mat)
        assert sc.n_tri == s.n_tri and sc.n_mat == s.n_mat
        assert abs(sc.diag - s.diag()) < 1e-5 * s.diag()
        assert s.n_tri <= sc.n_ref <= 64 * s.n_tri
        assert 1 <= sc.n_nodes <= sc.n_ref and 1 <= sc.depth <= 64


def test_build_tree_rejects_bad_meshes(rt):
    s = synth.shoebox_c1()
    bad_idx = s.tri.copy()
    bad_idx[3, 1] = 99
    with pytest.raises(rt.RtError, match="index"):
        rt.Scene(s.vtx, bad_idx, s.material, s.plane_id)
    degenerate = s.vtx.copy()
    t = s.tri[0]
    degenerate[t[1]] = degenerate[t[0]]
    with pytest.raises(rt.RtError):
        rt.Scene(degenerate, s.tri, s.material, s.plane_id)
    plane = s.plane_id.copy()
    plane[plane == plane[2]] = plane[0]          # two walls claimed coplanar
    with pytest.raises(rt.RtError, match="plane"):
        rt.Scene(s.vtx, s.tri, s.material, plane)
    mat = s.material.copy()
    mat[1] = (mat[0] + 1) % 6                    # same wall, two materials
    with pytest.raises(rt.RtError, match="material"):
        rt.Scene(s.vtx, s.tri, mat, s.plane_id)
    nan = s.vtx.copy()
    nan[0, 0] = np.nan
    with pytest.raises(rt.RtError):
        rt.Scene(nan, s.tri, s.material, s.plane_id)


def _query_parity(rt, oracle_lib, s, sc, o, u, lp, L, tag):
    n = len(o)
    tr = rt.trace_rays(sc, u, s.rcv, 1, origins=o, start_plane=lp, start_len=L, record_states=True)
    hit = tr.hit_seq[:, 0].cpu().numpy()
    det = tr.detections().cpu().numpy()
    gdet = np.zeros(n, np.uint32)
    d0 = det[det[:, 1] == 0]
    np.bitwise_or.at(gdet, d0[:, 0], (np.uint32(1) << d0[:, 2].astype(np.uint32)))
    nxt = tr.states[:, 1, :7].cpu().numpy()
    osc = oracle_lib.OracleScene.of(s)
    ref = oracle_lib.query_batch(osc, o, u, lp, L, s.rcv)
    flagged = ref["flags"] != 0
    bad_hit = (hit != ref["hit"]) & ~flagged
    # a detection mismatch is excused only by a near-tangent receiver or a changed hit
    tangent = (ref["flags"] & oracle_lib.FLAG_TANGENT) != 0
    bad_det = (gdet != ref["det"]) & ~(tangent | (hit != ref["hit"]))
    # a flagged hit mismatch must still be a valid answer within eps D
    epsD = 1e-6 * s.diag()
    for i in np.nonzero((hit != ref["hit"]) & flagged)[0]:
        if hit[i] >= 0:
            v = s.tri[hit[i]]
            t, miss = crossing_and_miss(o[i], u[i], s.vtx[v[0]], s.vtx[v[1]], s.vtx[v[2]])
            far = ref["delta"][i] if ref["hit"][i] >= 0 else np.inf
            # at most eps D beyond the oracle's hit, or beyond it only past triangles
            # crossed within eps D of their boundary (an open edge or vertex seam)
            assert t[0] > 0 and miss[0] <= epsD, (tag, i, t[0], miss[0], far)
            assert t[0] <= far + epsD or skips_only_at_boundaries(o[i], u[i], t[0], s.vtx, s.tri, epsD), (
                tag, i, t[0], far)
        else:
            assert ref["flags"][i] & (oracle_lib.FLAG_EDGE | oracle_lib.FLAG_NEAR_MISS), (tag, i)
            assert skips_only_at_boundaries(o[i], u[i], np.inf, s.vtx, s.tri, epsD), (tag, i)
    both = (hit == ref["hit"]) & (hit >= 0)
    on = ref["next"][both]
    gn = nxt[both]
    mag = np.maximum(np.abs(on[:, :3]), np.abs(o[both]).astype(np.float64)).max(1, keepdims=True)
    ulp_o = np.spacing(mag.astype(np.float32)).astype(np.float64)
    err_o = np.abs(gn[:, :3] - on[:, :3])
    err_u = ulp_diff(gn[:, 3:6], on[:, 3:6].astype(np.float32))
    err_L = np.abs(gn[:, 6] - on[:, 6]) / np.spacing(np.abs(on[:, 6]).astype(np.float32))
    _say("%s: n=%d flagged=%d hit-mismatch(flagged)=%d unflagged hit=%d det=%d escapes=%d max|do|/ulp=%.2f "
         "max du ulp=%d max dL ulp=%.2f" % (tag, n, flagged.sum(), ((hit != ref["hit"]) & flagged).sum(),
                                          bad_hit.sum(), bad_det.sum(), (hit < 0).sum(),
                                          (err_o / ulp_o).max() if len(gn) else 0,
                                          err_u.max() if len(gn) else 0, err_L.max() if len(gn) else 0))
    assert bad_hit.sum() == 0
    assert bad_det.sum() == 0
    assert np.all(err_o <= 2 * ulp_o)
    assert err_u.max() <= 2
    assert np.all(err_L <= 2)
    assert int(tr.counters[3]) == 0
    return flagged.mean()


@pytest.mark.parametrize("name,n", [("c1", 20_000), ("c2", 30_000), ("c2flat", 20_000), ("c3", 8_000)])
def test_surface_query_parity(rt, oracle_lib, scenes, name, n):
    s, sc = scenes[name]
    toward = (5.0, 3.5, 1.5) if name.startswith("c") and name != "c3" else None
    o, u, lp, L = synth.surface_query_states(s, n, seed=100 + n, toward=toward)
    frac = _query_parity(rt, oracle_lib, s, sc, o, u, lp, L, "surface " + name)
    assert frac < 0.02


@pytest.mark.parametrize("name,n", [("c2", 20_000), ("c3", 8_000)])
def test_interior_query_parity(rt, oracle_lib, scenes, name, n):
    s, sc = scenes[name]
    o, u, lp, L = synth.interior_query_states(s, n, seed=7 + n)
    _query_parity(rt, oracle_lib, s, sc, o, u, lp, L, "interior " + name)


@pytest.mark.parametrize("name", ["c2flat", "c3"])
def test_ties_at_shared_vertices_and_edges_are_order_robust(rt, oracle_lib, scenes, name):
    """Exact FP32 ties go to the lowest triangle id whatever order the search
    takes: rays aimed at shared vertices and edge midpoints (many ties and
    near ties) give the same first hit with the per-lane walk only, with the
    cooperative search (rays traced one, three and eight per launch, so one
    wavefront searches them with 64, 16 or 8 lanes per query), with LDS stack
    depths 8 and 32, another register budget, rays in index order and the rays
    split into other launches; and the hits match the oracle's query by query
    (flagged mismatches must be valid answers)."""
    s, sc = scenes[name]
    n = 20_000
    o, u, lp, L = synth.tie_query_states(s, n, seed=23)
    _query_parity(rt, oracle_lib, s, sc, o, u, lp, L, "ties " + name)
    osc = oracle_lib.OracleScene.of(s)
    flags = oracle_lib.query_batch(osc, o, u, lp, L, s.rcv)["flags"]
    _say("ties %s: oracle tie flags %d, edge flags %d of %d" % (
        name, ((flags & oracle_lib.FLAG_TIE) != 0).sum(), ((flags & oracle_lib.FLAG_EDGE) != 0).sum(), n))

    def first_hits(idx, **kw):
        tr = rt.trace_rays(sc, u[idx], s.rcv, 0, origins=o[idx], start_plane=lp[idx], start_len=L[idx], **kw)
        assert int(tr.counters[3]) == 0
        return tr.hit_seq[:, 0].cpu().numpy()

    every = np.arange(n)
    ref = first_hits(every)
    for kw in (dict(coop_queries=-1), dict(stack_depth=8), dict(stack_depth=32), dict(waves_per_simd=5),
               dict(keep_order=True)):
        assert np.array_equal(first_hits(every, **kw), ref), kw
    for part in (every[::3], every[1::3]):
        assert np.array_equal(first_hits(part), ref[part])
    sample = np.random.default_rng(5).choice(n, 120, replace=False)
    for size in (1, 3, 8):
        for c in range(0, len(sample), size):
            idx = sample[c:c + size]
            assert np.array_equal(first_hits(idx), ref[idx]), (size, idx)


def test_c1_trajectory_parity(rt, oracle_lib, scenes):
    s, sc = scenes["c1"]
    dirs = oracle_lib.fibonacci(s.n_rays)
    tr = rt.trace_rays(sc, dirs, s.rcv, s.max_reflections, src=s.src, max_path_length=s.max_path_length)
    hs = tr.hit_seq.cpu().numpy()
    osc = oracle_lib.OracleScene.of(s)
    ref = oracle_lib.trace(osc, s.src, dirs, s.rcv, s.max_reflections, max_len=s.max_path_length)
    diff = (hs != ref["hit_seq"]).any(axis=1)
    unflagged = 0
    for i in np.nonzero(diff)[0]:
        k = int(np.argmax(hs[i] != ref["hit_seq"][i]))
        if not ref["flags"][i, : k + 1].any():
            unflagged += 1
    # detections of rays whose whole sequence agrees and is unflagged
    good = ~diff & ~ref["flags"].any(axis=1)
    det = tr.detections().cpu().numpy()
    gbits = np.zeros_like(ref["det"])
    np.bitwise_or.at(gbits, (det[:, 0], det[:, 1]), (np.uint32(1) << det[:, 2].astype(np.uint32)))
    det_bad = (gbits[good] != ref["det"][good]).any(axis=1).sum()
    _say("c1 trajectories: rays=%d differing=%d unflagged-first-divergence=%d flagged-rays=%d det-bad=%d "
         "queries=%d" % (len(hs), diff.sum(), unflagged, ref["flags"].any(axis=1).sum(), det_bad,
                         int(tr.counters[1])))
    assert unflagged == 0
    assert det_bad == 0
    # closed room: nothing escapes, every ray ends by the path-length stop or R
    assert int(tr.counters[2]) == 0
    assert int(tr.counters[1]) == int((hs >= 0).sum())


def test_determinism_and_batch_invariance(rt, scenes):
    s, sc = scenes["c2"]
    dirs = rt.fibonacci_directions(50_000, device="cuda:0")
    a = rt.trace_rays(sc, dirs, s.rcv, 20, src=s.src)
    b = rt.trace_rays(sc, dirs, s.rcv, 20, src=s.src, shade_threshold=1, fetch_threshold=1, blocks_per_cu=1)
    assert torch.equal(a.hit_seq, b.hit_seq)
    sub = torch.arange(123, 50_000, 977, device="cuda:0")
    c = rt.trace_rays(sc, dirs[sub], s.rcv, 20, src=s.src)
    assert torch.equal(c.hit_seq, a.hit_seq[sub])
    da = a.detections().cpu().numpy()
    db = b.detections().cpu().numpy()
    sa = da[np.lexsort(da.T[::-1])]
    sb = db[np.lexsort(db.T[::-1])]
    assert np.array_equal(sa, sb)


def test_edge_cases(rt, scenes):
    s, sc = scenes["c1"]
    # no rays
    tr = rt.trace_rays(sc, np.zeros((0, 3), np.float32), s.rcv, 3, src=s.src)
    assert tr.hit_seq.shape == (0, 4) and int(tr.counters[1]) == 0
    # R = 0: one segment each; a zero direction escapes without detections
    d = np.array([[1, 0, 0], [0, 0, 0], [0, 0.6, 0.8]], np.float32)
    tr = rt.trace_rays(sc, d, s.rcv, 0, src=s.src)
    hs = tr.hit_seq.cpu().numpy()
    assert hs.shape == (3, 1) and hs[0, 0] >= 0 and hs[1, 0] == -1 and hs[2, 0] >= 0
    assert int(tr.counters[1]) == 3 and int(tr.counters[2]) == 1
    # single-triangle open scene: rays miss and escape
    one = rt.Scene(np.array([[0, 0, 5], [1, 0, 5], [0, 1, 5]], np.float32), np.array([[0, 1, 2]], np.int32),
                   np.zeros(1, np.int32))
    d = np.array([[0.04, 0.04, 1.0], [0, 0, -1.0], [0.02, 0.1, 1.0]], np.float32)
    tr = rt.trace_rays(one, d, np.array([[0, 0, -3, 0.8]], np.float32), 4, src=np.zeros(3))
    hs = tr.hit_seq.cpu().numpy()
    assert hs[0, 0] == 0 and hs[0, 1] == -1 and hs[1, 0] == -1 and hs[2, 0] == 0
    assert int(tr.counters[0]) == 2           # ray 0 after its reflection, ray 1 directly
    # detection capacity overflow: reported and retried by the wrapper
    dirs = rt.fibonacci_directions(20_000, device="cuda:0")
    small = rt.trace_rays(sc, dirs, s.rcv, 20, src=s.src, det_cap=16, check_capacity=False)
    need = int(small.counters[0])
    assert need > 16
    full = rt.trace_rays(sc, dirs, s.rcv, 20, src=s.src, det_cap=16)
    assert full.n_det() == need and full.det.shape[0] >= need


def _sorted_det(tr):
    d = tr.detections().cpu().numpy()
    return d[np.lexsort(d.T[::-1])]


@pytest.mark.parametrize("name,R,n,kw", [("c2", 20, 50_000, dict(suspend_after=1)),
                                         ("c2", 20, 50_000, dict(suspend_after=3)),
                                         ("c2", 20, 50_000, dict(suspend_after=20)),
                                         ("c2", 20, 50_000, dict(rounds=3, spill_threshold=40)),
                                         ("c3", 60, 200_000, dict(suspend_after=2)),
                                         ("c1", 20, 10_000, dict(coop_queries=-1)),
                                         ("c2", 20, 50_000, dict(coop_queries=-1)),
                                         ("c3", 60, 1_000_000, dict(coop_queries=-1)),
                                         ("c3", 60, 1_000_000, dict(coop_queries=-1, xcd_pools=-1)),
                                         ("c3", 60, 1_000_000, dict(stack_depth=8)),
                                         ("c3", 60, 1_000_000, dict(stack_depth=32, waves_per_simd=5)),
                                         ("c2", 20, 50_000, dict(stack_depth=8, waves_per_simd=5)),
                                         ("c2", 20, 50_000, dict(stack_depth=32))])
def test_scheduling_leaves_results_unchanged(rt, scenes, name, R, n, kw):
    """Suspension into a second launch, continuation rounds, per-XCD pools,
    single queries searched by whole wavefronts, other register budgets and
    LDS stack depths (8: the cooperative frontier holds 4 entries per lane)
    reorder work only: hit sequences, detections and counters are identical."""
    s, sc = scenes[name]
    dirs = rt.fibonacci_directions(n, device="cuda:0")
    mpl = s.max_path_length if name == "c3" else 0.0
    a = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl)
    b = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl, **kw)
    assert torch.equal(a.hit_seq, b.hit_seq)
    assert torch.equal(a.counters[:3], b.counters[:3]) and int(b.counters[3]) == 0
    assert np.array_equal(_sorted_det(a), _sorted_det(b))


def test_trace_before_scene_info_matches_after(rt):
    """rt_build_tree returns before its last kernels finish; a trace launched
    right away uses the node capacity and a depth bound, and must give the same
    results as one launched after rt_scene_info has read the exact node count
    and depth back (which lie within that capacity and bound)."""
    s = synth.tessellated_box_c2(jitter=True)
    sc = rt.Scene.from_synth(s, device="cuda:0")
    dirs = rt.fibonacci_directions(50_000, device="cuda:0")
    a = rt.trace_rays(sc, dirs, s.rcv, 20, src=s.src)
    n_nodes, depth, n_ref = sc.n_nodes, sc.depth, sc.n_ref
    assert 1 <= n_nodes <= n_ref - 1 and 1 <= depth <= 40 and n_ref >= s.n_tri
    b = rt.trace_rays(sc, dirs, s.rcv, 20, src=s.src)
    assert torch.equal(a.hit_seq, b.hit_seq)
    assert torch.equal(a.counters[:3], b.counters[:3]) and int(a.counters[3]) == 0 and int(b.counters[3]) == 0
    assert np.array_equal(_sorted_det(a), _sorted_det(b))


def test_trace_rays_graph_replay_matches_eager(rt, scenes):
    """rt_trace_rays captured in a HIP graph (reset, ray ordering, -1 fill of
    the hit rows, traversal): every replay, after eager work has zeroed the
    rows, equals the eager call."""
    s, sc = scenes["c2"]
    n, R = 50_000, 20
    dirs = rt.fibonacci_directions(n, device="cuda:0")
    rcv = torch.as_tensor(s.rcv, device="cuda:0")
    tr = rt.trace_rays(sc, dirs, rcv, R, src=s.src, det_cap=8 * n)
    torch.cuda.synchronize()
    ref_hs, ref_c, ref_det = tr.hit_seq.clone(), tr.counters[:3].clone(), _sorted_det(tr)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rt.trace_rays(sc, dirs, rcv, R, src=s.src, out=tr, check_capacity=False)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rt.trace_rays(sc, dirs, rcv, R, src=s.src, out=tr, check_capacity=False)
    for rep in range(3):
        tr.hit_seq.zero_()
        _ = torch.randn(1000, device="cuda:0").sum()     # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(tr.hit_seq, ref_hs), rep
        assert torch.equal(tr.counters[:3], ref_c) and int(tr.counters[3]) == 0, rep
        assert np.array_equal(_sorted_det(tr), ref_det), rep


@pytest.mark.parametrize("name,R,n", [("c1", 20, 300), ("c2", 50, 3_000), ("c3", 60, 5_000)])
def test_cooperative_search_small_calls(rt, scenes, name, R, n):
    """With few rays per wavefront the pool is empty at once, and many
    wavefronts end with one or two queries searched by all their lanes: the
    results equal those of the per-lane walk."""
    s, sc = scenes[name]
    dirs = rt.fibonacci_directions(n, device="cuda:0")
    mpl = s.max_path_length if name == "c3" else 0.0
    a = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl, coop_queries=-1)
    b = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl)
    assert torch.equal(a.hit_seq, b.hit_seq)
    assert torch.equal(a.counters[:3], b.counters[:3]) and int(b.counters[3]) == 0
    assert np.array_equal(_sorted_det(a), _sorted_det(b))


def test_cooperative_search_grazing_rays(rt, scenes):
    """Rays skimming the jittered floor of the 100k-triangle box within the
    jitter band cross many leaf boxes at once (wide frontiers for the
    breadth-first search of the last queries).  Results equal those of the
    per-lane walk."""
    s, sc = scenes["c2"]
    rng = np.random.default_rng(77)
    n = 2_000
    org = np.stack([rng.uniform(1, 9, n), rng.uniform(1, 6, n), rng.uniform(0.005, 0.04, n)], 1)
    phi = rng.uniform(0, 2 * np.pi, n)
    d = np.stack([np.cos(phi), np.sin(phi), rng.uniform(-0.004, 0.001, n)], 1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    org_t = torch.as_tensor(org.astype(np.float32), device="cuda:0")
    dirs = torch.as_tensor(d.astype(np.float32), device="cuda:0")
    a = rt.trace_rays(sc, dirs, s.rcv, 6, origins=org_t, coop_queries=-1)
    b = rt.trace_rays(sc, dirs, s.rcv, 6, origins=org_t)
    assert torch.equal(a.hit_seq, b.hit_seq)
    assert torch.equal(a.counters[:3], b.counters[:3]) and int(b.counters[3]) == 0
    assert np.array_equal(_sorted_det(a), _sorted_det(b))
    assert int((a.hit_seq[:, 0] >= 0).sum()) > n // 2


@pytest.mark.parametrize("name,R,n", [("c2", 20, 20_000), ("c3", 60, 20_000)])
def test_traversal_statistics(rt, scenes, name, R, n):
    """A call with traversal statistics gives the same results, and its counts
    are consistent: every query that hits a triangle visits the root, at least
    one leaf and tests at least one triangle."""
    s, sc = scenes[name]
    dirs = rt.fibonacci_directions(n, device="cuda:0")
    mpl = s.max_path_length if name == "c3" else 0.0
    a = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl)
    st = torch.full((4,), -1, dtype=torch.int64, device="cuda:0")
    b = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=mpl, stats=st)
    assert torch.equal(a.hit_seq, b.hit_seq) and torch.equal(a.counters[:3], b.counters[:3])
    nodes, leaves, tris, spills = st.cpu().tolist()
    hits = int(b.counters[1]) - int(b.counters[2])
    _say("stats %s: queries %d hits %d nodes %d leaves %d tris %d spills %d"
         % (name, int(b.counters[1]), hits, nodes, leaves, tris, spills))
    assert hits > 0 and nodes >= hits and leaves >= hits and tris >= hits and spills >= 0
    assert tris <= leaves * sc.leaf_size


@pytest.mark.parametrize("k", [1, 16, 91])
def test_tetra_one_iteration_matches_oracle(rt, oracle_lib, k):
    """The complexity study's workload ("Tree-base acceleration", Table 2):
    one iteration from the centre of a tessellated unit tetrahedron.  Every
    ray hits the oracle's triangle unless the oracle flags the query, and no
    ray escapes the watertight surface."""
    s = synth.tessellated_tetra(k)
    sc = rt.Scene.from_synth(s, device="cuda:0")
    n = s.n_tri
    dirs = rt.fibonacci_directions(n, device="cuda:0")
    tr = rt.trace_rays(sc, dirs, s.rcv, 0, src=s.src)
    gpu = tr.hit_seq[:, 0].cpu().numpy()
    assert int(tr.counters[2]) == 0 and np.all(gpu >= 0)
    osc = oracle_lib.OracleScene.of(s)
    q = oracle_lib.query_batch(osc, np.repeat(s.src[None, :], n, 0), oracle_lib.fibonacci(n))
    bad = (gpu != q["hit"]) & (q["flags"] == 0)
    _say("tetra k=%d M=%d flagged %d mismatches %d" % (k, n, int((q["flags"] != 0).sum()), int((gpu != q["hit"]).sum())))
    assert not bad.any()


def _trajectory_parity(rt, oracle_lib, s, sc, dirs, R, max_len, tag, **gpu_kw):
    """GPU trace vs FP64 oracle from the same FP32 directions: every ray's hit
    sequence equals the oracle's or first differs at a query the oracle
    flags; detections equal on rays that agree and are unflagged.  Returns
    the GPU result, the oracle's and the mask of those rays."""
    tr = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, **gpu_kw)
    hs = tr.hit_seq.cpu().numpy()
    ref = oracle_lib.trace(oracle_lib.OracleScene.of(s), s.src, dirs, s.rcv, R, max_len=max_len)
    diff = (hs != ref["hit_seq"]).any(axis=1)
    unflagged = sum(1 for i in np.nonzero(diff)[0]
                    if not ref["flags"][i, : int(np.argmax(hs[i] != ref["hit_seq"][i])) + 1].any())
    good = ~diff & ~ref["flags"].any(axis=1)
    det = tr.detections().cpu().numpy()
    gbits = np.zeros_like(ref["det"])
    np.bitwise_or.at(gbits, (det[:, 0], det[:, 1]), (np.uint32(1) << det[:, 2].astype(np.uint32)))
    det_bad = int((gbits[good] != ref["det"][good]).any(axis=1).sum())
    _say("%s: rays=%d differing=%d unflagged=%d flagged=%d det-bad=%d queries=%d" % (
        tag, len(hs), int(diff.sum()), unflagged, int(ref["flags"].any(axis=1).sum()), det_bad,
        int(tr.counters[1])))
    assert unflagged == 0 and det_bad == 0
    assert good.mean() > 0.98
    return tr, ref, good


@pytest.mark.parametrize("n,mpl", [(1, 0.0), (4, 0.0), (1, 9.0), (10_000, 0.0)])
def test_eq13_range_stop_matches_oracle(rt, oracle_lib, scenes, n, mpl):
    """Rays stop at the range of the discrete model, (r/2) sqrt(N/n) with the
    largest receiver radius (eq. 13), rounded to FP32, or at a shorter fixed
    path length; the oracle gets the same limit from its own eq. 13."""
    s, sc = scenes["c1"]
    N = s.n_rays
    dirs = oracle_lib.fibonacci(N)
    lim = float(np.float32(oracle_lib.range_limit(float(s.rcv[:, 3].astype(np.float64).max()), N, n)))
    if mpl > 0:
        lim = min(lim, mpl)
    R = 40
    tr, ref, good = _trajectory_parity(rt, oracle_lib, s, sc, dirs, R, lim, "eq13 n=%d mpl=%g" % (n, mpl),
                                       min_beam_rays=n, max_path_length=mpl, record_states=True)
    st = tr.states.cpu().numpy()
    hs = tr.hit_seq.cpu().numpy()
    nseg = (hs >= 0).sum(1)
    rows = np.arange(N)
    assert np.all(nseg < R + 1)                              # the range, not R, ends every ray
    assert np.all(st[rows, nseg, 6].astype(np.float64) >= lim)
    assert np.all(st[rows, nseg - 1, 6].astype(np.float64) < lim)
    assert int(tr.counters[2]) == 0


@pytest.mark.parametrize("level", [2, 3, 4])
def test_sphere_dirac_comb_matches_oracle(rt, oracle_lib, level):
    """The reflecting-sphere study ("Energy conservation by reflecting
    sphere"): 20 * 4^level flat facets, source and receiver at the centre,
    six reflections.  Trajectories, detections and image sources (keys,
    counts, positions) equal the oracle's on the rays whose trajectories
    agree and are unflagged."""
    s = synth.sphere_room(level)
    sc = rt.Scene.from_synth(s, device="cuda:0")
    N, R = 4000, 6
    dirs = oracle_lib.fibonacci(N)
    tr, ref, good = _trajectory_parity(rt, oracle_lib, s, sc, dirs, R, 0.0, "sphere level %d" % level)
    # a closed sphere loses no ray, except after a hit exactly on an edge (a
    # query the oracle flags): the ray then sits on the edge and may leave
    # through the neighbouring facet's plane
    hs = tr.hit_seq.cpu().numpy()
    assert np.all(hs[good] >= 0) and int(tr.counters[2]) <= int((~good).sum())
    det = tr.detections().cpu().numpy()
    det = det[good[det[:, 0]]]
    isrc = rt.collect_image_sources(sc, s.src, s.rcv, None, hit_seq=tr.hit_seq, det=det, max_reflections=R)
    g = gpu_is_dict(isrc)
    odet = oracle_lib.detections_from_bits(ref["det"])
    odet = odet[good[odet[:, 0]]]
    keys = oracle_lib.image_source_keys(s.plane_id, ref["hit_seq"], odet)
    assert set(g) == set(keys) and all(g[k][0] == c for k, c in keys.items())
    tab = oracle_lib.image_sources(oracle_lib.OracleScene.of(s), s.src, s.rcv, keys)
    gd = np.array([g[k][2] for k in tab["keys"]])
    gp = np.array([g[k][1] for k in tab["keys"]])
    assert np.abs(gd - tab["dist"]).max() <= 1e-9 * 16 and np.abs(gp - tab["pos"]).max() <= 1e-9 * 16


@pytest.mark.parametrize("name,n_random,n_long,min_good", [("c3", 300, 40, 0.95), ("c2", 200, 20, 0.8)])
def test_full_size_sampled(rt, oracle_lib, scenes, name, n_random, n_long, min_good):
    """The configurations at full size, default launch: the benchmarked
    theater (436,120 triangles, 10^6 Fibonacci rays, up to 60 reflections, 8
    receivers) and the jittered box (100,316 triangles, 10^6 rays, 50
    reflections, 3 receivers).  A seeded sample of rays plus the longest
    bounce chains (the drain of the launch, searched cooperatively) matches
    the oracle's trajectories, computed ray by ray from the same FP32
    directions (first difference only at a flagged query), and, on rays that
    agree and are unflagged, its detections.  In the closed box every ray
    runs 51 queries, so about one chain in ten meets a flagged query
    (flag rate ~0.2 % per query) and is compared only up to it."""
    s, sc = scenes[name]
    N, R = s.n_rays, s.max_reflections
    dirs = rt.fibonacci_directions(N, device="cuda:0")
    tr = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src, max_path_length=s.max_path_length, det_cap=6 * N)
    hs_all = tr.hit_seq.cpu().numpy()
    lens = (hs_all >= 0).sum(axis=1)
    rng = np.random.default_rng(61)
    idx = np.unique(np.concatenate([rng.choice(N, n_random, replace=False),
                                    np.argsort(-lens, kind="stable")[:n_long]]))
    odirs = np.ascontiguousarray(dirs.cpu().numpy()[idx])
    ref = oracle_lib.trace(oracle_lib.OracleScene.of(s), s.src, odirs, s.rcv, R, max_len=s.max_path_length)
    hs = hs_all[idx]
    diff = (hs != ref["hit_seq"]).any(axis=1)
    for i in np.nonzero(diff)[0]:
        k = int(np.argmax(hs[i] != ref["hit_seq"][i]))
        assert ref["flags"][i, : k + 1].any(), "unflagged divergence of ray %d" % idx[i]
    good = ~diff & ~ref["flags"].any(axis=1)
    det = tr.detections().cpu().numpy()
    sel = np.isin(det[:, 0], idx)
    gbits = np.zeros((len(idx), R + 1), np.uint32)
    rows = np.searchsorted(idx, det[sel, 0])
    np.bitwise_or.at(gbits, (rows, det[sel, 1]), (np.uint32(1) << det[sel, 2].astype(np.uint32)))
    assert np.array_equal(gbits[good], ref["det"][good])
    assert good.mean() > min_good and lens[idx].max() >= 20
    _say("%s full size: sample %d rays (longest %d segments), differing %d, flagged %d, queries %d" % (
        name, len(idx), int(lens[idx].max()), int(diff.sum()), int(ref["flags"].any(axis=1).sum()),
        int(tr.counters[1])))


def test_sphere_study_full_size_sampled(rt, oracle_lib):
    """The study at the paper's size: 10^5 rays, about 10^5 facets (level 6,
    81,920), six reflections.  Nothing escapes; a sample of 1,000 rays
    matches the oracle's trajectories and detections; the direct sound
    carries energy 1 and every later pulse lies within 1 % of 2k metres.
    Nothing escapes except, at most, a few rays after an exact edge hit."""
    s = synth.sphere_room(6)
    sc = rt.Scene.from_synth(s, device="cuda:0")
    N, R = 100_000, 6
    dirs = rt.fibonacci_directions(N, device="cuda:0")
    tr = rt.trace_rays(sc, dirs, s.rcv, R, src=s.src)
    assert int(tr.counters[2]) <= 10                     # only after exact edge hits
    idx = np.arange(7, N, 100)
    odirs = oracle_lib.fibonacci(N)[idx]
    ref = oracle_lib.trace(oracle_lib.OracleScene.of(s), s.src, odirs, s.rcv, R)
    hs = tr.hit_seq.cpu().numpy()[idx]
    diff = (hs != ref["hit_seq"]).any(axis=1)
    for i in np.nonzero(diff)[0]:
        k = int(np.argmax(hs[i] != ref["hit_seq"][i]))
        assert ref["flags"][i, : k + 1].any(), "unflagged divergence of ray %d" % idx[i]
    good = ~diff & ~ref["flags"].any(axis=1)
    assert np.all(hs[good] >= 0)
    det = tr.detections().cpu().numpy()
    gbits = np.zeros((N, R + 1), np.uint32)
    np.bitwise_or.at(gbits, (det[:, 0], det[:, 1]), (np.uint32(1) << det[:, 2].astype(np.uint32)))
    assert np.array_equal(gbits[idx][good], ref["det"][good])
    isrc = rt.collect_image_sources(sc, s.src, s.rcv, tr)
    key, cnt, pos, dist = [t.cpu().numpy() for t in isrc.valid()]
    order = key[:, 1]
    assert cnt[order == 0].sum() == N
    for k in range(1, R + 1):
        dk = dist[order == k]
        assert np.all(np.abs(dk - 2 * k) <= 0.01 * 2 * k)
    _say("sphere 81920: pulse energies " + " ".join("%.3f" % (cnt[order == k].sum() / N) for k in range(R + 1)))
