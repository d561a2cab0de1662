"""Scenes rebuilt in place (rt_rebuild_tree) and the whole path run on several
streams at once give the results of fresh scenes run one after another on
one stream.

The kernels' work does not depend on where a scene's memory lies, on what was
in it before, or on what runs beside them, so hit sequences, detection sets,
image-source counts and impulse responses are compared bit for bit.  The
streams reuse their scenes for meshes of 12 and 100,316 triangles in turn,
so the scenes' buffers grow and shrink while other streams are working (a
grown buffer's old block must not be handed to another stream before the
work queued on its own stream has passed)."""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

N_RAYS = 20_000
K_FIR = 255


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rt():
    import paper_1811_05784_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def meshes():
    return {"c1": synth.shoebox_c1(), "c2flat": synth.tessellated_box_c2(jitter=False),
            "c2": synth.tessellated_box_c2(jitter=True)}


def _run(rt, sc, s, taps):
    """Rays, trace, image sources and IR on the current stream (no host wait)."""
    dev = "cuda:0"
    dirs = rt.fibonacci_directions(N_RAYS, device=dev)
    cap = 8 * N_RAYS
    tr = rt.trace_rays(sc, dirs, s.rcv, s.max_reflections, src=s.src, max_path_length=s.max_path_length,
                       det_cap=cap, check_capacity=False, check_errors=False)
    isrc = rt.collect_image_sources(sc, s.src, s.rcv, tr, is_cap=cap, check_capacity=False)
    ir = rt.assemble_ir(sc, isrc, N_RAYS, len(s.rcv), s.alpha, s.beta, s.c, s.fs, s.ir_len, taps)
    return tr, isrc, ir


def _summary(res):
    tr, isrc, ir = res
    c = tr.counters.cpu()
    n_det = int(c[0])
    assert int(c[3]) == 0 and n_det <= tr.det.shape[0]
    det = tr.det[:n_det].cpu().numpy()
    det = det[np.lexsort(det.T[::-1])]
    n_is = int(isrc.n_is_dev.cpu()[0])
    return {"hit_seq": tr.hit_seq.cpu(), "det": det, "counters": c, "n_is": n_is,
            "band_energy": ir.band_energy.cpu(), "ir": ir.ir.cpu()}


def _same(a, b, what):
    assert torch.equal(a["hit_seq"], b["hit_seq"]), what + ": hit sequences differ"
    assert np.array_equal(a["det"], b["det"]), what + ": detections differ"
    assert torch.equal(a["counters"], b["counters"]), what
    assert a["n_is"] == b["n_is"], what
    assert torch.equal(a["band_energy"], b["band_energy"]), what + ": band energies differ"
    assert torch.equal(a["ir"], b["ir"]), what + ": impulse responses differ"


@pytest.fixture(scope="module")
def fresh(rt, meshes):
    """Reference results: a fresh scene per mesh, one stream, one at a time."""
    taps = synth.octave_fir_taps(K_FIR)
    out = {}
    for name, s in meshes.items():
        _say("fresh", name)
        sc = rt.Scene.from_synth(s, device="cuda:0")
        out[name] = (_summary(_run(rt, sc, s, taps)), (sc.n_nodes, sc.depth, sc.n_ref, sc.n_mat))
        sc.close()
    return out


def test_rebuild_in_place_reproduces_fresh_builds(rt, meshes, fresh):
    taps = synth.octave_fir_taps(K_FIR)
    s0 = meshes["c2flat"]
    sc = rt.Scene.from_synth(s0, device="cuda:0")
    for name in ["c2flat", "c1", "c2", "c1", "c2flat"]:
        _say("rebuild into", name)
        s = meshes[name]
        sc.rebuild(s.vtx, s.tri, s.material, s.plane_id)
        got = _summary(_run(rt, sc, s, taps))
        _same(got, fresh[name][0], "rebuilt " + name)
        assert (sc.n_nodes, sc.depth, sc.n_ref, sc.n_mat) == fresh[name][1]
    sc.close()


def test_rebuild_with_another_leaf_size(rt, meshes):
    """A rebuild may change the leaf size; the tree then matches a fresh build
    with that leaf size, and the results the fresh scene's."""
    taps = synth.octave_fir_taps(K_FIR)
    s = meshes["c2"]
    sc = rt.Scene.from_synth(s, device="cuda:0")
    for leaf in (4, 1, 8):
        _say("rebuild with leaf size %d" % leaf)
        ref_sc = rt.Scene.from_synth(s, leaf_size=leaf, device="cuda:0")
        want = _summary(_run(rt, ref_sc, s, taps))
        sc.rebuild(s.vtx, s.tri, s.material, s.plane_id, leaf_size=leaf)
        got = _summary(_run(rt, sc, s, taps))
        _same(got, want, "leaf size %d" % leaf)
        assert (sc.n_nodes, sc.depth, sc.n_ref, sc.leaf_size) == (ref_sc.n_nodes, ref_sc.depth, ref_sc.n_ref, leaf)
        ref_sc.close()
    sc.close()


def test_failed_rebuild_marks_the_scene_invalid_until_the_next_success(rt, meshes, fresh):
    taps = synth.octave_fir_taps(K_FIR)
    s = meshes["c1"]
    sc = rt.Scene.from_synth(s, device="cuda:0")
    bad = np.array(s.tri, copy=True)
    bad[3, 1] = len(s.vtx) + 5   # vertex index out of range: caught by the build's checks
    _say("rebuild with a bad mesh")
    with pytest.raises(RuntimeError, match="out of range"):
        sc.rebuild(s.vtx, bad, s.material, s.plane_id)
    dirs = rt.fibonacci_directions(64, device="cuda:0")
    with pytest.raises(RuntimeError, match="rebuild failed"):
        rt.trace_rays(sc, dirs, s.rcv, s.max_reflections, src=s.src)
    with pytest.raises(RuntimeError, match="rebuild failed"):
        _ = sc.n_nodes
    sc.rebuild(s.vtx, s.tri, s.material, s.plane_id)
    _same(_summary(_run(rt, sc, s, taps)), fresh["c1"][0], "rebuilt after a failure")
    sc.close()


def test_streams_running_at_once_give_the_serial_results(rt, meshes, fresh):
    taps = synth.octave_fir_taps(K_FIR)
    n_streams = 3
    order = ["c1", "c2flat", "c2", "c2", "c1", "c2flat", "c2flat", "c2", "c1", "c1", "c2", "c2flat"]
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    scenes = [None] * n_streams
    results = []
    torch.cuda.synchronize()
    for j, name in enumerate(order):
        k = j % n_streams
        s = meshes[name]
        _say("job %d: %s on stream %d" % (j, name, k))
        with torch.cuda.stream(streams[k]):
            if scenes[k] is None:
                scenes[k] = rt.Scene(s.vtx, s.tri, s.material, s.plane_id, device="cuda:0")
            else:
                scenes[k].rebuild(s.vtx, s.tri, s.material, s.plane_id)
            results.append((name, k, _run(rt, scenes[k], s, taps)))
    torch.cuda.synchronize()
    for j, (name, k, res) in enumerate(results):
        _same(_summary(res), fresh[name][0], "job %d (%s, stream %d)" % (j, name, k))
    for sc in scenes:
        sc.close()
