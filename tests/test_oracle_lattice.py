"""Shoe-box pins of the oracle (section "Analytical comparison by shoe box
model"): image sources found by ray tracing sit on the closed-form image
lattice of a rectangular room to machine precision; their reflection counts per
wall and their energies follow from the lattice indices; every well-resolved
lattice image is found with the expected ray count (solid-angle fraction,
section "Discrete model").  Also the invariants: retro-propagation of a
detected ray lands on its image source; alpha = 1 keeps only the direct
sound; alpha = beta = 0 makes all bands equal.
"""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_box_params():
    out = {}
    with open(os.path.join(GOLDEN, "shoebox_experiment.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                out[k] = [float(x) for x in v]
    return out


def _lattice_index(x, xs, L):
    """x = (1 - 2p) xs + 2 i L with p in {0,1}: return (i, p) or None."""
    for p in (0, 1):
        i = (x - (1 - 2 * p) * xs) / (2 * L)
        ir = round(i)
        if abs(i - ir) < 1e-9:
            return ir, p
    return None


def _material_of_plane(scene):
    m = np.full(scene.n_tri, -1, np.int64)
    for t in range(scene.n_tri - 1, -1, -1):
        m[scene.plane_id[t]] = scene.material[t]
    return m


@pytest.fixture(scope="module")
def paper_box_run(oracle_lib):
    prm = _paper_box_params()
    s = synth.paper_box(n_rays=int(prm["rays"][0]), max_reflections=6)
    assert tuple(s.vtx.max(0)) == tuple(prm["box"])
    assert np.allclose(s.src, prm["source"]) and np.allclose(s.rcv[0, :3], prm["receiver"])
    assert s.rcv[0, 3] == np.float32(prm["radius"][0])
    sc = oracle_lib.OracleScene.of(s)
    dirs = oracle_lib.fibonacci(s.n_rays)
    tr = oracle_lib.trace(sc, s.src, dirs, s.rcv, s.max_reflections, states=True)
    det = oracle_lib.detections_from_bits(tr["det"])
    keys = oracle_lib.image_source_keys(s.plane_id, tr["hit_seq"], det)
    tab = oracle_lib.image_sources(sc, s.src, s.rcv, keys)
    return s, sc, dirs, tr, det, keys, tab


def test_closed_room_nothing_escapes(paper_box_run):
    s, sc, dirs, tr, *_ = paper_box_run
    assert (tr["hit_seq"] >= 0).all()                 # R+1 segments, all ended on a wall


def test_image_sources_on_lattice(paper_box_run):
    s, sc, dirs, tr, det, keys, tab = paper_box_run
    dims = s.vtx.max(0).astype(np.float64)
    xs = s.src.astype(np.float64)
    mop = _material_of_plane(s)
    assert len(tab["keys"]) > 100
    for key, pos in zip(tab["keys"], tab["pos"]):
        k = key[1]
        walls = np.bincount(mop[list(key[2:])], minlength=6) if k else np.zeros(6, int)
        order = 0
        for a in range(3):
            li = _lattice_index(pos[a], xs[a], dims[a])
            assert li is not None, (key, pos)          # on the lattice to machine precision
            i, p = li
            assert walls[2 * a] == abs(i - p) and walls[2 * a + 1] == abs(i), (key, a, i, p)
            order += abs(2 * i - p)
        assert order == k
        # consecutive reflections are on different planes
        assert all(key[j] != key[j + 1] for j in range(2, len(key) - 1))


def test_lattice_completeness_and_counts(paper_box_run):
    s, sc, dirs, tr, det, keys, tab = paper_box_run
    dims = s.vtx.max(0).astype(np.float64)
    xs = s.src.astype(np.float64)
    xm = s.rcv[0, :3].astype(np.float64)
    r = float(s.rcv[0, 3])
    N, R = s.n_rays, s.max_reflections
    # merge keys by position (commuting reflections give equal positions)
    found = {}
    for key, pos, n in zip(tab["keys"], tab["pos"], tab["count"]):
        q = tuple(np.round(pos, 6))
        found[q] = found.get(q, 0) + int(n)
    checked = 0
    for i in range(-R, R + 1):
        for j in range(-R, R + 1):
            for kk in range(-R, R + 1):
                for p in (0, 1):
                    for q in (0, 1):
                        for w in (0, 1):
                            order = abs(2 * i - p) + abs(2 * j - q) + abs(2 * kk - w)
                            if order > R:
                                continue
                            pos = np.array([(1 - 2 * p) * xs[0] + 2 * i * dims[0],
                                            (1 - 2 * q) * xs[1] + 2 * j * dims[1],
                                            (1 - 2 * w) * xs[2] + 2 * kk * dims[2]])
                            d = np.linalg.norm(pos - xm)
                            e = N * (1 - np.sqrt(1 - r * r / (d * d))) / 2
                            if e < 5:
                                continue
                            n = found.get(tuple(np.round(pos, 6)), 0)
                            assert abs(n - e) <= 3 * np.sqrt(e) + 2, (order, d, n, e)
                            checked += 1
    assert checked >= 30


def test_energy_matches_lattice_exponents(paper_box_run, oracle_lib):
    s, sc, dirs, tr, det, keys, tab = paper_box_run
    mop = _material_of_plane(s)
    E = oracle_lib.is_energy(tab, s.n_rays, s.alpha, s.beta, mop)
    a = s.alpha.astype(np.float64)
    b = s.beta.astype(np.float64)
    for key, n, d, e in zip(tab["keys"], tab["count"], tab["dist"], E):
        walls = np.bincount(mop[list(key[2:])], minlength=6) if key[1] else np.zeros(6, int)
        want = n / s.n_rays * np.exp(-b * d) * np.prod((1 - a) ** walls[:, None], axis=0)
        assert np.allclose(e, want, rtol=1e-13)


def test_retro_propagation_lands_on_image_source(paper_box_run):
    s, sc, dirs, tr, det, keys, tab = paper_box_run
    idx = {k: i for i, k in enumerate(tab["keys"])}
    st = tr["states"]
    for ray, k, r in det[:: max(1, len(det) // 500)]:
        o, u, L = st[ray, k, :3], st[ray, k, 3:6], st[ray, k, 6]
        retro = o - L * u / np.linalg.norm(u)
        key = (int(r), int(k)) + tuple(int(s.plane_id[t]) for t in tr["hit_seq"][ray, :k])
        assert np.allclose(retro, tab["pos"][idx[key]], rtol=0, atol=1e-9)


def test_alpha_one_keeps_direct_sound_and_alpha_zero_flat_bands(paper_box_run, oracle_lib):
    s, sc, dirs, tr, det, keys, tab = paper_box_run
    mop = _material_of_plane(s)
    taps = synth.delta_taps(1)
    ones = oracle_lib.assemble_ir(tab, s.n_rays, 1, np.ones((6, 8)), s.beta, mop, 343.0, 48000.0,
                                  s.ir_len, taps)
    direct = [i for i, k in enumerate(tab["keys"]) if k[1] == 0]
    assert len(direct) == 1
    E0 = tab["count"][direct[0]] / s.n_rays * np.exp(-s.beta.astype(np.float64) * tab["dist"][direct[0]])
    assert np.allclose(ones["band_energy"][0], E0, rtol=1e-13)
    flat = oracle_lib.assemble_ir(tab, s.n_rays, 1, np.zeros((6, 8)), np.zeros(8), mop, 343.0, 48000.0,
                                  s.ir_len, taps)
    assert np.all(flat["band_energy"][0] == flat["band_energy"][0, 0])
    # histogram total equals the sum of the image-source energies inside the IR
    E = flat["energy"]
    keep = flat["bins"] < s.ir_len
    assert np.isclose(flat["hist"].sum(), E[keep].sum(), rtol=1e-12)
    # delta taps: the band IR is the pressure sqrt(H)
    assert np.array_equal(flat["band_ir"], np.sqrt(flat["hist"]))


def test_fir_perfect_reconstruction_over_bands(paper_box_run, oracle_lib):
    s, sc, dirs, tr, det, keys, tab = paper_box_run
    mop = _material_of_plane(s)
    rng = np.random.default_rng(2)
    K = 31
    taps = rng.standard_normal((8, K))
    taps -= taps.mean(axis=0, keepdims=True)          # bands sum to zero ...
    taps[:, K // 2] += 1.0 / 8                        # ... plus a shared delta
    out = oracle_lib.assemble_ir(tab, s.n_rays, 1, np.zeros((6, 8)), np.zeros(8), mop, 343.0, 48000.0,
                                 s.ir_len, taps)
    assert np.allclose(out["ir"][0], np.sqrt(out["hist"][0, 0]), atol=1e-12)
