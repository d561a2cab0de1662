"""Pin of the oracle's analytic absorption gradient.

For fixed ray paths the band energy is a polynomial in the absorption
coefficients (eq. for E_s with the product over reflections), so FP64 central
differences are exact up to O(h^2) with a tiny constant; the analytic
gradient must match them, including at alpha = 1 where the division form
breaks down.  Cross-band derivatives are zero by construction (band b only
uses alpha[:, b]).
"""
import numpy as np

import synth


def _setup(oracle_lib):
    s = synth.paper_box(n_rays=20_000, max_reflections=5)
    sc = oracle_lib.OracleScene.of(s)
    tr = oracle_lib.trace(sc, s.src, oracle_lib.fibonacci(s.n_rays), s.rcv, s.max_reflections, flags=False)
    det = oracle_lib.detections_from_bits(tr["det"])
    keys = oracle_lib.image_source_keys(s.plane_id, tr["hit_seq"], det)
    tab = oracle_lib.image_sources(sc, s.src, s.rcv, keys)
    mop = np.full(s.n_tri, -1, np.int64)
    for t in range(s.n_tri - 1, -1, -1):
        mop[s.plane_id[t]] = s.material[t]
    return s, tab, mop


def _loss(oracle_lib, s, tab, mop, alpha, g, L):
    out = oracle_lib.assemble_ir(tab, s.n_rays, 1, alpha, s.beta, mop, 343.0, 48000.0, L,
                                 synth.delta_taps(1))
    return float((out["band_energy"] * g).sum())


def test_gradient_matches_central_differences(oracle_lib):
    s, tab, mop = _setup(oracle_lib)
    rng = np.random.default_rng(3)
    g = rng.standard_normal((1, 8))
    L = 1500                      # cuts some late image sources off (they must not count)
    for alpha in (s.alpha.astype(np.float64), np.where(np.arange(8) % 3 == 0, 1.0, 0.4) * np.ones((6, 1))):
        grad = oracle_lib.band_energy_grad(tab, s.n_rays, 1, 6, alpha, s.beta, mop, 343.0, 48000.0, L, g)
        h = 1e-4
        fd = np.zeros_like(alpha)
        for m in range(6):
            for b in range(8):
                a1, a2 = alpha.copy(), alpha.copy()
                a1[m, b] += h
                a2[m, b] -= h
                fd[m, b] = (_loss(oracle_lib, s, tab, mop, a1, g, L) - _loss(oracle_lib, s, tab, mop, a2, g, L)) / (2 * h)
        scale = np.abs(fd).max()
        assert scale > 0
        assert np.allclose(grad, fd, rtol=1e-6, atol=1e-9 * scale), np.abs(grad - fd).max()


def test_gradient_single_source_closed_form(oracle_lib):
    # one image source with reflections on materials [0, 0, 1]: d/dalpha0 of
    # (1-a0)^2 (1-a1) is -2 (1-a0)(1-a1); d/dalpha1 is -(1-a0)^2
    tab = dict(keys=[(0, 3, 7, 9, 7)], count=np.array([4]), dist=np.array([2.0]))
    mop = np.zeros(10, np.int64)
    mop[9] = 1
    alpha = np.array([[0.3] * 8, [0.6] * 8])
    beta = np.full(8, 0.01)
    g = np.ones((1, 8))
    grad = oracle_lib.band_energy_grad(tab, 10, 1, 2, alpha, beta, mop, 343.0, 48000.0, 1000, g)
    base = 0.4 * np.exp(-0.02)
    assert np.allclose(grad[0], base * -2 * 0.7 * 0.4)
    assert np.allclose(grad[1], base * -(0.7 ** 2))
