"""Parity of the room-acoustic parameters (rt_room_params) with the FP64
oracle on seeded histograms: exponential decays of several rates with
Poisson-like sparsity, late-starting responses, a band without energy, a
receiver without energy, responses too short for T30.  Both sides sum in
FP64 (different order): EDT and T30 within 1e-6 relative, the others within
1e-9; NaN where the oracle has NaN."""
import numpy as np
import pytest
import torch

from oracle import params as oparams

pytestmark = pytest.mark.gpu
FS = 48_000.0


def _hist(seed, n_rcv, L):
    rng = np.random.default_rng(seed)
    h = np.zeros((n_rcv, 8, L), np.float32)
    for m in range(n_rcv):
        s0 = int(rng.integers(0, max(1, L // 10)))
        a = rng.uniform(3.0, 40.0, size=8)
        t = np.arange(L - s0) / FS
        for b in range(8):
            x = np.exp(-a[b] * t) * rng.exponential(size=len(t))
            x[rng.uniform(size=len(t)) < rng.uniform(0.2, 0.95)] = 0.0
            h[m, b, s0:] = x.astype(np.float32)
        h[m, int(rng.integers(0, 8))] *= 0.0 if m % 3 == 1 else 1.0
    if n_rcv > 2:
        h[2] = 0.0
    return h


@pytest.mark.parametrize("n_rcv,L", [(1, 1), (1, 100), (3, 4097), (4, 5000), (8, 96_000), (32, 24_001)])
def test_room_params_match_oracle(n_rcv, L):
    import paper_1811_05784_amd as rt
    h = _hist(n_rcv * 7 + L, n_rcv, L)
    got = rt.room_params(torch.as_tensor(h, device="cuda:0"), FS).cpu().numpy()
    ref = oparams.room_params(h.astype(np.float64), FS)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    rel = np.array([1e-6, 1e-6, 1e-9, 1e-9, 1e-9, 1e-9])
    tol = rel * np.maximum(np.abs(ref), 1e-12)
    assert np.all(np.abs(got - ref)[ok] <= np.broadcast_to(tol, ref.shape)[ok] + 1e-12)
    assert ok[..., 4].any()
    if L >= 1000:
        assert ok[..., 0].any() and ok[..., 1].any()
