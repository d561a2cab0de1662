"""Pins of the room-acoustic parameter oracle (oracle/params.py) against
closed forms: an exponentially decaying histogram H[s] = q^(s - s0) has a
geometric Schroeder curve, so every parameter follows from geometric sums
worked out by hand here; step histograms pin the windows and the origin."""
import math

import numpy as np
import pytest

from oracle import params

FS = 48_000.0


def _exp_hist(a, s0, L, fs=FS):
    q = math.exp(-a / fs)
    h = np.zeros((1, 8, L))
    h[0, :, s0:] = q ** np.arange(L - s0)
    return h, q


@pytest.mark.parametrize("a", [2.0, 7.0, 20.0])
def test_exponential_decay_closed_forms(a):
    s0 = 123
    L = s0 + int(FS * 12 * math.log(10) / a)             # the histogram ends ~120 dB down
    h, q = _exp_hist(a, s0, L)
    p = params.room_params(h, FS)[0, 3]
    n = L - s0
    # decay rate a (1/s) in energy: 10 log10 e per unit a t -> T60 = 60 / (10 a / ln 10)
    t60 = 6.0 * math.log(10.0) / a
    assert p[0] == pytest.approx(t60, rel=2e-3)          # EDT (curve straight to within the tail cut)
    assert p[1] == pytest.approx(t60, rel=2e-3)          # T30
    n80, n50 = round(0.08 * FS), round(0.05 * FS)
    e80 = (1 - q ** n80) / (1 - q)
    late = (q ** n80 - q ** n) / (1 - q)
    assert p[2] == pytest.approx(10 * math.log10(e80 / late), rel=1e-9)
    tot = (1 - q ** n) / (1 - q)
    assert p[3] == pytest.approx((1 - q ** n50) / (1 - q) / tot, rel=1e-9)
    # sum k q^k for k < n
    sk = (q - n * q ** n + (n - 1) * q ** (n + 1)) / (1 - q) ** 2
    assert p[4] == pytest.approx(sk / tot / FS, rel=1e-9)
    assert p[5] == pytest.approx(10 * math.log10(tot), rel=1e-12)


def test_windows_origin_and_undefined_values():
    L = 20_000
    h = np.zeros((2, 8, L))
    # receiver 0: direct sound in band 2 only at bin 100 sets the origin for every band
    h[0, 2, 100] = 1.0
    h[0, 5, 100 + 2000] = 3.0            # 2000 bins = 41.7 ms after the origin: early for D50 and C80
    h[0, 5, 100 + 3000] = 1.0            # 62.5 ms: early for C80 only
    p = params.room_params(h, FS)
    assert p[0, 5, 3] == pytest.approx(0.75)                   # D50
    assert math.isinf(p[0, 5, 2]) or np.isnan(p[0, 5, 2])       # no late energy
    assert p[0, 5, 4] == pytest.approx((3 * 2000 + 3000) / 4 / FS)
    assert p[0, 5, 5] == pytest.approx(10 * math.log10(4.0))
    assert np.isnan(p[0, 0]).all()                              # a band without energy
    assert np.isnan(p[1]).all()                                 # a receiver without energy
    # H = 2^-s for 8 bins: the curve falls ~3.01 dB per bin down to ~-21 dB and
    # then ends: an EDT from bins 0..3, no T30 (never reaches -35 dB)
    h2 = np.zeros((1, 8, L))
    h2[0, :, :8] = 0.5 ** np.arange(8)
    e = np.cumsum(h2[0, 0, :8][::-1])[::-1]
    y = 10 * np.log10(e[:4] / e[0])
    slope = np.polyfit(np.arange(4) / FS, y, 1)[0]
    q = params.room_params(h2, FS)[0, 0]
    assert np.isnan(q[1]) and q[0] == pytest.approx(-60.0 / slope, rel=1e-12)
