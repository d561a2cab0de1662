"""FP64 CPU oracle of the room-acoustic parameters computed from the
per-band energy histogram of an impulse response.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
CPU-baseline leg, never by the product library.  It shares no code with the
GPU path.

The paper derives perceptive factors (EDT, T30, SPL, C80, D50, Ts) from its
energy impulse responses (section on the Orange theater, Table 3).  It does
not restate their definitions; these follow the usual room-acoustics ones
(ISO 3382-1), on the histogram H[s] of energy per time bin of width 1/fs:

* time origin s0: the first bin with energy in any band of the receiver
  (arrival of the direct sound, or of the first reflection);
* Schroeder decay curve EDC(s) = sum_{s' >= s} H[s'], in dB re EDC(s0), on
  the bins up to the last one with energy (the response ends there);
* EDT = -60 / slope of the least-squares line of EDC_dB against
  t = (s - s0) / fs over the bins with 0 >= EDC_dB >= -10 (undefined unless
  the curve reaches -10 dB and at least 2 bins qualify);
* T30 = -60 / slope over -5 >= EDC_dB >= -35 (undefined unless the curve
  reaches -35 dB);
* C80 = 10 log10(E[s0, s0 + n80) / E[s0 + n80, L)), n80 = floor(0.08 fs + 1/2);
* D50 = E[s0, s0 + n50) / E[s0, L), n50 = floor(0.05 fs + 1/2);
* Ts = sum (s - s0) / fs H[s] / sum H[s] over s >= s0;
* SPL = 10 log10(sum H), the received energy relative to the emitted energy
  (every ray carries 1/N of it, section "Discrete model").

Undefined values are NaN.  Parity unpinned: none; tests/test_oracle_params.py
pins every parameter with closed forms of an exponentially decaying
histogram (geometric sums) and hand-built step histograms.
"""
from __future__ import annotations

import numpy as np

NAMES = ("EDT", "T30", "C80", "D50", "Ts", "SPL")


def _fit_slope(x, y):
    n = len(x)
    if n < 2:
        return np.nan
    xm, ym = x.mean(), y.mean()
    sxx = ((x - xm) ** 2).sum()
    if sxx == 0:
        return np.nan
    return ((x - xm) * (y - ym)).sum() / sxx


def room_params(hist, fs: float) -> np.ndarray:
    """hist [n_rcv, 8, L] energy per bin -> [n_rcv, 8, 6] (EDT s, T30 s,
    C80 dB, D50 fraction, Ts s, SPL dB)."""
    h = np.asarray(hist, np.float64)
    n_rcv, nb, L = h.shape
    out = np.full((n_rcv, nb, 6), np.nan)
    n80 = int(np.floor(0.08 * fs + 0.5))
    n50 = int(np.floor(0.05 * fs + 0.5))
    for m in range(n_rcv):
        any_e = np.nonzero((h[m] > 0).any(axis=0))[0]
        if len(any_e) == 0:
            continue
        s0 = int(any_e[0])
        for b in range(nb):
            x = h[m, b, s0:]
            tot = x.sum()
            if tot <= 0:
                continue
            t = np.arange(len(x)) / fs
            edc = np.cumsum(x[::-1])[::-1]
            live = edc > 0                      # bins after the last arrival are past the response
            db = np.full(len(x), -np.inf)
            db[live] = 10.0 * np.log10(edc[live] / edc[0])   # exactly 0 dB at the origin
            low = db[live].min()
            sel = live & (db <= 0) & (db >= -10)
            edt = -60.0 / _fit_slope(t[sel], db[sel]) if low <= -10 else np.nan
            sel = live & (db <= -5) & (db >= -35)
            t30 = -60.0 / _fit_slope(t[sel], db[sel]) if low <= -35 else np.nan
            e80, late = x[:n80].sum(), x[n80:].sum()
            c80 = 10.0 * np.log10(e80 / late) if late > 0 else np.nan
            d50 = x[:n50].sum() / tot
            ts = (t * x).sum() / tot
            out[m, b] = (edt, t30, c80, d50, ts, 10.0 * np.log10(tot))
    return out
