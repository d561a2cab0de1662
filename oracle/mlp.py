"""FP64 CPU oracle of the late-tail surrogate: a plain multilayer perceptron
with its loss, gradient and Adam update, and the feature / target transforms
that feed it.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the GPU path.

The surrogate is not part of the paper.  It extends the paper's observation
that late image sources are hit by few rays (discussion after the detection
probability, section "Discrete model"), so the late part of the response is
the noisiest and costliest part of a trace: the network maps the energy
histogram of reflection orders 0..8 to the decay curve of the full trace.

* ``forward`` / ``backward`` -- y = W_L relu(... relu(W_1 x + b_1) ...) + b_L,
  masked mean squared error, reverse-mode gradient by the chain rule.
* ``adam``                   -- Kingma & Ba (2015), Algorithm 1, with the bias
  corrections m/(1 - beta1^t) and v/(1 - beta2^t).
* ``schroeder_edc_db``       -- Schroeder (1965) backward integration of the
  per-band energy histogram, in dB relative to the total energy.
* ``hist_features``          -- per-bin energy in dB, clamped and scaled.

Parity unpinned: none; ``tests/test_oracle_mlp.py`` pins the gradient by
central differences of the forward pass, a one-layer network by its closed
form, the first Adam step by its closed form, and the decay curve by the
geometric series of an exponentially decaying histogram.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

FEAT_FLOOR_DB = -150.0
FEAT_OFFSET_DB = 75.0
FEAT_SCALE_DB = 25.0


def split_params(theta: np.ndarray, widths: Sequence[int]) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Flat parameter vector -> [(W_l [out, in], b_l [out])], layer after
    layer, each weight matrix row-major followed by its bias."""
    out, o = [], 0
    for i, j in zip(widths[:-1], widths[1:]):
        W = theta[o:o + i * j].reshape(j, i)
        o += i * j
        b = theta[o:o + j]
        o += j
        out.append((W, b))
    assert o == theta.size
    return out


def n_params(widths: Sequence[int]) -> int:
    return int(sum(i * j + j for i, j in zip(widths[:-1], widths[1:])))


def forward(theta, widths, x) -> List[np.ndarray]:
    """Activations [x, h_1, ..., h_{L-1}, y] in FP64; ReLU on hidden layers,
    identity on the output layer."""
    acts = [np.asarray(x, np.float64)]
    layers = split_params(np.asarray(theta, np.float64), widths)
    for li, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(np.maximum(z, 0.0) if li + 1 < len(layers) else z)
    return acts


def loss(y, target, mask) -> float:
    """Masked mean squared error: sum m (y - t)^2 / sum m."""
    m = np.asarray(mask, np.float64)
    d = np.asarray(y, np.float64) - np.asarray(target, np.float64)
    return float((m * d * d).sum() / max(m.sum(), 1e-300))


def backward(theta, widths, x, target, mask) -> Tuple[float, np.ndarray]:
    """Loss and its gradient with respect to the flat parameter vector."""
    acts = forward(theta, widths, x)
    layers = split_params(np.asarray(theta, np.float64), widths)
    m = np.asarray(mask, np.float64)
    msum = max(m.sum(), 1e-300)
    d = acts[-1] - np.asarray(target, np.float64)
    g = 2.0 * m * d / msum                         # dLoss/dy
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in = acts[li]
        grads.append((g.T @ a_in, g.sum(axis=0)))
        if li > 0:
            g = (g @ W) * (acts[li] > 0.0)         # through the ReLU of layer li
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return float((m * d * d).sum() / msum), flat


def adam(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step at step number t >= 1; returns (theta, m, v) in FP64."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def schroeder_edc_db(hist, floor_db: float = FEAT_FLOOR_DB):
    """hist [..., S] energy per time bin -> EDC_s = sum_{s' >= s} H_s' in dB
    relative to EDC_0, clamped below at floor_db (a band with no energy is
    all floor)."""
    h = np.asarray(hist, np.float64)
    edc = np.cumsum(h[..., ::-1], axis=-1)[..., ::-1]
    tot = edc[..., :1]
    with np.errstate(divide="ignore", invalid="ignore"):
        db = 10.0 * np.log10(edc / tot)
    db = np.where((tot > 0) & (edc > 0), db, floor_db)
    return np.maximum(db, floor_db)


def hist_features(hist):
    """hist [..., S] energy per bin -> (max(10 log10 H, floor) + offset) / scale."""
    h = np.asarray(hist, np.float64)
    with np.errstate(divide="ignore"):
        db = np.where(h > 0, 10.0 * np.log10(np.where(h > 0, h, 1.0)), FEAT_FLOOR_DB)
    return (np.maximum(db, FEAT_FLOOR_DB) + FEAT_OFFSET_DB) / FEAT_SCALE_DB


def band_rms_db(pred_db, full_db, min_db: float = -60.0):
    """Per-band RMS difference [.., bands] over the bins where the full
    decay curve is >= min_db."""
    p = np.asarray(pred_db, np.float64)
    f = np.asarray(full_db, np.float64)
    w = (f >= min_db).astype(np.float64)
    return np.sqrt((w * (p - f) ** 2).sum(-1) / np.maximum(w.sum(-1), 1.0))
