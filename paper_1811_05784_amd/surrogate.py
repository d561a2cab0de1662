"""Late-tail surrogate: binding of the rt_mlp_* / rt_hist_features /
rt_edc_db entry points and the pipeline from traces to network inputs and
targets.

The surrogate extends the method (it is not in the paper): the energy
histogram of reflection orders 0..8 (8 bands x 64 bins on [0, 0.25 s], dB)
goes in, the per-band decay curve of the full trace (8 bands x 128 bins,
Schroeder backward integration, dB re total) comes out.  Inference replaces
the bounces after the 8th; the full trace stays available as the fallback.

Every arithmetic step runs in librtac kernels; torch holds device memory.
"""
from __future__ import annotations

import ctypes
import math
import sys
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check
from .api import Batch, Scene, _dev, _ptr, _stream, assemble_batch, collect_batch, trace_batch

P = ctypes.c_void_p
WIDTHS = (512, 256, 256, 256, 1024)
N_BANDS = 8
FEAT_BINS = 64
FEAT_SECONDS = 0.25      # feature histogram span: orders 0..8 arrive early, so 3.9 ms bins
TARGET_BINS = 128
EARLY_ORDER = 8
FLOOR_DB = -150.0
OFFSET_DB = 75.0
SCALE_DB = 25.0
MASK_DB = -60.0


class Mlp:
    """A network handle (rt_mlp_create) with its FP32 master parameters, the
    BF16 copy, the gradient and the Adam moments as device tensors."""

    def __init__(self, theta, widths: Sequence[int] = WIDTHS, max_batch: int = 1024, device=None):
        lib = _lib.load()
        self.device = _dev(device)
        self.widths = tuple(int(w) for w in widths)
        w = (ctypes.c_int32 * len(self.widths))(*self.widths)
        h = P()
        with torch.cuda.device(self.device):
            check(lib.rt_mlp_create(w, len(self.widths) - 1, int(max_batch), ctypes.byref(h)), "rt_mlp_create")
        self.handle = h
        info = (ctypes.c_int64 * 4)()
        check(lib.rt_mlp_info(h, info), "rt_mlp_info")
        self.n_params = int(info[0])
        self.max_batch = int(info[2])
        theta = torch.as_tensor(np.asarray(theta, np.float32) if not isinstance(theta, torch.Tensor) else theta)
        if theta.numel() != self.n_params:
            raise ValueError("theta has %d entries, the network %d" % (theta.numel(), self.n_params))
        self.theta = theta.to(device=self.device, dtype=torch.float32).contiguous().clone()
        self.theta_bf16 = torch.empty(self.n_params, dtype=torch.bfloat16, device=self.device)
        self.grad = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        self.m = torch.zeros_like(self.grad)
        self.v = torch.zeros_like(self.grad)
        self.loss_terms = torch.zeros(2, dtype=torch.float64, device=self.device)
        self.step = 0
        to_bf16(self.theta, out=self.theta_bf16)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib._lib is not None:
            _lib._lib.rt_mlp_destroy(h)
            self.handle = None

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """x [B, w_0] bfloat16 -> y [B, w_L] float32."""
        lib = _lib.load()
        assert x.dtype == torch.bfloat16 and x.is_contiguous() and x.shape[1] == self.widths[0]
        B = x.shape[0]
        if out is None:
            out = torch.empty((B, self.widths[-1]), dtype=torch.float32, device=self.device)
        with torch.cuda.device(self.device):
            check(lib.rt_mlp_forward(self.handle, _ptr(self.theta_bf16), _ptr(self.theta), _ptr(x), B, _ptr(out),
                                     _stream(self.device)), "rt_mlp_forward")
        return out

    def backward(self, x: torch.Tensor, y: torch.Tensor, target: torch.Tensor,
                 mask: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Gradient of S = sum m (y - t)^2 into self.grad; returns the device
        (S, sum m) pair."""
        lib = _lib.load()
        with torch.cuda.device(self.device):
            check(lib.rt_mlp_backward(self.handle, _ptr(self.theta_bf16), _ptr(x), x.shape[0], _ptr(y), _ptr(target),
                                      _ptr(mask), _ptr(self.grad), _ptr(self.loss_terms), _stream(self.device)),
                  "rt_mlp_backward")
        return self.loss_terms

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             loss_terms: Optional[torch.Tensor] = "own") -> None:
        lib = _lib.load()
        self.step += 1
        lt = self.loss_terms if isinstance(loss_terms, str) else loss_terms
        with torch.cuda.device(self.device):
            check(lib.rt_mlp_adam(self.n_params, _ptr(self.theta), _ptr(self.theta_bf16), _ptr(self.grad),
                                  _ptr(self.m), _ptr(self.v), _ptr(lt), self.step, float(lr), float(beta1),
                                  float(beta2), float(eps), _stream(self.device)), "rt_mlp_adam")

    def train_step(self, x, target, mask, lr: float) -> torch.Tensor:
        y = self.forward(x)
        lt = self.backward(x, y, target, mask)
        self.adam(lr)
        return lt


def to_bf16(x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Round-to-nearest-even BF16 copy (rt_to_bf16)."""
    lib = _lib.load()
    x = x.contiguous()
    if out is None:
        out = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    with torch.cuda.device(x.device):
        check(lib.rt_to_bf16(_ptr(x), x.numel(), _ptr(out), _stream(x.device)), "rt_to_bf16")
    return out


def hist_features(hist: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Energy histogram -> BF16 features (max(10 log10 H, floor) + offset) / scale,
    same shape as hist."""
    lib = _lib.load()
    hist = hist.contiguous()
    if out is None:
        out = torch.empty(hist.shape, dtype=torch.bfloat16, device=hist.device)
    with torch.cuda.device(hist.device):
        check(lib.rt_hist_features(_ptr(hist), hist.numel(), FLOOR_DB, OFFSET_DB, SCALE_DB, _ptr(out),
                                   _stream(hist.device)), "rt_hist_features")
    return out


def edc_db(hist: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Schroeder decay curve in dB re total along the last axis of hist."""
    lib = _lib.load()
    hist = hist.contiguous()
    bins = hist.shape[-1]
    rows = hist.numel() // bins if bins else 0
    if out is None:
        out = torch.empty(hist.shape, dtype=torch.float32, device=hist.device)
    with torch.cuda.device(hist.device):
        check(lib.rt_edc_db(_ptr(hist), rows, bins, FLOOR_DB, _ptr(out), _stream(hist.device)), "rt_edc_db")
    return out


def _delta(device) -> torch.Tensor:
    t = torch.zeros((N_BANDS, 1), dtype=torch.float32, device=device)
    t[:, 0] = 1.0
    return t


def room_histograms(rooms, n_rays: int, orders: Sequence[int], bins: Sequence[int], c: float = 343.0,
                    T: float = 2.0, device=None, rooms_per_batch: int = 8, timers: Optional[Dict] = None,
                    spans: Optional[Sequence[float]] = None):
    """Per-band energy histograms of image sources for each room's (source,
    receiver) pairs (or, for a room with a single source, its receivers), one per (max reflection order, bin count) in
    zip(orders, bins): [n_pairs, 8, bins] each.  Rooms are traced in
    batches of rooms_per_batch in one persistent launch, once per distinct
    order.  timers (a dict) collects the milliseconds per order and batch.
    spans: time span in seconds of each histogram (default T for all)."""
    spans = list(spans) if spans is not None else [T] * len(orders)
    dev = _dev(device)
    outs = [[] for _ in orders]
    delta = _delta(dev)
    beta = torch.as_tensor(rooms[0].beta, dtype=torch.float32, device=dev)
    for r0 in range(0, len(rooms), rooms_per_batch):
        chunk = rooms[r0:r0 + rooms_per_batch]
        scenes = [Scene.from_synth(r, device=dev) for r in chunk]
        jobs = []
        for i, r in enumerate(chunk):
            src = np.asarray(r.src, np.float32)
            if src.ndim == 1:          # one source heard by all the scene's receivers
                jobs.append(dict(scene=i, src=src, rcv=r.rcv, n_rays=n_rays,
                                 max_path_length=c * T + float(np.max(r.rcv[:, 3]))))
                continue
            for p in range(len(src)):  # (source p, receiver p) pairs
                jobs.append(dict(scene=i, src=src[p], rcv=r.rcv[p:p + 1], n_rays=n_rays,
                                 max_path_length=c * T + float(r.rcv[p, 3])))
        b = Batch(scenes, jobs, device=dev)
        alpha = torch.as_tensor(np.concatenate([r.alpha for r in chunk]), dtype=torch.float32, device=dev)
        for R in sorted(set(orders)):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)] if timers is not None else None
            if ev:
                ev[0].record()
            tr = trace_batch(b, R)
            isb = collect_batch(b, tr)
            for o, (Ro, L) in enumerate(zip(orders, bins)):
                if Ro == R:
                    outs[o].append(assemble_batch(b, isb, alpha, beta, c, L / spans[o], L, delta).hist)
            if ev:
                ev[1].record()
                torch.cuda.synchronize()
                timers.setdefault(R, []).append(ev[0].elapsed_time(ev[1]))
    return [torch.cat(x) for x in outs]


def dataset(rooms, n_rays: int, full_order: int = 60, c: float = 343.0, T: float = 2.0, device=None,
            rooms_per_batch: int = 8):
    """(features [n, 512] bf16, targets [n, 1024] f32 in dB, mask [n, 1024],
    early-only decay curve [n, 1024] dB) for the rooms' pairs."""
    early_f, early_t, full = room_histograms(rooms, n_rays, (EARLY_ORDER, EARLY_ORDER, full_order),
                                             (FEAT_BINS, TARGET_BINS, TARGET_BINS), c, T, device, rooms_per_batch,
                                             spans=(FEAT_SECONDS, T, T))
    n = full.shape[0]
    x = hist_features(early_f).reshape(n, N_BANDS * FEAT_BINS)
    tgt = edc_db(full).reshape(n, N_BANDS * TARGET_BINS)
    base = edc_db(early_t).reshape(n, N_BANDS * TARGET_BINS)
    mask = (tgt >= MASK_DB).to(torch.float32)
    return x, tgt, mask, base


def band_rms_db(pred: torch.Tensor, full: torch.Tensor, min_db: float = MASK_DB) -> torch.Tensor:
    """Per-(pair, band) RMS dB difference over the bins where the full decay
    curve is >= min_db: [n, 8]."""
    p = pred.reshape(-1, N_BANDS, TARGET_BINS).double()
    f = full.reshape(-1, N_BANDS, TARGET_BINS).double()
    w = (f >= min_db).double()
    return torch.sqrt((w * (p - f) ** 2).sum(-1) / w.sum(-1).clamp_min(1.0))


def eval_loss(net: Mlp, x, tgt, mask) -> float:
    """Masked mean squared error of the network on (x, tgt, mask)."""
    y = net.forward(x)
    m = mask.double()
    return float(((y.double() - tgt.double()) ** 2 * m).sum() / m.sum().clamp_min(1.0))


def train(net: Mlp, x, tgt, mask, epochs: int = 200, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0, val=None) -> List[float]:
    """Adam on the masked squared error over shuffled minibatches, cosine
    learning-rate decay; returns the mean training loss per epoch.  val:
    optional held-out (x, tgt, mask) whose loss is printed with the log."""
    n = x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(x.device)
        acc = torch.zeros(2, dtype=torch.float64, device=x.device)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb = x[idx].contiguous()
            tb = tgt[idx].contiguous()
            mb = mask[idx].contiguous()
            lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / total))
            acc += net.train_step(xb, tb, mb, lr_k)
            k += 1
        a = acc.cpu()
        hist.append(float(a[0] / max(float(a[1]), 1.0)))
        if log_every and (ep % log_every == 0 or ep == epochs - 1):
            v = " held-out %.4f" % eval_loss(net, *val) if val is not None else ""
            print("epoch %d loss %.4f dB^2%s" % (ep, hist[-1], v), file=sys.stderr, flush=True)
    return hist
