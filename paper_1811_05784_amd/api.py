"""Torch-facing wrappers over the librtac C-ABI.

PyTorch provides device memory and the current HIP stream; every step of the
computation runs in librtac's kernels.  Functions mirror the C entry points:
``Scene`` (rt_build_tree), ``fibonacci_directions``, ``trace_rays``,
``collect_image_sources``, ``assemble_ir``, ``band_energy_adjoint`` and the
``BandEnergy`` autograd function built on the last two.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import BuildParams, Job, TraceParams, check

P = ctypes.c_void_p


def _dev(device=None) -> torch.device:
    if device is None:
        device = torch.device("cuda", torch.cuda.current_device())
    return torch.device(device)


def _stream(device=None):
    return P(torch.cuda.current_stream(_dev(device)).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else P(t.data_ptr())


def _to_dev(x, dtype, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)
    return t.contiguous()


def _host_f32(x, n):
    a = (ctypes.c_float * n)(*[float(v) for v in np.asarray(x, np.float64).reshape(-1)[:n]])
    return a


class Scene:
    """A mesh on the device plus its acceleration tree (rt_build_tree)."""

    def __init__(self, vtx, tri, material, plane_id=None, leaf_size: int = 1, device=None):
        lib = _lib.load()
        self.device = _dev(device)
        self.vtx = _to_dev(vtx, torch.float32, self.device)
        self.tri = _to_dev(tri, torch.int32, self.device)
        self.material = _to_dev(material, torch.int32, self.device)
        self.plane_id = None if plane_id is None else _to_dev(plane_id, torch.int32, self.device)
        self._h = P()
        prm = BuildParams(int(leaf_size))
        with torch.cuda.device(self.device):
            check(lib.rt_build_tree(_ptr(self.vtx), self.vtx.shape[0], _ptr(self.tri), self.tri.shape[0],
                                    _ptr(self.material), _ptr(self.plane_id), ctypes.byref(prm),
                                    _stream(self.device), ctypes.byref(self._h)), "rt_build_tree")
        self.n_tri = int(self.tri.shape[0])
        self.leaf_size = int(leaf_size)
        self._info = None   # read on first use: rt_scene_info waits for the build to finish

    def _scene_info(self):
        if self._info is None:
            info = (ctypes.c_int64 * 6)()
            diag = (ctypes.c_double * 1)()
            check(_lib.load().rt_scene_info(self.handle, info, diag), "rt_scene_info")
            self._info = [int(v) for v in info] + [float(diag[0])]
        return self._info

    def rebuild(self, vtx, tri, material, plane_id=None, leaf_size=None) -> "Scene":
        """Replace this scene's mesh and tree with those of a new (or the same)
        mesh, built on the current stream into the scene's own device memory
        (rt_rebuild_tree).  Earlier calls on the scene must be on the same
        stream or finished; batches made from it must be recreated."""
        lib = _lib.load()
        v = _to_dev(vtx, torch.float32, self.device)
        t = _to_dev(tri, torch.int32, self.device)
        m = _to_dev(material, torch.int32, self.device)
        pid = None if plane_id is None else _to_dev(plane_id, torch.int32, self.device)
        leaf = self.leaf_size if leaf_size is None else int(leaf_size)
        prm = BuildParams(leaf)
        with torch.cuda.device(self.device):
            rc = lib.rt_rebuild_tree(self.handle, _ptr(v), v.shape[0], _ptr(t), t.shape[0], _ptr(m), _ptr(pid),
                                     ctypes.byref(prm), _stream(self.device))
        # the build reads its inputs after the call returns: keep them with the scene
        self.vtx, self.tri, self.material, self.plane_id = v, t, m, pid
        self._info = None
        check(rc, "rt_rebuild_tree")
        self.n_tri = int(t.shape[0])
        self.leaf_size = leaf
        return self

    n_mat = property(lambda self: self._scene_info()[1])
    n_nodes = property(lambda self: self._scene_info()[2])
    depth = property(lambda self: self._scene_info()[3])
    n_ref = property(lambda self: self._scene_info()[5])
    diag = property(lambda self: self._scene_info()[6])

    @classmethod
    def from_synth(cls, s, leaf_size: int = 1, device=None) -> "Scene":
        return cls(s.vtx, s.tri, s.material, s.plane_id, leaf_size=leaf_size, device=device)

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("scene destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().rt_scene_destroy(self._h)
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fibonacci_directions(n: int, device=None) -> torch.Tensor:
    dev = _dev(device)
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    check(_lib.load().rt_fibonacci_directions(int(n), _ptr(out), _stream(dev)), "rt_fibonacci_directions")
    return out


def icosahedral_directions(f: int, device=None) -> torch.Tensor:
    """rt_icosahedral_directions: the 10 f^2 + 2 grid directions of the
    icosahedron subdivided at frequency f."""
    dev = _dev(device)
    out = torch.empty((10 * int(f) * int(f) + 2, 3), dtype=torch.float32, device=dev)
    check(_lib.load().rt_icosahedral_directions(int(f), _ptr(out), _stream(dev)), "rt_icosahedral_directions")
    return out


def directional_directions(n: int, m: float, axis, device=None) -> torch.Tensor:
    """rt_directional_directions: n directions of a source radiating energy
    per solid angle proportional to (1 + cos theta)^m about `axis`."""
    dev = _dev(device)
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    check(_lib.load().rt_directional_directions(int(n), float(m), _host_f32(axis, 3), _ptr(out), _stream(dev)),
          "rt_directional_directions")
    return out


@dataclasses.dataclass
class TraceResult:
    hit_seq: torch.Tensor          # [N, R+1] int32
    det: torch.Tensor              # [cap, 3] int32 (first n_det rows valid)
    counters: torch.Tensor         # [4] int64 (device)
    states: Optional[torch.Tensor]  # [N, R+2, 8] float32
    max_reflections: int

    def n_det(self) -> int:
        return int(self.counters[0].item())

    def detections(self) -> torch.Tensor:
        return self.det[: min(self.n_det(), self.det.shape[0])]


def trace_rays(scene: Scene, dirs: torch.Tensor, rcv, max_reflections: int, src=None, origins=None,
               start_plane=None, start_len=None, max_path_length: float = 0.0, record_states: bool = False,
               det_cap: Optional[int] = None, fetch_threshold: int = 0, shade_threshold: int = 0,
               blocks_per_cu: int = 0, check_capacity: bool = True, out: Optional[TraceResult] = None,
               check_errors: bool = True, keep_order: bool = False,
               stats: Optional[torch.Tensor] = None, rounds: int = 0, spill_threshold: int = 0,
               waves_per_simd: int = 0, kernel_events=None, suspend_after: int = 0,
               min_beam_rays: int = 0, xcd_pools: int = 0, coop_queries: int = 0,
               record_rows=None, stack_depth: int = 0) -> TraceResult:
    """rt_trace_rays.  With check_capacity the call synchronises, and re-runs
    with a larger detection buffer if the first one overflowed.
    record_rows: with record_states, an int32 [n] map ray -> row of `states`
    (-1: not recorded); states then has max(record_rows) + 1 rows.
    min_beam_rays: n >= 1 stops each ray at the eq. 13 range (r/2) sqrt(N/n)
    of the largest receiver radius r and the N rays of the call.
    kernel_events: optional (start, stop) torch.cuda.Event pair (timing
    enabled) recorded around the traversal-kernel launches only."""
    lib = _lib.load()
    dev = scene.device
    dirs = _to_dev(dirs, torch.float32, dev)
    n = dirs.shape[0]
    R1 = max_reflections + 1
    rcv_t = _to_dev(rcv, torch.float32, dev).reshape(-1, 4)
    org = None if origins is None else _to_dev(origins, torch.float32, dev)
    spl = None if start_plane is None else _to_dev(start_plane, torch.int32, dev)
    sln = None if start_len is None else _to_dev(start_len, torch.float32, dev)
    src_h = _host_f32(src if src is not None else [0, 0, 0], 3)
    rrows = None if record_rows is None else _to_dev(record_rows, torch.int32, dev)
    if rrows is not None:
        assert rrows.shape == (n,)
    n_rec = n if rrows is None else (int(rrows.max().item()) + 1 if n else 0)
    if det_cap is None:
        det_cap = max(4 * n, 1024)
    if out is None:
        out = TraceResult(
            hit_seq=torch.empty((n, R1), dtype=torch.int32, device=dev),
            det=torch.empty((det_cap, 3), dtype=torch.int32, device=dev),
            counters=torch.zeros(4, dtype=torch.int64, device=dev),
            states=torch.full((max(n_rec, 0), R1 + 1, 8), float("nan"), dtype=torch.float32, device=dev)
            if record_states else None,
            max_reflections=max_reflections)
    prm = TraceParams(int(max_reflections), float(max_path_length), int(bool(record_states)), int(fetch_threshold),
                      int(shade_threshold), int(blocks_per_cu), int(bool(keep_order)), _ptr(stats),
                      int(rounds), int(spill_threshold), int(waves_per_simd), *_event_ptrs(kernel_events),
                      int(suspend_after), int(min_beam_rays), int(xcd_pools), int(coop_queries), _ptr(rrows),
                      int(stack_depth))
    with torch.cuda.device(dev):
        check(lib.rt_trace_rays(scene.handle, src_h, _ptr(org), _ptr(dirs), _ptr(spl), _ptr(sln), n, _ptr(rcv_t),
                                rcv_t.shape[0], ctypes.byref(prm), _ptr(out.hit_seq), _ptr(out.det),
                                out.det.shape[0], _ptr(out.counters), _ptr(out.states), _stream(dev)),
              "rt_trace_rays")
    if check_capacity:
        c = out.counters.cpu()
        if check_errors and int(c[3]) != 0:
            raise _lib.RtError("rt_trace_rays: device error word %d" % int(c[3]))
        if int(c[0]) > out.det.shape[0]:
            return trace_rays(scene, dirs, rcv_t, max_reflections, src, org, spl, sln, max_path_length,
                              record_states, det_cap=int(c[0]) + 1024, fetch_threshold=fetch_threshold,
                              shade_threshold=shade_threshold, blocks_per_cu=blocks_per_cu,
                              keep_order=keep_order, stats=stats, rounds=rounds,
                              spill_threshold=spill_threshold, waves_per_simd=waves_per_simd,
                              suspend_after=suspend_after, min_beam_rays=min_beam_rays, xcd_pools=xcd_pools,
                              coop_queries=coop_queries, record_rows=rrows, stack_depth=stack_depth)
    return out


PARAM_NAMES = ("EDT", "T30", "C80", "D50", "Ts", "SPL")


def room_params(hist, fs: float, device=None) -> torch.Tensor:
    """rt_room_params: [n_rcv, 8, L] energy histogram -> [n_rcv, 8, 6] float64
    (EDT s, T30 s, C80 dB, D50, Ts s, SPL dB); NaN where undefined."""
    lib = _lib.load()
    dev = hist.device if isinstance(hist, torch.Tensor) else _dev(device)
    h = _to_dev(hist, torch.float32, dev)
    assert h.dim() == 3 and h.shape[1] == 8
    out = torch.empty((h.shape[0], 8, 6), dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        check(lib.rt_room_params(_ptr(h), h.shape[0], h.shape[2], float(fs), _ptr(out), _stream(dev)),
              "rt_room_params")
    return out


def _event_ptrs(events):
    """(start, stop) torch.cuda.Event pair -> their hipEvent_t handles (the
    events are created by a first record on the current stream)."""
    if events is None:
        return (None, None)
    out = []
    for ev in events:
        if ev.cuda_event == 0:
            ev.record()
        out.append(ev.cuda_event)
    return tuple(out)


@dataclasses.dataclass
class ImageSources:
    key: torch.Tensor      # [cap, R+2] int32
    count: torch.Tensor    # [cap] int32
    pos: torch.Tensor      # [cap, 3] float64
    dist: torch.Tensor     # [cap] float64
    n_is_dev: torch.Tensor  # [1] int64 (device)
    max_reflections: int

    def n_is(self) -> int:
        return int(self.n_is_dev.item())

    def valid(self):
        n = min(self.n_is(), self.key.shape[0])
        return self.key[:n], self.count[:n], self.pos[:n], self.dist[:n]


def collect_image_sources(scene: Scene, src, rcv, tr: TraceResult, is_cap: Optional[int] = None,
                          check_capacity: bool = True, hit_seq=None, det=None, n_det_dev=None,
                          max_reflections: Optional[int] = None) -> ImageSources:
    """rt_collect_image_sources on a trace result (or on given hit_seq/det)."""
    lib = _lib.load()
    dev = scene.device
    hs = tr.hit_seq if tr is not None else _to_dev(hit_seq, torch.int32, dev)
    dt = tr.det if tr is not None else _to_dev(det, torch.int32, dev).reshape(-1, 3)
    nd = tr.counters[0:1] if tr is not None else (
        n_det_dev if n_det_dev is not None else torch.tensor([dt.shape[0]], dtype=torch.int64, device=dev))
    R = tr.max_reflections if tr is not None else int(max_reflections)
    rcv_t = _to_dev(rcv, torch.float32, dev).reshape(-1, 4)
    if is_cap is None:
        is_cap = max(dt.shape[0], 1)
    out = ImageSources(key=torch.empty((is_cap, R + 2), dtype=torch.int32, device=dev),
                       count=torch.empty(is_cap, dtype=torch.int32, device=dev),
                       pos=torch.empty((is_cap, 3), dtype=torch.float64, device=dev),
                       dist=torch.empty(is_cap, dtype=torch.float64, device=dev),
                       n_is_dev=torch.zeros(1, dtype=torch.int64, device=dev), max_reflections=R)
    with torch.cuda.device(dev):
        check(lib.rt_collect_image_sources(scene.handle, _host_f32(src, 3), _ptr(rcv_t), rcv_t.shape[0], _ptr(hs),
                                           hs.shape[0], R, _ptr(dt), dt.shape[0], _ptr(nd), _ptr(out.key),
                                           _ptr(out.count), _ptr(out.pos), _ptr(out.dist), is_cap,
                                           _ptr(out.n_is_dev), _stream(dev)), "rt_collect_image_sources")
    if check_capacity and out.n_is() > is_cap:
        return collect_image_sources(scene, src, rcv, tr, out.n_is(), True, hit_seq, det, n_det_dev,
                                     max_reflections)
    return out


@dataclasses.dataclass
class ImpulseResponse:
    band_energy: torch.Tensor   # [n_rcv, 8]
    hist: torch.Tensor          # [n_rcv, 8, L]
    band_ir: torch.Tensor       # [n_rcv, 8, L]
    ir: torch.Tensor            # [n_rcv, L]


def assemble_ir(scene: Scene, isrc: ImageSources, n_rays: int, n_rcv: int, alpha, beta, c: float, fs: float,
                L: int, fir, out: Optional[ImpulseResponse] = None) -> ImpulseResponse:
    lib = _lib.load()
    dev = scene.device
    a = _to_dev(alpha, torch.float32, dev)
    b = _to_dev(beta, torch.float32, dev)
    f = _to_dev(fir, torch.float32, dev)
    K = f.shape[1]
    if out is None:
        out = ImpulseResponse(band_energy=torch.empty((n_rcv, 8), dtype=torch.float32, device=dev),
                              hist=torch.empty((n_rcv, 8, L), dtype=torch.float32, device=dev),
                              band_ir=torch.empty((n_rcv, 8, L), dtype=torch.float32, device=dev),
                              ir=torch.empty((n_rcv, L), dtype=torch.float32, device=dev))
    with torch.cuda.device(dev):
        check(lib.rt_assemble_ir(scene.handle, _ptr(isrc.key), _ptr(isrc.count), _ptr(isrc.dist),
                                 _ptr(isrc.n_is_dev), isrc.key.shape[0], isrc.max_reflections, int(n_rays),
                                 int(n_rcv), _ptr(a), _ptr(b), float(c), float(fs), int(L), _ptr(f), int(K),
                                 _ptr(out.band_energy), _ptr(out.hist), _ptr(out.band_ir), _ptr(out.ir),
                                 _stream(dev)), "rt_assemble_ir")
    return out


def band_energy_adjoint(scene: Scene, isrc: ImageSources, n_rays: int, n_rcv: int, alpha, beta, c: float,
                        fs: float, L: int, grad_band_energy, n_mat: Optional[int] = None) -> torch.Tensor:
    lib = _lib.load()
    dev = scene.device
    a = _to_dev(alpha, torch.float32, dev)
    b = _to_dev(beta, torch.float32, dev)
    g = _to_dev(grad_band_energy, torch.float32, dev)
    n_mat = int(a.shape[0]) if n_mat is None else n_mat
    out = torch.empty((n_mat, 8), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(lib.rt_band_energy_adjoint(scene.handle, _ptr(isrc.key), _ptr(isrc.count), _ptr(isrc.dist),
                                         _ptr(isrc.n_is_dev), isrc.key.shape[0], isrc.max_reflections, int(n_rays),
                                         int(n_rcv), _ptr(a), n_mat, _ptr(b), float(c), float(fs), int(L), _ptr(g),
                                         _ptr(out), _stream(dev)), "rt_band_energy_adjoint")
    return out


class BandEnergy(torch.autograd.Function):
    """band_energy[r, b] as a differentiable function of alpha [n_mat, 8]
    for fixed ray paths (image sources); backward = rt_band_energy_adjoint."""

    @staticmethod
    def forward(ctx, alpha, scene, isrc, n_rays, n_rcv, beta, c, fs, L):
        taps = torch.zeros((8, 1), dtype=torch.float32, device=alpha.device)
        taps[:, 0] = 1.0
        ir = assemble_ir(scene, isrc, n_rays, n_rcv, alpha.detach(), beta, c, fs, L, taps)
        ctx.save_for_backward(alpha.detach())
        ctx.args = (scene, isrc, n_rays, n_rcv, beta, c, fs, L)
        return ir.band_energy.clone()

    @staticmethod
    def backward(ctx, grad):
        (alpha,) = ctx.saved_tensors
        scene, isrc, n_rays, n_rcv, beta, c, fs, L = ctx.args
        g = band_energy_adjoint(scene, isrc, n_rays, n_rcv, alpha, beta, c, fs, L, grad.contiguous(),
                                n_mat=alpha.shape[0])
        return g, None, None, None, None, None, None, None, None


class Batch:
    """Many jobs (source + receivers in one of several scenes) traced by one
    persistent launch (rt_batch_create / rt_trace_batch and friends).

    jobs: list of dicts with keys scene (index), src (3), rcv ([n, 4] array),
    n_rays, max_path_length.  Receivers of all jobs are stacked in job order
    (global rows); materials of all scenes are stacked in scene order."""

    def __init__(self, scenes, jobs, device=None):
        lib = _lib.load()
        self.device = _dev(device)
        self.scenes = list(scenes)
        self.jobs = [dict(j) for j in jobs]
        arr = (P * len(self.scenes))(*[sc.handle for sc in self.scenes])
        jt = (Job * len(self.jobs))()
        for i, j in enumerate(self.jobs):
            rcv = np.asarray(j["rcv"], np.float32).reshape(-1, 4)
            jt[i].scene = int(j["scene"])
            jt[i].n_rcv = len(rcv)
            jt[i].n_rays = int(j["n_rays"])
            for c in range(3):
                jt[i].src[c] = float(j["src"][c])
            jt[i].max_path_length = float(j.get("max_path_length", 0.0))
        self.rcv = torch.as_tensor(np.concatenate([np.asarray(j["rcv"], np.float32).reshape(-1, 4)
                                                   for j in self.jobs]), device=self.device)
        self._h = P()
        with torch.cuda.device(self.device):
            check(lib.rt_batch_create(arr, len(self.scenes), jt, len(self.jobs), _stream(self.device),
                                      ctypes.byref(self._h)), "rt_batch_create")
        info = (ctypes.c_int64 * 4)()
        check(lib.rt_batch_info(self._h, info), "rt_batch_info")
        self.n_jobs, self.n_rays, self.n_rcv, self.n_mat = [int(v) for v in info]
        self.ray_off = np.concatenate([[0], np.cumsum([int(j["n_rays"]) for j in self.jobs])]).astype(np.int64)
        self.rcv_off = np.concatenate([[0], np.cumsum([len(np.asarray(j["rcv"]).reshape(-1, 4))
                                                       for j in self.jobs])]).astype(np.int64)
        self.mat_off = np.concatenate([[0], np.cumsum([sc.n_mat for sc in self.scenes])]).astype(np.int64)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().rt_batch_destroy(self._h)
            self._h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trace_batch(b: Batch, max_reflections: int, det_cap: Optional[int] = None, out: Optional[TraceResult] = None,
                check_capacity: bool = True, min_beam_rays: int = 0, record_rows=None, **tune) -> TraceResult:
    """rt_trace_batch.  min_beam_rays as in trace_rays, per job (its rays and
    its receivers).  record_rows: int32 [total rays] map global ray -> row of
    the recorded states (-1: not recorded), or None (no states)."""
    lib = _lib.load()
    dev = b.device
    R1 = max_reflections + 1
    rrows = None if record_rows is None else _to_dev(record_rows, torch.int32, dev)
    if det_cap is None:
        det_cap = max(2 * b.n_rays, 1024)
    if out is None:
        states = None
        if rrows is not None:
            assert rrows.shape == (b.n_rays,)
            states = torch.full((int(rrows.max().item()) + 1, R1 + 1, 8), float("nan"), dtype=torch.float32,
                                device=dev)
        out = TraceResult(hit_seq=torch.empty((b.n_rays, R1), dtype=torch.int32, device=dev),
                          det=torch.empty((det_cap, 3), dtype=torch.int32, device=dev),
                          counters=torch.zeros(4, dtype=torch.int64, device=dev), states=states,
                          max_reflections=max_reflections)
    prm = TraceParams(int(max_reflections), 0.0, int(rrows is not None), int(tune.get("fetch_threshold", 0)),
                      int(tune.get("shade_threshold", 0)), int(tune.get("blocks_per_cu", 0)), 1, None,
                      int(tune.get("rounds", 0)), int(tune.get("spill_threshold", 0)),
                      int(tune.get("waves_per_simd", 0)), *_event_ptrs(tune.get("kernel_events")),
                      int(tune.get("suspend_after", 0)), int(min_beam_rays), int(tune.get("xcd_pools", 0)), 0,
                      _ptr(rrows), int(tune.get("stack_depth", 0)))
    with torch.cuda.device(dev):
        check(lib.rt_trace_batch(b.handle, _ptr(b.rcv), ctypes.byref(prm), _ptr(out.hit_seq), _ptr(out.det),
                                 out.det.shape[0], _ptr(out.counters), _ptr(out.states), _stream(dev)),
              "rt_trace_batch")
    if check_capacity:
        c = out.counters.cpu()
        if int(c[3]) != 0:
            raise _lib.RtError("rt_trace_batch: device error word %d" % int(c[3]))
        if int(c[0]) > out.det.shape[0]:
            return trace_batch(b, max_reflections, det_cap=int(c[0]) + 1024, min_beam_rays=min_beam_rays,
                               record_rows=rrows, **tune)
    return out


def collect_batch(b: Batch, tr: TraceResult, is_cap: Optional[int] = None, check_capacity: bool = True,
                  out: Optional[ImageSources] = None) -> ImageSources:
    lib = _lib.load()
    dev = b.device
    R = tr.max_reflections
    if is_cap is None:
        is_cap = max(tr.det.shape[0], 1)
    if out is None:
        out = ImageSources(key=torch.empty((is_cap, R + 2), dtype=torch.int32, device=dev),
                           count=torch.empty(is_cap, dtype=torch.int32, device=dev),
                           pos=torch.empty((is_cap, 3), dtype=torch.float64, device=dev),
                           dist=torch.empty(is_cap, dtype=torch.float64, device=dev),
                           n_is_dev=torch.zeros(1, dtype=torch.int64, device=dev), max_reflections=R)
    with torch.cuda.device(dev):
        check(lib.rt_collect_batch(b.handle, _ptr(b.rcv), _ptr(tr.hit_seq), R, _ptr(tr.det), tr.det.shape[0],
                                   _ptr(tr.counters[0:1]), _ptr(out.key), _ptr(out.count), _ptr(out.pos),
                                   _ptr(out.dist), out.key.shape[0], _ptr(out.n_is_dev), _stream(dev)),
              "rt_collect_batch")
    if check_capacity and out.n_is() > out.key.shape[0]:
        return collect_batch(b, tr, out.n_is(), True)
    return out


def assemble_batch(b: Batch, isrc: ImageSources, alpha, beta, c: float, fs: float, L: int, fir,
                   out: Optional[ImpulseResponse] = None) -> ImpulseResponse:
    lib = _lib.load()
    dev = b.device
    a = _to_dev(alpha, torch.float32, dev)
    be = _to_dev(beta, torch.float32, dev)
    f = _to_dev(fir, torch.float32, dev)
    n = b.n_rcv
    if out is None:
        out = ImpulseResponse(band_energy=torch.empty((n, 8), dtype=torch.float32, device=dev),
                              hist=torch.empty((n, 8, L), dtype=torch.float32, device=dev),
                              band_ir=torch.empty((n, 8, L), dtype=torch.float32, device=dev),
                              ir=torch.empty((n, L), dtype=torch.float32, device=dev))
    with torch.cuda.device(dev):
        check(lib.rt_assemble_batch(b.handle, _ptr(isrc.key), _ptr(isrc.count), _ptr(isrc.dist), _ptr(isrc.n_is_dev),
                                    isrc.key.shape[0], isrc.max_reflections, _ptr(a), _ptr(be), float(c), float(fs),
                                    int(L), _ptr(f), int(f.shape[1]), _ptr(out.band_energy), _ptr(out.hist),
                                    _ptr(out.band_ir), _ptr(out.ir), _stream(dev)), "rt_assemble_batch")
    return out


def adjoint_batch(b: Batch, isrc: ImageSources, alpha, beta, c: float, fs: float, L: int, grad_band_energy,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    lib = _lib.load()
    dev = b.device
    a = _to_dev(alpha, torch.float32, dev)
    be = _to_dev(beta, torch.float32, dev)
    g = _to_dev(grad_band_energy, torch.float32, dev)
    if out is None:
        out = torch.empty((b.n_mat, 8), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(lib.rt_adjoint_batch(b.handle, _ptr(isrc.key), _ptr(isrc.count), _ptr(isrc.dist), _ptr(isrc.n_is_dev),
                                   isrc.key.shape[0], isrc.max_reflections, _ptr(a), _ptr(be), float(c), float(fs),
                                   int(L), _ptr(g), _ptr(out), _stream(dev)), "rt_adjoint_batch")
    return out


def version() -> str:
    return _lib.load().rt_version().decode()
