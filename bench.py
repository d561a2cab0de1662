"""Benchmark of the whole hot path on the synthetic open-air theater.

Workload (one "step"): 436,120-triangle open-air theater, 1e6 Fibonacci rays
from a point source, up to 60 reflections, 8 receiver spheres (r = 2 m), 2 s
impulse response at 48 kHz, 8 octave bands (K = 4095 FIR taps):
scene ingest + tree build, ray generation, trace, image-source collection,
impulse-response assembly.  Inputs are resident in HBM before timing.

value = device-counted ray segments (rays x bounces) / step time.
roofline: the traversal kernel's algorithmic bytes per query
B(M) = 76 + 48 ceil(log2 M) + 40 (ray state, one root-to-leaf path of 2-child
boxes, one triangle) times queries per launch, over the traversal kernel's
own HIP-event time (events recorded by the library around its launch, on
its stream), vs the 8 TB/s HBM peak.  cpu_baseline: the FP64 brute-force oracle on a bounded
sample of the same rays.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_query(m: int) -> int:
    return 76 + 48 * math.ceil(math.log2(m)) + 40


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rays", type=int, default=1_000_000)
    ap.add_argument("--cpu-rays", type=int, default=3000, help="oracle sample size (rays)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--leaf", type=int, default=1)
    ap.add_argument("--shade", type=int, default=0)
    ap.add_argument("--fetch", type=int, default=0)
    ap.add_argument("--bpc", type=int, default=0)
    ap.add_argument("--keep-order", action="store_true")
    ap.add_argument("--rounds", type=int, default=0)
    ap.add_argument("--spill", type=int, default=0)
    ap.add_argument("--wps", type=int, default=0, help="trace kernel waves per SIMD (4, 5, 6, 8)")
    ap.add_argument("--stats", action="store_true", help="count traversal work (extra pass, not timed)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the ray set would be split "
              "by ray id across GPUs with the scene replicated; not implemented). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1811_05784_amd as rt
    import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    s = synth.theater_c3(n_rays=args.rays)
    R = s.max_reflections
    L = s.ir_len
    taps = synth.octave_fir_taps(4095)
    n_rcv = len(s.rcv)
    # inputs resident in HBM
    vtx = torch.as_tensor(s.vtx, device=dev)
    tri = torch.as_tensor(s.tri, device=dev)
    mat = torch.as_tensor(s.material, device=dev)
    pid = torch.as_tensor(s.plane_id, device=dev)
    rcv = torch.as_tensor(s.rcv, device=dev)
    alpha = torch.as_tensor(s.alpha, device=dev)
    beta = torch.as_tensor(s.beta, device=dev)
    fir = torch.as_tensor(taps, device=dev)
    det_cap = 6 * args.rays
    stream = torch.cuda.current_stream()

    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("build", "raygen", "trace", "collect", "assemble", "k_trace")}
    state = {}

    def step(record=False):
        def mark(name, i):
            if record:
                ev[name][i].record(stream)
        mark("build", 0)
        sc = rt.Scene(vtx, tri, mat, pid, leaf_size=args.leaf, device=dev)
        mark("build", 1)
        mark("raygen", 0)
        dirs = rt.fibonacci_directions(args.rays, device=dev)
        mark("raygen", 1)
        mark("trace", 0)
        tr = rt.trace_rays(sc, dirs, rcv, R, src=s.src, max_path_length=s.max_path_length, det_cap=det_cap,
                           check_capacity=False, out=state.get("tr"), shade_threshold=args.shade,
                           fetch_threshold=args.fetch, blocks_per_cu=args.bpc, keep_order=args.keep_order,
                           rounds=args.rounds, spill_threshold=args.spill, waves_per_simd=args.wps,
                           kernel_events=ev["k_trace"] if record else None)
        mark("trace", 1)
        state["tr"] = tr
        mark("collect", 0)
        isrc = rt.collect_image_sources(sc, s.src, rcv, tr, is_cap=det_cap, check_capacity=False)
        mark("collect", 1)
        mark("assemble", 0)
        ir = rt.assemble_ir(sc, isrc, args.rays, n_rcv, alpha, beta, s.c, s.fs, L, fir, out=state.get("ir"))
        mark("assemble", 1)
        state["ir"] = ir
        state["isrc"] = isrc
        state["scene"] = sc
        return sc

    if args.calib_copy_mb:
        src_buf = torch.ones(args.calib_copy_mb * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst_buf = torch.empty_like(src_buf)
        torch.cuda.synchronize()
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    c = state["tr"].counters.cpu()
    if int(c[0]) > det_cap or int(c[3]) != 0 or state["isrc"].n_is() > det_cap:
        raise SystemExit("capacity or device error: counters=%s n_is=%d" % (c.tolist(), state["isrc"].n_is()))
    phase = {k: 0.0 for k in ev}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(record=True)
        torch.cuda.synchronize()
        for k, (a, b) in ev.items():
            phase[k] += a.elapsed_time(b)
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    phase = {k: v / args.steps for k, v in phase.items()}
    c = state["tr"].counters.cpu()
    queries = int(c[1])
    value = queries / (ms * 1e-3)
    B = algorithmic_bytes_per_query(s.n_tri)
    trace_ms = phase["trace"]
    kernel_ms = phase.pop("k_trace")
    achieved = queries * B / (kernel_ms * 1e-3) / 1e9

    out = {
        "metric": "rays·bounces/s at 436k tris, 1e6 rays (HBM roofline %); IR band error vs oracle",
        "value": value,
        "unit": "rays·bounces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 traversal, f64 shading/image sources, f32 MFMA FIR",
        "data": "synthetic (seeded theater stand-in for the 436k-face mesh; Fibonacci rays)",
        "config": {"workload": "open-air theater 436,120 tris, 1e6 rays, R=60, 8 receivers r=2 m, 2 s IR "
                               "@48 kHz, 8 bands, K=4095", "n_tri": s.n_tri, "rays": args.rays,
                   "max_reflections": R, "receivers": n_rcv, "ir_samples": L, "leaf_size": args.leaf},
        "queries": queries,
        "detections": int(c[0]),
        "escapes": int(c[2]),
        "image_sources": state["isrc"].n_is(),
        "phase_ms": phase,
        "trace_rays_bounces_per_s": queries / (trace_ms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_trace", "bytes_per_query": B, "kernel_ms": kernel_ms},
    }
    if args.stats:
        st = torch.zeros(4, dtype=torch.int64, device=dev)
        sc = state["scene"]
        rt.trace_rays(sc, rt.fibonacci_directions(args.rays, device=dev), rcv, R, src=s.src,
                      max_path_length=s.max_path_length, det_cap=det_cap, stats=st, keep_order=args.keep_order)
        st = st.cpu().tolist()
        out["traversal_per_query"] = {"inner_nodes": st[0] / queries, "leaves": st[1] / queries,
                                      "triangles": st[2] / queries, "spills": st[3] / queries,
                                      "tree_nodes": sc.n_nodes, "tree_depth": sc.depth}
    out["roofline"]["traffic"] = measured_traffic()
    # IR band error vs the oracle on a seeded image-source table of this shape
    try:
        out["ir_band_error"] = band_error(rt, state["scene"], s, taps)
    except Exception as e:  # report, never hide
        out["ir_band_error"] = "failed: %r" % (e,)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_rays)
    print(json.dumps(out), flush=True)


def measured_traffic():
    """HBM bytes per k_trace launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-kernel calibrated), or None when the kernel
    source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_trace_theater_436k_counters.txt")
    src = os.path.join(ROOT, "paper_1811_05784_amd", "csrc", "trace.hip")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k] = v
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if kv.get("trace_source_sha256_16") != sha:
        return None
    return int(kv["traffic_bytes_per_launch"])


def band_error(rt, sc, s, taps):
    import torch

    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from tests._util import material_of_plane, synthetic_is_table
    n_rays, R, n_rcv, L = 1_000_000, 60, 2, s.ir_len
    tab, arr = synthetic_is_table(s, 20_000, R, n_rcv, seed=31, L=L, c=s.c, fs=s.fs, n_rays=n_rays)
    dev = "cuda:0"
    n = len(arr)
    isrc = rt.ImageSources(key=torch.as_tensor(arr, device=dev),
                           count=torch.as_tensor(tab["count"].astype(np.int32), device=dev),
                           pos=torch.zeros((n, 3), dtype=torch.float64, device=dev),
                           dist=torch.as_tensor(tab["dist"], device=dev),
                           n_is_dev=torch.tensor([n], dtype=torch.int64, device=dev), max_reflections=R)
    ir = rt.assemble_ir(sc, isrc, n_rays, n_rcv, s.alpha, s.beta, s.c, s.fs, L, taps)
    ref = oracle.assemble_ir(tab, n_rays, n_rcv, s.alpha, s.beta, material_of_plane(s), s.c, s.fs, L, taps)
    be = ir.band_energy.cpu().numpy().astype(np.float64)
    eb = (ir.band_ir.cpu().numpy().astype(np.float64) ** 2).sum(-1)
    er = (ref["band_ir"] ** 2).sum(-1)
    return {"band_energy_max_rel": float(np.max(np.abs(be - ref["band_energy"]) / ref["band_energy"])),
            "fir_energy_max_rel": float(np.max(np.abs(eb - er) / er)),
            "sample": "seeded image-source table, %d sources, 2 receivers, L=%d, K=4095" % (n, L)}


def cpu_baseline(s, n_cpu):
    import oracle
    dirs_all = oracle.fibonacci(s.n_rays)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(s.n_rays, size=n_cpu, replace=False))
    dirs = np.ascontiguousarray(dirs_all[pick])
    sc = oracle.OracleScene.of(s)
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    tr = oracle.trace(sc, s.src, dirs, s.rcv, s.max_reflections, max_len=s.max_path_length, flags=False,
                      threads=threads)
    dt = time.perf_counter() - t0
    q = int(tr["tests"] // s.n_tri)          # every brute-force query tests all triangles once
    return {"value": q / dt, "unit": "rays·bounces/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the 1e6 Fibonacci rays (seeded choice), full trajectories, FP64 brute force over "
                      "all %d triangles; %d queries in %.1f s" % (n_cpu, s.n_tri, q, dt),
            "triangle_tests_per_s": tr["tests"] / dt}


if __name__ == "__main__":
    main()
