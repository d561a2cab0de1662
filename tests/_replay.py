"""Stepwise replay of recorded trace states through the FP64 oracle.

Every query a recorded ray made is re-run by ``oracle.query_batch`` from the
FP32 input state the GPU recorded for it (section "Standard algorithm": one
nearest-hit query per segment, from the ray's position, direction and
travelled length), continuing past any divergence on the GPU's own states.
Per query the GPU must give the oracle's hit triangle and detections and its
next state within 4 FP32 ulp, and stop where the oracle stops, unless the
oracle flags the query.  A flagged mismatch must still be a valid answer:

* a GPU hit on triangle g: g's FP64 plane crossing lies ahead of the ray,
  within eps*D of the triangle, and not more than eps*D beyond the oracle's
  nearest hit (a tie, an edge, or a near miss in front of it), or, beyond it,
  only past triangles the ray crosses within eps*D of their boundary (an
  edge or vertex seam where the mesh is open, decided by rounding);
* a GPU escape: only where the oracle's hit lies within eps*D of its edges
  (flags EDGE or NEAR_MISS) and the ray crosses every triangle within eps*D
  of its boundary;
* a detection mismatch: only with the oracle's TANGENT flag or a changed hit;
* a different stop: only with the LENGTH flag.
"""
import numpy as np

from tests._util import crossing_and_miss, skips_only_at_boundaries


def det_bits(det, rows_of_ray, n_rows, R1, rcv_off=None):
    """(ray, k, receiver) rows -> [n_rows, R1] bit masks for the rays in
    rows_of_ray (dict ray -> row)."""
    bits = np.zeros((n_rows, R1), np.uint32)
    for ray, k, m in det:
        row = rows_of_ray.get(int(ray))
        if row is not None:
            mm = int(m) - (0 if rcv_off is None else int(rcv_off[row]))
            bits[row, int(k)] |= np.uint32(1) << np.uint32(mm)
    return bits


def replay(oracle_lib, osc, vtx, tri, states, hit_seq, bits, rcv_of_row, lim_of_row, R, diag, eps=1e-6):
    """states [n, R+2, 8] FP32 as recorded; hit_seq [n, R+1] and bits [n, R+1]
    of the same rays; rcv_of_row(row) -> [n_rcv, 4] receivers of that ray's
    call or job; lim_of_row [n] FP32 path-length limits (inf: none).  Returns
    counts and the list of problems (unflagged or invalid mismatches)."""
    O = oracle_lib
    n, R1 = hit_seq.shape
    # every state a query may have started from: segment 0, and each segment
    # after a hit (the GPU may have stopped there by R or length: checked below)
    qs = []
    for i in range(n):
        for k in range(R1):
            if k > 0 and hit_seq[i, k - 1] < 0:
                break
            if np.isnan(states[i, k, 0]):
                break
            qs.append((i, k))
    qs = np.array(qs, np.int64).reshape(-1, 2)
    st = states[qs[:, 0], qs[:, 1]]
    o, u, L = st[:, 0:3], st[:, 3:6], st[:, 6]
    lp = st[:, 7].copy().view(np.int32)
    # one oracle batch per receiver set (jobs may differ)
    groups = {}
    for q, (i, k) in enumerate(qs):
        groups.setdefault(id(rcv_of_row(i)), (rcv_of_row(i), []))[1].append(q)
    ref = dict(hit=np.empty(len(qs), np.int32), delta=np.empty(len(qs)), det=np.empty(len(qs), np.uint32),
               next=np.empty((len(qs), 7)), flags=np.empty(len(qs), np.uint32))
    for rcv, idx in groups.values():
        idx = np.array(idx)
        lims = lim_of_row[qs[idx, 0]]
        for lim in np.unique(lims):
            sel = idx[lims == lim]
            r = O.query_batch(osc, o[sel], u[sel], lp[sel], L[sel], rcv,
                              max_len=0.0 if not np.isfinite(lim) else float(lim), eps=eps)
            for key in ref:
                ref[key][sel] = r[key]
    at = {(int(i), int(k)): q for q, (i, k) in enumerate(qs)}
    epsD = eps * diag
    out = dict(n_queries=0, n_flagged=0, n_flagged_mismatch=0, problems=[])
    for i in range(n):
        k = 0
        while k < R1:
            q = at.get((i, k))
            if q is None:
                out["problems"].append("ray row %d: no recorded state for segment %d" % (i, k))
                break
            out["n_queries"] += 1
            fl = int(ref["flags"][q])
            g, h = int(hit_seq[i, k]), int(ref["hit"][q])
            gd, hd = int(bits[i, k]), int(ref["det"][q])
            if fl:
                out["n_flagged"] += 1
                if g != h or gd != hd:
                    out["n_flagged_mismatch"] += 1
            where = "ray row %d segment %d (flags %d, gpu %d, oracle %d)" % (i, k, fl, g, h)
            if g != h:
                if not fl:
                    out["problems"].append("unflagged hit mismatch at " + where)
                elif g >= 0:
                    v = tri[g]
                    t, miss = crossing_and_miss(o[q], u[q], vtx[v[0]], vtx[v[1]], vtx[v[2]])
                    far = ref["delta"][q] if h >= 0 else np.inf
                    if not (t[0] > 0 and miss[0] <= epsD and
                            (t[0] <= far + epsD or skips_only_at_boundaries(o[q], u[q], t[0], vtx, tri, epsD))):
                        out["problems"].append("invalid GPU hit at %s: t %.9g miss %.3g oracle t %.9g"
                                               % (where, t[0], miss[0], far))
                elif not (fl & (O.FLAG_EDGE | O.FLAG_NEAR_MISS) and
                          skips_only_at_boundaries(o[q], u[q], np.inf, vtx, tri, epsD)):
                    out["problems"].append("GPU escape not at an edge or near miss at " + where)
            if gd != hd and g == h and not fl & O.FLAG_TANGENT:
                out["problems"].append("detection mismatch (gpu %x oracle %x) at %s" % (gd, hd, where))
            if g < 0:
                break                                   # the GPU's ray ended here (escape)
            if g == h:
                nx = states[i, k + 1]
                ro = ref["next"][q]
                mag = np.maximum(np.abs(ro[:3]), np.abs(o[q]).astype(np.float64)).max()
                e_o = np.abs(nx[:3].astype(np.float64) - ro[:3]).max() / float(np.spacing(np.float32(mag)))
                # direction components: 4 ulp of each, or FP64 noise for components near 0
                du = np.abs(nx[3:6].astype(np.float64) - ro[3:6])
                e_u = float((du / (np.spacing(np.abs(ro[3:6]).astype(np.float32)).astype(np.float64) + 1e-13)).max())
                e_L = abs(float(nx[6]) - ro[6]) / float(np.spacing(np.float32(abs(ro[6]))))
                if (e_o > 4 or e_u > 4 or e_L > 4) and not fl:
                    out["problems"].append("next state off by %.1f / %.1f / %.1f ulp at %s" % (e_o, e_u, e_L, where))
            # the oracle's stop after this segment (its next length, or the
            # GPU's where the hits differ)
            L_next = ref["next"][q, 6] if g == h else float(states[i, k + 1, 6])
            stop_o = k == R1 - 1 or L_next >= lim_of_row[i]
            gpu_more = k + 1 < R1 and (hit_seq[i, k + 1] >= 0 or bits[i, k + 1] != 0)
            if stop_o and gpu_more and not fl & O.FLAG_LENGTH:
                out["problems"].append("GPU continued past the oracle's stop at " + where)
            if not gpu_more and (stop_o or fl & O.FLAG_LENGTH):
                break
            # otherwise the GPU traced segment k + 1 (it may have escaped there)
            k += 1
    return out
