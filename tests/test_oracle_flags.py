"""The oracle's flags cover rays through shared edges and vertices.

A ray aimed at a mesh vertex or at the midpoint of an axis-aligned edge of an
axis-aligned mesh reaches that point at parameter 1, and the point lies on
the mesh (its coordinates are exact in FP32), so the nearest hit lies at a
parameter of at most 1 (section "Standard algorithm": the nearest crossing of
a closed triangle, 0 <= lambda, mu and lambda + mu <= 1).  In floating point
the closed-triangle test can reject every triangle of the fan by the rounding
of lambda and mu; the query must then carry a flag (the triangles pass within
the tolerance of the ray), so that a different answer on the GPU is judged
by the validity checks and not taken for an error."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("make,n", [(lambda: synth.tessellated_box_c2(jitter=False), 6000),
                                    (synth.shoebox_c1, 20000)])
def test_rays_through_vertices_and_edges_hit_there_or_are_flagged(oracle_lib, make, n):
    s = make()
    o, u, lp, L = synth.tie_query_states(s, n, seed=23)
    ref = oracle_lib.query_batch(oracle_lib.OracleScene.of(s), o, u, lp, L, s.rcv)
    beyond = (ref["hit"] < 0) | (ref["delta"] > 1.0 + 1e-9)
    assert np.all(ref["flags"][beyond] != 0), np.nonzero(beyond & (ref["flags"] == 0))[0][:10]
    # most of these queries meet several triangles at the target: most are flagged
    assert (ref["flags"] != 0).mean() > 0.5
