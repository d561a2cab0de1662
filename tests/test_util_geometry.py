"""Pins of the test-side geometry used to check flagged queries: crossing
distance and point-to-triangle distance on cases worked out by hand."""
import math

import numpy as np

from tests._util import crossing_and_miss


def test_crossing_inside_outside_and_parallel():
    v0, v1, v2 = [0, 0, 5], [2, 0, 5], [0, 2, 5]
    o = np.zeros((5, 3))
    u = np.array([[0.25, 0.25, 1],      # (1.25, 1.25, 5): beyond the hypotenuse
                  [0.1, 0.1, 1],        # inside at (0.5, 0.5, 5)
                  [-0.2, 0.1, 1],       # (-1, 0.5, 5): 1 m left of the x = 0 edge
                  [1, 0, 0],            # parallel to the plane
                  [0.6, -0.2, 1]])      # (3, -1, 5): nearest point is the vertex (2, 0, 5)
    t, miss = crossing_and_miss(o, u, [v0] * 5, [v1] * 5, [v2] * 5)
    assert np.allclose(t[[0, 1, 2, 4]], 5.0) and t[3] == np.inf and miss[3] == np.inf
    # (1.25, 1.25) lies beyond the hypotenuse x + y = 2 by (2.5 - 2) / sqrt 2
    assert math.isclose(miss[0], 0.5 / math.sqrt(2), rel_tol=1e-12)
    assert miss[1] == 0.0
    assert math.isclose(miss[2], 1.0, rel_tol=1e-12)
    assert math.isclose(miss[4], math.sqrt(2.0), rel_tol=1e-12)


def test_crossing_behind_and_on_edge():
    t, miss = crossing_and_miss([[0, 0, 10]], [[0, 0, 1]], [[0, 0, 5]], [[2, 0, 5]], [[0, 2, 5]])
    assert t[0] == -5.0 and miss[0] == 0.0          # behind the origin: negative t
    t, miss = crossing_and_miss([[1, 0, 0]], [[0, 0, 2]], [[0, 0, 5]], [[2, 0, 5]], [[0, 2, 5]])
    assert t[0] == 2.5 and miss[0] == 0.0           # on the edge y = 0


def test_skips_only_at_boundaries():
    """Two unit triangles side by side in z = 0 that share no vertices (a seam
    along x = 1, y in [0, 1]) and a third in z = 2: a ray straight down
    through the seam may be answered by the far triangle (it passes the near
    ones at their boundary); through a near triangle's interior it may not;
    an escape is judged the same way."""
    from tests._util import skips_only_at_boundaries
    vtx = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0],       # near triangle A (edge x = 1)
                    [1, 0, 0], [2, 0, 0], [1, 1, 0],       # near triangle B, separate copies of the vertices
                    [-5, -5, -2], [5, -5, -2], [0, 5, -2]], np.float64)
    tri = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]])
    down = np.array([0.0, 0.0, -1.0])
    eps = 1e-9
    assert skips_only_at_boundaries([1.0, 0.5, 1.0], down, 3.0, vtx, tri, eps)          # through the seam
    assert not skips_only_at_boundaries([0.9, 0.5, 1.0], down, 3.0, vtx, tri, eps)      # through A's interior
    assert skips_only_at_boundaries([0.9, 0.5, 1.0], down, 1.0, vtx, tri, eps)          # A itself answered
    assert skips_only_at_boundaries([1.0, 1.0, 1.0], down, np.inf, vtx, tri, 1e-9) is False  # far one missed
    assert skips_only_at_boundaries([7.0, 7.0, 1.0], down, np.inf, vtx, tri, eps)       # crosses nothing
