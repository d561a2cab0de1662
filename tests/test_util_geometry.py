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
