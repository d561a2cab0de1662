"""The trace kernel rejects a receiver sphere before its FP64 test when the
ray's line clears the sphere in FP32 by 64 units of 2^-24 |w|^2 (w = centre -
origin).  This checks that bound on the CPU: the FP32 evaluation of the
squared line distance, in numpy float32 (each operation rounded), never
rejects a sphere that the exact line distance (rational arithmetic) reaches,
on rays aimed within a relative 1e-5 of tangency from up to 2 km away, and it
does reject the spheres far from the line."""
from fractions import Fraction

import numpy as np


def _screen_rejects(o, u, c, r):
    f = np.float32
    o = o.astype(f)
    u = u.astype(f)
    c = c.astype(f)
    r = f(r)
    inv_uu = f(1.0) / (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])
    w = c - o
    a = w[0] * w[0] + w[1] * w[1] + w[2] * w[2]
    b = w[0] * u[0] + w[1] * u[1] + w[2] * u[2]
    return bool(a - b * b * inv_uu > r * r + f(2.0 ** -18) * a)


def _exact_line_d2(o, u, c):
    o = [Fraction(float(x)) for x in o.astype(np.float32)]
    u = [Fraction(float(x)) for x in u.astype(np.float32)]
    c = [Fraction(float(x)) for x in c.astype(np.float32)]
    w = [c[i] - o[i] for i in range(3)]
    a = sum(x * x for x in w)
    b = sum(w[i] * u[i] for i in range(3))
    uu = sum(x * x for x in u)
    return a - b * b / uu


def test_screen_never_rejects_a_reachable_sphere():
    rng = np.random.default_rng(12)
    bad = 0
    near = 0
    for _ in range(4000):
        o = rng.uniform(-1000, 1000, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        u *= rng.uniform(0.5, 2.0)                  # directions are not exactly unit
        r = float(np.float32(rng.uniform(0.1, 5.0)))
        t = rng.uniform(-50, 2000)
        side = rng.normal(size=3)
        side -= side.dot(u) / u.dot(u) * u
        side /= np.linalg.norm(side)
        d = r * (1 + rng.uniform(-1e-5, 1e-5))       # within 1e-5 of tangency
        c = o + t * u + d * side
        exact_r2 = Fraction(float(np.float32(r))) ** 2
        if _exact_line_d2(o, u, c) <= exact_r2:
            near += 1
            if _screen_rejects(o, u, c, r):
                bad += 1
    assert near > 1000 and bad == 0


def test_screen_rejects_spheres_far_from_the_line():
    rng = np.random.default_rng(13)
    rejected = 0
    for _ in range(2000):
        o = rng.uniform(-100, 100, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = rng.uniform(-100, 100, 3)
        r = 2.0
        if float(_exact_line_d2(o, u, c)) > 4.0 * 1.01:
            rejected += _screen_rejects(o, u, c, r)
            continue
        rejected += 1
    assert rejected == 2000
