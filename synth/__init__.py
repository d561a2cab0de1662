"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only *describes* inputs: meshes, materials, sources, receivers,
absorption tables, band filters, seeded query states and seeded ray-path
tables.  It performs none of the method's arithmetic (no intersection,
reflection, detection, image-source or impulse-response computation), so it
can feed both the FP64 oracle and the HIP library without coupling them.
"""
from .scenes import *  # noqa: F401,F403
