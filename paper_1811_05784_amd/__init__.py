"""MI355X-native hot path of the hybrid ray-tracing / image-source room
acoustics method (Aussal & Gueguen 2018): tree build, ray generation,
specular propagation with receiver detection, image-source collection,
8-band impulse-response assembly and the absorption adjoint, as gfx950 HIP
kernels behind the C-ABI in include/rtac.h.  This package is the thin
binding (ctypes + torch tensors for device memory and streams).
"""
from ._lib import RtError, load  # noqa: F401
from .api import (BandEnergy, Batch, ImageSources, ImpulseResponse, Scene, TraceResult,  # noqa: F401
                  adjoint_batch, assemble_batch, assemble_ir, band_energy_adjoint, collect_batch,
                  collect_image_sources, directional_directions, fibonacci_directions,
                  icosahedral_directions, room_params, trace_batch, trace_rays, version)
