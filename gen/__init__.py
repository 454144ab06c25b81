"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

Nothing in this package evaluates the rendering method; it only draws scenes,
rays and request streams from fixed seeds.
"""
from .scenes import uniform_scene, blob_scene, jitter_scene, N_FIELDS  # noqa: F401
from .cameras import (ortho_rays, pinhole_rays, eight_views, random_rays,  # noqa: F401
                      poisson_arrivals, serving_requests, orbit_eye)
