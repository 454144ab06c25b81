"""MI355X (gfx950) Gabor-field rendering: HIP kernels behind a C ABI.

``paper_2602_05081_amd._lib`` holds the thin ctypes binding (one Python
function per C entry point); ``paper_2602_05081_amd.autograd`` wraps the
optical depth and its adjoint in a ``torch.autograd.Function``.
"""
from . import _lib  # noqa: F401
from ._lib import (Scene, GfError, gf_mask, make_mask, gf_scene_create, gf_scene_export_lbvh,  # noqa: F401
                   gf_scene_cells, gf_mask_lod_cells, gf_mask_cone, gf_optical_depth, gf_optical_depth_counts,
                   gf_density, gf_transmittance_ratio, gf_render_rays, gf_render, gf_render_workspace_size, gf_render_noalloc,
                   gf_render_counts, render_desc, camera, gf_camera_rays, LEVEL, BIN,
                   gf_optical_depth_backward, gf_server_simulate, FULL_CELLS)
