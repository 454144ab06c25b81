"""ctypes binding of libgaborfields.so (argument marshalling only).

Every function here has the name of the C entry point it calls (see
include/gaborfields.h) and takes torch tensors that already live on the GPU;
the work is done by the HIP kernels of the library.  The library is loaded
from the package directory; a missing library is an error (no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgaborfields.so")

GF_OK, GF_EINVAL, GF_ENOMEM, GF_EDEVICE, GF_ESTATE, GF_EBUSY = 0, -1, -2, -3, -4, -5
FULL_CELLS = (1 << 12) - 1


class GfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("gaborfields status %d: %s" % (status, msg))
        self.status = status


class gf_mask(C.Structure):
    _fields_ = [("cells", C.c_uint64), ("prim_bits", C.c_void_p), ("lod_k", C.c_float)]


class gf_scene_desc(C.Structure):
    _fields_ = [("rho", C.c_float), ("trunc_r", C.c_float), ("majorant_grid", C.c_int), ("clamp_eps", C.c_float)]


class gf_scene_info_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("rho", C.c_float), ("trunc_r", C.c_float), ("clamp_eps", C.c_float),
                ("fmax", C.c_double),
                ("nonempty_cells", C.c_uint64), ("cell_count", C.c_int64 * 12),
                ("cell_median_kw", C.c_float * 12), ("grid_res", C.c_int), ("bounds_lo", C.c_float * 3),
                ("bounds_hi", C.c_float * 3), ("device_bytes", C.c_size_t)]


class gf_render_desc(C.Structure):
    _fields_ = [("spp", C.c_int), ("multiple", C.c_int), ("max_scatter", C.c_int), ("albedo", C.c_float),
                ("hg_g", C.c_float), ("env", C.c_float), ("stochastic", C.c_int), ("level_strategy", C.c_int),
                ("bin_strategy", C.c_int), ("beta", C.c_float), ("delta", C.c_float), ("free_flight", C.c_int),
                ("transmittance", C.c_int), ("shadow_cells", C.c_uint64), ("mask", gf_mask), ("seed", C.c_uint64)]


# strategy codes of the per-segment stochastic masks (gf_level_strategy / gf_bin_strategy)
LEVEL = dict(deterministic=0, uniform=1, power=2, uniform_cv=3, power_cv=4, power_cv_accum=5)
BIN = dict(deterministic=0, threshold=1, uniform=2, importance=3, threshold_uniform=4, mixture=5)


class gf_camera(C.Structure):
    _fields_ = [("kind", C.c_int), ("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_y_deg", C.c_float), ("width", C.c_int), ("height", C.c_int)]


class gf_request(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("camera", gf_camera), ("render", gf_render_desc), ("out", C.c_void_p)]


_lib = None
_vp, _i64, _u64, _i = C.c_void_p, C.c_int64, C.c_uint64, C.c_int

_SIGS = {
    "gf_scene_create": [_vp, _i64, C.POINTER(gf_scene_desc), _vp, C.POINTER(_vp)],
    "gf_scene_destroy": [_vp],
    "gf_scene_info": [_vp, C.POINTER(gf_scene_info_t)],
    "gf_scene_export_lbvh": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "gf_scene_cells": [_vp, _vp, _vp],
    "gf_mask_cone": [_vp, C.POINTER(C.c_float), C.c_float, _vp, _vp],
    "gf_optical_depth": [_vp, _vp, _i64, _i, gf_mask, _vp, _vp, _vp],
    "gf_optical_depth_counts": [_vp, _vp, _i64, _i, gf_mask, _vp, _vp, _vp],
    "gf_density": [_vp, _vp, _i64, gf_mask, _vp, _vp, _vp],
    "gf_transmittance_ratio": [_vp, _vp, _i64, _i, gf_mask, _i, _u64, _vp, _vp, _vp],
    "gf_render_rays": [_vp, _vp, _i64, _i, C.POINTER(gf_render_desc), _vp, _vp, _vp, _vp, _vp],
    "gf_render_workspace_size": [_vp, C.POINTER(gf_camera), C.POINTER(gf_render_desc), C.POINTER(C.c_size_t)],
    "gf_render": [_vp, C.POINTER(gf_camera), C.POINTER(gf_render_desc), _vp, C.c_size_t, _vp, _vp, _vp],
    "gf_render_noalloc": [_vp, C.POINTER(gf_camera), C.POINTER(gf_render_desc), _vp, _vp, _vp],
    "gf_render_counts": [_vp, _vp, _i64, _i, C.POINTER(gf_render_desc), _vp, _vp],
    "gf_camera_rays": [C.POINTER(gf_camera), _vp, _vp],
    "gf_optical_depth_backward": [_vp, _vp, _i64, _i, gf_mask, _vp, _vp, _vp, _vp, _vp],
    "gf_server_create": [C.c_size_t, _i, _i, _vp, C.POINTER(_vp)],
    "gf_server_destroy": [_vp],
    "gf_server_submit": [_vp, C.POINTER(gf_request), C.POINTER(_u64)],
    "gf_server_step": [_vp, _i],
    "gf_server_poll": [_vp, C.POINTER(_u64), _i, C.POINTER(_i)],
    "gf_server_stats": [_vp, C.POINTER(_i), C.POINTER(_i), C.POINTER(C.c_size_t)],
    "gf_server_simulate": [C.c_size_t, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, C.c_double, _vp, _vp,
                           C.POINTER(C.c_size_t)],
}


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgaborfields.so is not built (run paper_2602_05081_amd.build.build())")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = C.c_int
        L.gf_last_error.restype = C.c_char_p
        L.gf_mask_lod_cells.restype = C.c_uint64
        L.gf_mask_lod_cells.argtypes = [C.c_int]
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS) + ["gf_last_error", "gf_mask_lod_cells"]


def _check(status):
    if status != GF_OK:
        raise GfError(status, lib().gf_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError("tensor required")
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected %s, got %s" % (dtype, t.dtype))
    return C.c_void_p(t.data_ptr())


def make_mask(cells=FULL_CELLS, prim_bits=None, lod_k=0.0) -> gf_mask:
    return gf_mask(cells, None if prim_bits is None else prim_bits.data_ptr(), lod_k)


class Scene:
    """A resident scene (owns the C handle)."""

    def __init__(self, params: torch.Tensor, rho: float, trunc_r: float = 3.0, majorant_grid: int = 0,
                 clamp_eps: float = 0.0):
        h = C.c_void_p()
        desc = gf_scene_desc(rho, trunc_r, majorant_grid, clamp_eps)
        _check(lib().gf_scene_create(_ptr(params, torch.float32), params.shape[0], C.byref(desc), _stream(),
                                     C.byref(h)))
        self.handle = h
        self.n = int(params.shape[0])

    def info(self) -> gf_scene_info_t:
        out = gf_scene_info_t()
        _check(lib().gf_scene_info(self.handle, C.byref(out)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().gf_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gf_scene_create(params, rho, trunc_r=3.0, majorant_grid=0, clamp_eps=0.0) -> Scene:
    return Scene(params, rho, trunc_r, majorant_grid, clamp_eps)


def gf_scene_export_lbvh(scene: Scene):
    n = scene.n
    dev = torch.device("cuda")
    out = dict(keys=torch.empty(n, dtype=torch.int64, device=dev),
               perm=torch.empty(n, dtype=torch.int32, device=dev),
               left=torch.empty(max(n - 1, 1), dtype=torch.int32, device=dev),
               right=torch.empty(max(n - 1, 1), dtype=torch.int32, device=dev),
               parent=torch.empty(2 * n - 1, dtype=torch.int32, device=dev),
               aabb=torch.empty((2 * n - 1, 6), dtype=torch.float32, device=dev),
               cellor=torch.empty(2 * n - 1, dtype=torch.int64, device=dev))
    _check(lib().gf_scene_export_lbvh(scene.handle, *[_ptr(out[k]) for k in
                                                       ("keys", "perm", "left", "right", "parent", "aabb",
                                                        "cellor")], _stream()))
    if n == 1:
        out["left"] = out["left"][:0]
        out["right"] = out["right"][:0]
    return out


def gf_scene_cells(scene: Scene):
    out = torch.empty(scene.n, dtype=torch.int32, device="cuda")
    _check(lib().gf_scene_cells(scene.handle, _ptr(out), _stream()))
    return out


def gf_mask_lod_cells(lod: int) -> int:
    return int(lib().gf_mask_lod_cells(lod))


def gf_mask_cone(scene: Scene, axis=(0.0, 0.0, 1.0), half_angle=0.7853981633974483):
    bits = torch.empty((scene.n + 31) // 32, dtype=torch.int32, device="cuda")
    ax = (C.c_float * 3)(*axis)
    _check(lib().gf_mask_cone(scene.handle, ax, half_angle, _ptr(bits), _stream()))
    return bits


def gf_optical_depth(scene: Scene, rays, mask: gf_mask = None, image_width=0, want_T=True):
    n = rays.shape[0]
    tau = torch.empty(n, dtype=torch.float32, device=rays.device)
    T = torch.empty(n, dtype=torch.float32, device=rays.device) if want_T else None
    m = mask if mask is not None else make_mask()
    _check(lib().gf_optical_depth(scene.handle, _ptr(rays, torch.float32), n, image_width, m, _ptr(tau),
                                  _ptr(T, optional=True), _stream()))
    return tau, T


def gf_optical_depth_counts(scene: Scene, rays, mask: gf_mask = None, image_width=0):
    n = rays.shape[0]
    nodes = torch.empty(n, dtype=torch.int32, device=rays.device)
    hits = torch.empty(n, dtype=torch.int32, device=rays.device)
    m = mask if mask is not None else make_mask()
    _check(lib().gf_optical_depth_counts(scene.handle, _ptr(rays, torch.float32), n, image_width, m, _ptr(nodes),
                                         _ptr(hits), _stream()))
    return nodes, hits


def gf_density(scene: Scene, pts, mask: gf_mask = None):
    n = pts.shape[0]
    kap = torch.empty(n, dtype=torch.float32, device=pts.device)
    kb = torch.empty(n, dtype=torch.float32, device=pts.device)
    m = mask if mask is not None else make_mask()
    _check(lib().gf_density(scene.handle, _ptr(pts, torch.float32), n, m, _ptr(kap), _ptr(kb), _stream()))
    return kap, kb


def gf_transmittance_ratio(scene: Scene, rays, spp, seed, mask: gf_mask = None, image_width=0):
    n = rays.shape[0]
    Tm = torch.empty(n, dtype=torch.float32, device=rays.device)
    Tv = torch.empty(n, dtype=torch.float32, device=rays.device)
    m = mask if mask is not None else make_mask()
    _check(lib().gf_transmittance_ratio(scene.handle, _ptr(rays, torch.float32), n, image_width, m, spp, seed,
                                        _ptr(Tm), _ptr(Tv), _stream()))
    return Tm, Tv


def render_desc(spp=1, multiple=False, max_scatter=16, albedo=0.9, hg_g=0.0, env=1.0, stochastic=False,
                mask: gf_mask = None, seed=0, level="uniform_cv", bin="importance", beta=0.0, delta=1.0,
                analytic=False, exact_shadow=False, shadow_cells=0) -> gf_render_desc:
    """level / bin: strategy names (LEVEL, BIN) or codes; analytic: free
    flights by CDF inversion with exact transmittances; exact_shadow:
    closed-form shadow transmittance with delta-tracked free flights;
    shadow_cells: cells the single-scattering shadow rays trace (0: their
    own mask)."""
    lv = LEVEL[level] if isinstance(level, str) else int(level)
    bn = BIN[bin] if isinstance(bin, str) else int(bin)
    return gf_render_desc(spp, int(multiple), max_scatter, albedo, hg_g, env, int(stochastic), lv, bn, beta, delta,
                          int(analytic), int(exact_shadow), shadow_cells, mask if mask is not None else make_mask(),
                          seed)


def gf_render_rays(scene: Scene, rays, desc: gf_render_desc, image_width=0, want_var=True):
    n = rays.shape[0]
    f = lambda: torch.empty(n, dtype=torch.float32, device=rays.device)  # noqa: E731
    Lm, Tm = f(), f()
    Lv, Tv = (f(), f()) if want_var else (None, None)
    _check(lib().gf_render_rays(scene.handle, _ptr(rays, torch.float32), n, image_width, C.byref(desc), _ptr(Lm),
                                _ptr(Lv, optional=True), _ptr(Tm), _ptr(Tv, optional=True), _stream()))
    return Lm, Lv, Tm, Tv


def gf_render_workspace_size(scene: Scene, cam, desc: gf_render_desc) -> int:
    out = C.c_size_t()
    _check(lib().gf_render_workspace_size(scene.handle, C.byref(cam), C.byref(desc), C.byref(out)))
    return out.value


def gf_render(scene: Scene, cam, desc: gf_render_desc, workspace: torch.Tensor, want_T=True):
    """Camera image (height x width radiance, and the primary transmittance)
    rendered in a caller-owned workspace (a uint8 device tensor of at least
    gf_render_workspace_size bytes)."""
    rad = torch.empty((cam.height, cam.width), dtype=torch.float32, device="cuda")
    T = torch.empty_like(rad) if want_T else None
    _check(lib().gf_render(scene.handle, C.byref(cam), C.byref(desc), _ptr(workspace), workspace.numel(),
                           _ptr(rad), _ptr(T, optional=True), _stream()))
    return rad, T


GF_RENDER_COUNTS = 7


def gf_render_noalloc(scene: Scene, cam, desc: gf_render_desc, want_T=True):
    """gf_render with the library's own fixed workspace (no allocation in
    the call; the output tensors are allocated here, by the caller)."""
    rad = torch.empty((cam.height, cam.width), dtype=torch.float32, device="cuda")
    T = torch.empty_like(rad) if want_T else None
    _check(lib().gf_render_noalloc(scene.handle, C.byref(cam), C.byref(desc), _ptr(rad), _ptr(T, optional=True),
                                   _stream()))
    return rad, T


def gf_render_counts(scene: Scene, rays, desc: gf_render_desc, image_width=0):
    """(tentative points, nodes visited, primitive records read, windows,
    points consumed, their point-query nodes, their covering primitives)"""
    out = torch.zeros(GF_RENDER_COUNTS, dtype=torch.int64, device=rays.device)
    _check(lib().gf_render_counts(scene.handle, _ptr(rays, torch.float32), rays.shape[0], image_width,
                                  C.byref(desc), _ptr(out), _stream()))
    return [int(x) for x in out.cpu()]


def camera(kind=1, eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0), fov_y_deg=40.0, width=64,
           height=64) -> gf_camera:
    return gf_camera(kind, (C.c_float * 3)(*eye), (C.c_float * 3)(*target), (C.c_float * 3)(*up), fov_y_deg,
                     width, height)


def gf_camera_rays(cam: gf_camera):
    out = torch.empty((cam.width * cam.height, 8), dtype=torch.float32, device="cuda")
    _check(lib().gf_camera_rays(C.byref(cam), _ptr(out), _stream()))
    return out


def gf_optical_depth_backward(scene: Scene, rays, dL_dtau, mask: gf_mask = None, dL_dT=None, T=None,
                              image_width=0, out=None):
    n = rays.shape[0]
    g = out if out is not None else torch.empty((scene.n, 15), dtype=torch.float32, device=rays.device)
    m = mask if mask is not None else make_mask()
    _check(lib().gf_optical_depth_backward(scene.handle, _ptr(rays, torch.float32), n, image_width, m,
                                           _ptr(dL_dtau, torch.float32), _ptr(dL_dT, optional=True),
                                           _ptr(T, optional=True), _ptr(g), _stream()))
    return g


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
class Server:
    """Continuous-batching render server (owns the C handle)."""

    def __init__(self, mem_budget: int, tile_rays: int = 4096, max_tiles: int = 64):
        h = C.c_void_p()
        _check(lib().gf_server_create(mem_budget, tile_rays, max_tiles, _stream(), C.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, scene: Scene, cam: gf_camera, desc: gf_render_desc, out: torch.Tensor) -> int:
        req = gf_request(scene.handle, cam, desc, _ptr(out, torch.float32))
        rid = C.c_uint64()
        _check(lib().gf_server_submit(self.handle, C.byref(req), C.byref(rid)))
        self._keep[rid.value] = out
        return rid.value

    def step(self, wait: bool = False):
        _check(lib().gf_server_step(self.handle, int(wait)))

    def poll(self, max_ids: int = 256):
        ids = (C.c_uint64 * max_ids)()
        n = C.c_int()
        _check(lib().gf_server_poll(self.handle, ids, max_ids, C.byref(n)))
        done = [ids[k] for k in range(n.value)]
        for d in done:
            self._keep.pop(d, None)
        return done

    def stats(self):
        q, f, b = C.c_int(), C.c_int(), C.c_size_t()
        _check(lib().gf_server_stats(self.handle, C.byref(q), C.byref(f), C.byref(b)))
        return q.value, f.value, b.value

    def close(self):
        if getattr(self, "handle", None):
            lib().gf_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gf_server_create(mem_budget, tile_rays=4096, max_tiles=64) -> Server:
    return Server(mem_budget, tile_rays, max_tiles)


def gf_server_simulate(mem_budget: int, tile_rays: int, max_tiles: int, width, height, spp, multiple, arrival_s,
                       work_per_s: float):
    """The server's admission and batching policy on a virtual clock (host
    only, no device).  Returns (admit_s, done_s, max_bytes_held) as numpy
    arrays and an int."""
    import numpy as np

    i32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.int32))  # noqa: E731
    w, h, s, m = i32(width), i32(height), i32(spp), i32(multiple)
    arr = np.ascontiguousarray(np.asarray(arrival_s, dtype=np.float64))
    n = len(w)
    admit, done = np.empty(n), np.empty(n)
    held = C.c_size_t()
    p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    _check(lib().gf_server_simulate(mem_budget, tile_rays, max_tiles, n, p(w), p(h), p(s), p(m), p(arr),
                                    float(work_per_s), p(admit), p(done), C.byref(held)))
    return admit, done, held.value
