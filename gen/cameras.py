"""Seeded camera rays and request streams (input generation only).

Ray record, 8 float32 per ray: ``o[3] v[3] tmin tmax``; the ray is
x(t) = o + t v for t in [tmin, tmax] (Sec. 3, the ray r = x0 + v t).
Images are row-major: ray index = j * width + i, j = 0 is the top row.
"""
from __future__ import annotations

import numpy as np

INF = np.float32(np.inf)


def ortho_rays(width: int = 64, height: int = 64, z0: float = -1.0) -> np.ndarray:
    """Orthographic rays along +z through pixel centres of the unit square."""
    j, i = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    r = np.zeros((height, width, 8), dtype=np.float64)
    r[..., 0] = (i + 0.5) / width
    r[..., 1] = (j + 0.5) / height
    r[..., 2] = z0
    r[..., 5] = 1.0
    r[..., 6] = 0.0
    r[..., 7] = np.inf
    return np.ascontiguousarray(r.reshape(-1, 8).astype(np.float32))


def look_at_basis(eye, target, up):
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(np.asarray(up, np.float64), fwd)
    right /= np.linalg.norm(right)
    upv = np.cross(fwd, right)
    return fwd, right, upv


def pinhole_rays(width: int, height: int, eye=(0.5, 0.5, -1.5), target=(0.5, 0.5, 0.5),
                 up=(0.0, 1.0, 0.0), fov_y_deg: float = 40.0) -> np.ndarray:
    """Pinhole rays through pixel centres; unit directions, t in [0, inf)."""
    fwd, right, upv = look_at_basis(eye, target, up)
    th = np.tan(np.deg2rad(fov_y_deg) * 0.5)
    aspect = width / height
    j, i = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    px = (2.0 * (i + 0.5) / width - 1.0) * th * aspect
    py = (1.0 - 2.0 * (j + 0.5) / height) * th
    d = fwd[None, None, :] + px[..., None] * right[None, None, :] + py[..., None] * upv[None, None, :]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    r = np.zeros((height, width, 8), dtype=np.float64)
    r[..., 0:3] = np.asarray(eye, np.float64)
    r[..., 3:6] = d
    r[..., 6] = 0.0
    r[..., 7] = np.inf
    return np.ascontiguousarray(r.reshape(-1, 8).astype(np.float32))


def orbit_eye(theta_deg: float, elev_deg: float, dist: float = 2.0, centre=(0.5, 0.5, 0.5)):
    th, el = np.deg2rad(theta_deg), np.deg2rad(elev_deg)
    c = np.asarray(centre, np.float64)
    return c + dist * np.array([np.cos(el) * np.sin(th), np.sin(el), -np.cos(el) * np.cos(th)])


def eight_views(width: int = 256, height: int = 256) -> np.ndarray:
    """Eight pinhole views around the cube centre at 30 degrees elevation, 45 degree steps."""
    out = [pinhole_rays(width, height, eye=orbit_eye(45.0 * k, 30.0), target=(0.5, 0.5, 0.5))
           for k in range(8)]
    return np.ascontiguousarray(np.concatenate(out, axis=0))


def random_rays(n: int, seed: int, lo=-0.2, hi=1.2) -> np.ndarray:
    """Rays with random origins in a box around the unit cube and random unit
    directions, finite [tmin, tmax] windows (used for clipped-chord coverage)."""
    g = np.random.Generator(np.random.PCG64(seed))
    o = g.uniform(lo, hi, size=(n, 3))
    d = g.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tmin = g.uniform(-0.5, 0.5, size=n)
    tmax = tmin + g.uniform(0.0, 1.5, size=n)
    r = np.concatenate([o, d, tmin[:, None], tmax[:, None]], axis=1)
    return np.ascontiguousarray(r.astype(np.float32))


def poisson_arrivals(n: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of rate ``qps``."""
    g = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(g.exponential(1.0 / qps, size=n))


def serving_requests(n: int, seed: int, n_scenes: int = 4):
    """Request mix of the serving workload: uniform scene, resolution in
    {128,256,512,1024}^2, LOD level in {0..3}, 1..4 spp, single/multiple 50/50,
    and an orbit camera (azimuth U[0,360), elevation U[-30,60] degrees, distance 2)."""
    g = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(n):
        reqs.append(dict(
            scene=int(g.integers(n_scenes)),
            res=int(g.choice([128, 256, 512, 1024])),
            lod=int(g.integers(4)),
            spp=int(g.integers(1, 5)),
            multiple=int(g.integers(2)),
            az=float(g.uniform(0.0, 360.0)),
            el=float(g.uniform(-30.0, 60.0)),
            seed=int(g.integers(1, 2**62)),
        ))
    return reqs
