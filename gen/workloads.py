"""Named synthetic workloads (sizes, seeds, cameras) and their extinction scales.

The extinction scale ``rho`` of each scene is a stored number: it was written
by ``gen/calibrate_rho.py`` (which calls only the FP64 oracle) so that the
median envelope optical depth rho * sum_i |alpha_i| int env_i over the
workload's hitting camera rays equals 4.  Scene, rays and rho are what both the
oracle and the HIP path receive.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import cameras, scenes

_HERE = os.path.dirname(os.path.abspath(__file__))
RHO_PATH = os.path.join(_HERE, "rho.json")

WORKLOADS = {
    # 256 Gabors, uniform means, scales logU[0.02, 0.1]; 64x64 orthographic rays along +z
    "tiny256": dict(kind="uniform", n=256, seed=0, smin=0.02, smax=0.1, camera=("ortho", 64, 64)),
    # 100k Gabors from the 64-blob field, scales logU[0.003, 0.05]; 512^2 pinhole
    "blob100k": dict(kind="blob", n=100_000, seed=1, camera=("pinhole", 512, 512)),
    # 1M Gabors, same generator; 1024^2 pinhole
    "blob1m": dict(kind="blob", n=1_000_000, seed=2, camera=("pinhole", 1024, 1024)),
    # the same scenes with a Gaussian low-pass level (every fourth primitive
    # f = 0, phi = 0, alpha x 4): a mostly positive field like the paper's assets
    "blob100k_lp": dict(kind="blob", n=100_000, seed=1, camera=("pinhole", 512, 512), base_level=True),
    "blob1m_lp": dict(kind="blob", n=1_000_000, seed=2, camera=("pinhole", 1024, 1024), base_level=True),
    # 50k Gabors, eight 256^2 views; the target scene is a 5% jitter (seed 4)
    "diff50k": dict(kind="blob", n=50_000, seed=3, camera=("eight", 256, 256), jitter_seed=4),
    # resident serving scenes
    "serve10k": dict(kind="blob", n=10_000, seed=10, camera=("pinhole", 256, 256)),
    "serve100k": dict(kind="blob", n=100_000, seed=11, camera=("pinhole", 256, 256)),
    "serve500k": dict(kind="blob", n=500_000, seed=12, camera=("pinhole", 256, 256)),
    "serve2m": dict(kind="blob", n=2_000_000, seed=13, camera=("pinhole", 256, 256)),
}

SERVE_SCENES = ["serve10k", "serve100k", "serve500k", "serve2m"]


def describe(name: str) -> str:
    """One-line description of a workload's scene (for benchmark records)."""
    w = WORKLOADS[name]
    if w["kind"] == "uniform":
        return "%d Gabors, uniform means, scales logU[%g, %g], seed %d" % (w["n"], w["smin"], w["smax"], w["seed"])
    lp = w.get("base_level", False)
    return "%d %s, 64-blob field, scales logU[0.003, 0.05], seed %d" % (
        w["n"], "primitives (every 4th a Gaussian of the low-pass level, alpha x4)" if lp else "Gabors (Gabor-only)",
        w["seed"])


def scene(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if w["kind"] == "uniform":
        return scenes.uniform_scene(w["n"], w["seed"], w["smin"], w["smax"])
    return scenes.blob_scene(w["n"], w["seed"], base_level=w.get("base_level", False))


def target_scene(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    return scenes.jitter_scene(scene(name), w["jitter_seed"])


def rays(name: str) -> np.ndarray:
    kind, width, height = WORKLOADS[name]["camera"]
    if kind == "ortho":
        return cameras.ortho_rays(width, height)
    if kind == "pinhole":
        return cameras.pinhole_rays(width, height)
    if kind == "eight":
        return cameras.eight_views(width, height)
    raise KeyError(kind)


def pixel_subset(n_rays: int, k: int = 4096, seed: int = 99) -> np.ndarray:
    """A fixed, seeded subset of ray indices (sorted)."""
    if n_rays <= k:
        return np.arange(n_rays)
    g = np.random.Generator(np.random.PCG64(seed))
    return np.sort(g.choice(n_rays, size=k, replace=False))


def rho(name: str) -> float:
    with open(RHO_PATH) as fh:
        return float(json.load(fh)[name])
