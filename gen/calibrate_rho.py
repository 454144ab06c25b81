"""Writes gen/rho.json: the extinction scale of every named workload.

rho is chosen so that the median, over the workload's hitting camera rays (a
fixed 4096-ray subset for the large ones), of the envelope optical depth
sum_i |alpha_i| int env_i  (Gaussian envelope only, omega = 0, phi = 0)
times rho equals 4.  Computed with the FP64 oracle only.

    python -m gen.calibrate_rho
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from gen import workloads  # noqa: E402

TARGET = 4.0


def calibrate(name: str) -> float:
    params = workloads.scene(name)
    rays = workloads.rays(name)
    sub = workloads.pixel_subset(rays.shape[0])
    env, _, hits = oracle.tau(params, rays[sub], rho=1.0, envelope=True)
    hit = hits > 0
    return float(TARGET / np.median(env[hit]))


def main():
    out = {}
    for name in workloads.WORKLOADS:
        out[name] = calibrate(name)
        print(name, out[name], flush=True)
    with open(workloads.RHO_PATH, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
