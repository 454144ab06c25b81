#!/usr/bin/env python3
"""Benchmark of the Gabor-field hot path on one MI355X.

Workload (default): 100k Gabor primitives from the 64-blob field, a 512x512
pinhole camera, LOD masks {full, 1/2 band, 1/4 band, 45-degree cone about +z}.
One step runs the whole path on that batch:
  scene build (validation, Morton keys, radix sort, Karras tree, refit,
  traversal records, majorant grid) + cone mask, then for every mask
  deterministic optical depth / transmittance of the 512^2 rays and an 8-spp
  single-scattering render (weighted delta tracking, ratio-tracked shadow rays,
  isotropic phase, albedo 0.9).
value = (transmittance rays + render camera samples) / s over the step.

After the timed steps (not part of them) the run measures the serving trace
(four resident scenes, Poisson arrivals) against the plain per-request
renderer and times the FP64 CPU oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# bytes each unit of work must touch (per-unit figures; see the design notes)
# optical depth: per ray, per child-box hit (half a 64 B node record), per chord
# (a 60 B primitive record); tracking: per internal-node visit (its 64 B
# record) and per primitive record read at a leaf
RAY_BYTES, OUT_BYTES, PRIM_BYTES, NODE_BYTES, VISIT_BYTES = 32, 8, 60, 32, 64


def log(*a):
    """progress on stderr (the JSON result alone goes to stdout)"""
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="blob100k")
    ap.add_argument("--spp", type=int, default=8)
    ap.add_argument("--no-render", dest="render", action="store_false",
                    help="leave the single-scattering render out of the step (optical depth only)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2602_05081_amd as gf
    from gen import workloads as W

    torch.cuda.init()
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    name = args.workload
    params_h, rays_h, rho = W.scene(name), W.rays(name), W.rho(name)
    width = int(math.isqrt(rays_h.shape[0]))
    params = torch.as_tensor(params_h).cuda()
    rays = torch.as_tensor(rays_h).cuda()
    npix = rays.shape[0]
    lod = [gf.gf_mask_lod_cells(k) for k in (0, 1, 2)]
    mask_names = ["full", "half_band", "quarter_band", "cone45"]

    def masks_for(scene):
        bits = gf.gf_mask_cone(scene)
        return [gf.make_mask(lod[0]), gf.make_mask(lod[1]), gf.make_mask(lod[2]),
                gf.make_mask(gf.FULL_CELLS, bits)], bits

    def desc(mask):
        return gf.render_desc(spp=args.spp, multiple=False, albedo=0.9, env=1.0, mask=mask, seed=1234)

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    timings = {"build": [], "tau": [[] for _ in range(4)], "render": [[] for _ in range(4)]}

    def step(record):
        e0 = ev()
        e0.record()
        scene = gf.Scene(params, rho)
        masks, bits = masks_for(scene)
        e1 = ev()
        e1.record()
        evs = []
        for k, m in enumerate(masks):
            a, b, c = ev(), ev(), ev()
            a.record()
            gf.gf_optical_depth(scene, rays, m, image_width=width)
            b.record()
            if args.render:
                gf.gf_render(scene, rays, desc(m), image_width=width, want_var=False)
            c.record()
            evs.append((a, b, c))
        if record is not None:
            record.append((e0, e1, evs))
        return scene, bits

    for k in range(args.warmup):
        scene, bits = step(None)
        scene.close()
        torch.cuda.synchronize()
        log("warmup step %d done" % k)
    rec = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        scene, bits = step(rec)
        scene.close()
        # progress only; the GPU work of the steps stays queued back to back
        log("step %d queued" % k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("timed steps done: %.1f ms per step" % (1e3 * (t1 - t0) / args.steps))
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    for e0, e1, evs in rec:
        timings["build"].append(e0.elapsed_time(e1))
        for k, (a, b, c) in enumerate(evs):
            timings["tau"][k].append(a.elapsed_time(b))
            timings["render"][k].append(b.elapsed_time(c))
    tau_ms = [float(np.mean(t)) for t in timings["tau"]]
    ren_ms = [float(np.mean(t)) for t in timings["render"]]
    spp_r = args.spp if args.render else 0
    units = 4 * npix * (1 + spp_r)
    value = units / (ms_per_step * 1e-3) / 1e6

    # algorithmic work of the timed launches (same inputs and seeds)
    scene = gf.Scene(params, rho)
    masks, bits = masks_for(scene)
    tau_bytes, ren_bytes = [], []
    for k, m in enumerate(masks):
        log("counting work of mask %s" % mask_names[k])
        nodes, hits = gf.gf_optical_depth_counts(scene, rays, m, image_width=width)
        nn, nh = int(nodes.sum().item()), int(hits.sum().item())
        tau_bytes.append(npix * (RAY_BYTES + OUT_BYTES) + PRIM_BYTES * nh + NODE_BYTES * nn)
        if args.render:
            tent, qn, qp, nwin = gf.gf_render_counts(scene, rays, desc(m), image_width=width)
            ren_bytes.append(npix * (RAY_BYTES + OUT_BYTES) + VISIT_BYTES * qn + PRIM_BYTES * qp)
        else:
            ren_bytes.append(0)
    torch.cuda.synchronize()
    tau_gbs = [b / (t * 1e-3) / 1e9 for b, t in zip(tau_bytes, tau_ms)]
    ren_gbs = [b / (t * 1e-3) / 1e9 if t > 0 else 0.0 for b, t in zip(ren_bytes, ren_ms)]
    dominant = "render" if args.render and sum(ren_ms) >= sum(tau_ms) else "optical_depth"
    if dominant == "render":
        ach = sum(ren_bytes) / (sum(ren_ms) * 1e-3) / 1e9
    else:
        ach = sum(tau_bytes) / (sum(tau_ms) * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": measured_traffic(name, dominant),
                "kernel": dominant}

    result = {
        "metric": "Mrays/s transmittance at full & masked LOD; p50/p99 render-request latency",
        "value": round(value, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 geometry setup)", "data": "synthetic",
        "config": {"workload": "%s: %d Gabors (64-blob field), %dx%d pinhole, masks %s%s"
                   % (name, params.shape[0], width, width, "/".join(mask_names),
                      ", %d-spp single scattering" % args.spp if args.render else ", optical depth and transmittance"),
                   "global_batch": npix, "parallelism": "single GPU"},
        "roofline": roofline,
        "per_mask": {mask_names[k]: {"tau_ms": round(tau_ms[k], 3), "tau_Mrays_s": round(npix / tau_ms[k] / 1e3, 1),
                                     "tau_alg_GBs": round(tau_gbs[k], 1), "render_ms": round(ren_ms[k], 3),
                                     "render_Msamples_s": round(npix * spp_r / max(ren_ms[k], 1e-9) / 1e3, 2),
                                     "render_alg_GBs": round(ren_gbs[k], 1)} for k in range(4)},
        "build_ms": round(float(np.mean(timings["build"])), 3),
    }

    if not args.no_serving:
        log("serving trace")
        result["serving"] = serving(args, gf, W, np, torch)
    if not args.no_cpu:
        log("oracle on the host")
        result["cpu_baseline"] = cpu_baseline(args, np, params_h, rays_h, rho, tau_ms, ren_ms, npix, units,
                                              ms_per_step)
    scene.close()
    print(json.dumps(result), flush=True)


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/<kernel>_<workload>_pmc.txt), scaled by the calibration
    factors recorded there; None when no summary exists or the HIP sources
    changed since it was taken."""
    sys.path.insert(0, ROOT)
    import profile_summary
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read().splitlines()
    if not any(l.startswith("# source hash: %s" % profile_summary.source_hash()) for l in text):
        return None
    name = {"optical_depth": "void k_tau<false>", "render": "void k_render<false>"}[kernel]
    for line in text:
        if line.startswith(name):
            return int(float(line.split()[-1]) * 1e6)
    return None


def serving(args, gf, W, np, torch):
    """Poisson trace over four resident scenes, continuous batching vs FIFO plain."""
    import gen
    from paper_2602_05081_amd import serve
    scenes = [gf.Scene(torch.as_tensor(W.scene(s)).cuda(), rho=W.rho(s)) for s in W.SERVE_SCENES]
    n = args.serving_requests
    reqs = gen.serving_requests(n, seed=5)
    # warm both paths
    serve.run_plain(scenes, reqs[:1], np.zeros(1))
    # saturation throughput of the plain renderer on this trace decides the rate
    t0 = time.perf_counter()
    serve.run_plain(scenes, reqs[:3], np.zeros(3))
    plain_rate = 3 / (time.perf_counter() - t0)
    qps = 0.7 * plain_rate
    arrivals = gen.poisson_arrivals(n, qps, seed=6)
    log("serving: plain renderer saturates at %.3f requests/s; replaying %d requests at %.3f/s" % (plain_rate, n, qps))
    def done(tag):
        return lambda k, t: log("serving (%s): request %d done at %.1f s" % (tag, k, t))

    lat_s, mk_s, _, held = serve.run_server(scenes, reqs, arrivals, mem_budget=1 << 30, tile_rays=4096,
                                            max_tiles=192, time_limit=600, on_done=done("batching"))
    log("serving: continuous batching done in %.1f s" % mk_s)
    lat_p, mk_p, _ = serve.run_plain(scenes, reqs, arrivals, time_limit=600, on_done=done("plain"))
    log("serving: plain renderer done in %.1f s" % mk_p)
    out = {"qps": round(qps, 2), "requests": n, "scenes": W.SERVE_SCENES,
           "continuous_batching": serve.summarize(lat_s, mk_s, reqs),
           "plain_per_request": serve.summarize(lat_p, mk_p, reqs), "max_bytes_held": held}
    for s in scenes:
        s.close()
    return out


def cpu_baseline(args, np, params, rays, rho, tau_ms, ren_ms, npix, units, ms_per_step):
    """FP64 oracle on the host cores on a bounded sample of the same workload,
    scaled to the step's work mix."""
    import oracle
    from gen import workloads as W
    sub = W.pixel_subset(rays.shape[0], k=512, seed=5)
    t0 = time.perf_counter()
    oracle.tau(params, rays[sub], rho=rho)
    t_tau = (time.perf_counter() - t0) / len(sub)
    spp_r = args.spp if args.render else 0
    sub_r = W.pixel_subset(rays.shape[0], k=16, seed=6)
    t_ren = 0.0
    if spp_r:
        t0 = time.perf_counter()
        oracle.render(params, rays[sub_r], args.spp, seed=3, rho=rho, multiple=False, albedo=0.9)
        t_ren = (time.perf_counter() - t0) / (len(sub_r) * args.spp)
    # one step: 4 masks x (npix transmittance rays + npix*spp samples) at full mask cost
    step_s = 4 * npix * (t_tau + spp_r * t_ren)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or 1)
    return {"value": round(units / step_s / 1e6, 6), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": ("%d transmittance rays" % len(sub)) +
                      (" and %d rays x %d spp single scattering" % (len(sub_r), spp_r) if spp_r else "") +
                      " at the full mask, scaled to one step",
            "tau_ms_per_ray": round(1e3 * t_tau, 4), "render_ms_per_sample": round(1e3 * t_ren, 3)}


if __name__ == "__main__":
    main()
