#!/usr/bin/env python3
"""Benchmark of the Gabor-field hot path on one MI355X.

Workload (default): 100k Gabor primitives from the 64-blob field, a 512x512
pinhole camera, LOD masks {full, 1/2 band, 1/4 band, 45-degree cone about +z}.
One step runs the whole path on that batch:
  scene build (validation, Morton keys, radix sort, Karras tree, refit,
  traversal records) + cone mask, then for every mask
  deterministic optical depth / transmittance of the 512^2 rays and an 8-spp
  single-scattering render (weighted delta tracking of the camera segment,
  shadow transmittance in closed form -- or ratio-tracked with
  --ratio-shadow --, isotropic phase, albedo 0.9).
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
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# VALU issue peak: 256 CUs x one wave64 instruction per cycle (4 SIMD16 units,
# 4 cycles each) x 2.4 GHz; 64 lanes x 2 (FMA) x 614.4e9 = 78.6 TFLOP/s, the
# float32 peak without packed instructions (the library is compiled without them)
PEAK_VALU_INSTS = 256 * 2.4e9
# bytes each unit of work must touch (the per-unit byte model of the
# measurement): optical depth per ray 32 (ray) + 8 (tau, T) + 60 per primitive with
# a non-empty chord + 32 per box met (half a 64 B node record); tracking per
# consumed tentative point 32 per node a point query visits + 60 per
# primitive whose support contains the point, plus 40 per camera ray
RAY_BYTES, OUT_BYTES, PRIM_BYTES, NODE_BYTES = 32, 8, 60, 32


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
    ap.add_argument("--serving", action="store_true",
                    help="add the serving trace (continuous batching vs plain renderer; ~10 minutes)")
    ap.add_argument("--no-serving", action="store_true", help="(default) no serving trace")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=12)
    ap.add_argument("--serving-sweep", action="store_true", help="serving at 0.35, 0.7, 1.0, 1.4 x saturation")
    ap.add_argument("--serving-max-tiles", type=int, default=192, help="tiles of 4096 rays per serving batch")
    ap.add_argument("--serving-loads", default="",
                    help="comma-separated loads (multiples of the plain renderer's saturation rate) to serve at")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for hardware byte counters)")
    ap.add_argument("--bin", default="mixture", help="orientation-bin strategy of the multiple-scattering workload")
    ap.add_argument("--rows", type=int, default=0,
                    help="1M multiple-scattering workload: render only this many central rows (0: the full frame)")
    ap.add_argument("--ratio-shadow", action="store_true",
                    help="ratio-tracked shadow transmittance (default: closed form exp(-tau))")
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
    if args.workload.startswith("blob1m"):
        return multiple_scattering_bench(args)
    if args.ratio_shadow:
        KERNELS["render"] = "void k_render<false, 0>"
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
        return gf.render_desc(spp=args.spp, multiple=False, albedo=0.9, env=1.0, mask=mask, seed=1234,
                              exact_shadow=not args.ratio_shadow)

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
                gf.gf_render_rays(scene, rays, desc(m), image_width=width, want_var=False)
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

    # algorithmic work of the timed launches: optical depth counted exactly on
    # the same launch; the render's work per sample counted with one sample
    # per ray on every 4th pixel row (the counting variant walks a point query
    # per consumed tentative point, far slower than the render; samples are
    # independent, so the work per sample does not depend on their number)
    # and scaled to the frame's rays and samples
    scene = gf.Scene(params, rho)
    masks, bits = masks_for(scene)
    tau_bytes, ren_bytes, ren_counts = [], [], []
    stride = 4
    sub_rays = rays.view(width, width, 8)[::stride].reshape(-1, 8).contiguous()

    def count_desc(mask):
        d = desc(mask)
        d.spp = 1
        return d
    for k, m in enumerate(masks):
        log("counting work of mask %s" % mask_names[k])
        nodes, hits = gf.gf_optical_depth_counts(scene, rays, m, image_width=width)
        nn, nh = int(nodes.sum().item()), int(hits.sum().item())
        tau_bytes.append(npix * (RAY_BYTES + OUT_BYTES) + PRIM_BYTES * nh + NODE_BYTES * nn)
        if args.render:
            c = [v * stride * args.spp for v in gf.gf_render_counts(scene, sub_rays, count_desc(m), image_width=width)]
            ren_counts.append(c)
            ren_bytes.append(npix * (RAY_BYTES + OUT_BYTES) + NODE_BYTES * c[5] + PRIM_BYTES * c[6])
        else:
            ren_bytes.append(0)
    torch.cuda.synchronize()
    tau_gbs = [b / (t * 1e-3) / 1e9 for b, t in zip(tau_bytes, tau_ms)]
    ren_gbs = [b / (t * 1e-3) / 1e9 if t > 0 else 0.0 for b, t in zip(ren_bytes, ren_ms)]
    dominant = "render" if args.render and sum(ren_ms) >= sum(tau_ms) else "optical_depth"
    if dominant == "render":
        per_launch_s = sum(ren_ms) * 1e-3 / 4
        alg = sum(ren_bytes) / 4
    else:
        per_launch_s = sum(tau_ms) * 1e-3 / 4
        alg = sum(tau_bytes) / 4
    ach = alg / per_launch_s / 1e9
    prof = profile_figures(name, dominant)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": prof.get("traffic"), "kernel": KERNELS[dominant],
                "algorithmic_bytes_per_launch": int(alg), "launch_ms": round(1e3 * per_launch_s, 3)}
    if dominant == "render" and ren_counts:
        # the same rate with the kernel's own reads (32 B per internal node it
        # visits, 60 B per primitive record it reads) in place of point queries
        kr = sum(npix * (RAY_BYTES + OUT_BYTES) + NODE_BYTES * c[1] + PRIM_BYTES * c[2] for c in ren_counts) / 4
        roofline["frac_kernel_reads"] = round(kr / per_launch_s / 1e9 / PEAK_HBM_GBS, 4)
    if prof.get("traffic"):
        roofline["measured_frac"] = round(prof["traffic"] / per_launch_s / 1e9 / PEAK_HBM_GBS, 4)
    if prof.get("valu_insts"):
        roofline["valu_frac"] = round(prof["valu_insts"] / per_launch_s / PEAK_VALU_INSTS, 4)

    result = {
        "metric": "Mrays/s transmittance at full & masked LOD; p50/p99 render-request latency",
        "value": round(value, 3), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 geometry setup)", "data": "synthetic",
        "config": {"workload": "%s: %s, %dx%d pinhole, masks %s%s"
                   % (name, W.describe(name), width, width, "/".join(mask_names),
                      (", %d-spp single scattering (delta-tracked free flights, %s shadow transmittance)"
                       % (args.spp, "ratio-tracked" if args.ratio_shadow else "closed-form"))
                      if args.render else ", optical depth and transmittance"),
                   "global_batch": npix, "parallelism": "single GPU"},
        "roofline": roofline,
        "per_mask": {mask_names[k]: {"tau_ms": round(tau_ms[k], 3), "tau_Mrays_s": round(npix / tau_ms[k] / 1e3, 1),
                                     "tau_alg_GBs": round(tau_gbs[k], 1), "render_ms": round(ren_ms[k], 3),
                                     "render_Msamples_s": round(npix * spp_r / max(ren_ms[k], 1e-9) / 1e3, 2),
                                     "render_alg_GBs": round(ren_gbs[k], 1),
                                     "render_work_per_sample": work_per_sample(ren_counts, k, npix * spp_r)}
                     for k in range(4)},
        "build_ms": round(float(np.mean(timings["build"])), 3),
    }

    if args.serving and not args.no_serving:
        log("serving trace")
        result["serving"] = serving(args, gf, W, np, torch)
    if not args.no_cpu:
        log("oracle on the host")
        result["cpu_baseline"] = cpu_baseline(args, np, params_h, rays_h, rho, tau_ms, ren_ms, npix, units,
                                              ms_per_step)
    scene.close()
    print(json.dumps(result), flush=True)


KERNELS = {"render": "void k_render<false, 1>", "optical_depth": "void k_tau<false>"}


def work_per_sample(counts, k, samples):
    if not counts or not samples:
        return None
    c = counts[k]
    names = ["tentative_points", "kernel_node_visits", "kernel_prim_reads", "windows", "points_used",
             "point_query_nodes", "covering_prims"]
    return {n: round(v / samples, 2) for n, v in zip(names, c)}


def profile_figures(workload, kernel, rows=0):
    """Per-launch figures of the dominant kernel from the committed rocprofv3
    summaries, used only while their recorded source hash matches the HIP
    sources and their command rendered the same rows (rows > 0: `--rows
    rows`; 0: the full frame): measured HBM bytes
    (profiles/<kernel>_<workload>_pmc.txt, FETCH_SIZE and WRITE_SIZE scaled
    by the calibration factors recorded there) and VALU instructions
    (profiles/<kernel>_<workload>_sq.txt)."""
    sys.path.insert(0, ROOT)
    import profile_summary
    out = {}
    name = KERNELS[kernel]
    for kind in ("pmc", "sq"):
        path = os.path.join(ROOT, "profiles", "%s_%s_%s.txt" % (kernel, workload, kind))
        if not os.path.exists(path):
            continue
        text = open(path).read().splitlines()
        if not any(l.startswith("# source hash: %s" % profile_summary.source_hash()) for l in text):
            continue
        cmds = [l for l in text if l.startswith("# command") or l.startswith("# fetch command")]
        m = re.search(r"--rows (\d+)", cmds[0]) if cmds else None
        if (int(m.group(1)) if m else 0) != rows:
            continue
        header = next((l for l in text if l.startswith("kernel ")), None)
        for line in text:
            if not line.startswith(name):
                continue
            if kind == "pmc":
                out["traffic"] = int(float(line.split()[-1]) * 1e6)
            elif header:
                cols = header.split()
                vals = line[48:].split()
                if "SQ_INSTS_VALU" in cols:
                    out["valu_insts"] = float(vals[cols.index("SQ_INSTS_VALU") - 1])
            break
    return out


def multiple_scattering_bench(args):
    """The 1M-primitive multiple-scattering workload: a 1024x1024 pinhole
    frame, 4 spp, Henyey-Greenstein g = 0.3, albedo 0.9, up to 16 bounces,
    per-segment stochastic masks (uniform + control variate levels, --bin
    orientation strategy).  One step: scene build, optical depth of every
    pixel at the full mask, the render.  Reports camera paths and
    transmittance rays per second, the work per sample (counted on a
    64-row band at the frame's centre), and the primary transmittance's
    bias and variance against the full-mask FP64 optical depth of a
    4096-pixel subset (in the CPU leg)."""
    import numpy as np
    import torch

    import paper_2602_05081_amd as gf
    from gen import workloads as W

    name, spp = args.workload, 4
    KERNELS["render"] = "void k_render<false, 0>"  # delta tracking, ratio-tracked transmittances
    params_h, rays_h, rho = W.scene(name), W.rays(name), W.rho(name)
    width = int(math.isqrt(rays_h.shape[0]))
    rows = args.rows if 0 < args.rows < width else width
    r0 = (width - rows) // 2
    rays_h = np.ascontiguousarray(rays_h[r0 * width:(r0 + rows) * width])
    params, rays = torch.as_tensor(params_h).cuda(), torch.as_tensor(rays_h).cuda()
    npix = rays.shape[0]
    desc = gf.render_desc(spp=spp, multiple=True, max_scatter=16, albedo=0.9, hg_g=0.3, env=1.0, stochastic=True,
                          level="uniform_cv", bin=args.bin, seed=4321)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    rec = []
    out = None
    t0 = None
    for k in range(args.warmup + args.steps):
        if k == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        e = [ev() for _ in range(4)]
        e[0].record()
        scene = gf.Scene(params, rho)
        e[1].record()
        gf.gf_optical_depth(scene, rays, image_width=width)
        e[2].record()
        out = gf.gf_render_rays(scene, rays, desc, image_width=width)
        e[3].record()
        if k >= args.warmup:
            rec.append(e)
        torch.cuda.synchronize()
        log("%s step %d done" % ("warmup" if k < args.warmup else "timed", k))
        scene.close()
    t1 = time.perf_counter()
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    build_ms = float(np.mean([a.elapsed_time(b) for a, b, c, d in rec]))
    tau_ms = float(np.mean([b.elapsed_time(c) for a, b, c, d in rec]))
    ren_ms = float(np.mean([c.elapsed_time(d) for a, b, c, d in rec]))
    L, _, Tm, Tv = (x.cpu().numpy() for x in out)
    units = npix * (1 + spp)
    # work per sample counted with one sample per ray on every 16th row
    # (the counting variant walks a point query per consumed point, far
    # slower than the render), scaled to the frame's rays and samples
    scene = gf.Scene(params, rho)
    band = rays.view(rows, width, 8)[::16].reshape(-1, 8).contiguous()
    cdesc = gf.render_desc(spp=1, multiple=True, max_scatter=16, albedo=0.9, hg_g=0.3, env=1.0, stochastic=True,
                           level="uniform_cv", bin=args.bin, seed=4321)
    log("counting work on every 16th row (%d rays, 1 spp)" % band.shape[0])
    c = gf.gf_render_counts(scene, band, cdesc, image_width=width)
    log("counting done")
    band_samples = band.shape[0]
    alg_frame = npix * (RAY_BYTES + OUT_BYTES) + (NODE_BYTES * c[5] + PRIM_BYTES * c[6]) * (npix * spp / band_samples)
    ach = alg_frame / (ren_ms * 1e-3) / 1e9
    prof = profile_figures(name, "render", rows if rows != width else 0)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": prof.get("traffic"), "kernel": KERNELS["render"],
                "algorithmic_bytes_per_launch": int(alg_frame), "launch_ms": round(ren_ms, 3),
                "note": "algorithmic bytes counted at 1 spp on every 16th row, scaled to the frame"}
    if prof.get("traffic"):
        roofline["measured_frac"] = round(prof["traffic"] / (ren_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    if prof.get("valu_insts"):
        roofline["valu_frac"] = round(prof["valu_insts"] / (ren_ms * 1e-3) / PEAK_VALU_INSTS, 4)
    result = {
        "metric": "Mrays/s transmittance at full & masked LOD; p50/p99 render-request latency",
        "value": round(units / (ms_per_step * 1e-3) / 1e6, 4), "unit": "Mrays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 (f64 geometry setup)",
        "data": "synthetic",
        "config": {"workload": "%s: %s, %dx%d pinhole%s, %d spp, multiple scattering (HG 0.3, albedo 0.9, <= 16 "
                               "bounces), per-segment stochastic masks (uniform+CV levels, %s bins)"
                               % (name, W.describe(name), width, width,
                                  "" if rows == width else " (the central %d rows)" % rows, spp, args.bin),
                   "global_batch": npix, "parallelism": "single GPU"},
        "roofline": roofline,
        "build_ms": round(build_ms, 2), "tau_ms": round(tau_ms, 2), "tau_Mrays_s": round(npix / tau_ms / 1e3, 2),
        "render_ms": round(ren_ms, 1), "camera_paths_per_s": round(npix * spp / (ren_ms * 1e-3), 1),
        "frame_mean_radiance": round(float(L.mean()), 5), "frame_mean_primary_T": round(float(Tm.mean()), 5),
        "render_work_per_sample_band": {k: round(v / band_samples, 2) for k, v in zip(
            ["tentative_points", "kernel_node_visits", "kernel_prim_reads", "windows", "points_used",
             "point_query_nodes", "covering_prims"], c)},
    }
    if not args.no_cpu:
        log("oracle on the host")
        result["cpu_baseline"], result["primary_T_vs_full_mask"] = multiple_scattering_cpu(
            args, np, params_h, rays_h, rho, Tm, Tv, spp, units, ms_per_step)
    scene.close()
    print(json.dumps(result), flush=True)


def multiple_scattering_cpu(args, np, params, rays, rho, Tm, Tv, spp, units, ms_per_step):
    """FP64 oracle on the host: a bounded sample of the workload (optical
    depth of 64 rays, 8 rays x 4 spp of the multiple-scattering render with
    the same strategies), scaled to one step; and the GPU's stochastic
    primary transmittance against exp(-tau) of the full-mask FP64 optical
    depth on a fixed 4096-pixel subset (bias and mean per-sample variance)."""
    import oracle
    from gen import workloads as W
    sub = W.pixel_subset(rays.shape[0], k=64, seed=5)
    t0 = time.perf_counter()
    oracle.tau(params, rays[sub], rho=rho)
    t_tau = (time.perf_counter() - t0) / len(sub)
    sub_r = W.pixel_subset(rays.shape[0], k=8, seed=6)
    t0 = time.perf_counter()
    oracle.render(params, rays[sub_r], spp, seed=3, rho=rho, multiple=True, max_scatter=16, albedo=0.9, hg_g=0.3,
                  stochastic=True, level="uniform_cv", bin=args.bin)
    t_ren = (time.perf_counter() - t0) / (len(sub_r) * spp)
    step_s = rays.shape[0] * (t_tau + spp * t_ren)
    cores = min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1)
    cpu = {"value": round(units / step_s / 1e6, 8), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
           "sample": "%d optical-depth rays and %d rays x %d spp multiple scattering, scaled to one step"
                     % (len(sub), len(sub_r), spp),
           "tau_ms_per_ray": round(1e3 * t_tau, 3), "render_ms_per_sample": round(1e3 * t_ren, 2)}
    bsub = W.pixel_subset(rays.shape[0], k=4096, seed=7)
    log("full-mask optical depth of 4096 pixels (oracle)")
    tau, _, _ = oracle.tau(params, rays[bsub], rho=rho)
    ref = np.exp(-tau)
    d = Tm[bsub].astype(np.float64) - ref
    bias = {"pixels": len(bsub), "mean_T_gpu": round(float(Tm[bsub].mean()), 6),
            "mean_T_full_mask": round(float(ref.mean()), 6), "bias": round(float(d.mean()), 6),
            "bias_se": round(float(np.sqrt((Tv[bsub] / spp).sum()) / len(bsub)), 6),
            "mean_abs_error": round(float(np.abs(d).mean()), 6),
            "mean_sample_variance": round(float(Tv[bsub].mean()), 6)}
    return cpu, bias


def serving(args, gf, W, np, torch):
    """Poisson trace over four resident scenes, continuous batching vs the
    plain per-request renderer (FIFO, one request at a time, caller
    workspace).  The request rate is a multiple of the plain renderer's
    saturation rate on this trace (0.7 by default; --serving-sweep runs
    several), and the server's memory budget (96 MB: two 1024^2 requests at
    4 spp, rays and per-sample radiance) makes admission bind."""
    import gen
    from paper_2602_05081_amd import serve
    scenes = [gf.Scene(torch.as_tensor(W.scene(s)).cuda(), rho=W.rho(s)) for s in W.SERVE_SCENES]
    n = args.serving_requests
    reqs = gen.serving_requests(n, seed=5)
    budget = 96 << 20
    # warm both paths
    serve.run_plain(scenes, reqs[:1], np.zeros(1))
    # saturation throughput of the plain renderer on this trace decides the rate
    t0 = time.perf_counter()
    k = min(4, n)
    serve.run_plain(scenes, reqs[:k], np.zeros(k))
    plain_rate = k / (time.perf_counter() - t0)
    out = {"requests": n, "scenes": W.SERVE_SCENES, "mem_budget": budget, "max_tiles": args.serving_max_tiles,
           "plain_saturation_qps": round(plain_rate, 4), "points": []}

    def done(tag):
        return lambda k, t: log("serving (%s): request %d done at %.1f s" % (tag, k, t))

    loads = [0.35, 0.7, 1.0, 1.4] if args.serving_sweep else [0.7]
    if args.serving_loads:
        loads = [float(x) for x in args.serving_loads.split(",")]
    for f in loads:
        qps = f * plain_rate
        arrivals = gen.poisson_arrivals(n, qps, seed=6)
        log("serving: %.2f x saturation = %.3f requests/s, %d requests" % (f, qps, n))
        lat_s, mk_s, _, held = serve.run_server(scenes, reqs, arrivals, mem_budget=budget, tile_rays=4096,
                                                max_tiles=args.serving_max_tiles, time_limit=1800,
                                                on_done=done("batching"))
        lat_p, mk_p, _ = serve.run_plain(scenes, reqs, arrivals, time_limit=1800, on_done=done("plain"))
        out["points"].append({"load": f, "qps": round(qps, 4),
                              "continuous_batching": serve.summarize(lat_s, mk_s, reqs),
                              "plain_per_request": serve.summarize(lat_p, mk_p, reqs),
                              "max_bytes_held": held})
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
