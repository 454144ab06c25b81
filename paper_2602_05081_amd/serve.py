"""Serving front-end: replays a request trace (Poisson arrivals) against the
continuous-batching server and against the plain per-request renderer, and
reports per-request latency (arrival -> result on the host).

Only orchestration lives here: ray generation and rendering run in the HIP
library (gf_render / gf_server_*).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib


def request_camera(req) -> _lib.gf_camera:
    th, el = np.deg2rad(req["az"]), np.deg2rad(req["el"])
    eye = (0.5 + 2.0 * np.cos(el) * np.sin(th), 0.5 + 2.0 * np.sin(el), 0.5 - 2.0 * np.cos(el) * np.cos(th))
    return _lib.camera(1, eye=tuple(float(x) for x in eye), target=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0),
                       fov_y_deg=40.0, width=req["res"], height=req["res"])


def request_desc(req) -> _lib.gf_render_desc:
    return _lib.render_desc(spp=req["spp"], multiple=bool(req["multiple"]), max_scatter=16, albedo=0.9,
                            hg_g=0.3 if req["multiple"] else 0.0, env=1.0, stochastic=False,
                            mask=_lib.make_mask(_lib.gf_mask_lod_cells(req["lod"])), seed=req["seed"])


def _percentiles(lat):
    lat = np.asarray(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def run_server(scenes, reqs, arrivals, mem_budget=512 << 20, tile_rays=4096, max_tiles=64, outputs=None,
               time_limit=None, on_done=None):
    """Replays the trace in wall-clock time.  Returns (latencies, makespan,
    outputs, max bytes held).  on_done(k, seconds) is called as request k
    completes."""
    srv = _lib.Server(mem_budget, tile_rays, max_tiles)
    outs = outputs if outputs is not None else [torch.empty(r["res"] * r["res"], device="cuda") for r in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt = 0
    id2k, t_arr, t_done = {}, {}, {}
    max_held = 0
    while len(t_done) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrivals[nxt] <= now:
            r = reqs[nxt]
            rid = srv.submit(scenes[r["scene"]], request_camera(r), request_desc(r), outs[nxt])
            id2k[rid] = nxt
            t_arr[nxt] = arrivals[nxt]
            nxt += 1
        srv.step(wait=False)
        for rid in srv.poll():
            t_done[id2k[rid]] = time.perf_counter() - t0
            if on_done:
                on_done(id2k[rid], t_done[id2k[rid]])
        max_held = max(max_held, srv.stats()[2])
        if nxt < len(reqs) and srv.stats()[1] == 0 and srv.stats()[0] == 0:
            time.sleep(max(0.0, min(0.001, arrivals[nxt] - (time.perf_counter() - t0))))
        if time_limit and time.perf_counter() - t0 > time_limit:
            raise TimeoutError("serving trace exceeded %.0f s" % time_limit)
    torch.cuda.synchronize()
    lat = [t_done[k] - t_arr[k] for k in range(len(reqs))]
    makespan = max(t_done.values())
    srv.close()
    return lat, makespan, outs, max_held


def run_plain(scenes, reqs, arrivals, outputs=None, time_limit=None, on_done=None):
    """FIFO plain renderer: each request rendered alone, in arrival order.
    on_done(k, seconds) is called as request k completes."""
    outs = outputs if outputs is not None else [torch.empty(r["res"] * r["res"], device="cuda") for r in reqs]
    # one workspace of the largest size any request needs, allocated up front
    need = max(_lib.gf_render_workspace_size(scenes[r["scene"]], request_camera(r), request_desc(r)) for r in reqs)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = []
    for k, r in enumerate(reqs):
        now = time.perf_counter() - t0
        if arrivals[k] > now:
            time.sleep(arrivals[k] - now)
        L, _ = _lib.gf_render(scenes[r["scene"]], request_camera(r), request_desc(r), ws, want_T=False)
        outs[k].copy_(L.view(-1))
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - arrivals[k])
        if on_done:
            on_done(k, time.perf_counter() - t0)
        if time_limit and time.perf_counter() - t0 > time_limit:
            raise TimeoutError("plain trace exceeded %.0f s" % time_limit)
    return lat, time.perf_counter() - t0, outs


def summarize(lat, makespan, reqs):
    rays = sum(r["res"] * r["res"] * r["spp"] for r in reqs)
    p50, p99 = _percentiles(lat)
    return {"p50_ms": 1e3 * p50, "p99_ms": 1e3 * p99, "Mrays_per_s": rays / makespan / 1e6,
            "requests": len(reqs), "makespan_s": makespan}
