"""Open-loop replay of a timed request stream through the request server.

Each request is submitted at its arrival time (seconds after the start);
the loop polls the server, fetches every finished request's per-ray
outputs to the host and records its latency (arrival to fetched).  The
server batches whatever has queued up whenever one of its slots frees, so
requests that arrive while others run join the next launch.  A request
with an 'ionogram' entry is an ionogram-synthesis request: once its sweep
is fetched, rt_ionogram extracts the traces (inside its latency).
"""
from __future__ import annotations

import time

import numpy as np


def replay(server, grids, requests, opts: dict, keep_results: bool = False):
    """Replay `requests` (dicts with t_arrive, snapshot, fan, optional
    per-request trace options 'opts' over `opts`, sorted by t_arrive)
    against `grids` (one rtgd.Grid per snapshot).  Returns a dict
    with per-request latency (s), ray-steps, wall time and, if asked, the
    results keyed by request index."""
    n = len(requests)
    lat = np.zeros(n)
    steps = np.zeros(n, dtype=np.int64)
    rays = np.zeros(n, dtype=np.int64)
    results = {} if keep_results else None
    ids = {}
    arrive = {}
    t0 = time.perf_counter()
    i = done = 0
    while done < n:
        now = time.perf_counter() - t0
        while i < n and requests[i]["t_arrive"] <= now:
            r = requests[i]
            rid = server.submit(grids[r["snapshot"]], r["fan"], **dict(opts, **r.get("opts", {})))
            ids[rid] = i
            arrive[rid] = t0 + r["t_arrive"]
            i += 1
        finished = server.poll()
        for d in finished:
            k = ids.pop(d["id"])
            out = server.fetch(d["id"], d["n_rays"])
            io = requests[k].get("ionogram")
            if io is not None:
                from . import rtgd
                out["ionogram"] = rtgd.ionogram(server.ctx, requests[k]["fan"], out,
                                                io["range_km"], io["max_points"])
            lat[k] = time.perf_counter() - arrive.pop(d["id"])
            steps[k] = d["total_steps"]
            rays[k] = d["n_rays"]
            if keep_results:
                results[k] = out
            done += 1
        if not finished:
            # nothing to collect: sleep until the next arrival or a short poll interval
            nxt = requests[i]["t_arrive"] - (time.perf_counter() - t0) if i < n else 1e-4
            time.sleep(min(max(nxt, 0.0), 1e-4))
    wall = time.perf_counter() - t0
    return dict(latency_s=lat, ray_steps=steps, rays=rays, wall_s=wall, results=results)
