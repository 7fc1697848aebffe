"""Small driver for rocprofv3 runs: optional plain device copy of a known
size (calibrates the FETCH_SIZE / WRITE_SIZE counters), then `reps` traces
of one workload.

    python -m paper_2506_18579_amd.profile_run --workload ionogram --precision fp64 \
        --reps 3 --copy-mb 256
"""
from __future__ import annotations

import argparse
import json

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("ionogram", "aniso", "iso", "serving", "sweeps8"),
                    default="ionogram",
                    help="serving: the 400-request serving mix, every request queued at once "
                         "(the saturation run of the benchmark), through the request server; "
                         "sweeps8: eight ionogram sweeps (two per snapshot) queued at once there")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--copy-mb", type=int, default=0)
    ap.add_argument("--single", default="", help="elev,freq,mode,replicas: one ray of the "
                    "workload's grid and transmitter, replicated")
    ap.add_argument("--tail", type=int, default=0)
    ap.add_argument("--waves-per-simd", type=int, default=0)
    ap.add_argument("--ray-order", type=int, default=0)
    ap.add_argument("--promote-waves", type=int, default=0)
    ap.add_argument("--promote-age", type=int, default=0)
    ap.add_argument("--cu-layout", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner first and trace with the settings it picks "
                         "(the knob options above are then ignored)")
    a = ap.parse_args()
    import torch
    from paper_2506_18579_amd import rtgd, synth
    if a.copy_mb:
        n = a.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy {a.copy_mb} MiB read + {a.copy_mb} MiB write", flush=True)
    if a.workload in ("serving", "sweeps8"):
        serving(a, rtgd, synth)
        return
    wl = {"ionogram": lambda: synth.ionogram_workload(0),
          "aniso": lambda: synth.aniso_fan_workload(0),
          "iso": synth.iso_chapman_workload}[a.workload]()
    if a.single:
        el, fr, md, reps = a.single.split(",")
        wl.fan = synth.Fan(wl.fan.tx_lat_deg, wl.fan.tx_lon_deg, wl.fan.tx_h_km,
                           np.array([float(el)]), np.zeros(int(reps)), np.array([float(fr)]),
                           (int(md),))
    ctx = rtgd.Context(0)
    grid = rtgd.Grid(ctx, wl.grid)
    wkw = dict(step_km=wl.step_km, max_group_km=wl.max_group_km, exit_h_km=wl.exit_km)
    knobs = dict(tail_threshold=a.tail, waves_per_simd=a.waves_per_simd, ray_order=a.ray_order,
                 promote_waves=a.promote_waves, promote_age=a.promote_age, cu_layout=a.cu_layout)
    if a.autotune:
        tune = rtgd.autotune(ctx, grid, wl.fan, precision=a.precision, **wkw)
        knobs = {k: tune[k] for k in knobs}
        print(json.dumps({"autotuned": knobs}), flush=True)
    out = None
    for i in range(a.reps):
        out = rtgd.trace(ctx, grid, wl.fan, precision=a.precision, device_results=True, out=out,
                         **wkw, **knobs)
        print(json.dumps({"rep": i, "workload": wl.name, "precision": a.precision,
                          "ray_steps": out["total_steps"], "kernel_ms": out["kernel_ms"],
                          "trace_ms": out["trace_ms"], "tail_ms": out["tail_ms"],
                          "phase_steps": out["phase_steps"],
                          "one_lane_occupancy": out["phase_steps"][0] / max(1, 64 * out["one_lane_wave_iters"])}),
              flush=True)
    grid.close()
    ctx.close()


def serving(a, rtgd, synth):
    """The benchmark's serving mix at saturation: 400 requests (90 % ray fans
    of 1-20,000 rays, 10 % ionogram syntheses) over 4 resident snapshots,
    all queued at t = 0, `reps` times after a warm-up of 8 requests; or
    (sweeps8) eight 112,400-ray ionogram sweeps, two per snapshot, queued at
    t = 0."""
    from paper_2506_18579_amd import serve
    ctx = rtgd.Context(0)
    snaps = [rtgd.Grid(ctx, synth.ionosphere_grid(synth.GEOM_ANISO, s)) for s in range(4)]
    reqs = synth.serving_requests(400, seed=1234, n_snapshots=4, max_rays=20000, qps=200.0,
                                  ionogram_fraction=0.1)
    o = dict(step_km=1.0, max_group_km=4000.0, exit_h_km=600.0, precision=a.precision)
    srv = rtgd.Server(ctx, mem_budget_bytes=256 << 20)
    serve.replay(srv, snaps, reqs[:8], o)
    if a.workload == "sweeps8":
        wl = synth.ionogram_workload(0)
        burst = [dict(t_arrive=0.0, snapshot=s % 4, fan=wl.fan) for s in range(8)]
        o = dict(step_km=wl.step_km, max_group_km=wl.max_group_km, exit_h_km=wl.exit_km, precision=a.precision)
        name = "eight_ionogram_sweeps"
    else:
        burst = [dict(q, t_arrive=0.0) for q in reqs]
        name = "serving_400_requests"
    for i in range(a.reps):
        r = serve.replay(srv, snaps, burst, o)
        print(json.dumps({"rep": i, "workload": name, "precision": a.precision,
                          "wall_ms": r["wall_s"] * 1e3, "ray_steps": int(r["ray_steps"].sum()),
                          "ray_steps_per_s": float(r["ray_steps"].sum() / r["wall_s"])}), flush=True)
    srv.close()
    for g in snaps:
        g.close()
    ctx.close()


if __name__ == "__main__":
    main()
