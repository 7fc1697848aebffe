"""Benchmark: ray-steps/s of batched GD ray tracing on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one rt_trace of the whole oblique-ionogram sweep (181x181x226
anisotropic grid, 281 frequencies x 2 modes x 200 elevations = 112,400
rays, FP64), grid and output buffers resident in HBM.  The same sweep is
timed in mixed precision, the 24,576-ray anisotropic fan in both
precisions, and fan latency percentiles are reported.  Accuracy is measured
on a sample against the FP64 CPU oracle, which is also timed on the host
cores as the CPU baseline.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per RK4 step (4 right-hand sides + combine),
# counted from the method (add/mul = 1, FMA = 2, div/sqrt/sincos = 1):
# per RHS: cell location 13, 1-D GD weights 3 x 65, 4x4x4 contraction of
# value + 3 partials 352 (+7 scaling), dipole 16, A-H setup 15, A-H partials
# 42, Hamiltonian partials 50, ray equations 40 -> 730 (anisotropic);
# isotropic RHS 617.  Per step 4 RHS + 136 (RK4 stages, termination).
FLOPS_PER_STEP_ANISO = 4 * 730 + 136
FLOPS_PER_STEP_ISO = 4 * 617 + 136
PEAK_FP64_VALU_TFLOPS = 78.6      # MI355X vector FP64 (256 CU x 2.4 GHz x 128)
PEAK_FP32_VALU_TFLOPS = 157.3     # packed FP32; 78.6 without packed math

# HBM bytes of one FP64 ionogram launch (k_start, k_trace, k_tail and
# k_finish; the autotuned setting: hand-off at 4096 rays, 32 promotion waves
# for trapped and grazing rays) from rocprofv3: FETCH_SIZE x 2.000 +
# WRITE_SIZE x 1.000 (factors from a 1 GiB device copy in the same runs).
# Valid only for the device sources (per-step arithmetic and trace kernels)
# with these hashes; otherwise reported as null.
TRAFFIC_BYTES = (76280 + 48017) * 1024
TRAFFIC_SOURCES = {
    "rtgd_device.h": "fc2671d864d65019d61ee6dcdc3f5df412c22267d5495bb45054fd1589ddab48",
    "rtgd_kernels.h": "3700c5caf5f3c2d5f2c992a4bc176ea4ea361702d9c0259e38cdf231dc9335a1",
}


# launch settings the autotuner chooses (results do not depend on them)
TUNED_KNOBS = ("tail_threshold", "waves_per_simd", "ray_order", "promote_waves", "promote_age")


def measured_traffic():
    import hashlib
    csrc = os.path.join(ROOT, "paper_2506_18579_amd", "csrc")
    for name, digest in TRAFFIC_SOURCES.items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return TRAFFIC_BYTES


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample-stride", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-qps", type=float, default=200.0,
                    help="rate the request stream is drawn at (rescaled to each offered load)")
    return ap.parse_args()


def time_trace(rtgd, torch, ctx, grid, wl, precision, steps, warmup, tune=None):
    out = None
    kw = {k: tune[k] for k in TUNED_KNOBS} if tune else {}
    for _ in range(warmup):
        out = rtgd.trace(ctx, grid, wl.fan, step_km=wl.step_km, max_group_km=wl.max_group_km,
                         exit_h_km=wl.exit_km, precision=precision, device_results=True, out=out, **kw)
    torch.cuda.synchronize()
    walls, kms, total = [], [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        out = rtgd.trace(ctx, grid, wl.fan, step_km=wl.step_km, max_group_km=wl.max_group_km,
                         exit_h_km=wl.exit_km, precision=precision, device_results=True, out=out, **kw)
        walls.append(time.perf_counter() - ts)
        kms.append(out["kernel_ms"])
        total += out["total_steps"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return dict(out=out, elapsed=elapsed, walls=walls, kernel_ms=kms, ray_steps=total)


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: rays are independent, so one GPU's share of a "
              "sharded fan is the same workload at its real shape; multi-GPU runs are not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2506_18579_amd import rtgd, synth

    ctx = rtgd.Context(0)
    wl = synth.ionogram_workload(0)
    grid = rtgd.Grid(ctx, wl.grid)

    wkw = dict(step_km=wl.step_km, max_group_km=wl.max_group_km, exit_h_km=wl.exit_km)
    tune64 = rtgd.autotune(ctx, grid, wl.fan, precision="fp64", **wkw)
    tune32 = rtgd.autotune(ctx, grid, wl.fan, precision="mixed", **wkw)
    fp64 = time_trace(rtgd, torch, ctx, grid, wl, "fp64", a.steps, a.warmup, tune64)
    mixed = time_trace(rtgd, torch, ctx, grid, wl, "mixed", max(1, a.steps), 1, tune32)
    # end to end: per-ray results copied back to host memory inside each call
    e2e = []
    for _ in range(3):
        t = time.perf_counter()
        r = rtgd.trace(ctx, grid, wl.fan, step_km=wl.step_km, max_group_km=wl.max_group_km,
                       exit_h_km=wl.exit_km, precision="fp64", **{k: tune64[k] for k in TUNED_KNOBS})
        e2e.append((time.perf_counter() - t, r["total_steps"]))
    e2e_ms = float(np.median([x[0] for x in e2e])) * 1e3
    fan_wl = synth.aniso_fan_workload(0)
    fan_grid = rtgd.Grid(ctx, fan_wl.grid)
    # fan latency: 20 launches each, with the library defaults and with the
    # settings the autotuner picks for this fan
    fan64 = time_trace(rtgd, torch, ctx, fan_grid, fan_wl, "fp64", 20, 2)
    fan32 = time_trace(rtgd, torch, ctx, fan_grid, fan_wl, "mixed", 20, 2)
    fkw = dict(step_km=fan_wl.step_km, max_group_km=fan_wl.max_group_km, exit_h_km=fan_wl.exit_km)
    ftune64 = rtgd.autotune(ctx, fan_grid, fan_wl.fan, precision="fp64", **fkw)
    ftune32 = rtgd.autotune(ctx, fan_grid, fan_wl.fan, precision="mixed", **fkw)
    fan64t = time_trace(rtgd, torch, ctx, fan_grid, fan_wl, "fp64", 20, 2, ftune64)
    fan32t = time_trace(rtgd, torch, ctx, fan_grid, fan_wl, "mixed", 20, 2, ftune32)
    fan_grid.close()

    serving = {}
    if a.serve_requests > 0:
        from paper_2506_18579_amd import serve
        snaps = [rtgd.Grid(ctx, synth.ionosphere_grid(synth.GEOM_ANISO, s)) for s in range(4)]
        reqs = synth.serving_requests(a.serve_requests, seed=1234, n_snapshots=4, max_rays=20000,
                                      qps=a.serve_qps, ionogram_fraction=0.1)
        sopts = dict(step_km=1.0, max_group_km=4000.0, exit_h_km=600.0)
        burst = [dict(q, t_arrive=0.0) for q in reqs]

        def stats(r):
            lat = r["latency_s"] * 1e3
            return {"ray_steps_per_s": float(r["ray_steps"].sum() / r["wall_s"]),
                    "requests_per_s": len(reqs) / r["wall_s"],
                    "latency_ms_p50": float(np.percentile(lat, 50)),
                    "latency_ms_p99": float(np.percentile(lat, 99)),
                    "latency_ms_max": float(lat.max()), "wall_s": r["wall_s"]}
        for prec in ("fp64", "mixed"):
            srv = rtgd.Server(ctx, n_slots=4, mem_budget_bytes=256 << 20)
            o = dict(sopts, precision=prec)
            serve.replay(srv, snaps, reqs[:8], o)                       # warm-up
            # saturation: every request queued at t = 0
            rs = serve.replay(srv, snaps, burst, o)
            sat = stats(rs)
            res = dict(rays=int(rs["rays"].sum()), ray_steps=int(rs["ray_steps"].sum()),
                       saturation=sat)
            # Poisson arrivals (the same stream, time-scaled) at 25, 50 and 90 % of
            # the measured saturation request rate
            for frac in (0.25, 0.5, 0.9):
                qps = frac * sat["requests_per_s"]
                scaled = [dict(q, t_arrive=q["t_arrive"] * a.serve_qps / qps) for q in reqs]
                res[f"load_{int(frac * 100)}pct"] = dict(stats(serve.replay(srv, snaps, scaled, o)),
                                                         offered_requests_per_s=qps)
            srv.close()
            serving[prec] = res
        for g in snaps:
            g.close()

    steps_per_trace = fp64["ray_steps"] / a.steps
    ms_per_step = fp64["elapsed"] / a.steps * 1e3
    value = steps_per_trace / (ms_per_step / 1e3)
    kms = float(np.mean(fp64["kernel_ms"]))
    achieved = steps_per_trace * FLOPS_PER_STEP_ANISO / (kms * 1e-3) / 1e12

    res64 = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in fp64["out"].items()}
    res32 = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in mixed["out"].items()}

    cpu = None
    cpu_1thread = None
    accuracy = {}
    if not a.no_cpu:
        from oracle import oracle as O
        idx = np.arange(0, wl.fan.n_rays, a.cpu_sample_stride)
        e, az, f, m = wl.fan.expand()
        med = O.OracleMedium.from_grid(wl.grid)
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t = time.perf_counter()
        o = O.trace(med, e[idx], az[idx], f[idx], m[idx], B0=wl.grid.B0_T,
                    R=wl.grid.geom.earth_radius_km,
                    tx=(wl.fan.tx_lat_deg, wl.fan.tx_lon_deg, wl.fan.tx_h_km),
                    step=wl.step_km, max_group=wl.max_group_km, exit_h=wl.exit_km,
                    nthreads=nthreads)
        dt = time.perf_counter() - t
        cpu = {"value": o["total_steps"] / dt, "unit": "ray-steps/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"every {a.cpu_sample_stride}. ray of the 112,400-ray ionogram sweep "
                         f"({idx.size} rays, {o['total_steps']} ray-steps, {dt:.1f} s, "
                         f"plain FP64 C, OpenMP over rays)"}
        # one host thread on a bounded sample (every 64th ray)
        idx1 = np.arange(0, wl.fan.n_rays, 64)
        t = time.perf_counter()
        o1 = O.trace(med, e[idx1], az[idx1], f[idx1], m[idx1], B0=wl.grid.B0_T,
                     R=wl.grid.geom.earth_radius_km,
                     tx=(wl.fan.tx_lat_deg, wl.fan.tx_lon_deg, wl.fan.tx_h_km),
                     step=wl.step_km, max_group=wl.max_group_km, exit_h=wl.exit_km, nthreads=1)
        dt1 = time.perf_counter() - t
        cpu_1thread = {"value": o1["total_steps"] / dt1, "unit": "ray-steps/s", "cores": 1,
                       "sample": f"every 64th ray ({idx1.size} rays, {o1['total_steps']} ray-steps, "
                                 f"{dt1:.1f} s)"}
        same = (res64["status"][idx] == o["status"])
        scale = lambda k, fl: np.abs(res64[k][idx][same] - o[k][same]) / np.maximum(np.abs(o[k][same]), fl)
        relv = np.max([scale(k, 1.0) for k in ("group_km", "phase_km", "range_km", "az_dev_deg")], axis=0)
        accuracy["fp64_max_rel_vs_oracle"] = float(relv.max())
        accuracy["fp64_median_rel_vs_oracle"] = float(np.median(relv))
        accuracy["fp64_rays_over_1e-9_rel"] = int((relv > 1e-9).sum())
        accuracy["fp64_status_mismatch"] = int((~same).sum())
        same32 = (res32["status"][idx] == o["status"]) & (o["status"] != 3)
        for k in ("group_km", "range_km", "az_dev_deg"):
            d = res32[k][idx][same32] - o[k][same32]
            accuracy[f"mixed_{k}_max_all"] = float(np.abs(d).max())
            accuracy[f"mixed_{k}_rms_all"] = float(np.sqrt(np.mean(d * d)))
        accuracy["mixed_status_mismatch"] = int((~same32 & (o["status"] != 3)).sum())
        accuracy["sample_rays"] = int(idx.size)
        # FP32 evaluation perturbs every right-hand side at the 1e-7 level: a
        # ray whose FP64 outputs already move by more than the tolerance when
        # its elevation moves by 1e-6 deg or its frequency by 5e-8 (X by
        # 1e-7) -- near the penetration boundary, near reflection -- is
        # counted apart.  Probed on every 8th sampled ray.
        sub = np.arange(0, idx.size, 8)
        k_idx = idx[sub]
        pe = np.concatenate([e[k_idx] - 1e-6, e[k_idx] + 1e-6, e[k_idx], e[k_idx]])
        pf = np.concatenate([f[k_idx], f[k_idx], f[k_idx] * (1 - 5e-8), f[k_idx] * (1 + 5e-8)])
        rep4 = lambda v: np.concatenate([v[k_idx]] * 4)
        pr = O.trace(med, pe, rep4(az), pf, rep4(m), B0=wl.grid.B0_T,
                     R=wl.grid.geom.earth_radius_km,
                     tx=(wl.fan.tx_lat_deg, wl.fan.tx_lon_deg, wl.fan.tx_h_km),
                     step=wl.step_km, max_group=wl.max_group_km, exit_h=wl.exit_km,
                     nthreads=nthreads)
        ns = sub.size
        ill = np.zeros(ns, dtype=bool)
        for half in range(4):
            sl = slice(half * ns, (half + 1) * ns)
            ill |= pr["status"][sl] != o["status"][sub]
            ill |= np.abs(pr["range_km"][sl] - o["range_km"][sub]) > 0.1
            ill |= np.abs(pr["group_km"][sl] - o["group_km"][sub]) > 0.1
            ill |= np.abs(pr["az_dev_deg"][sl] - o["az_dev_deg"][sub]) > 0.001
        good = ~ill & (res32["status"][k_idx] == o["status"][sub]) & (o["status"][sub] != 3)
        for k in ("group_km", "range_km", "az_dev_deg"):
            d = res32[k][k_idx][good] - o[k][sub][good]
            accuracy[f"mixed_{k}_max"] = float(np.abs(d).max())
            accuracy[f"mixed_{k}_rms"] = float(np.sqrt(np.mean(d * d)))
        within = good & (np.abs(res32["range_km"][k_idx] - o["range_km"][sub]) <= 0.1) & \
            (np.abs(res32["group_km"][k_idx] - o["group_km"][sub]) <= 0.1) & \
            (np.abs(res32["az_dev_deg"][k_idx] - o["az_dev_deg"][sub]) <= 0.001)
        accuracy["mixed_conditioned_within_tolerance"] = int(within.sum())
        accuracy["mixed_conditioned_rays"] = int(good.sum())
        accuracy["mixed_ill_conditioned_rays"] = int(ill.sum())
        accuracy["mixed_tolerance"] = "0.1 km ground range and group path, 0.001 deg azimuth"

    lat = np.array(fan64["walls"]) * 1e3
    lat32 = np.array(fan32["walls"]) * 1e3
    latt = np.array(fan64t["walls"]) * 1e3
    latt32 = np.array(fan32t["walls"]) * 1e3
    line = {
        "metric": "ray-steps/s at stated accuracy, FP64 vs mixed; p50/p99 ray-fan latency",
        "value": value,
        "unit": "ray-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "rays": wl.fan.n_rays, "grid": "181x181x226",
                   "ray_steps_per_step": int(steps_per_trace), "field": "axial dipole 3.12e-5 T",
                   "modes": "O+X", "step_km": wl.step_km, "exit_km": wl.exit_km,
                   "max_group_km": wl.max_group_km},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU_TFLOPS,
                     "traffic": measured_traffic(),
                     "kernel": "trace launch: k_start + k_trace<double,0> + k_tail<double,0> + k_finish",
                     "kernel_ms_avg": kms, "flops_per_ray_step": FLOPS_PER_STEP_ANISO},
        "tuning": {"fp64": tune64, "mixed": tune32},
        "cpu_baseline": cpu,
        "cpu_oracle_1thread": cpu_1thread,
        "end_to_end_host_results": {"ms_per_sweep": e2e_ms,
                                    "ray_steps_per_s": e2e[-1][1] / (e2e_ms * 1e-3),
                                    "note": "fan upload, the four kernels and the 8 MB result copy "
                                            "to pageable host memory"},
        "accuracy": accuracy,
        "mixed": {"value": mixed["ray_steps"] / mixed["elapsed"],
                  "kernel_ms_avg": float(np.mean(mixed["kernel_ms"])),
                  "speedup_vs_fp64": (mixed["ray_steps"] / mixed["elapsed"]) / value},
        "aniso_fan_24576": {
            "fp64_ray_steps_per_s": fan64["ray_steps"] / fan64["elapsed"],
            "mixed_ray_steps_per_s": fan32["ray_steps"] / fan32["elapsed"],
            "fp64_latency_ms_p50": float(np.percentile(lat, 50)),
            "fp64_latency_ms_p99": float(np.percentile(lat, 99)),
            "mixed_latency_ms_p50": float(np.percentile(lat32, 50)),
            "mixed_latency_ms_p99": float(np.percentile(lat32, 99)),
            "tuned_fp64_latency_ms_p50": float(np.percentile(latt, 50)),
            "tuned_fp64_latency_ms_p99": float(np.percentile(latt, 99)),
            "tuned_mixed_latency_ms_p50": float(np.percentile(latt32, 50)),
            "tuned_mixed_latency_ms_p99": float(np.percentile(latt32, 99)),
            "tuning": {"fp64": {k: ftune64[k] for k in TUNED_KNOBS},
                       "mixed": {k: ftune32[k] for k in TUNED_KNOBS}},
            "note": "wall time of one rt_trace call (device results), 20 calls each; "
                    "library defaults, then the autotuned settings for this fan"},
        "serving": dict(serving, workload=f"{a.serve_requests} requests, 90 % ray fans of "
                        "1-20,000 rays (log-uniform) and 10 % ionogram syntheses (500-4,000-ray "
                        "sweeps of the 1200 km link), 4 resident 181x181x226 snapshots, 4 slots, "
                        "256 MiB output "
                        "arena; all requests at once (saturation), then Poisson arrivals at 25, "
                        "50 and 90 % of the saturation request rate") if serving else None,
    }
    print(json.dumps(line), flush=True)
    grid.close()
    ctx.close()


if __name__ == "__main__":
    main()
