"""Parity helpers: compare GPU per-ray outputs with the FP64 oracle.

FP64 path: |gpu - oracle| <= 1e-9 * max(|oracle|, floor), with a floor of 1 km
for lengths and 1 deg for angles, identical status and step count.  A ray
that misses this is re-traced by the oracle at elevations beta (1 +- 1e-10);
if that perturbation alone moves an output by more than 1e-7 (relative, same
floors) or flips its status, the ray is ill-conditioned (near the
penetration boundary the outputs jump with beta): it then passes if it
agrees to 1e-6 with one of the three oracle results (same status).

Mixed path: ground range and group path within 0.1 km and azimuth deviation
within 0.001 deg, same status.  FP32 evaluation perturbs every right-hand
side at the 1e-7 level, so a ray that misses is re-traced by the oracle with
its launch direction tilted by +-1e-6 deg in the launch plane (the elevation)
and across it, and with its frequency scaled by 1 +- 5e-8 (X by about 1e-7).
If any of those moves an output by more than the tolerance or flips its
status, the ray is ill-conditioned at FP32 level and counted apart; a ray
that misses while conditioned is a failure.  (The tilt across the launch
plane matters where the ground range is short: a near-vertical ray lands a
few hundred metres from the transmitter, and the bearing of that point
moves by more than 0.001 deg when it moves sideways by a few millimetres.)

Every function takes whole arrays and re-traces only the rays that miss, in
one oracle call, so that a full 112,400-ray sweep is classified in seconds.
"""
from __future__ import annotations

import numpy as np

LEN_KEYS = ("group_km", "phase_km", "range_km", "apogee_km")
ANG_KEYS = ("az_dev_deg", "land_lat_deg", "land_lon_deg")
# angles defined modulo 360 deg: the landing longitude is reported nearest the
# transmitter's and the azimuth deviation in (-180, 180], and both choices
# are ties where the landing point lies on the antipodal meridian or the
# deviation is 180 deg, which a last-bit difference in atan2 decides either
# way; their differences are compared modulo 360
PERIODIC_KEYS = ("az_dev_deg", "land_lon_deg")
NUMERIC = 3
TOL_KM, TOL_DEG = 0.1, 0.001


def diff(k, a, b):
    """a - b for output k, periodic angles reduced to [-180, 180]."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return d - 360.0 * np.round(d / 360.0) if k in PERIODIC_KEYS else d


def _scaled_err(g, o):
    """Per-ray max over the float outputs of |g - o| / max(|o|, 1); rays
    NUMERIC on both sides score 0 (their outputs are NaN)."""
    err = np.zeros(len(o["status"]))
    for k in LEN_KEYS + ANG_KEYS:
        d = diff(k, g[k], o[k])
        err = np.maximum(err, np.abs(d) / np.maximum(np.abs(np.asarray(o[k], dtype=np.float64)), 1.0))
    both_numeric = (np.asarray(g["status"]) == NUMERIC) & (np.asarray(o["status"]) == NUMERIC)
    err[both_numeric] = 0.0
    return np.where(np.isnan(err), np.inf, err)


def _take(res, idx):
    return {k: np.asarray(v)[idx] for k, v in res.items() if k in LEN_KEYS + ANG_KEYS +
            ("status", "n_steps")}


def ray_err(gpu, ora, i, j=None):
    """Max scaled error over the float outputs of ray i (gpu) vs j (oracle)."""
    j = i if j is None else j
    return float(_scaled_err(_take(gpu, [i]), _take(ora, [j]))[0])


def classify_fp64(gpu, ora, rays, trace_oracle, gpu_idx=None, tol=1e-9, ill_tol=1e-6, sens_tol=1e-7):
    """FP64 gate on every ray.  gpu: dict of host arrays (whole fan); ora:
    oracle results of the rays (elev, az, freq, mode) listed in `rays`;
    gpu_idx[k] is the gpu index of sample k (default: identity).
    trace_oracle(elev, az, freq, mode) re-traces rays.  Returns a report:
    n, n_within (met the gate directly), worst_rel and median_rel over
    those, ill_conditioned (tuples: gpu ray, elev, freq, mode, error against
    the nearest oracle result) and failures (dicts)."""
    elev, az, freq, mode = (np.asarray(v) for v in rays)
    n = elev.size
    gpu_idx = np.arange(n) if gpu_idx is None else np.asarray(gpu_idx)
    g = _take(gpu, gpu_idx)
    o = _take(ora, np.arange(n))
    same = g["status"] == o["status"]
    err = np.where(same, _scaled_err(g, o), np.inf)
    ok = same & (err <= tol) & (g["n_steps"] == o["n_steps"])
    miss = np.flatnonzero(~ok)
    ill, fails = [], []
    if miss.size:
        m2 = np.concatenate([miss, miss])
        pe = np.concatenate([elev[miss] * (1 - 1e-10), elev[miss] * (1 + 1e-10)])
        pr = trace_oracle(pe, az[m2], freq[m2], mode[m2])
        for j, k in enumerate(miss):
            sens, best = 0.0, ray_err(g, o, k) if same[k] else np.inf
            for p in (j, j + miss.size):
                if int(pr["status"][p]) != int(o["status"][k]):
                    sens = np.inf
                else:
                    sens = max(sens, ray_err(pr, o, p, k))
                if int(pr["status"][p]) == int(g["status"][k]):
                    best = min(best, ray_err(g, pr, k, p))
            i = int(gpu_idx[k])
            if sens > sens_tol and best <= ill_tol:
                ill.append((i, float(elev[k]), float(freq[k]), int(mode[k]), float(best)))
            else:
                fails.append(dict(ray=i, elev=float(elev[k]), az=float(az[k]), freq=float(freq[k]),
                                  mode=int(mode[k]), gpu_status=int(g["status"][k]),
                                  ora_status=int(o["status"][k]), err=float(err[k]),
                                  gpu_steps=int(g["n_steps"][k]), ora_steps=int(o["n_steps"][k]),
                                  sens=float(sens), best=float(best)))
    within = err[ok]
    return dict(n=n, n_within=int(ok.sum()), worst_rel=float(within.max()) if within.size else 0.0,
                median_rel=float(np.median(within)) if within.size else 0.0,
                ill_conditioned=ill, failures=fails)


def compare(gpu, ora, rays, trace_oracle, tol=1e-9, ill_tol=1e-6, gpu_idx=None):
    """classify_fp64, raising AssertionError if any ray fails."""
    rep = classify_fp64(gpu, ora, rays, trace_oracle, gpu_idx=gpu_idx, tol=tol, ill_tol=ill_tol)
    fails = rep["failures"]
    assert not fails, f"{len(fails)} of {rep['n']} rays out of tolerance: {fails[:5]}"
    return rep


def _mixed_ok(g, o, tol_km=TOL_KM, tol_deg=TOL_DEG):
    same = g["status"] == o["status"]
    num = same & (o["status"] == NUMERIC)
    d_r = np.abs(g["range_km"] - o["range_km"])
    d_g = np.abs(g["group_km"] - o["group_km"])
    d_a = np.abs(diff("az_dev_deg", g["az_dev_deg"], o["az_dev_deg"]))
    close = (d_r <= tol_km) & (d_g <= tol_km) & (d_a <= tol_deg)
    return num | (same & close)


def tilt_across(elev, az, delta_deg):
    """Launch direction (elevation, azimuth in deg) tilted by delta_deg
    across the launch plane (toward azimuth + 90 deg); for a vertical launch
    this tilts it toward azimuth + 90 deg."""
    b, a, d = np.radians(elev), np.radians(az), np.radians(delta_deg)
    up = np.sin(b)
    north = np.cos(b) * np.cos(a) - d * np.sin(a)
    east = np.cos(b) * np.sin(a) + d * np.cos(a)
    return np.degrees(np.arctan2(up, np.hypot(north, east))), np.degrees(np.arctan2(east, north))


def classify_mixed(gpu, ora, rays, trace_oracle, gpu_idx=None, tol_km=TOL_KM, tol_deg=TOL_DEG):
    """Mixed-precision tolerance on every ray.  Returns counts (n, n_within,
    n_ill, n_fail), the failures, and the max / RMS absolute errors of group
    path, ground range and azimuth deviation over the rays within tolerance
    and over all rays with the same (non-NUMERIC) status."""
    elev, az, freq, mode = (np.asarray(v) for v in rays)
    n = elev.size
    gpu_idx = np.arange(n) if gpu_idx is None else np.asarray(gpu_idx)
    g = _take(gpu, gpu_idx)
    o = _take(ora, np.arange(n))
    ok = _mixed_ok(g, o, tol_km, tol_deg)
    miss = np.flatnonzero(~ok)
    ill = np.zeros(n, dtype=bool)
    if miss.size:
        m6 = np.concatenate([miss] * 6)
        e_m, a_m = elev[miss], az[miss]
        (e_l, a_l), (e_r, a_r) = tilt_across(e_m, a_m, -1e-6), tilt_across(e_m, a_m, 1e-6)
        pe = np.concatenate([e_m - 1e-6, e_m + 1e-6, e_m, e_m, e_l, e_r])
        pa = np.concatenate([a_m, a_m, a_m, a_m, a_l, a_r])
        pf = np.concatenate([freq[miss], freq[miss], freq[miss] * (1 - 5e-8), freq[miss] * (1 + 5e-8),
                             freq[miss], freq[miss]])
        pr = _take(trace_oracle(pe, pa, pf, mode[m6]), np.arange(6 * miss.size))
        ref = _take(o, m6)
        moved = ~_mixed_ok(pr, ref, tol_km, tol_deg)
        ill[miss] = moved.reshape(6, miss.size).any(axis=0)
    fail = ~ok & ~ill
    same = (g["status"] == o["status"]) & (o["status"] != NUMERIC)
    stats = {}
    for k in ("group_km", "range_km", "az_dev_deg"):
        d = np.abs(diff(k, g[k], o[k]))
        for name, sel in (("within", ok & same), ("all", same)):
            v = d[sel]
            stats[f"{k}_max_{name}"] = float(v.max()) if v.size else 0.0
            stats[f"{k}_rms_{name}"] = float(np.sqrt(np.mean(v * v))) if v.size else 0.0
    fails = [dict(ray=int(gpu_idx[k]), elev=float(elev[k]), freq=float(freq[k]), mode=int(mode[k]),
                  gpu_status=int(g["status"][k]), ora_status=int(o["status"][k]),
                  d_range=float(g["range_km"][k] - o["range_km"][k]),
                  d_group=float(g["group_km"][k] - o["group_km"][k]),
                  d_az=float(diff("az_dev_deg", g["az_dev_deg"][k], o["az_dev_deg"][k]))) for k in np.flatnonzero(fail)]
    return dict(n=n, n_within=int(ok.sum()), n_ill=int(ill.sum()), n_fail=int(fail.sum()),
                n_status_mismatch=int((g["status"] != o["status"]).sum()), failures=fails, **stats)


def host(res):
    """Torch device results -> numpy."""
    out = {}
    for k, v in res.items():
        out[k] = v.cpu().numpy() if hasattr(v, "cpu") else v
    return out


def error_stats(gpu, ora, gpu_idx=None):
    """Max and RMS absolute differences (km, km, km, deg) over rays with the
    same status: group path, ground range, phase path, azimuth deviation."""
    gpu_idx = np.arange(len(ora["status"])) if gpu_idx is None else np.asarray(gpu_idx)
    same = np.asarray(gpu["status"])[gpu_idx] == np.asarray(ora["status"])
    same &= np.asarray(ora["status"]) != 3
    out = {"n_compared": int(same.sum()), "n_status_mismatch": int((~same).sum())}
    for k in ("group_km", "range_km", "phase_km", "az_dev_deg", "apogee_km"):
        d = diff(k, np.asarray(gpu[k])[gpu_idx][same], np.asarray(ora[k])[same])
        out[k] = {"max": float(np.abs(d).max()) if d.size else 0.0,
                  "rms": float(np.sqrt(np.mean(d ** 2))) if d.size else 0.0}
    return out


def oracle_tracer(orc, wl, fan=None, **kw):
    med = orc.OracleMedium.from_grid(wl.grid)
    fan = fan or wl.fan
    opts = dict(B0=wl.grid.B0_T, R=wl.grid.geom.earth_radius_km,
                tx=(fan.tx_lat_deg, fan.tx_lon_deg, fan.tx_h_km), step=wl.step_km,
                max_group=wl.max_group_km, exit_h=wl.exit_km)
    opts.update(kw)

    def tr(e, a, f, m, **extra):
        o = dict(opts)
        o.update(extra)
        return orc.trace(med, e, a, f, m, **o)
    return tr


def gpu_trace(rt, ctx, grid, wl, fan=None, **kw):
    args = dict(step_km=wl.step_km, max_group_km=wl.max_group_km, exit_h_km=wl.exit_km)
    args.update(kw)
    return rt.trace(ctx, grid, fan or wl.fan, **args)
