"""The parity classification itself, on the CPU: the oracle against copies
of its own results with planted errors.  A ray that is well conditioned and
moved beyond the tolerance must be reported as a failure; a ray within the
tolerance must not; NUMERIC rays on both sides agree."""
import numpy as np

from paper_2506_18579_amd import synth

from parity import classify_fp64, classify_mixed, oracle_tracer


def _setup(orc):
    wl = synth.iso_chapman_workload()
    fan = synth.sub_fan(wl.fan, elev_idx=list(range(0, 90, 6)))
    rays = fan.expand()
    tr = oracle_tracer(orc, wl, fan)
    return rays, tr, tr(*rays)


def _copy(res):
    return {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in res.items()}


def test_fp64_classification(orc):
    rays, tr, o = _setup(orc)
    rep = classify_fp64(o, o, rays, tr)
    assert rep["n_within"] == rep["n"] and not rep["failures"] and rep["worst_rel"] == 0.0
    g = _copy(o)
    g["range_km"][3] *= 1 + 3e-9          # a conditioned ray moved beyond 1e-9
    g["group_km"][5] *= 1 + 5e-10         # within the gate
    g["n_steps"][7] += 1                  # a step count that differs
    rep = classify_fp64(g, o, rays, tr)
    assert sorted(f["ray"] for f in rep["failures"]) == [3, 7]
    assert abs(rep["worst_rel"] - 5e-10) < 1e-12


def test_fp64_gpu_index_map(orc):
    rays, tr, o = _setup(orc)
    n = rays[0].size
    big = {k: np.concatenate([np.full(2, np.nan) if v.dtype.kind == "f" else np.zeros(2, v.dtype), v])
           for k, v in o.items() if isinstance(v, np.ndarray)}
    rep = classify_fp64(big, o, rays, tr, gpu_idx=np.arange(2, n + 2))
    assert rep["n_within"] == n


def test_mixed_classification(orc):
    rays, tr, o = _setup(orc)
    g = _copy(o)
    g["group_km"][2] += 0.05              # within 0.1 km
    g["range_km"][4] += 0.3               # beyond, on a conditioned ray
    g["az_dev_deg"][6] += 0.002           # beyond 0.001 deg
    g["status"][8] = 3                    # a status that differs
    rep = classify_mixed(g, o, rays, tr)
    assert rep["n_fail"] == 3 and sorted(f["ray"] for f in rep["failures"]) == [4, 6, 8]
    assert rep["n_within"] == rep["n"] - 3
    assert abs(rep["group_km_max_within"] - 0.05) < 1e-9


def test_periodic_angles_compared_modulo_360(orc):
    """The landing longitude and the azimuth deviation are angles: a result
    that names the same angle another way (a landing point on the antipodal
    meridian reported as lon + 360) is the same result."""
    rays, tr, o = _setup(orc)
    g = _copy(o)
    g["land_lon_deg"][1] += 360.0           # the same longitude
    g["az_dev_deg"][2] -= 360.0             # the same deviation
    g["land_lon_deg"][4] += 360.0 + 1e-3    # another longitude
    rep = classify_fp64(g, o, rays, tr)
    assert [f["ray"] for f in rep["failures"]] == [4]
