"""GPU (HIP, FP64) vs the FP64 CPU oracle, through the C-ABI.

Element-by-element parity on small fans that span several 64-lane waves
and a ragged tail; sampled parity at the full workload sizes in the launch
configuration the benchmark uses; edge cases (empty fan, grid edges, maximum
path, invalid arguments, trajectories, determinism, batch independence).
"""
import dataclasses

import numpy as np
import pytest

from paper_2506_18579_amd import synth

from parity import compare, error_stats, gpu_trace, host, oracle_tracer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    from paper_2506_18579_amd import rtgd
    rtgd.lib()
    return rtgd


@pytest.fixture(scope="module")
def ctx(rt):
    c = rt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def iso_wl():
    return synth.iso_chapman_workload()


@pytest.fixture(scope="module")
def aniso_wl():
    return synth.aniso_fan_workload(0)


@pytest.fixture(scope="module")
def iso_grid(rt, ctx, iso_wl):
    g = rt.Grid(ctx, iso_wl.grid)
    yield g
    g.close()


@pytest.fixture(scope="module")
def aniso_grid(rt, ctx, aniso_wl):
    g = rt.Grid(ctx, aniso_wl.grid)
    yield g
    g.close()


def test_iso_chapman_every_ray(rt, ctx, orc, iso_wl, iso_grid):
    """Isotropic 61x61x201 Chapman grid, 90 rays 1..90 deg: all rays."""
    g = gpu_trace(rt, ctx, iso_grid, iso_wl)
    rays = iso_wl.fan.expand()
    tr = oracle_tracer(orc, iso_wl)
    o = tr(*rays)
    rep = compare(g, o, rays, tr)
    assert g["total_steps"] == int(g["n_steps"].sum()) == o["total_steps"]
    print("iso worst rel err", rep["worst_rel"], "ill-conditioned", rep["ill_conditioned"])
    # 1..51 deg return to ground, 52..90 escape (10 MHz through foF2 = 8 MHz)
    assert np.all(g["status"][:51] == 0) and np.all(g["status"][51:] == 1)


def test_grazing_returns_match_oracle(rt, ctx, orc, iso_wl, iso_grid):
    """Rays from a transmitter at 50 km launched below about 7 deg come back
    below the grid bottom on vacuum lines that miss the Earth and climb back
    into the grid (the grazing branch of the landing rule), hop after hop, up
    to the maximum group path.  Every ray against the oracle; the 16-lane
    path (every ray handed to the tail kernel at once) is bit-identical.
    The azimuths keep the hops away from the poles: a meridional ray that
    crosses a pole reaches the antipodal meridian, where the longitude of
    the spherical state is a tie between -180 and +180 deg from the
    transmitter that rounding decides."""
    fan = synth.Fan(30.0, 110.0, 50.0, np.array([1.0, 4.0, 6.5]), np.array([90.0, 135.0]),
                    np.array([6.0, 8.0]), (1,))
    wl = dataclasses.replace(iso_wl, max_group_km=8000.0)
    g = gpu_trace(rt, ctx, iso_grid, wl, fan, tail_threshold=-1)
    rays = fan.expand()
    tr = oracle_tracer(orc, wl, fan)
    o = tr(*rays)
    rep = compare(g, o, rays, tr)
    print("grazing worst rel err", rep["worst_rel"])
    assert np.all(g["status"] == 2)
    # chords add path without steps: fewer steps than max_group / step
    assert np.all(g["n_steps"] < 7000)
    t16 = gpu_trace(rt, ctx, iso_grid, wl, fan, tail_threshold=fan.n_rays)
    for k in ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km", "land_lat_deg",
              "land_lon_deg", "status", "n_steps"):
        assert np.array_equal(g[k], t16[k], equal_nan=True), k


def _subfan(wl):
    return synth.sub_fan(wl.fan, elev_idx=[0, 9, 21, 40, 63], az_idx=[0, 7, 13, 22, 31, 50, 63])


def test_aniso_subfan_every_ray(rt, ctx, orc, aniso_wl, aniso_grid):
    """Anisotropic grid, O and X, 3 frequencies: 210 rays (3 full waves and a
    ragged tail of 18), every ray against the oracle."""
    fan = _subfan(aniso_wl)
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    rays = fan.expand()
    tr = oracle_tracer(orc, aniso_wl, fan)
    o = tr(*rays)
    rep = compare(g, o, rays, tr)
    print("aniso subfan worst rel err", rep["worst_rel"], "ill", len(rep["ill_conditioned"]))
    assert len(rep["ill_conditioned"]) <= 3


def test_long_steps_match_oracle(rt, ctx, orc, aniso_wl, aniso_grid):
    """400 km RK4 steps: a stage's colatitude then lies beyond the range of the
    series around the ray's anchor colatitude, so those stages take sin and cos
    from the library; every ray still matches the oracle."""
    fan = _subfan(aniso_wl)
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, step_km=400.0)
    rays = fan.expand()
    tr = oracle_tracer(orc, aniso_wl, fan, step=400.0)
    o = tr(*rays)
    rep = compare(g, o, rays, tr)
    print("400 km steps worst rel err", rep["worst_rel"], "ill", len(rep["ill_conditioned"]),
          "steps", int(g["n_steps"].sum()))
    assert len(rep["ill_conditioned"]) <= 3


def test_aniso_full_fan_sampled(rt, ctx, orc, aniso_wl, aniso_grid):
    """All 24,576 rays on the GPU (device-resident outputs, as benchmarked);
    a seeded sample of 160 checked against the oracle one by one."""
    g = host(gpu_trace(rt, ctx, aniso_grid, aniso_wl, device_results=True))
    n = aniso_wl.fan.n_rays
    assert g["status"].size == n
    assert np.all((g["status"] >= 0) & (g["status"] <= 3))
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 158, replace=False)]))
    e, a, f, m = aniso_wl.fan.expand()
    rays = (e[idx], a[idx], f[idx], m[idx])
    tr = oracle_tracer(orc, aniso_wl)
    o = tr(*rays)
    rep = compare(g, o, rays, tr, gpu_idx=idx)
    print("aniso full sampled worst", rep["worst_rel"], "ill", len(rep["ill_conditioned"]))
    print("status histogram", np.bincount(g["status"], minlength=4))


def test_two_million_ray_fan_sampled(rt, ctx, orc, aniso_wl, aniso_grid):
    """A fan of 2^21 = 2,097,152 rays (128 elevations x 128 azimuths x 64
    frequencies x O/X; queue tickets, ray records and outputs at scale), 300 km
    of group path each: the per-ray step counts add up to the launch total,
    every status is valid, and a seeded sample of 256 rays, the first and the
    last included, matches the oracle."""
    fan = synth.Fan(30.0, 110.0, 0.0, np.linspace(2.0, 80.0, 128), np.linspace(-60.0, 60.0, 128),
                    np.linspace(3.0, 25.0, 64), (1, -1))
    wl = dataclasses.replace(aniso_wl, max_group_km=300.0)
    n = fan.n_rays
    assert n == 1 << 21
    g = host(gpu_trace(rt, ctx, aniso_grid, wl, fan, device_results=True))
    assert g["status"].size == n
    assert np.all((g["status"] >= 0) & (g["status"] <= 3))
    assert g["total_steps"] == int(g["n_steps"].astype(np.int64).sum())
    rng = np.random.default_rng(21)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 254, replace=False)]))
    e, a, f, m = fan.expand()
    rays = (e[idx], a[idx], f[idx], m[idx])
    tr = oracle_tracer(orc, wl, fan)
    o = tr(*rays)
    rep = compare(g, o, rays, tr, gpu_idx=idx)
    print("2^21-ray fan sampled worst", rep["worst_rel"], "ill", len(rep["ill_conditioned"]))


def test_ionogram_every_ray(rt, ctx, ionogram_sweep, ionogram_sweep_oracle):
    """Ionogram sweep, all 112,400 rays (exit 1000 km, 8000 km max group path),
    device-resident outputs and the library's default launch settings,
    against the oracle ray by ray.  Every ray meets the 1e-9 gate or is
    ill-conditioned (its oracle outputs move by more than 1e-7 when the
    elevation moves by 1e-10 relative) and within 1e-6 of an oracle result."""
    wl = ionogram_sweep
    grid = rt.Grid(ctx, wl.grid)
    try:
        g = host(gpu_trace(rt, ctx, grid, wl, device_results=True))
    finally:
        grid.close()
    o, tr = ionogram_sweep_oracle
    rep = compare(g, o, wl.fan.expand(), tr)
    assert g["total_steps"] == o["total_steps"] == sum(g["phase_steps"])
    assert g["phase_steps"][1] > 0 and g["phase_steps"][2] > 0    # promotion and tail both ran
    # lane occupancy of the one-lane waves: each iteration steps at most 64 rays
    assert 0 < g["phase_steps"][0] <= 64 * g["one_lane_wave_iters"] < 64 * g["phase_steps"][0]
    print("ionogram every ray: one-lane occupancy", g["phase_steps"][0] / (64 * g["one_lane_wave_iters"]))
    print("ionogram every ray: within 1e-9", rep["n_within"], "of", rep["n"], "worst", rep["worst_rel"],
          "median", rep["median_rel"], "ill-conditioned", rep["ill_conditioned"])
    assert len(rep["ill_conditioned"]) <= 50


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_numeric_status_matches_oracle(rt, ctx, orc, iso_wl, iso_grid, precision):
    """A frequency whose square underflows (1e-170 MHz) makes X = f_N^2 / f^2
    infinite at the first right-hand side inside the grid: the Hamiltonian
    is not finite, the ray ends NUMERIC after one step with NaN outputs, on
    the oracle and on the GPU alike.  Rays of an ordinary frequency in the
    same launch are unaffected."""
    fan = synth.Fan(30.0, 110.0, 0.0, np.array([10.0, 45.0, 80.0]), np.array([0.0]),
                    np.array([1e-170, 10.0]), (1,))
    g = gpu_trace(rt, ctx, iso_grid, iso_wl, fan, precision=precision)
    rays = fan.expand()
    tr = oracle_tracer(orc, iso_wl, fan)
    o = tr(*rays)
    assert list(o["status"][:3]) == [3, 3, 3] and list(o["n_steps"][:3]) == [1, 1, 1]
    assert np.array_equal(g["status"], o["status"]) and np.array_equal(g["n_steps"], o["n_steps"])
    for k in ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km"):
        assert np.all(np.isnan(g[k][:3])), k
        assert np.all(np.isfinite(g[k][3:])), k
    if precision == "fp64":
        compare(g, o, rays, tr)


def test_trajectory_records_match_oracle(rt, ctx, orc, aniso_wl, aniso_grid):
    fan = synth.sub_fan(aniso_wl.fan, elev_idx=[5, 30], az_idx=[10], freq_idx=[0, 2])
    stride, per_ray = 7, 800
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, traj_stride=stride, traj_per_ray=per_ray)
    rays = fan.expand()
    tr = oracle_tracer(orc, aniso_wl, fan)
    o = tr(*rays, traj_stride=stride, traj_per_ray=per_ray)
    assert np.array_equal(g["traj_count"], o["traj_count"])
    for i in range(rays[0].size):
        nrec = g["traj_count"][i]
        a, b = g["traj"][i, :nrec], o["traj"][i, :nrec]
        scale = np.maximum(np.abs(b), 1.0)
        assert np.max(np.abs(a - b) / scale) < 1e-9


def test_trajectories_identical_with_promotion(rt, ctx, aniso_wl, aniso_grid):
    """The whole 24,576-ray fan with trajectories: the default promotion
    waves (which record their rays' points themselves) give the same records
    as a launch without promotion, and the same outputs."""
    kw = dict(traj_stride=100, traj_per_ray=45)
    a = gpu_trace(rt, ctx, aniso_grid, aniso_wl, **kw)
    b = gpu_trace(rt, ctx, aniso_grid, aniso_wl, promote_waves=-1, **kw)
    assert np.array_equal(a["traj_count"], b["traj_count"])
    for k in ("group_km", "range_km", "status", "n_steps"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    for i in range(a["status"].size):
        n = a["traj_count"][i]
        assert np.array_equal(a["traj"][i, :n], b["traj"][i, :n]), i


def test_trajectory_truncation_is_reported(rt, ctx, aniso_wl, aniso_grid):
    fan = synth.sub_fan(aniso_wl.fan, elev_idx=[5], az_idx=[10], freq_idx=[0], modes=(1,))
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, traj_stride=1, traj_per_ray=10)
    assert g["truncated"] and g["traj_count"][0] == 10


def test_bitwise_deterministic(rt, ctx, aniso_wl, aniso_grid):
    fan = _subfan(aniso_wl)
    a = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    b = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    for k in ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km", "status", "n_steps"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_ray_independent_of_batch(rt, ctx, aniso_wl, aniso_grid):
    """A ray's outputs do not depend on the fan it is traced in."""
    fan = _subfan(aniso_wl)
    big = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    e, a, f, m = fan.expand()
    for i in (0, 37, 141, 209):
        one = synth.Fan(fan.tx_lat_deg, fan.tx_lon_deg, fan.tx_h_km, np.array([e[i]]),
                        np.array([a[i]]), np.array([f[i]]), (int(m[i]),))
        s = gpu_trace(rt, ctx, aniso_grid, aniso_wl, one)
        for k in ("group_km", "phase_km", "range_km", "az_dev_deg", "status", "n_steps"):
            assert np.array_equal(s[k][0], big[k][i]), (i, k)


def test_device_and_host_results_identical(rt, ctx, iso_wl, iso_grid):
    a = gpu_trace(rt, ctx, iso_grid, iso_wl)
    b = host(gpu_trace(rt, ctx, iso_grid, iso_wl, device_results=True))
    for k in ("group_km", "range_km", "status", "n_steps"):
        assert np.array_equal(a[k], b[k]), k


def test_max_path_limit(rt, ctx, orc, iso_wl, iso_grid):
    g = gpu_trace(rt, ctx, iso_grid, iso_wl, max_group_km=300.0)
    rays = iso_wl.fan.expand()
    tr = oracle_tracer(orc, iso_wl, max_group=300.0)
    o = tr(*rays)
    compare(g, o, rays, tr)
    assert np.all(g["status"] == 2) and np.all(g["group_km"] >= 300.0)


def test_rays_leaving_the_grid_box(rt, ctx, orc, aniso_wl, aniso_grid):
    """Transmitter near the south-west corner, rays heading out of the box:
    the density is continued as a constant outside (clamped axes)."""
    fan = synth.Fan(9.0, 89.0, 0.0, np.array([5.0, 15.0, 30.0]), np.array([200.0, 250.0, 300.0]),
                    np.array([6.0, 9.0]), (1, -1))
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    rays = fan.expand()
    tr = oracle_tracer(orc, aniso_wl, fan)
    compare(g, tr(*rays), rays, tr)


def test_degenerate_launch_directions(rt, ctx, orc, aniso_wl, aniso_grid):
    """Horizontal and vertical launches (elevation 0 and 90 deg, where the
    azimuth only names the plane), azimuths on both sides of north and of
    180 deg, O and X."""
    fan = synth.Fan(30.0, 110.0, 0.0, np.array([0.0, 0.5, 89.5, 90.0]),
                    np.array([0.0, 90.0, 179.99, 180.0, -90.0, 359.99]), np.array([6.0, 12.0]), (1, -1))
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    rays = fan.expand()
    tr = oracle_tracer(orc, aniso_wl, fan)
    compare(g, tr(*rays), rays, tr)


@pytest.mark.parametrize("tx_h_km", [12.5, 59.9])
def test_elevated_transmitter(rt, ctx, orc, aniso_wl, aniso_grid, tx_h_km):
    """A transmitter above the ground (an aircraft; one 100 m below the grid
    bottom, so that the launch's vacuum segment is nearly empty)."""
    fan = synth.Fan(30.0, 110.0, tx_h_km, np.array([0.0, 2.0, 10.0, 45.0]), np.array([0.0, 45.0, 135.0]),
                    np.array([6.0, 12.0]), (1, -1))
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    rays = fan.expand()
    tr = oracle_tracer(orc, aniso_wl, fan)
    compare(g, tr(*rays), rays, tr)


@pytest.mark.parametrize("interp", ["gd", "cr"])
@pytest.mark.parametrize("B0", [0.0, synth.B0_DIPOLE_T])
def test_smallest_grid(rt, ctx, orc, aniso_wl, B0, interp):
    """A grid of 4 x 5 x 6 nodes, the fewest an axis may have plus one and
    two: every axis has one or two cells, so the weights are evaluated on the
    edge cells' extended range s in [-1, 2] almost everywhere (GD and the
    Catmull-Rom comparator)."""
    geom = synth.GridGeom(4, 5, 6, 28.5, 1.0, 108.0, 1.0, 60.0, 90.0)
    small = synth.ionosphere_grid(geom, 3, B0_T=B0)
    wl = dataclasses.replace(aniso_wl, grid=small)
    fan = synth.Fan(30.0, 110.0, 0.0, np.array([5.0, 20.0, 40.0, 70.0]), np.array([0.0, 90.0, 200.0]),
                    np.array([4.0, 8.0]), (1, -1))
    grid = rt.Grid(ctx, small, interp=interp)
    try:
        g = gpu_trace(rt, ctx, grid, wl, fan)
    finally:
        grid.close()
    rays = fan.expand()
    med = orc.OracleMedium.from_grid(small, interp=interp)

    def tr(e, a, f, m):
        return orc.trace(med, e, a, f, m, B0=B0, R=geom.earth_radius_km, tx=(fan.tx_lat_deg, fan.tx_lon_deg, 0.0),
                         step=wl.step_km, max_group=wl.max_group_km, exit_h=wl.exit_km)
    compare(g, tr(*rays), rays, tr)


def test_paths_over_the_pole(rt, ctx, orc, aniso_wl, aniso_grid):
    """A transmitter 3 deg from the north pole with rays heading north: the
    colatitude passes through zero (sin theta changes sign) on the way, far
    outside the grid box, where the density is continued as a constant."""
    fan = synth.Fan(87.0, 110.0, 0.0, np.array([3.0, 8.0, 15.0, 25.0]), np.array([0.0, 1.0, 30.0]),
                    np.array([5.0, 9.0]), (1, -1))
    g = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan)
    rays = fan.expand()
    tr = oracle_tracer(orc, aniso_wl, fan)
    o = tr(*rays)
    compare(g, o, rays, tr)
    # some of these rays do cross the pole: their landing longitude differs
    # from the transmitter's by more than 90 deg
    assert np.any(np.abs(((o["land_lon_deg"] - 110.0) + 180.0) % 360.0 - 180.0) > 90.0)


def test_empty_fan_is_a_noop(rt, ctx, iso_wl, iso_grid):
    fan = synth.Fan(30.0, 110.0, 0.0, np.array([]), np.array([0.0]), np.array([10.0]), (1,))
    g = gpu_trace(rt, ctx, iso_grid, iso_wl, fan)
    assert g["status"].size == 0 and g["total_steps"] == 0


def test_invalid_arguments(rt, ctx, iso_wl, iso_grid, aniso_wl, aniso_grid):
    with pytest.raises(rt.RTError) as e:
        gpu_trace(rt, ctx, iso_grid, iso_wl, step_km=0.0)
    assert e.value.code == rt.RT_E_INVALID
    bad = synth.Fan(30.0, 110.0, 0.0, np.array([-1.0]), np.array([0.0]), np.array([10.0]), (1,))
    with pytest.raises(rt.RTError) as e:
        gpu_trace(rt, ctx, iso_grid, iso_wl, bad)
    assert e.value.code == rt.RT_E_INVALID
    low = synth.Fan(30.0, 110.0, 0.0, np.array([10.0]), np.array([0.0]), np.array([1.5]), (1,))
    with pytest.raises(rt.RTError) as e:
        gpu_trace(rt, ctx, aniso_grid, aniso_wl, low)
    assert e.value.code == rt.RT_E_UNSUPPORTED
    high_tx = synth.Fan(30.0, 110.0, 70.0, np.array([10.0]), np.array([0.0]), np.array([10.0]), (1,))
    with pytest.raises(rt.RTError) as e:
        gpu_trace(rt, ctx, iso_grid, iso_wl, high_tx)
    assert e.value.code == rt.RT_E_UNSUPPORTED
    for kw in (dict(promote_waves=65), dict(promote_waves=-2), dict(promote_age=-2),
               dict(ray_order=4), dict(waves_per_simd=3), dict(tail_threshold=-3),
               dict(cu_layout=3), dict(cu_layout=-1)):
        with pytest.raises(rt.RTError) as e:
            gpu_trace(rt, ctx, iso_grid, iso_wl, **kw)
        assert e.value.code == rt.RT_E_INVALID, kw
    # the context stays usable after errors
    ok = gpu_trace(rt, ctx, iso_grid, iso_wl)
    assert ok["status"].size == 90


def test_promotion_timeout_is_reported(rt, ctx, aniso_wl, aniso_grid, monkeypatch):
    """An idle promotion wave's wait is bounded in wall-clock time.  With the
    bound forced down to a microsecond from the host, the promotion waves give
    up at once: the launch reports a device error instead of hanging, and the
    context stays usable."""
    monkeypatch.setenv("RTGD_PROMOTE_IDLE_MS", "0.001")
    with pytest.raises(rt.RTError) as e:
        gpu_trace(rt, ctx, aniso_grid, aniso_wl, promote_waves=16, promote_age=-1)
    assert e.value.code == rt.RT_E_DEVICE
    monkeypatch.delenv("RTGD_PROMOTE_IDLE_MS")
    a = gpu_trace(rt, ctx, aniso_grid, aniso_wl, promote_waves=16, promote_age=-1)
    b = gpu_trace(rt, ctx, aniso_grid, aniso_wl, promote_waves=-1)
    for k in ("group_km", "range_km", "status", "n_steps"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_grid_create_rejects_bad_values(rt, ctx):
    geom = synth.GridGeom(6, 6, 8, 28.0, 0.5, 108.0, 0.5, 100.0, 3.0)
    vals = np.ones((6, 6, 8)) * 1e11
    vals[2, 3, 4] = np.nan
    with pytest.raises(rt.RTError) as e:
        rt.Grid(ctx, synth.Grid(geom, vals))
    assert e.value.code == rt.RT_E_INVALID
    vals[2, 3, 4] = -1.0
    with pytest.raises(rt.RTError):
        rt.Grid(ctx, synth.Grid(geom, vals))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tail_kernel_is_bit_identical(rt, ctx, aniso_wl, aniso_grid, precision):
    """The sixteen-lanes-per-ray path splits only the stencil contraction
    and combines it in the one-lane order: outputs are identical whether a
    ray finishes in the one-lane kernel (hand-off off), runs entirely in the
    tail kernel (threshold above the ray count, so every ray is handed off
    at the first check), is handed off midway, or finishes on a 16-lane row
    of its own wave (in-wave switch), in either visiting order."""
    fan = _subfan(aniso_wl)
    one = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, precision=precision, tail_threshold=-1)
    tail = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, precision=precision,
                     tail_threshold=1 << 20)
    mid = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, precision=precision, tail_threshold=100)
    inwave = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, precision=precision, tail_threshold=-2)
    strided = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, precision=precision, tail_threshold=-2,
                        ray_order=2)
    for k in ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km", "status", "n_steps"):
        for other in (tail, mid, inwave, strided):
            assert np.array_equal(one[k], other[k], equal_nan=True), k
    assert one["total_steps"] == tail["total_steps"] == mid["total_steps"] == inwave["total_steps"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_promotion_is_bit_identical(rt, ctx, precision):
    """Promotion waves take trapped, grazing and old rays over while the
    one-lane waves run; outputs are identical with promotion off, at the
    default (32 waves for this fan, trapped and grazing rays, one four-wave
    work-group per CU), with one-wave work-groups, with the most waves, with
    a small age (many rays promoted, the queue kept full), and with the tail
    kernel off (promoted rays run to the end)."""
    wl = synth.ionogram_workload(0)
    grid = rt.Grid(ctx, wl.grid)
    try:
        runs = [host(gpu_trace(rt, ctx, grid, wl, precision=precision, device_results=True,
                               **kw))
                for kw in (dict(promote_waves=-1), dict(), dict(cu_layout=1), dict(ray_order=3),
                           dict(promote_waves=64),
                           dict(promote_waves=8, promote_age=200),
                           dict(promote_waves=4, promote_age=-1, tail_threshold=-1))]
    finally:
        grid.close()
    for r in runs:      # every ray finished (a ray no kernel finished keeps status -1)
        assert (r["status"] >= 0).all()
    for k in ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km", "land_lat_deg",
              "land_lon_deg", "status", "n_steps"):
        for other in runs[1:]:
            assert np.array_equal(runs[0][k], other[k], equal_nan=True), k
    assert len({r["total_steps"] for r in runs}) == 1


def test_single_ray_is_handed_off(rt, ctx, aniso_wl, aniso_grid):
    """A lone ray with the hand-off on runs in the tail kernel (at most
    `threshold` live rays) and still equals the one-lane result."""
    fan = synth.sub_fan(aniso_wl.fan, elev_idx=[30], az_idx=[10], freq_idx=[1])
    a = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, tail_threshold=-1)
    b = gpu_trace(rt, ctx, aniso_grid, aniso_wl, fan, tail_threshold=1)
    for k in ("group_km", "range_km", "az_dev_deg", "status", "n_steps"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_mode_sorted_queue_is_result_neutral(rt, ctx, iso_wl, iso_grid, aniso_wl, aniso_grid):
    """The queue sorted by wave mode (ray_order 3: a counting sort, O and
    isotropic rays first, then X) gives the same outputs as index order for
    fans with both modes, one mode, and no field; and in a server launch that
    batches requests of different mode sets, each result equals its fan
    traced alone."""
    base = aniso_wl.fan
    fans = [(aniso_grid, aniso_wl, synth.sub_fan(base, elev_idx=list(range(0, 64, 5)),
                                                 az_idx=[3, 40], freq_idx=[0, 1])),
            (aniso_grid, aniso_wl, synth.sub_fan(base, elev_idx=list(range(0, 64, 7)), az_idx=[9],
                                                 modes=(-1,))),
            (aniso_grid, aniso_wl, synth.sub_fan(base, elev_idx=list(range(2, 64, 7)), az_idx=[20],
                                                 modes=(1,))),
            (iso_grid, iso_wl, iso_wl.fan)]
    for grid, wl, fan in fans:
        a = gpu_trace(rt, ctx, grid, wl, fan, ray_order=1)
        b = gpu_trace(rt, ctx, grid, wl, fan, ray_order=3)
        for k in ("group_km", "phase_km", "range_km", "az_dev_deg", "status", "n_steps"):
            assert np.array_equal(a[k], b[k], equal_nan=True), k
    srv = rt.Server(ctx, n_slots=1, mem_budget_bytes=64 << 20)
    try:
        kw = dict(step_km=1.0, max_group_km=4000.0, exit_h_km=600.0, ray_order=3)
        ids = {srv.submit(aniso_grid, f, **kw): f for _, _, f in fans[:3]}
        done = {}
        while len(done) < len(ids):
            for d in srv.poll():
                done[d["id"]] = d
        for rid, f in ids.items():
            got = srv.fetch(rid, done[rid]["n_rays"])
            alone = rt.trace(ctx, aniso_grid, f, **kw)
            for k in ("group_km", "range_km", "status", "n_steps"):
                assert np.array_equal(got[k], alone[k], equal_nan=True), k
    finally:
        srv.close()
