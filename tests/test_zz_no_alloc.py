"""rt_trace_noalloc (every launch buffer in the library's per-device scratch
region, no allocation) against rt_trace, through the C ABI: the same kernels
on the same inputs, so results must be bit-identical.  Three calls in a row
with shrinking inputs (the 112,400-ray sweep with promotion waves, the
24,576-ray anisotropic fan, a 160-ray sub-fan), so that each call also shows
that nothing of the previous call's scratch contents leaks into the next;
then the limits, which are refused before anything is launched."""
import numpy as np
import pytest

from paper_2506_18579_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km", "land_lat_deg",
        "land_lon_deg", "status", "n_steps")


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


def _limits(wl):
    return dict(step_km=wl.step_km, max_group_km=wl.max_group_km, exit_h_km=wl.exit_km)


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy(), equal_nan=True), k
    assert a["total_steps"] == b["total_steps"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_equals_trace_on_shrinking_inputs(rt, ctx, precision):
    sweep = synth.ionogram_workload(0)
    fan = synth.aniso_fan_workload(0)
    small = synth.sub_fan(fan.fan, elev_idx=list(range(0, 64, 9)), az_idx=list(range(0, 64, 13)),
                          freq_idx=[0, 2])
    cases = [(sweep, sweep.fan), (fan, fan.fan), (fan, small)]
    assert [f.n_rays for _, f in cases] == [112400, 24576, 160]
    grids = {}
    for wl, f in cases:
        key = id(wl.grid)
        if key not in grids:
            grids[key] = rt.Grid(ctx, wl.grid)
        g = grids[key]
        print(f"noalloc {precision}: {f.n_rays} rays", flush=True)
        ref = rt.trace(ctx, g, f, precision=precision, device_results=True, **_limits(wl))
        got = rt.trace_noalloc(ctx, g, f, precision=precision, **_limits(wl))
        _same(got, ref)
    for g in grids.values():
        g.close()


def test_noalloc_limits(rt, ctx):
    wl = synth.aniso_fan_workload(0)
    g = rt.Grid(ctx, wl.grid)
    try:
        f = synth.sub_fan(wl.fan, elev_idx=[3], az_idx=[4], freq_idx=[0])
        with pytest.raises(rt.RTError) as e:          # host results
            rt.trace(ctx, g, f, _entry="rt_trace_noalloc", **_limits(wl))
        assert e.value.code == rt.RT_E_INVALID
        with pytest.raises(rt.RTError) as e:          # trajectories
            rt.trace(ctx, g, f, traj_stride=1, traj_per_ray=10, device_results=True,
                     _entry="rt_trace_noalloc", **_limits(wl))
        assert e.value.code == rt.RT_E_INVALID
        big = synth.Fan(30.0, 110.0, 0.0, np.linspace(5.0, 60.0, 257), np.linspace(-30.0, 30.0, 256),
                        np.array([9.0, 11.0]), (1,))
        assert big.n_rays > rt.RT_NOALLOC_MAX_RAYS
        with pytest.raises(rt.RTError) as e:          # too many rays
            rt.trace_noalloc(ctx, g, big, **_limits(wl))
        assert e.value.code == rt.RT_E_INVALID
        wide = synth.Fan(30.0, 110.0, 0.0, np.linspace(5.0, 60.0, rt.RT_NOALLOC_MAX_AXIS - 1),
                         np.array([0.0, 1.0]), np.array([9.0]), (1,))
        with pytest.raises(rt.RTError) as e:          # too many fan axis values
            rt.trace_noalloc(ctx, g, wide, **_limits(wl))
        assert e.value.code == rt.RT_E_INVALID
    finally:
        g.close()
