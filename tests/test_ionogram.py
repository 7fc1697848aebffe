"""Oblique-ionogram synthesis (Sec. IV-B-4, joint frequency-elevation scan).

The oracle's extraction follows the definition on plain Python loops.  Its
own pins (CPU): on a spherically symmetric Chapman layer the received rays
must reproduce, to interpolation accuracy, rays launched directly at the
interpolated elevations.  GPU: the extraction kernel on the GPU's ray
outputs against the oracle's extraction on the same outputs (identical
decisions, values to rounding), and end to end against oracle rays.
"""
import numpy as np
import pytest

from paper_2506_18579_amd import synth


def _chapman_sweep(orc, freqs, elevs, D):
    med = orc.OracleMedium.chapman(8.0, 300.0, 50.0, floor_km=60.0)
    fan = synth.Fan(30.0, 110.0, 0.0, np.asarray(elevs), np.array([0.0]), np.asarray(freqs), (1,))
    e, a, f, m = fan.expand()
    r = orc.trace(med, e, a, f, m, exit_h=500.0)
    return med, fan, r


def test_oracle_ionogram_hits_the_receiver(orc):
    D = 1200.0
    elevs = np.linspace(2.0, 60.0, 59)
    med, fan, r = _chapman_sweep(orc, [6.0, 9.0, 11.0], elevs, D)
    pts, cnt = orc.ionogram(r, elevs, 3, 1, D)
    assert cnt.sum() > 0
    for t in range(3):
        for k in range(min(cnt[t], 8)):
            el, gp = pts[t, k, 0], pts[t, k, 1]
            chk = orc.trace(med, [el], 0.0, fan.freq_mhz[t], exit_h=500.0)
            # linear interpolation over a 1 deg elevation step: the ray
            # launched at the interpolated elevation lands within a few km
            assert chk["status"][0] == orc.GROUND
            assert abs(chk["range_km"][0] - D) < 15.0
            assert abs(chk["group_km"][0] - gp) < 15.0


def test_oracle_ionogram_low_and_high_rays(orc):
    """Chapman layer, foF2 = 8 MHz, 1200 km link: below foF2 the ground
    range falls monotonically with elevation (one ray); just below the MUF
    the skip distance is shorter than the link and a low and a high ray
    arrive (the high ray steeper, with the longer group path); above the
    MUF nothing arrives."""
    elevs = np.linspace(1.0, 80.0, 159)
    _, _, r = _chapman_sweep(orc, [6.0, 13.0, 30.0], elevs, 1200.0)
    pts, cnt = orc.ionogram(r, elevs, 3, 1, 1200.0)
    assert list(cnt) == [1, 2, 0]
    assert pts[1, 0, 0] < pts[1, 1, 0] and pts[1, 0, 1] < pts[1, 1, 1]


@pytest.mark.gpu
def test_gpu_ionogram_matches_oracle_extraction(orc):
    from paper_2506_18579_amd import rtgd
    from parity import host
    wl = synth.ionogram_workload(0)
    ctx = rtgd.Context(0)
    grid = rtgd.Grid(ctx, wl.grid)
    res = rtgd.trace(ctx, grid, wl.fan, step_km=wl.step_km, max_group_km=wl.max_group_km,
                     exit_h_km=wl.exit_km, device_results=True)
    pts, cnt = rtgd.ionogram(ctx, wl.fan, res, 1200.0, 8)
    pts, cnt = pts.cpu().numpy(), cnt.cpu().numpy()
    h = host(res)
    # same extraction on host-resident inputs through the C ABI
    pts_h, cnt_h = rtgd.ionogram(ctx, wl.fan, h, 1200.0, 8)
    grid.close()
    ctx.close()
    assert np.array_equal(cnt, cnt_h) and np.array_equal(pts, pts_h)
    opts, ocnt = orc.ionogram(h, wl.fan.elev_deg, len(wl.fan.freq_mhz), len(wl.fan.modes), 1200.0, 8)
    assert np.array_equal(cnt, ocnt)
    assert np.allclose(pts, opts, rtol=1e-13, atol=1e-10)
    n = int(np.minimum(cnt, 8).sum())
    print("ionogram traces", cnt.size, "received rays", n, "max per trace", cnt.max())
    assert n > 200


@pytest.mark.gpu
def test_gpu_ionogram_end_to_end_against_oracle_rays(orc):
    """Traces of a few frequencies: GPU rays + GPU extraction against
    oracle rays + oracle extraction."""
    from paper_2506_18579_amd import rtgd
    from parity import oracle_tracer
    wl = synth.ionogram_workload(0)
    fan = synth.sub_fan(wl.fan, freq_idx=[20, 60, 100, 140])
    ctx = rtgd.Context(0)
    grid = rtgd.Grid(ctx, wl.grid)
    g = rtgd.trace(ctx, grid, fan, step_km=1.0, max_group_km=8000.0, exit_h_km=1000.0)
    gp, gc = rtgd.ionogram(ctx, fan, g, 1200.0, 8)
    grid.close()
    ctx.close()
    o = oracle_tracer(orc, wl, fan)(*fan.expand())
    op, oc = orc.ionogram(o, fan.elev_deg, 4, 2, 1200.0, 8)
    assert np.array_equal(gc, oc)
    k = np.minimum(gc, 8)
    for t in range(gc.size):
        np.testing.assert_allclose(gp[t, :k[t]], op[t, :k[t]], rtol=1e-8, atol=1e-8)
