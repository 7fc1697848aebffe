"""The seeded synthetic inputs (CPU): deterministic, of the stated shapes,
sizes and value ranges, and the request stream's mix as documented."""
import math

import numpy as np
import pytest

from paper_2506_18579_amd import synth


def test_ionosphere_grid_is_seeded_and_in_range():
    g = synth.GridGeom(21, 23, 50, 20.0, 1.0, 100.0, 1.0, 60.0, 11.0)
    a = synth.ionosphere_grid(g, 3)
    b = synth.ionosphere_grid(g, 3)
    c = synth.ionosphere_grid(g, 4)
    assert a.values.shape == (21, 23, 50)
    assert np.array_equal(a.values, b.values)
    assert not np.array_equal(a.values, c.values)
    assert np.all(np.isfinite(a.values)) and np.all(a.values >= 0.0)
    # peak N_e of a foF2 in [5, 12] MHz layer with +-10 % TIDs and an E layer
    nm_hi = (12.0e6) ** 2 / 80.61638587963628 * 1.1 * 1.05
    assert 1e10 < a.values.max() < nm_hi


def test_chapman_grid_peak_and_uniformity():
    g = synth.GridGeom(5, 6, 201, 15.0, 0.5, 95.0, 0.5, 60.0, 2.2)
    grid = synth.chapman_grid(g, 8.0, 300.0, 50.0)
    v = grid.values
    assert np.allclose(v, v[:1, :1, :])                     # horizontally uniform
    k = int(np.argmax(v[0, 0]))
    assert abs(60.0 + 2.2 * k - 300.0) <= 1.1               # peak at hmF2
    assert v[0, 0, k] == pytest.approx((8.0e6) ** 2 / 80.61638587963628, rel=1e-3)


def test_workload_shapes():
    iso = synth.iso_chapman_workload()
    assert iso.fan.n_rays == 90 and iso.grid.values.shape == (61, 61, 201)
    fan = synth.aniso_fan_workload(0).fan
    assert fan.n_rays == 64 * 64 * 3 * 2
    io = synth.ionogram_workload(0)
    assert io.fan.n_rays == 281 * 2 * 200
    (la, lo), (lb, _) = synth.link_endpoints()
    assert synth.R_EARTH_KM * math.radians(lb - la) == pytest.approx(1200.0)
    assert io.fan.tx_lat_deg == pytest.approx(la)


def test_serving_stream_sizes_and_determinism():
    a = synth.serving_requests(300, seed=5, qps=100.0)
    b = synth.serving_requests(300, seed=5, qps=100.0)
    assert [r["t_arrive"] for r in a] == [r["t_arrive"] for r in b]
    n = np.array([r["fan"].n_rays for r in a])
    assert n.min() >= 1 and n.max() <= 20000
    # log-uniform sizes: the median of N is near exp(ln(20000)/2) ~ 141
    assert 40 < np.median(n) < 500
    t = np.array([r["t_arrive"] for r in a])
    assert np.all(np.diff(t) > 0) and 2.0 < t[-1] < 4.5     # Poisson at 100 req/s
    modes = [r["fan"].modes for r in a]
    for m in ((1,), (-1,), (1, -1)):
        assert 0.2 < modes.count(m) / len(modes) < 0.47


def test_serving_stream_ionogram_fraction():
    plain = synth.serving_requests(200, seed=9, qps=50.0)
    assert not any("ionogram" in r for r in plain)
    mixed = synth.serving_requests(200, seed=9, qps=50.0, ionogram_fraction=0.25)
    io = [r for r in mixed if "ionogram" in r]
    assert 0.15 < len(io) / len(mixed) < 0.35
    for r in io:
        f = r["fan"]
        assert len(f.elev_deg) == 50 and len(f.az_deg) == 1 and tuple(f.modes) == (1, -1)
        assert 5 <= len(f.freq_mhz) <= 40 and 2.0 <= f.freq_mhz[0] and f.freq_mhz[-1] <= 30.0
        assert r["opts"] == dict(max_group_km=8000.0, exit_h_km=1000.0)
        assert r["ionogram"]["range_km"] == 1200.0
