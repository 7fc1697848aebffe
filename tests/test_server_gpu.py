"""Request server (continuous batching) on the GPU.

A Poisson stream of uneven ray fans against resident grid snapshots is
pushed through rt_server_* with several slots, so that requests overlap on
the device and later ones are admitted as slots and arena memory free up.
Every request's per-ray outputs must equal, bit for bit, those of the same
fan traced alone with rt_trace (the per-ray arithmetic does not depend on
what else runs), and served results are checked against the FP64 oracle
directly: a seeded sample of every request (every ray of the ionogram
requests, and their extracted traces), in both precisions.  Admission by
memory, cancellation and the error paths are checked too.
"""
import time

import numpy as np
import pytest

from paper_2506_18579_amd import synth

from parity import classify_mixed, compare, oracle_tracer

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


@pytest.fixture(scope="module")
def grids(rt, ctx):
    gs = [rt.Grid(ctx, synth.ionosphere_grid(synth.GEOM_ANISO, seed)) for seed in (0, 1)]
    yield gs
    for g in gs:
        g.close()


def opts(precision):
    return dict(step_km=1.0, max_group_km=4000.0, exit_h_km=600.0, precision=precision)


def drain(srv, want, timeout_s=60.0):
    done = {}
    t0 = time.time()
    while len(done) < want:
        for d in srv.poll():
            done[d["id"]] = d
        assert time.time() - t0 < timeout_s, f"server stalled: {srv.stats()}"
        time.sleep(0.0005)
    return done


def same(a, b):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k]), equal_nan=True), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_each_result_same_alone_and_in_mix(rt, ctx, grids, precision):
    reqs = synth.serving_requests(24, seed=7, n_snapshots=len(grids), max_rays=3000, qps=1e9)
    srv = rt.Server(ctx, n_slots=4, mem_budget_bytes=64 << 20)
    try:
        ids = {}
        peak_running = 0
        for r in reqs:
            ids[srv.submit(grids[r["snapshot"]], r["fan"], **opts(precision))] = r
            peak_running = max(peak_running, srv.stats()["running"])
        done = drain(srv, len(reqs))
        assert peak_running >= 2          # work overlapped on the device
        mixed = {rid: srv.fetch(rid, done[rid]["n_rays"]) for rid in ids}
        st = srv.stats()
        assert st == dict(queued=0, running=0, arena_used=0)
    finally:
        srv.close()
    for rid, r in ids.items():
        alone = rt.trace(ctx, grids[r["snapshot"]], r["fan"], **opts(precision))
        assert done[rid]["n_rays"] == alone["status"].size
        assert done[rid]["total_steps"] == alone["total_steps"]
        same(mixed[rid], alone)


@pytest.mark.parametrize("cu_layout", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_merged_launch_matches_alone(rt, ctx, grids, precision, cu_layout):
    """Three 6,000-ray requests queued behind one slot are launched together
    (18,000 rays: enough for the default promotion waves), in the default
    grouped layout (four-wave work-groups, one per CU) and in one-wave
    work-groups (where the FP32 kernel holds two one-lane waves per SIMD).
    Every result equals, bit for bit, its fan traced alone (6,000 rays: no
    promotion)."""
    fans = [synth.Fan(30.0, 110.0, 0.0, np.linspace(5.0, 65.0, 60), np.linspace(-60.0, 60.0, 100),
                      np.array([f]), (m,)) for f, m in ((7.0, 1), (9.5, -1), (12.0, 1))]
    srv = rt.Server(ctx, n_slots=1, mem_budget_bytes=64 << 20)
    try:
        ids = {srv.submit(grids[k % len(grids)], fan, **opts(precision), cu_layout=cu_layout): k
               for k, fan in enumerate(fans)}
        done = drain(srv, len(fans))
        got = {rid: srv.fetch(rid, done[rid]["n_rays"]) for rid in ids}
    finally:
        srv.close()
    for rid, k in ids.items():
        alone = rt.trace(ctx, grids[k % len(grids)], fans[k], **opts(precision))
        assert done[rid]["total_steps"] == alone["total_steps"]
        same(got[rid], alone)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_staggered_large_batches_match_alone(rt, ctx, grids, precision):
    """Two requests of 65,536 rays (the smallest batch that starts
    staggered) that cannot share a launch (different maximum group paths),
    on a two-slot server whose slot buffers first held a small request.  The
    first large launch grows its slot's buffers while the second waits for
    that launch's one-lane phase to end; then both finish.  Every result
    equals, bit for bit, its fan traced alone, fetched to host memory for
    one request and to device memory for the other."""
    big = synth.Fan(30.0, 110.0, 0.0, np.linspace(3.0, 65.0, 64), np.linspace(-60.0, 60.0, 128),
                    np.array([5.0, 7.5, 10.0, 12.5]), (1, -1))
    small = synth.Fan(30.0, 110.0, 0.0, np.linspace(5.0, 60.0, 10), np.linspace(-30.0, 30.0, 10),
                      np.array([8.0]), (1,))
    assert rt.fan_count(big) == 1 << 16
    o_a = opts(precision)
    o_b = dict(opts(precision), max_group_km=3000.0)
    srv = rt.Server(ctx, n_slots=2, mem_budget_bytes=64 << 20)
    try:
        s_id = srv.submit(grids[0], small, **o_a)
        d_small = drain(srv, 1)
        srv.fetch(s_id, d_small[s_id]["n_rays"])
        a_id = srv.submit(grids[0], big, **o_a)
        b_id = srv.submit(grids[1], big, **o_b)
        # the second large batch waits (its one-lane phase alone takes
        # milliseconds; these calls return within microseconds)
        st = srv.stats()
        assert st["running"] == 1 and st["queued"] == 1, st
        done = drain(srv, 2)
        got_a = srv.fetch(a_id, done[a_id]["n_rays"])
        got_b = srv.fetch(b_id, done[b_id]["n_rays"], device=True)
        got_b = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in got_b.items()}
        assert srv.stats() == dict(queued=0, running=0, arena_used=0)
    finally:
        srv.close()
    for rid, g, o, got in ((a_id, grids[0], o_a, got_a), (b_id, grids[1], o_b, got_b)):
        alone = rt.trace(ctx, g, big, **o)
        assert done[rid]["total_steps"] == alone["total_steps"]
        same(got, alone)


def test_admission_by_memory(rt, ctx, grids):
    """An arena that holds one request at a time: all requests still finish,
    in submission order, with the same results."""
    wl = synth.aniso_fan_workload(0)
    fans = [synth.sub_fan(wl.fan, elev_idx=list(range(k, 64, 8)), az_idx=list(range(0, 64, 4)))
            for k in range(4)]
    n = [rt.fan_count(f) for f in fans]
    per_ray = 7 * 8 + 2 * 4
    srv = rt.Server(ctx, n_slots=4, mem_budget_bytes=max(n) * per_ray + 4096)
    try:
        ids = [srv.submit(grids[0], f, **opts("fp64")) for f in fans]
        s = srv.stats()
        assert s["running"] == 1 and s["queued"] == 3
        order = []
        out = {}
        t0 = time.time()
        while len(out) < len(ids):
            for d in srv.poll():
                order.append(d["id"])
                out[d["id"]] = srv.fetch(d["id"], d["n_rays"])   # frees the arena block
            assert time.time() - t0 < 60
        assert order == ids
    finally:
        srv.close()
    for rid, f in zip(ids, fans):
        same(out[rid], rt.trace(ctx, grids[0], f, **opts("fp64")))


def test_cancel_and_errors(rt, ctx, grids):
    wl = synth.aniso_fan_workload(0)
    fan = synth.sub_fan(wl.fan, elev_idx=list(range(0, 64, 4)), az_idx=list(range(0, 64, 4)))
    n = rt.fan_count(fan)
    srv = rt.Server(ctx, n_slots=1, mem_budget_bytes=1 << 20)
    try:
        a = srv.submit(grids[0], fan, **opts("fp64"))
        b = srv.submit(grids[0], fan, **opts("fp64"))
        c = srv.submit(grids[1], fan, **opts("mixed"))
        srv.cancel(b)                                    # queued: dropped
        srv.cancel(a)                                    # running: discarded on completion
        done = drain(srv, 1)
        assert list(done) == [c]
        s = srv.stats()
        assert s["queued"] == 0 and s["running"] == 0
        out = srv.fetch(c, n)
        same(out, rt.trace(ctx, grids[1], fan, **opts("mixed")))
        assert srv.stats()["arena_used"] == 0
        with pytest.raises(rt.RTError):
            srv.fetch(c, n)                              # already fetched
        with pytest.raises(rt.RTError):
            srv.cancel(12345)
        big = synth.sub_fan(wl.fan, elev_idx=list(range(64)), az_idx=list(range(64)))
        with pytest.raises(rt.RTError) as e:
            srv.submit(grids[0], big, **opts("fp64"))    # larger than the arena
        assert e.value.code == rt.RT_E_NOMEM
        empty = synth.Fan(30.0, 110.0, 0.0, np.zeros(0), np.zeros(1), np.array([10.0]), (1,))
        z = srv.submit(grids[0], empty, **opts("fp64"))
        assert [d["id"] for d in srv.poll()] == [z]
        assert srv.fetch(z, 0)["status"].size == 0
    finally:
        srv.close()


def test_ionogram_requests_in_the_mix(rt, ctx, grids):
    """Ionogram-synthesis requests among fan requests: each sweep and its
    extracted traces equal those computed alone."""
    from paper_2506_18579_amd import serve
    reqs = synth.serving_requests(16, seed=11, n_snapshots=len(grids), max_rays=2000, qps=1e9,
                                  ionogram_fraction=0.4)
    assert sum("ionogram" in r for r in reqs) >= 3
    srv = rt.Server(ctx, n_slots=4, mem_budget_bytes=64 << 20)
    try:
        out = serve.replay(srv, grids, reqs, opts("mixed"), keep_results=True)
    finally:
        srv.close()
    for k, r in enumerate(reqs):
        o = dict(opts("mixed"), **r.get("opts", {}))
        alone = rt.trace(ctx, grids[r["snapshot"]], r["fan"], **o)
        same(out["results"][k], alone)
        if "ionogram" in r:
            pts, cnt = rt.ionogram(ctx, r["fan"], alone, 1200.0, 8)
            mp, mc = out["results"][k]["ionogram"]
            assert np.array_equal(cnt, mc) and np.array_equal(pts, mp, equal_nan=True)


def _served_mix():
    """A Poisson mix of fan and ionogram requests, plus fans whose azimuth
    span crosses +-180 deg (pointing away from the grid box) and a fan from
    the box's south-west corner heading out of it."""
    reqs = synth.serving_requests(18, seed=23, n_snapshots=2, max_rays=3000, qps=1e9,
                                  ionogram_fraction=0.25)
    extra = [(30.0, 110.0, np.linspace(4.0, 40.0, 12), np.linspace(170.0, 190.0, 5), 8.5, (1, -1)),
             (30.0, 110.0, np.linspace(10.0, 60.0, 9), np.linspace(-185.0, -175.0, 3), 13.0, (-1,)),
             (9.0, 89.0, np.linspace(5.0, 30.0, 6), np.linspace(200.0, 300.0, 6), 6.0, (1, -1))]
    for k, (la, lo, el, az, f, modes) in enumerate(extra):
        reqs.append(dict(id=100 + k, t_arrive=0.0, snapshot=k % 2,
                         fan=synth.Fan(la, lo, 0.0, el, az, np.array([f]), modes)))
    return reqs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_requests_match_oracle(rt, ctx, orc, grids, precision):
    """Requests served concurrently (4 slots, batched launches) against the
    FP64 oracle: FP64 at the 1e-9 gate, mixed at 0.1 km / 0.001 deg (rays
    ill-conditioned at FP32 level counted apart).  Fan requests: a seeded
    sample of 12 rays plus the first and the last; ionogram requests: every
    ray, and (FP64) the extracted traces against the oracle's extraction."""
    from paper_2506_18579_amd import serve
    reqs = _served_mix()
    assert sum("ionogram" in r for r in reqs) >= 3
    assert any(np.any(np.abs(r["fan"].az_deg) > 150.0) for r in reqs)
    srv = rt.Server(ctx, n_slots=4, mem_budget_bytes=64 << 20)
    try:
        out = serve.replay(srv, grids, reqs, opts(precision), keep_results=True)
    finally:
        srv.close()
    snaps = [synth.ionosphere_grid(synth.GEOM_ANISO, seed) for seed in (0, 1)]
    rng = np.random.default_rng(5)
    n_ill = n_checked = 0
    for k, r in enumerate(reqs):
        o_kw = dict(opts(precision), **r.get("opts", {}))
        wl = synth.Workload("served", snaps[r["snapshot"]], r["fan"], o_kw["step_km"],
                            o_kw["max_group_km"], o_kw["exit_h_km"])
        got = out["results"][k]
        n = got["status"].size
        assert n == r["fan"].n_rays
        if "ionogram" in r or n <= 14:
            idx = np.arange(n)
        else:
            idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 12, replace=False)]))
        e, a, f, m = r["fan"].expand()
        rays = (e[idx], a[idx], f[idx], m[idx])
        tr = oracle_tracer(orc, wl)
        o = tr(*rays)
        if precision == "fp64":
            rep = compare(got, o, rays, tr, gpu_idx=idx)
            n_ill += len(rep["ill_conditioned"])
            if "ionogram" in r:
                io = r["ionogram"]
                pts, cnt = orc.ionogram(o, r["fan"].elev_deg, len(r["fan"].freq_mhz), 2,
                                        io["range_km"], io["max_points"])
                gp, gc = got["ionogram"]
                if not rep["ill_conditioned"]:
                    assert np.array_equal(gc, cnt)
                    assert np.allclose(gp, pts, rtol=1e-8, atol=1e-8)
        else:
            rep = classify_mixed(got, o, rays, tr, gpu_idx=idx)
            assert rep["n_fail"] == 0, (k, rep["failures"][:3])
            n_ill += rep["n_ill"]
        n_checked += idx.size
    print(f"served {len(reqs)} requests ({precision}): {n_checked} rays checked against the oracle, "
          f"{n_ill} ill-conditioned")
    assert n_ill <= 0.05 * n_checked
