"""Seeded synthetic inputs: electron-density grids and ray fans.

This module only builds inputs (grids of N_e, launch fans, request streams).
It holds none of the ray-tracing arithmetic and is the one module that both
the GPU path and the CPU oracle consume, so that both see identical bytes.

The paper drives its experiments with IRI-2020 densities and an IGRF-13
field, which are not available here.  Synthetic stand-ins of the same shape
are used instead: alpha-Chapman F2 and E layers, seeded Gaussian travelling
ionospheric disturbance (TID) blobs, and a centred axial dipole.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

R_EARTH_KM = 6371.0
# f_N^2 = K_N N_e  (Hz^2, N_e in m^-3), CODATA 2022.  Used only to turn a
# layer's critical frequency into its peak density.
K_N = 80.61638587963628
B0_DIPOLE_T = 3.12e-5


@dataclasses.dataclass
class GridGeom:
    n_lat: int
    n_lon: int
    n_h: int
    lat0_deg: float
    dlat_deg: float
    lon0_deg: float
    dlon_deg: float
    h0_km: float
    dh_km: float
    earth_radius_km: float = R_EARTH_KM

    def heights(self):
        return self.h0_km + self.dh_km * np.arange(self.n_h)

    def lats(self):
        return self.lat0_deg + self.dlat_deg * np.arange(self.n_lat)

    def lons(self):
        return self.lon0_deg + self.dlon_deg * np.arange(self.n_lon)

    @property
    def top_km(self):
        return self.h0_km + self.dh_km * (self.n_h - 1)


@dataclasses.dataclass
class Grid:
    geom: GridGeom
    values: np.ndarray          # N_e in m^-3, float64, shape (n_lat, n_lon, n_h)
    B0_T: float = 0.0           # centred axial dipole; 0 = no field
    meta: dict = dataclasses.field(default_factory=dict)


@dataclasses.dataclass
class Fan:
    """A launch fan: ray index = ((i_f * n_mode + i_m) * n_elev + i_e) * n_az + i_a."""
    tx_lat_deg: float
    tx_lon_deg: float
    tx_h_km: float
    elev_deg: np.ndarray
    az_deg: np.ndarray
    freq_mhz: np.ndarray
    modes: tuple = (1,)         # +1 = O, -1 = X

    @property
    def n_rays(self) -> int:
        return len(self.freq_mhz) * len(self.modes) * len(self.elev_deg) * len(self.az_deg)

    def expand(self):
        """Per-ray (elev, az, freq, mode) arrays in ray-index order."""
        f, m, e, a = np.meshgrid(np.asarray(self.freq_mhz, dtype=np.float64),
                                 np.asarray(self.modes, dtype=np.int32),
                                 np.asarray(self.elev_deg, dtype=np.float64),
                                 np.asarray(self.az_deg, dtype=np.float64), indexing="ij")
        return (e.ravel().copy(), a.ravel().copy(), f.ravel().copy(),
                m.ravel().astype(np.int32))


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    fan: Fan
    step_km: float = 1.0
    max_group_km: float = 4000.0
    exit_h_km: float = 0.0      # <= 0: grid top
    precision: str = "fp64"     # "fp64" or "mixed"

    @property
    def exit_km(self):
        return self.exit_h_km if self.exit_h_km > 0 else self.grid.geom.top_km


def chapman(h_km, fc_mhz, hm_km, scale_km):
    """alpha-Chapman layer N_e (m^-3) with peak plasma frequency fc."""
    nm = (fc_mhz * 1e6) ** 2 / K_N
    z = (np.asarray(h_km, dtype=np.float64) - hm_km) / scale_km
    return nm * np.exp(0.5 * (1.0 - z - np.exp(-z)))


def _central_angle(lat1, lon1, lat2, lon2):
    p1, p2 = np.radians(lat1), np.radians(lat2)
    dl = np.radians(lon2 - lon1)
    s = np.sin((p2 - p1) / 2) ** 2 + np.cos(p1) * np.cos(p2) * np.sin(dl / 2) ** 2
    return 2.0 * np.arcsin(np.sqrt(np.clip(s, 0.0, 1.0)))


def chapman_grid(geom: GridGeom, fc_mhz=8.0, hm_km=300.0, scale_km=50.0) -> Grid:
    """Horizontally uniform Chapman layer on a grid; no field."""
    prof = chapman(geom.heights(), fc_mhz, hm_km, scale_km)
    vals = np.broadcast_to(prof, (geom.n_lat, geom.n_lon, geom.n_h)).copy()
    return Grid(geom, vals, 0.0, dict(kind="chapman", fc=fc_mhz, hm=hm_km, H=scale_km))


def ionosphere_grid(geom: GridGeom, seed: int = 0, B0_T: float = B0_DIPOLE_T,
                    n_tid: int = 3) -> Grid:
    """F2 + E Chapman layers times (1 + sum of seeded Gaussian TID blobs).

    foF2 ~ U[5, 12] MHz, hmF2 ~ U[250, 350] km, H ~ U[40, 60] km (drawn once);
    E layer foE = 3 MHz, hmE = 110 km, H_E = 10 km.  Each TID has amplitude
    +-10 % (random sign), 200 km horizontal and 50 km vertical Gaussian
    widths, a centre uniform in the inner 80 % of the box and a height
    uniform in hmF2 +- 50 km.  numpy PCG64(seed), draws in this order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    fo_f2 = rng.uniform(5.0, 12.0)
    hm_f2 = rng.uniform(250.0, 350.0)
    h_f2 = rng.uniform(40.0, 60.0)
    lats, lons, hs = geom.lats(), geom.lons(), geom.heights()
    lat_span = lats[-1] - lats[0]
    lon_span = lons[-1] - lons[0]
    tids = []
    for _ in range(n_tid):
        tl = lats[0] + lat_span * rng.uniform(0.1, 0.9)
        tn = lons[0] + lon_span * rng.uniform(0.1, 0.9)
        th = rng.uniform(hm_f2 - 50.0, hm_f2 + 50.0)
        amp = 0.10 if rng.uniform() < 0.5 else -0.10
        tids.append((tl, tn, th, amp))
    prof = chapman(hs, fo_f2, hm_f2, h_f2) + chapman(hs, 3.0, 110.0, 10.0)
    LA, LO = np.meshgrid(lats, lons, indexing="ij")
    pert = np.ones((geom.n_lat, geom.n_lon, geom.n_h))
    for tl, tn, th, amp in tids:
        d = geom.earth_radius_km * _central_angle(LA, LO, tl, tn)
        horiz = np.exp(-d ** 2 / (2.0 * 200.0 ** 2))
        vert = np.exp(-(hs - th) ** 2 / (2.0 * 50.0 ** 2))
        pert += amp * horiz[:, :, None] * vert[None, None, :]
    vals = prof[None, None, :] * pert
    meta = dict(kind="ionosphere", seed=seed, foF2=fo_f2, hmF2=hm_f2, H=h_f2, tids=tids)
    return Grid(geom, np.ascontiguousarray(vals), B0_T, meta)


# ---------------------------------------------------------------------------
# The five benchmark workloads (grid + fan + integration limits)
# ---------------------------------------------------------------------------
GEOM_ISO = GridGeom(61, 61, 201, 15.0, 0.5, 95.0, 0.5, 60.0, 2.2)
GEOM_ANISO = GridGeom(181, 181, 226, 7.5, 0.25, 87.5, 0.25, 60.0, 2.4)


def iso_chapman_workload() -> Workload:
    """Isotropic FP64: 61x61x201 grid (0.5 deg, 2.2 km), Chapman foF2 = 8 MHz,
    hmF2 = 300 km, H = 50 km; 90 rays at 1..90 deg elevation, azimuth 0,
    10 MHz, from (30N, 110E); 1 km steps, 4000 km max group path."""
    grid = chapman_grid(GEOM_ISO, 8.0, 300.0, 50.0)
    fan = Fan(30.0, 110.0, 0.0, np.arange(1.0, 91.0), np.array([0.0]), np.array([10.0]), (1,))
    return Workload("iso_chapman_61x61x201_90rays", grid, fan, 1.0, 4000.0, 500.0)


def aniso_fan_workload(seed: int = 0) -> Workload:
    """Anisotropic FP64 O and X: 181x181x226 grid (0.25 deg, 2.4 km), F2 + E +
    3 TIDs, dipole B0 = 3.12e-5 T; 64 elevations (2..65) x 64 azimuths
    (-30..30) x 3 frequencies (7, 12, 18 MHz) x 2 modes = 24,576 rays."""
    grid = ionosphere_grid(GEOM_ANISO, seed)
    fan = Fan(30.0, 110.0, 0.0, np.linspace(2.0, 65.0, 64), np.linspace(-30.0, 30.0, 64),
              np.array([7.0, 12.0, 18.0]), (1, -1))
    return Workload("aniso_fan_181x181x226_24576rays", grid, fan, 1.0, 4000.0, 600.0)


def link_endpoints(range_km=1200.0, centre_lat=30.0, lon=110.0, R=R_EARTH_KM):
    half = math.degrees(range_km / R) / 2.0
    return (centre_lat - half, lon), (centre_lat + half, lon)


def ionogram_workload(seed: int = 0, precision: str = "fp64") -> Workload:
    """Oblique-ionogram sweep on the anisotropic grid: transmitter and receiver
    1200 km apart on the 110E meridian, azimuth 0; 281 frequencies
    (2.0..30.0 MHz, 0.1 MHz) x 2 modes x 200 elevations (1..80 deg) =
    112,400 rays; exit at 1000 km, 8000 km max group path."""
    grid = ionosphere_grid(GEOM_ANISO, seed)
    (tlat, tlon), _ = link_endpoints()
    freqs = np.round(2.0 + 0.1 * np.arange(281), 10)
    fan = Fan(tlat, tlon, 0.0, np.linspace(1.0, 80.0, 200), np.array([0.0]), freqs, (1, -1))
    name = "ionogram_181x181x226_112400rays_" + precision
    return Workload(name, grid, fan, 1.0, 8000.0, 1000.0, precision)


def sub_fan(fan: Fan, elev_idx=None, az_idx=None, freq_idx=None, modes=None) -> Fan:
    """A fan built from subsets of another fan's axes."""
    pick = lambda arr, idx: np.asarray(arr)[idx] if idx is not None else np.asarray(arr)
    return Fan(fan.tx_lat_deg, fan.tx_lon_deg, fan.tx_h_km, pick(fan.elev_deg, elev_idx),
               pick(fan.az_deg, az_idx), pick(fan.freq_mhz, freq_idx),
               tuple(modes) if modes is not None else fan.modes)


def serving_requests(n_requests: int, seed: int = 1234, n_snapshots: int = 4,
                     max_rays: int = 20000, qps: float = 50.0, ionogram_fraction: float = 0.0):
    """Poisson request stream of ray fans of log-uniform size 1..max_rays.

    Each request: arrival time, snapshot id, fan (elevation start U[1, 60],
    width U[1, 30]; azimuth centre U[-180, 180], width U[0, 60]; one
    frequency U[3, 30] MHz; O, X or both with probability 1/3 each), laid
    out as n_el x n_az with n_az = ceil(sqrt(N)/2).

    With ionogram_fraction > 0, that fraction of the requests (decided by a
    second PCG64 stream, seed + 1, so the fan draws are unchanged) are
    ionogram-synthesis requests instead: the 1200 km link of
    ionogram_workload, 50 elevations (1..80 deg) x O/X x a run of 5..40
    consecutive 0.1 MHz frequencies starting at U{2.0..26.0} MHz, with an
    'ionogram' entry (receiver range, points per trace) and that
    workload's exit height and maximum group path in 'opts'."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rng_kind = np.random.Generator(np.random.PCG64(seed + 1))
    (tlat, tlon), _ = link_endpoints()
    t = 0.0
    reqs = []
    for k in range(n_requests):
        if ionogram_fraction > 0.0 and rng_kind.uniform() < ionogram_fraction:
            t += rng.exponential(1.0 / qps)
            snap = int(rng_kind.integers(0, n_snapshots))
            n_f = int(rng_kind.integers(5, 41))
            f0 = 2.0 + 0.1 * int(rng_kind.integers(0, 241))
            freqs = np.round(f0 + 0.1 * np.arange(n_f), 10)
            fan = Fan(tlat, tlon, 0.0, np.linspace(1.0, 80.0, 50), np.array([0.0]), freqs, (1, -1))
            reqs.append(dict(id=k, t_arrive=t, snapshot=snap, fan=fan,
                             ionogram=dict(range_km=1200.0, max_points=8),
                             opts=dict(max_group_km=8000.0, exit_h_km=1000.0)))
            continue
        t += rng.exponential(1.0 / qps)
        n = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_rays)))))
        n = max(1, min(n, max_rays))
        f = rng.uniform(3.0, 30.0)
        e0, ew = rng.uniform(1.0, 60.0), rng.uniform(1.0, 30.0)
        ac, aw = rng.uniform(-180.0, 180.0), rng.uniform(0.0, 60.0)
        mpick = int(rng.integers(0, 3))
        snap = int(rng.integers(0, n_snapshots))
        modes = ((1,), (-1,), (1, -1))[mpick]
        per_mode = max(1, n // len(modes))
        n_az = max(1, int(math.ceil(math.sqrt(per_mode) / 2.0)))
        n_el = max(1, per_mode // n_az)
        fan = Fan(30.0, 110.0, 0.0, np.linspace(e0, e0 + ew, n_el),
                  np.linspace(ac - aw / 2, ac + aw / 2, n_az), np.array([f]), modes)
        reqs.append(dict(id=k, t_arrive=t, snapshot=snap, fan=fan))
    return reqs
