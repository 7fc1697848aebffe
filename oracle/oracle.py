"""ctypes wrapper of the FP64 CPU oracle (``oracle/rtgd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark.  The product path never imports it.
It shares nothing with the GPU library except the seeded inputs the callers
pass in.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rtgd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
COUNT_SRC = os.path.join(HERE, "op_count.cpp")
COUNT_LIB = os.path.join(HERE, "liboracle_count.so")

GRID, CHAPMAN, QP, GRID_CR = 0, 1, 2, 3
GROUND, ESCAPE, MAX_PATH, NUMERIC = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no fast-math, no FMA contraction;
    and its operation-counting build (op_count.cpp, the same source as C++
    with a counting number type, no OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    if force or not os.path.exists(COUNT_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-Wall", "-Wno-unknown-pragmas", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-I", HERE, "-o", COUNT_LIB + ".tmp",
               COUNT_SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(COUNT_LIB + ".tmp", COUNT_LIB)
    return LIB


class Medium(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("n_lat", ctypes.c_int), ("n_lon", ctypes.c_int), ("n_h", ctypes.c_int),
        ("lat0_deg", ctypes.c_double), ("dlat_deg", ctypes.c_double),
        ("lon0_deg", ctypes.c_double), ("dlon_deg", ctypes.c_double),
        ("h0_km", ctypes.c_double), ("dh_km", ctypes.c_double),
        ("ne", ctypes.POINTER(ctypes.c_double)),
        ("fc_mhz", ctypes.c_double), ("hm_km", ctypes.c_double),
        ("thick_km", ctypes.c_double), ("floor_km", ctypes.c_double),
    ]


class Field(ctypes.Structure):
    _fields_ = [("B0_T", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("R_km", ctypes.c_double),
        ("tx_lat_deg", ctypes.c_double), ("tx_lon_deg", ctypes.c_double),
        ("tx_h_km", ctypes.c_double),
        ("step_km", ctypes.c_double), ("max_group_km", ctypes.c_double),
        ("exit_h_km", ctypes.c_double),
        ("traj_stride", ctypes.c_int), ("nthreads", ctypes.c_int),
    ]


class Ham(ctypes.Structure):
    _fields_ = [("H", ctypes.c_double), ("G", ctypes.c_double),
                ("Hn", ctypes.c_double * 3), ("Hq", ctypes.c_double * 3),
                ("X", ctypes.c_double), ("mu2", ctypes.c_double)]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def _bind(L):
    L.or_gd_weights.argtypes = [ctypes.c_double, _DP, _DP]
    L.or_cr_weights.argtypes = [ctypes.c_double, _DP, _DP]
    L.or_medium_eval.argtypes = [ctypes.POINTER(Medium), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, _DP]
    L.or_dipole.argtypes = [ctypes.c_double] * 5 + [_DP, _DP, _DP]
    L.or_appleton.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, _DP]
    L.or_appleton.restype = ctypes.c_int
    L.or_hamiltonian.argtypes = [ctypes.POINTER(Medium), ctypes.POINTER(Field),
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, _DP,
                                 ctypes.POINTER(Ham)]
    L.or_hamiltonian.restype = ctypes.c_int
    L.or_rhs.argtypes = [ctypes.POINTER(Medium), ctypes.POINTER(Field), ctypes.c_double,
                         ctypes.c_double, ctypes.c_int, _DP, _DP]
    L.or_rhs.restype = ctypes.c_int
    L.or_launch.argtypes = [ctypes.POINTER(Opts), ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, _DP]
    L.or_launch.restype = ctypes.c_double
    L.or_trace.argtypes = [ctypes.POINTER(Medium), ctypes.POINTER(Field),
                           ctypes.POINTER(Opts), ctypes.c_int, _DP, _DP, _DP, _IP, _DP,
                           _IP, _IP, _DP, ctypes.c_int, _IP]
    L.or_trace.restype = ctypes.c_longlong
    return L


def lib():
    """The oracle's shared object.  RTGD_ORACLE_LIB names another build of
    the same interface instead (the pin tests' mutation check loads copies
    of the oracle with planted mistakes this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("RTGD_ORACLE_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        _lib = _bind(ctypes.CDLL(path))
    return _lib


_count_lib = None


def count_lib():
    """The operation-counting build: the same entry points (serial), plus
    or_count_reset() and or_count_get(out[4]) = {add/sub, mul, div, libm}."""
    global _count_lib
    if _count_lib is None:
        if not os.path.exists(COUNT_LIB):
            build(force=False)
        L = _bind(ctypes.CDLL(COUNT_LIB))
        L.or_count_get.argtypes = [ctypes.POINTER(ctypes.c_ulonglong)]
        _count_lib = L
    return _count_lib


def counted(fn, *args):
    """Run fn(*args) and return (result, ops) with ops = {add, mul, div, lib,
    total} counted by the counting build (fn must call count_lib())."""
    L = count_lib()
    L.or_count_reset()
    r = fn(*args)
    c = (ctypes.c_ulonglong * 4)()
    L.or_count_get(c)
    ops = dict(add=int(c[0]), mul=int(c[1]), div=int(c[2]), lib=int(c[3]))
    ops["total"] = sum(ops.values())
    return r, ops


def _dp(a):
    return a.ctypes.data_as(_DP)


def _ip(a):
    return a.ctypes.data_as(_IP)


class OracleMedium:
    """Holds a Medium struct and keeps the grid array alive."""

    def __init__(self, kind=GRID, grid=None, fc_mhz=0.0, hm_km=0.0, thick_km=0.0,
                 floor_km=60.0):
        self.m = Medium()
        self.m.kind = kind
        self._ne = None
        if grid is not None:
            g = grid.geom
            self._ne = np.ascontiguousarray(grid.values, dtype=np.float64)
            if self._ne.shape != (g.n_lat, g.n_lon, g.n_h):
                raise ValueError(f"grid values of shape {self._ne.shape}, geometry "
                                 f"({g.n_lat}, {g.n_lon}, {g.n_h})")
            self.m.n_lat, self.m.n_lon, self.m.n_h = g.n_lat, g.n_lon, g.n_h
            self.m.lat0_deg, self.m.dlat_deg = g.lat0_deg, g.dlat_deg
            self.m.lon0_deg, self.m.dlon_deg = g.lon0_deg, g.dlon_deg
            self.m.h0_km, self.m.dh_km = g.h0_km, g.dh_km
            self.m.ne = _dp(self._ne)
            floor_km = g.h0_km
        self.m.fc_mhz, self.m.hm_km, self.m.thick_km = fc_mhz, hm_km, thick_km
        self.m.floor_km = floor_km

    @classmethod
    def from_grid(cls, grid, interp="gd"):
        return cls(GRID_CR if interp == "cr" else GRID, grid=grid)

    @classmethod
    def chapman(cls, fc_mhz, hm_km, scale_km, floor_km=60.0):
        return cls(CHAPMAN, fc_mhz=fc_mhz, hm_km=hm_km, thick_km=scale_km, floor_km=floor_km)

    @classmethod
    def qp(cls, fc_mhz, hm_km, ym_km, floor_km=60.0):
        return cls(QP, fc_mhz=fc_mhz, hm_km=hm_km, thick_km=ym_km, floor_km=floor_km)

    def eval(self, R, r, th, ph):
        out = np.zeros(4)
        lib().or_medium_eval(ctypes.byref(self.m), R, r, th, ph, _dp(out))
        return out


def gd_weights(s):
    w, dw = np.zeros(4), np.zeros(4)
    lib().or_gd_weights(float(s), _dp(w), _dp(dw))
    return w, dw


def cr_weights(s):
    w, dw = np.zeros(4), np.zeros(4)
    lib().or_cr_weights(float(s), _dp(w), _dp(dw))
    return w, dw


def dipole(B0, R, f_mhz, r, th):
    Y, Yr, Yt = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().or_dipole(B0, R, f_mhz, r, th, _dp(Y), _dp(Yr), _dp(Yt))
    return Y, Yr, Yt


def appleton(X, a, b, mode):
    out = np.zeros(4)
    ok = lib().or_appleton(X, a, b, mode, _dp(out))
    return out, bool(ok)


def hamiltonian(med: OracleMedium, B0, R, f_mhz, mode, y):
    y = np.ascontiguousarray(y[:6], dtype=np.float64)
    h = Ham()
    fld = Field(B0)
    ok = lib().or_hamiltonian(ctypes.byref(med.m), ctypes.byref(fld), R, f_mhz, mode,
                              _dp(y), ctypes.byref(h))
    return {"H": h.H, "G": h.G, "Hn": np.array(h.Hn[:]), "Hq": np.array(h.Hq[:]),
            "X": h.X, "mu2": h.mu2, "ok": bool(ok)}


def rhs(med: OracleMedium, B0, R, f_mhz, mode, y):
    y = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.zeros(7)
    fld = Field(B0)
    lib().or_rhs(ctypes.byref(med.m), ctypes.byref(fld), R, f_mhz, mode, _dp(y), _dp(dy))
    return dy


def make_opts(R=6371.0, tx=(30.0, 110.0, 0.0), step=1.0, max_group=4000.0, exit_h=500.0,
              traj_stride=0, nthreads=0):
    return Opts(R, tx[0], tx[1], tx[2], step, max_group, exit_h, traj_stride, nthreads)


def launch(opts: Opts, floor_km, elev, az):
    y = np.zeros(7)
    s = lib().or_launch(ctypes.byref(opts), floor_km, elev, az, _dp(y))
    return y, s


OUT_NAMES = ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km",
             "land_lat_deg", "land_lon_deg")


def trace(med: OracleMedium, elev, az, freq, mode=None, B0=0.0, R=6371.0,
          tx=(30.0, 110.0, 0.0), step=1.0, max_group=4000.0, exit_h=500.0,
          traj_stride=0, traj_per_ray=0, nthreads=0, counting=False):
    """Trace rays given per-ray elevation/azimuth (deg), frequency (MHz) and
    mode (+1 O, -1 X).  Returns a dict of numpy arrays.  counting=True runs
    the operation-counting build (serial; see counted())."""
    elev = np.ascontiguousarray(elev, dtype=np.float64)
    n = elev.size
    az = np.ascontiguousarray(np.broadcast_to(az, (n,)), dtype=np.float64)
    freq = np.ascontiguousarray(np.broadcast_to(freq, (n,)), dtype=np.float64)
    if mode is None:
        mode = np.ones(n, dtype=np.int32)
    mode = np.ascontiguousarray(np.broadcast_to(mode, (n,)), dtype=np.int32)
    out7 = np.zeros((n, 7))
    status = np.zeros(n, dtype=np.int32)
    nsteps = np.zeros(n, dtype=np.int32)
    opts = make_opts(R, tx, step, max_group, exit_h, traj_stride, nthreads)
    fld = Field(B0)
    traj = tcount = None
    if traj_stride > 0 and traj_per_ray > 0:
        traj = np.zeros((n, traj_per_ray, 8))
        tcount = np.zeros(n, dtype=np.int32)
    L = count_lib() if counting else lib()
    total = L.or_trace(ctypes.byref(med.m), ctypes.byref(fld), ctypes.byref(opts), n,
                           _dp(elev), _dp(az), _dp(freq), _ip(mode), _dp(out7), _ip(status),
                           _ip(nsteps), _dp(traj) if traj is not None else None,
                           traj_per_ray, _ip(tcount) if tcount is not None else None)
    res = {k: out7[:, i].copy() for i, k in enumerate(OUT_NAMES)}
    res["status"] = status
    res["n_steps"] = nsteps
    res["total_steps"] = int(total)
    if traj is not None:
        res["traj"] = traj
        res["traj_count"] = tcount
    return res


def ionogram(res, elev_deg, n_freq, n_mode, range_km, max_points=8):
    """Oblique ionogram from a frequency x mode x elevation sweep (one
    azimuth), following its definition: for each (frequency, mode) trace,
    each adjacent elevation pair whose rays both reach the ground with
    ground ranges on opposite sides of range_km (range - range_km changes
    sign, zero counting as positive) gives one received ray, linearly
    interpolated in elevation.  Returns (points[n_trace, max_points, 4] =
    elevation, group, phase, apogee; counts[n_trace])."""
    elev = np.asarray(elev_deg, dtype=np.float64)
    n_elev = elev.size
    n_trace = n_freq * n_mode
    pts = np.zeros((n_trace, max_points, 4))
    cnt = np.zeros(n_trace, dtype=np.int32)
    for t in range(n_trace):
        found = 0
        for e in range(n_elev - 1):
            i0 = t * n_elev + e
            i1 = i0 + 1
            if res["status"][i0] != GROUND or res["status"][i1] != GROUND:
                continue
            d0 = res["range_km"][i0] - range_km
            d1 = res["range_km"][i1] - range_km
            if (d0 < 0.0) == (d1 < 0.0):
                continue
            if found < max_points:
                w = d0 / (d0 - d1)
                pts[t, found, 0] = elev[e] + w * (elev[e + 1] - elev[e])
                for j, k in ((1, "group_km"), (2, "phase_km"), (3, "apogee_km")):
                    pts[t, found, j] = res[k][i0] + w * (res[k][i1] - res[k][i0])
            found += 1
        cnt[t] = found
    return pts, cnt
