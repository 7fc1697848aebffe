"""Thin ctypes binding of librtgd (the HIP C-ABI declared in include/rtgd.h).

Argument marshalling only: every step of the ray tracing runs in the HIP
kernels of librtgd.so.  PyTorch is used, when results are requested on the
device, for device memory and the current stream.  If the library has not
been built, importing works but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtgd.so")

RT_OK, RT_W_TRAJ_TRUNCATED = 0, 1
RT_E_INVALID, RT_E_NOMEM, RT_E_DEVICE, RT_E_UNSUPPORTED = -1, -2, -3, -4
RT_F64, RT_F32 = 0, 1
RT_NE_M3, RT_FN2_MHZ2 = 0, 1
RT_INTERP_GD, RT_INTERP_CR = 0, 1
RT_MODE_O, RT_MODE_X = 1, 2
RT_FP64, RT_MIXED = 0, 1
RT_MEM_HOST, RT_MEM_DEVICE = 0, 1
# limits of rt_trace_noalloc (include/rtgd.h)
RT_NOALLOC_SCRATCH_BYTES = 40 << 20
RT_NOALLOC_MAX_RAYS = 131072
RT_NOALLOC_MAX_AXIS = 4096
GROUND, ESCAPE, MAX_PATH, NUMERIC = 0, 1, 2, 3
STATUS_NAMES = {RT_OK: "RT_OK", RT_W_TRAJ_TRUNCATED: "RT_W_TRAJ_TRUNCATED",
                RT_E_INVALID: "RT_E_INVALID", RT_E_NOMEM: "RT_E_NOMEM",
                RT_E_DEVICE: "RT_E_DEVICE", RT_E_UNSUPPORTED: "RT_E_UNSUPPORTED"}

_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)


class GridGeom(ctypes.Structure):
    _fields_ = [("n_lat", ctypes.c_int32), ("n_lon", ctypes.c_int32), ("n_h", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("quantity", ctypes.c_int32),
                ("interp", ctypes.c_int32),
                ("lat0_deg", ctypes.c_double), ("dlat_deg", ctypes.c_double),
                ("lon0_deg", ctypes.c_double), ("dlon_deg", ctypes.c_double),
                ("h0_km", ctypes.c_double), ("dh_km", ctypes.c_double),
                ("earth_radius_km", ctypes.c_double)]


class Dipole(ctypes.Structure):
    _fields_ = [("B0_tesla", ctypes.c_double), ("pole_lat_deg", ctypes.c_double),
                ("pole_lon_deg", ctypes.c_double)]


class Fan(ctypes.Structure):
    _fields_ = [("tx_lat_deg", ctypes.c_double), ("tx_lon_deg", ctypes.c_double),
                ("tx_h_km", ctypes.c_double),
                ("elev_deg", _DP), ("n_elev", ctypes.c_int32), ("n_az", ctypes.c_int32),
                ("az_deg", _DP), ("freq_mhz", _DP), ("n_freq", ctypes.c_int32),
                ("modes", ctypes.c_uint32)]


class TraceOpts(ctypes.Structure):
    _fields_ = [("step_km", ctypes.c_double), ("max_group_km", ctypes.c_double),
                ("exit_h_km", ctypes.c_double), ("precision", ctypes.c_int32),
                ("traj_stride", ctypes.c_int32), ("traj_capacity", ctypes.c_int64),
                ("results_mem", ctypes.c_int32), ("tail_threshold", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32), ("ray_order", ctypes.c_int32),
                ("promote_waves", ctypes.c_int32), ("promote_age", ctypes.c_int32),
                ("cu_layout", ctypes.c_int32)]


class Results(ctypes.Structure):
    _fields_ = [("group_km", _DP), ("phase_km", _DP), ("range_km", _DP),
                ("az_dev_deg", _DP), ("apogee_km", _DP), ("land_lat_deg", _DP),
                ("land_lon_deg", _DP), ("status", _IP), ("n_steps", _IP),
                ("traj", _DP), ("traj_count", _IP), ("total_steps", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("steps_one_lane", ctypes.c_int64),
                ("steps_promoted", ctypes.c_int64), ("steps_rows", ctypes.c_int64),
                ("trace_ms", ctypes.c_double), ("tail_ms", ctypes.c_double),
                ("one_lane_wave_iters", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_int64), ("n_slots", ctypes.c_int32),
                ("max_batch_requests", ctypes.c_int32), ("max_batch_rays", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("n_rays", ctypes.c_int64),
                ("total_steps", ctypes.c_int64), ("kernel_ms", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("n_candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32)]


OUT_DOUBLE = ("group_km", "phase_km", "range_km", "az_dev_deg", "apogee_km",
              "land_lat_deg", "land_lon_deg")
OUT_INT = ("status", "n_steps")

_lib = None


class RTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load librtgd.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2506_18579_amd.build` (there is no CPU fallback)")
    # PyTorch ships its own HIP runtime with the same soname as the system
    # one; loading torch first makes librtgd bind to that single runtime
    # instead of bringing a second copy into the process.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.rt_ctx_create.argtypes = [ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.rt_ctx_create.restype = ctypes.c_int32
    L.rt_ctx_destroy.argtypes = [vp]
    L.rt_ctx_destroy.restype = None
    L.rt_last_error.argtypes = [vp]
    L.rt_last_error.restype = ctypes.c_char_p
    L.rt_grid_create.argtypes = [vp, ctypes.POINTER(GridGeom), vp, ctypes.c_int32,
                                 ctypes.POINTER(vp)]
    L.rt_grid_create.restype = ctypes.c_int32
    L.rt_grid_destroy.argtypes = [vp]
    L.rt_grid_destroy.restype = None
    L.rt_field_set.argtypes = [vp, ctypes.POINTER(Dipole)]
    L.rt_field_set.restype = ctypes.c_int32
    L.rt_trace.argtypes = [vp, vp, ctypes.POINTER(Fan), ctypes.POINTER(TraceOpts),
                           ctypes.POINTER(Results)]
    L.rt_trace.restype = ctypes.c_int32
    L.rt_trace_noalloc.argtypes = L.rt_trace.argtypes
    L.rt_trace_noalloc.restype = ctypes.c_int32
    L.rt_fan_count.argtypes = [ctypes.POINTER(Fan), ctypes.POINTER(ctypes.c_int64)]
    L.rt_fan_count.restype = ctypes.c_int32
    L.rt_check_geom.argtypes = [ctypes.POINTER(GridGeom)]
    L.rt_check_geom.restype = ctypes.c_int32
    L.rt_default_opts.argtypes = [ctypes.POINTER(TraceOpts)]
    L.rt_default_opts.restype = None
    L.rt_ionogram.argtypes = [vp, ctypes.POINTER(Fan), ctypes.POINTER(Results), ctypes.c_double,
                              ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.rt_ionogram.restype = ctypes.c_int32
    L.rt_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.rt_server_create.restype = ctypes.c_int32
    L.rt_server_destroy.argtypes = [vp]
    L.rt_server_destroy.restype = None
    L.rt_server_submit.argtypes = [vp, vp, ctypes.POINTER(Fan), ctypes.POINTER(TraceOpts),
                                   ctypes.POINTER(ctypes.c_int64)]
    L.rt_server_submit.restype = ctypes.c_int32
    L.rt_server_poll.argtypes = [vp, ctypes.POINTER(RequestInfo), ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32)]
    L.rt_server_poll.restype = ctypes.c_int32
    L.rt_server_fetch.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(Results), ctypes.c_int32]
    L.rt_server_fetch.restype = ctypes.c_int32
    L.rt_server_cancel.argtypes = [vp, ctypes.c_int64]
    L.rt_server_cancel.restype = ctypes.c_int32
    L.rt_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int64)]
    L.rt_server_stats.restype = ctypes.c_int32
    L.rt_plan_create.argtypes = [vp, vp, ctypes.POINTER(Fan), ctypes.POINTER(TraceOpts),
                                 ctypes.POINTER(Results), ctypes.POINTER(vp)]
    L.rt_plan_create.restype = ctypes.c_int32
    L.rt_plan_launch.argtypes = [vp]
    L.rt_plan_launch.restype = ctypes.c_int32
    L.rt_plan_wait.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    L.rt_plan_wait.restype = ctypes.c_int32
    L.rt_plan_destroy.argtypes = [vp]
    L.rt_plan_destroy.restype = None
    L.rt_autotune.argtypes = [vp, vp, ctypes.POINTER(Fan), ctypes.POINTER(TraceOpts),
                              ctypes.POINTER(TraceOpts), ctypes.POINTER(TuneInfo)]
    L.rt_autotune.restype = ctypes.c_int32
    L.rt_tune_cache_save.argtypes = [ctypes.c_char_p]
    L.rt_tune_cache_save.restype = ctypes.c_int32
    L.rt_tune_cache_load.argtypes = [ctypes.c_char_p]
    L.rt_tune_cache_load.restype = ctypes.c_int32
    L.rt_tune_cache_clear.argtypes = []
    L.rt_tune_cache_clear.restype = None
    _lib = L
    return L


def make_geom(geom, dtype=RT_F64, quantity=RT_NE_M3, interp="gd") -> GridGeom:
    g = GridGeom()
    g.n_lat, g.n_lon, g.n_h = geom.n_lat, geom.n_lon, geom.n_h
    g.dtype, g.quantity = dtype, quantity
    g.interp = RT_INTERP_CR if interp == "cr" else RT_INTERP_GD
    g.lat0_deg, g.dlat_deg = geom.lat0_deg, geom.dlat_deg
    g.lon0_deg, g.dlon_deg = geom.lon0_deg, geom.dlon_deg
    g.h0_km, g.dh_km = geom.h0_km, geom.dh_km
    g.earth_radius_km = geom.earth_radius_km
    return g


class FanArgs:
    """rt_fan with its arrays kept alive."""

    def __init__(self, fan):
        self.elev = np.ascontiguousarray(fan.elev_deg, dtype=np.float64)
        self.az = np.ascontiguousarray(fan.az_deg, dtype=np.float64)
        self.freq = np.ascontiguousarray(fan.freq_mhz, dtype=np.float64)
        modes = 0
        for m in fan.modes:
            modes |= RT_MODE_O if m > 0 else RT_MODE_X
        if list(fan.modes) not in ([1], [-1], [1, -1]):
            raise ValueError("fan.modes must be (1,), (-1,) or (1, -1)")
        self.s = Fan(fan.tx_lat_deg, fan.tx_lon_deg, fan.tx_h_km,
                     self.elev.ctypes.data_as(_DP), self.elev.size, self.az.size,
                     self.az.ctypes.data_as(_DP), self.freq.ctypes.data_as(_DP),
                     self.freq.size, modes)


def fan_count(fan) -> int:
    fa = FanArgs(fan)
    n = ctypes.c_int64(0)
    st = lib().rt_fan_count(ctypes.byref(fa.s), ctypes.byref(n))
    if st != RT_OK:
        raise RTError(st, "invalid fan")
    return int(n.value)


def _torch_stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch  # device memory and streams come from PyTorch
        if not torch.cuda.is_available():
            raise RuntimeError("librtgd needs a ROCm GPU (torch.cuda.is_available() is False)")
        torch.cuda.set_device(device)
        self.device = device
        if stream is None:
            sptr = _torch_stream_ptr()
        elif isinstance(stream, int):
            sptr = ctypes.c_void_p(stream)
        else:
            sptr = ctypes.c_void_p(stream.cuda_stream)
        self.h = ctypes.c_void_p()
        st = lib().rt_ctx_create(device, sptr, ctypes.byref(self.h))
        if st != RT_OK:
            raise RTError(st, "rt_ctx_create failed: " + lib().rt_last_error(None).decode())

    def error(self) -> str:
        return lib().rt_last_error(self.h).decode()

    def check(self, st, what):
        if st not in (RT_OK, RT_W_TRAJ_TRUNCATED):
            raise RTError(st, f"{what}: {self.error()}")
        return st

    def close(self):
        if self.h:
            lib().rt_ctx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid:
    """A grid resident on the device (rt_grid_create + rt_field_set)."""

    def __init__(self, ctx: Context, grid, interp: str = "gd", values_f32_fn2=None):
        self.ctx = ctx
        if values_f32_fn2 is not None:
            vals = np.ascontiguousarray(values_f32_fn2, dtype=np.float32)
            g = make_geom(grid.geom, RT_F32, RT_FN2_MHZ2, interp)
        else:
            vals = np.ascontiguousarray(grid.values, dtype=np.float64)
            g = make_geom(grid.geom, RT_F64, RT_NE_M3, interp)
        self.geom = grid.geom
        self.h = ctypes.c_void_p()
        ctx.check(lib().rt_grid_create(ctx.h, ctypes.byref(g), vals.ctypes.data_as(ctypes.c_void_p),
                                       RT_MEM_HOST, ctypes.byref(self.h)), "rt_grid_create")
        self.set_field(grid.B0_T)

    def set_field(self, B0_T: float):
        d = Dipole(float(B0_T), 90.0, 0.0)
        self.ctx.check(lib().rt_field_set(self.h, ctypes.byref(d)), "rt_field_set")
        self.B0 = float(B0_T)

    def close(self):
        if self.h:
            lib().rt_grid_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(step_km=1.0, max_group_km=4000.0, exit_h_km=0.0, precision="fp64",
              tail_threshold=0, waves_per_simd=0, ray_order=0, promote_waves=0,
              promote_age=0, cu_layout=0) -> TraceOpts:
    o = TraceOpts()
    lib().rt_default_opts(ctypes.byref(o))
    o.step_km, o.max_group_km, o.exit_h_km = step_km, max_group_km, exit_h_km
    o.precision = RT_MIXED if precision == "mixed" else RT_FP64
    o.tail_threshold = tail_threshold
    o.waves_per_simd = waves_per_simd
    o.ray_order = ray_order
    o.promote_waves = promote_waves
    o.promote_age = promote_age
    o.cu_layout = cu_layout
    return o


def trace(ctx: Context, grid: Grid, fan, step_km=1.0, max_group_km=4000.0, exit_h_km=0.0,
          precision="fp64", traj_stride=0, traj_per_ray=0, device_results=False, out=None,
          tail_threshold=0, waves_per_simd=0, ray_order=0, promote_waves=0, promote_age=0,
          cu_layout=0, _entry="rt_trace"):
    """Trace every ray of `fan` (synth.Fan) through `grid`.

    Returns a dict of per-ray arrays (numpy on the host, or torch tensors on
    the device with device_results=True; pass `out` to reuse device
    tensors), plus total_steps, kernel_ms and how the launch ran:
    phase_steps (one lane, promotion rows, 16-lane rows), trace_ms,
    tail_ms and one_lane_wave_iters (one-lane wave iterations that stepped a
    ray)."""
    fa = FanArgs(fan)
    n = ctypes.c_int64(0)
    st = lib().rt_fan_count(ctypes.byref(fa.s), ctypes.byref(n))
    if st != RT_OK:
        raise RTError(st, "invalid fan")
    n = int(n.value)
    o = make_opts(step_km, max_group_km, exit_h_km, precision, tail_threshold, waves_per_simd,
                  ray_order, promote_waves, promote_age, cu_layout)
    o.traj_stride = traj_stride
    o.traj_capacity = traj_per_ray * n if traj_stride > 0 else 0
    o.results_mem = RT_MEM_DEVICE if device_results else RT_MEM_HOST
    r = Results()
    if device_results:
        import torch
        dev = torch.device("cuda", ctx.device)
        if out is None:
            out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in OUT_DOUBLE}
            out.update({k: torch.empty(n, dtype=torch.int32, device=dev) for k in OUT_INT})
            if traj_stride > 0:
                out["traj"] = torch.empty((n, traj_per_ray, 8), dtype=torch.float64, device=dev)
                out["traj_count"] = torch.empty(n, dtype=torch.int32, device=dev)
        ptr = lambda t, P: ctypes.cast(ctypes.c_void_p(t.data_ptr()), P)
    else:
        out = {k: np.empty(n, dtype=np.float64) for k in OUT_DOUBLE}
        out.update({k: np.empty(n, dtype=np.int32) for k in OUT_INT})
        if traj_stride > 0:
            out["traj"] = np.empty((n, traj_per_ray, 8), dtype=np.float64)
            out["traj_count"] = np.empty(n, dtype=np.int32)
        ptr = lambda a, P: a.ctypes.data_as(P)
    for k in OUT_DOUBLE:
        setattr(r, k, ptr(out[k], _DP))
    for k in OUT_INT:
        setattr(r, k, ptr(out[k], _IP))
    if traj_stride > 0:
        r.traj = ptr(out["traj"], _DP)
        r.traj_count = ptr(out["traj_count"], _IP)
    st = getattr(lib(), _entry)(ctx.h, grid.h, ctypes.byref(fa.s), ctypes.byref(o), ctypes.byref(r))
    ctx.check(st, _entry)
    res = dict(out)
    res["total_steps"] = int(r.total_steps)
    res["kernel_ms"] = float(r.kernel_ms)
    res["phase_steps"] = (int(r.steps_one_lane), int(r.steps_promoted), int(r.steps_rows))
    res["one_lane_wave_iters"] = int(r.one_lane_wave_iters)
    res["trace_ms"] = float(r.trace_ms)
    res["tail_ms"] = float(r.tail_ms)
    res["truncated"] = st == RT_W_TRAJ_TRUNCATED
    return res


def trace_noalloc(ctx: Context, grid: Grid, fan, step_km=1.0, max_group_km=4000.0, exit_h_km=0.0,
                  precision="fp64", out=None, tail_threshold=0, waves_per_simd=0, ray_order=0,
                  promote_waves=0, promote_age=0, cu_layout=0):
    """rt_trace_noalloc: trace() with device results and no trajectories,
    every launch buffer taken from the library's per-device scratch region
    (the library allocates nothing; `out`, if given, is reused)."""
    return trace(ctx, grid, fan, step_km, max_group_km, exit_h_km, precision, 0, 0, True, out,
                 tail_threshold, waves_per_simd, ray_order, promote_waves, promote_age, cu_layout,
                 _entry="rt_trace_noalloc")


def trace_raw(ctx: Context, grid: Grid, fan_struct: Fan, opts: TraceOpts, res: Results) -> int:
    """Direct rt_trace call on prepared structs (returns the status)."""
    return lib().rt_trace(ctx.h, grid.h, ctypes.byref(fan_struct), ctypes.byref(opts),
                          ctypes.byref(res))


def ionogram(ctx: Context, fan, res, range_km: float, max_points: int = 8):
    """Synthetic oblique ionogram (rt_ionogram) from the per-ray results of a
    frequency x elevation sweep `fan` (one azimuth).  `res` is the dict
    returned by trace() (numpy on the host or torch on the device).  Returns
    (points[n_trace, max_points, 4] = elevation, group, phase, apogee;
    counts[n_trace]) with trace t = i_freq * n_mode + i_mode."""
    fa = FanArgs(fan)
    n_trace = len(fan.freq_mhz) * len(fan.modes)
    r = Results()
    on_device = hasattr(res["group_km"], "data_ptr")
    if on_device:
        import torch
        dev = res["group_km"].device
        pts = torch.zeros((n_trace, max_points, 4), dtype=torch.float64, device=dev)
        cnt = torch.zeros(n_trace, dtype=torch.int32, device=dev)
        ptr = lambda t, P: ctypes.cast(ctypes.c_void_p(t.data_ptr()), P)
        vptr = lambda t: ctypes.c_void_p(t.data_ptr())
    else:
        pts = np.zeros((n_trace, max_points, 4), dtype=np.float64)
        cnt = np.zeros(n_trace, dtype=np.int32)
        ptr = lambda a, P: np.ascontiguousarray(a).ctypes.data_as(P)
        vptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    keep = {k: (res[k] if on_device else np.ascontiguousarray(res[k]))
            for k in ("group_km", "phase_km", "range_km", "apogee_km", "status")}
    r.group_km = ptr(keep["group_km"], _DP)
    r.phase_km = ptr(keep["phase_km"], _DP)
    r.range_km = ptr(keep["range_km"], _DP)
    r.apogee_km = ptr(keep["apogee_km"], _DP)
    r.status = ptr(keep["status"], _IP)
    st = lib().rt_ionogram(ctx.h, ctypes.byref(fa.s), ctypes.byref(r), float(range_km),
                           int(max_points), RT_MEM_DEVICE if on_device else RT_MEM_HOST,
                           vptr(pts), vptr(cnt))
    ctx.check(st, "rt_ionogram")
    return pts, cnt


class Server:
    """Request server (rt_server_*): continuous batching of ray-fan
    requests (queued requests are launched together, as slots free up) over
    `n_slots` streams (0: the library default, 2) with a device output arena
    of `mem_budget_bytes`.  submit() never blocks; poll() launches queued work
    and returns finished requests; fetch() copies a finished request's
    per-ray outputs out and frees its arena block."""

    def __init__(self, ctx: Context, n_slots: int = 0, mem_budget_bytes: int = 256 << 20,
                 max_batch_requests: int = 0, max_batch_rays: int = 0):
        self.ctx = ctx
        self.h = ctypes.c_void_p()
        so = ServerOpts(int(mem_budget_bytes), int(n_slots), int(max_batch_requests),
                        int(max_batch_rays), 0)
        ctx.check(lib().rt_server_create(ctx.h, ctypes.byref(so), ctypes.byref(self.h)),
                  "rt_server_create")
        self._n = {}
        self._buf = (RequestInfo * 64)()

    def submit(self, grid: Grid, fan, **opts) -> int:
        fa = FanArgs(fan)
        o = make_opts(**opts)
        rid = ctypes.c_int64(0)
        self.ctx.check(lib().rt_server_submit(self.h, grid.h, ctypes.byref(fa.s), ctypes.byref(o),
                                              ctypes.byref(rid)), "rt_server_submit")
        return int(rid.value)

    def poll(self) -> list:
        """Finished requests since the last poll: dicts with id, n_rays,
        total_steps, kernel_ms, status."""
        out = []
        while True:
            n = ctypes.c_int32(0)
            self.ctx.check(lib().rt_server_poll(self.h, self._buf, len(self._buf), ctypes.byref(n)),
                           "rt_server_poll")
            for i in range(n.value):
                b = self._buf[i]
                out.append(dict(id=int(b.id), n_rays=int(b.n_rays), total_steps=int(b.total_steps),
                                kernel_ms=float(b.kernel_ms), status=int(b.status)))
            if n.value < len(self._buf):
                return out

    def fetch(self, rid: int, n_rays: int, device: bool = False) -> dict:
        """Per-ray outputs of a finished request: numpy arrays on the host,
        or (device=True) torch tensors on the context's GPU."""
        r = Results()
        if device:
            import torch
            dev = torch.device("cuda", self.ctx.device)
            out = {k: torch.empty(n_rays, dtype=torch.float64, device=dev) for k in OUT_DOUBLE}
            out.update({k: torch.empty(n_rays, dtype=torch.int32, device=dev) for k in OUT_INT})
            ptr = lambda t, P: ctypes.cast(ctypes.c_void_p(t.data_ptr()), P)
        else:
            out = {k: np.empty(n_rays, dtype=np.float64) for k in OUT_DOUBLE}
            out.update({k: np.empty(n_rays, dtype=np.int32) for k in OUT_INT})
            ptr = lambda a, P: a.ctypes.data_as(P)
        for k in OUT_DOUBLE:
            setattr(r, k, ptr(out[k], _DP))
        for k in OUT_INT:
            setattr(r, k, ptr(out[k], _IP))
        self.ctx.check(lib().rt_server_fetch(self.h, int(rid), ctypes.byref(r),
                                             RT_MEM_DEVICE if device else RT_MEM_HOST), "rt_server_fetch")
        out["total_steps"] = int(r.total_steps)
        out["kernel_ms"] = float(r.kernel_ms)
        return out

    def cancel(self, rid: int):
        self.ctx.check(lib().rt_server_cancel(self.h, int(rid)), "rt_server_cancel")

    def stats(self):
        q, r, a = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int64(0)
        self.ctx.check(lib().rt_server_stats(self.h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(a)),
                       "rt_server_stats")
        return dict(queued=q.value, running=r.value, arena_used=a.value)

    def close(self):
        if self.h:
            lib().rt_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ctx: Context, grid: Grid, fan, step_km=1.0, max_group_km=4000.0, exit_h_km=0.0,
             precision="fp64") -> dict:
    """rt_autotune: the fastest (tail_threshold, waves_per_simd, ray_order,
    promote_waves, promote_age, cu_layout) for this fan, from the process cache or by
    timing every candidate."""
    fa = FanArgs(fan)
    base = make_opts(step_km, max_group_km, exit_h_km, precision)
    tuned = TraceOpts()
    info = TuneInfo()
    ctx.check(lib().rt_autotune(ctx.h, grid.h, ctypes.byref(fa.s), ctypes.byref(base),
                                ctypes.byref(tuned), ctypes.byref(info)), "rt_autotune")
    return dict(tail_threshold=int(tuned.tail_threshold), waves_per_simd=int(tuned.waves_per_simd),
                ray_order=int(tuned.ray_order), promote_waves=int(tuned.promote_waves),
                promote_age=int(tuned.promote_age), cu_layout=int(tuned.cu_layout),
                best_ms=float(info.best_ms),
                default_ms=float(info.default_ms), n_candidates=int(info.n_candidates),
                from_cache=bool(info.from_cache))


def tune_cache_save(path: str):
    if lib().rt_tune_cache_save(os.fsencode(path)) != RT_OK:
        raise RTError(RT_E_INVALID, f"cannot write {path}")


def tune_cache_load(path: str):
    if lib().rt_tune_cache_load(os.fsencode(path)) != RT_OK:
        raise RTError(RT_E_INVALID, f"cannot read {path} or a line is malformed")


def tune_cache_clear():
    lib().rt_tune_cache_clear()


class Plan:
    """A trace captured once into a HIP graph (rt_plan_*) and replayed.
    Results go to device tensors (self.out), rewritten by every replay."""

    def __init__(self, ctx: Context, grid: Grid, fan, step_km=1.0, max_group_km=4000.0,
                 exit_h_km=0.0, precision="fp64", tail_threshold=0, waves_per_simd=0, ray_order=0,
                 promote_waves=0, promote_age=0, cu_layout=0):
        import torch
        self.ctx, self.grid = ctx, grid
        n = fan_count(fan)
        dev = torch.device("cuda", ctx.device)
        self.out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in OUT_DOUBLE}
        self.out.update({k: torch.empty(n, dtype=torch.int32, device=dev) for k in OUT_INT})
        r = Results()
        for k in OUT_DOUBLE:
            setattr(r, k, ctypes.cast(ctypes.c_void_p(self.out[k].data_ptr()), _DP))
        for k in OUT_INT:
            setattr(r, k, ctypes.cast(ctypes.c_void_p(self.out[k].data_ptr()), _IP))
        o = make_opts(step_km, max_group_km, exit_h_km, precision, tail_threshold, waves_per_simd,
                      ray_order, promote_waves, promote_age, cu_layout)
        o.results_mem = RT_MEM_DEVICE
        fa = FanArgs(fan)
        self.h = ctypes.c_void_p()
        ctx.check(lib().rt_plan_create(ctx.h, grid.h, ctypes.byref(fa.s), ctypes.byref(o),
                                       ctypes.byref(r), ctypes.byref(self.h)), "rt_plan_create")

    def launch(self):
        self.ctx.check(lib().rt_plan_launch(self.h), "rt_plan_launch")

    def wait(self):
        steps, ms = ctypes.c_int64(0), ctypes.c_double(0.0)
        self.ctx.check(lib().rt_plan_wait(self.h, ctypes.byref(steps), ctypes.byref(ms)), "rt_plan_wait")
        return int(steps.value), float(ms.value)

    def close(self):
        if self.h:
            lib().rt_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
