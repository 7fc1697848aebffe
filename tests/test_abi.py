"""The C-ABI library loads and exports every entry point include/rtgd.h
declares; host-only helpers validate geometry, fans and options.  No
compute call is made here (CPU-only)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtgd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def rt():
    from paper_2506_18579_amd import rtgd
    if not os.path.exists(rtgd.LIB_PATH):
        from paper_2506_18579_amd import build
        build.build(verbose=False)
    return rtgd


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("rt_ctx_create", "rt_ctx_destroy", "rt_last_error", "rt_grid_create",
                 "rt_grid_destroy", "rt_field_set", "rt_trace", "rt_fan_count",
                 "rt_check_geom", "rt_default_opts"):
        assert must in names


def test_library_exports_every_declared_symbol(rt):
    lib = rt.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rt_[a-z_]+)\b", out))
    assert set(_declared_functions()) <= exported


def test_library_has_gfx950_code_object(rt):
    """The offload bundle embedded in our own build targets gfx950."""
    data = open(rt.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def _geom(rt, **kw):
    from paper_2506_18579_amd.synth import GEOM_ISO
    g = rt.make_geom(GEOM_ISO)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("field,value", [("n_lat", 3), ("n_h", 0), ("dlat_deg", 0.0),
                                         ("dlon_deg", -1.0), ("dh_km", float("nan")),
                                         ("lat0_deg", -95.0), ("dtype", 7), ("quantity", 5),
                                         ("interp", 9), ("earth_radius_km", 0.0)])
def test_check_geom_rejects(rt, field, value):
    g = _geom(rt, **{field: value})
    assert rt.lib().rt_check_geom(ctypes.byref(g)) == rt.RT_E_INVALID


def test_check_geom_accepts_workload_grids(rt):
    from paper_2506_18579_amd.synth import GEOM_ANISO, GEOM_ISO
    for geom in (GEOM_ISO, GEOM_ANISO):
        g = rt.make_geom(geom)
        assert rt.lib().rt_check_geom(ctypes.byref(g)) == rt.RT_OK
    # latitude range must stay inside (-90, 90)
    g = _geom(rt, lat0_deg=60.0, dlat_deg=1.0)
    assert rt.lib().rt_check_geom(ctypes.byref(g)) == rt.RT_E_INVALID


def test_fan_count_index_space(rt):
    from paper_2506_18579_amd.synth import Fan
    fan = Fan(30.0, 110.0, 0.0, np.linspace(2, 65, 64), np.linspace(-30, 30, 64),
              np.array([7.0, 12.0, 18.0]), (1, -1))
    assert rt.fan_count(fan) == 24576
    fan1 = Fan(30.0, 110.0, 0.0, np.arange(1.0, 91.0), np.array([0.0]), np.array([10.0]), (1,))
    assert rt.fan_count(fan1) == 90
    empty = Fan(30.0, 110.0, 0.0, np.array([]), np.array([0.0]), np.array([10.0]), (1,))
    assert rt.fan_count(empty) == 0


def test_fan_count_rejects_bad_modes(rt):
    f = rt.Fan(30.0, 110.0, 0.0, None, 1, 1, None, None, 1, 4)
    n = ctypes.c_int64(0)
    assert rt.lib().rt_fan_count(ctypes.byref(f), ctypes.byref(n)) == rt.RT_E_INVALID
    f.modes = 3
    f.n_elev = -1
    assert rt.lib().rt_fan_count(ctypes.byref(f), ctypes.byref(n)) == rt.RT_E_INVALID


def test_default_opts(rt):
    o = rt.TraceOpts()
    rt.lib().rt_default_opts(ctypes.byref(o))
    assert o.step_km == 1.0 and o.max_group_km == 4000.0 and o.exit_h_km == 0.0
    assert o.precision == rt.RT_FP64 and o.results_mem == rt.RT_MEM_HOST


def test_struct_layout_matches_header(rt):
    """Offsets the C side uses, compiled from the header with the host compiler."""
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "rtgd.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(rt_grid_geom), sizeof(rt_fan), sizeof(rt_trace_opts),
         sizeof(rt_results), sizeof(rt_dipole));
  printf("%zu %zu %zu %zu %zu\n", offsetof(rt_grid_geom, lat0_deg), offsetof(rt_fan, az_deg),
         offsetof(rt_trace_opts, results_mem), offsetof(rt_results, kernel_ms),
         offsetof(rt_results, tail_ms));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = list(map(int, out))
    want = [ctypes.sizeof(rt.GridGeom), ctypes.sizeof(rt.Fan), ctypes.sizeof(rt.TraceOpts),
            ctypes.sizeof(rt.Results), ctypes.sizeof(rt.Dipole),
            rt.GridGeom.lat0_deg.offset, rt.Fan.az_deg.offset, rt.TraceOpts.results_mem.offset,
            rt.Results.kernel_ms.offset, rt.Results.tail_ms.offset]
    assert got == want


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package never imports the oracle and raises without its library."""
    pkg = os.path.join(ROOT, "paper_2506_18579_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", text).lower() or f == "synth.py", f


def test_tune_cache_text_roundtrip(rt, tmp_path):
    """The autotuner's cache file format (host-only, no device)."""
    src = tmp_path / "tune.txt"
    src.write_text("# comment\n256 181 181 226 0 0 1 17 16384 1 2 16 -1 2\n256 61 61 201 0 1 0 7 -1 2 1 0 0 0\n")
    rt.tune_cache_clear()
    rt.tune_cache_load(str(src))
    dst = tmp_path / "out.txt"
    rt.tune_cache_save(str(dst))
    lines = [l for l in dst.read_text().splitlines() if not l.startswith("#")]
    assert sorted(lines) == sorted(["256 181 181 226 0 0 1 17 16384 1 2 16 -1 2",
                                    "256 61 61 201 0 1 0 7 -1 2 1 0 0 0"])
    rt.tune_cache_clear()
    rt.tune_cache_save(str(dst))
    assert [l for l in dst.read_text().splitlines() if not l.startswith("#")] == []


@pytest.mark.parametrize("bad", ["256 181 181\n", "1 2 3 4 5 6 7 8 9 1 4 0 0 0\n", "1 2 3 4 5 6 7 8 9 1 1\n",
                                 "1 2 3 4 5 6 7 8 9 1 1 0 0 0 7\n", "a b c d e f g h i j k l m n\n",
                                 "1 2 3 4 5 6 7 8 9 1 1 65 0 0\n", "1 2 3 4 5 6 7 8 9 1 1 16 -2 0\n",
                                 "1 2 3 4 5 6 7 8 9 1 1 16 0 3\n", "1 2 3 4 5 6 7 8 9 1 1 16 0\n"])
def test_tune_cache_rejects_malformed_lines(rt, tmp_path, bad):
    p = tmp_path / "bad.txt"
    p.write_text(bad)
    with pytest.raises(rt.RTError):
        rt.tune_cache_load(str(p))
    with pytest.raises(rt.RTError):
        rt.tune_cache_load(str(tmp_path / "missing.txt"))


def test_noalloc_limits_match_header(rt):
    """The binding's copies of the rt_trace_noalloc limits are the header's."""
    src = open(os.path.join(ROOT, "include", "rtgd.h")).read()
    for name in ("RT_NOALLOC_SCRATCH_BYTES", "RT_NOALLOC_MAX_RAYS", "RT_NOALLOC_MAX_AXIS"):
        m = re.search(r"#define " + name + r" \(?([0-9]+)(?: << ([0-9]+))?\)?", src)
        assert m, name
        val = int(m.group(1)) << int(m.group(2) or 0)
        assert getattr(rt, name) == val, name
