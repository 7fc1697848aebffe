"""The paper's comparison of its GD interpolant (Sec. II-B-2, Appendix A)
with Catmull-Rom (Sec. II-B-1, eq. cr_basis), on media with an exact answer:
a Chapman layer gridded at several height spacings, traced by the oracle
with each interpolant, against the same layer evaluated analytically.

Pinned: both interpolants converge to the analytic rays as the grid is
refined (group path and ground range RMS fall by more than 4x from 10 km to
5 km and by more than 3x from 5 km to 2.2 km: third-order values and
second-order gradients, Sec. III-A-2), and on these smooth layers their
errors agree to within a factor of 1.5 at every spacing.  The paper's
Table II finds GD well ahead of CR on IRI-2020 grids; on smooth synthetic
layers the two schemes, which share their orders of accuracy, are level.
"""
import numpy as np
import pytest

from paper_2506_18579_amd import synth

ELEV = np.arange(1.0, 90.0, 2.0)


def rms(orc, dh, interp, B0, mode, az):
    geom = synth.GridGeom(61, 61, int(round(440.0 / dh)) + 1, 15.0, 0.5, 95.0, 0.5, 60.0, dh)
    grid = synth.chapman_grid(geom, 8.0, 300.0, 50.0)
    m = np.full(ELEV.size, mode, np.int32)
    kw = dict(B0=B0, tx=(30.0, 110.0, 0.0), step=1.0, max_group=4000.0, exit_h=500.0)
    ref = orc.trace(orc.OracleMedium.chapman(8.0, 300.0, 50.0, floor_km=60.0), ELEV, az, 10.0, m, **kw)
    r = orc.trace(orc.OracleMedium.from_grid(grid, interp), ELEV, az, 10.0, m, **kw)
    same = (r["status"] == ref["status"]) & (ref["status"] != 3)
    assert same.sum() >= ELEV.size - 1
    return np.array([np.sqrt(np.mean((r[k][same] - ref[k][same]) ** 2)) for k in ("group_km", "range_km")])


@pytest.mark.parametrize("B0,mode,az", [(0.0, 1, 0.0), (3.12e-5, 1, 45.0), (3.12e-5, -1, 45.0)])
def test_gd_and_cr_converge_and_are_level_on_smooth_layers(orc, B0, mode, az):
    e = {(dh, ip): rms(orc, dh, ip, B0, mode, az) for dh in (10.0, 5.0, 2.2) for ip in ("gd", "cr")}
    for ip in ("gd", "cr"):
        assert np.all(e[(10.0, ip)] > 4.0 * e[(5.0, ip)]), (ip, e)
        assert np.all(e[(5.0, ip)] > 3.0 * e[(2.2, ip)]), (ip, e)
    for dh in (10.0, 5.0, 2.2):
        ratio = e[(dh, "gd")] / e[(dh, "cr")]
        assert np.all((ratio > 1 / 1.5) & (ratio < 1.5)), (dh, ratio)
