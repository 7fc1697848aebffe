"""Pins of the oracle's GD p=3 interpolant (Sec. II-B-2, Appendix A).

The oracle's weight table is checked against the pieces as printed in the
paper (golden fixture) and against properties the mathematics fixes:
interpolation of the four stencil nodes, central-difference derivatives at
the cell ends, partition of unity, exact reproduction of quadratics in 3-D,
C1 continuity across faces, and the convergence orders of the error bounds
(value O(h^3), gradient O(h^2) for p = 3).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _pieces():
    rows = {}
    for line in open(os.path.join(GOLD, "gd_p3_appendix_pieces.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        rows[int(tok[0])] = [Fraction(t) for t in tok[1:]]   # t^5 .. t^0
    return rows


def _piece_value(coefs, t):
    v = Fraction(0)
    for c in coefs:
        v = v * t + c
    return v


def _piece_deriv(coefs, t):
    deg = len(coefs) - 1
    v = Fraction(0)
    for i, c in enumerate(coefs[:-1]):
        v = v * t + c * (deg - i)
    return v


def test_weights_match_appendix_pieces(orc):
    """Node j+a of cell j contributes psi_{-a} at its shifted variable s."""
    rows = _pieces()
    for s in [Fraction(k, 17) for k in range(-17, 35)]:
        w, dw = orc.gd_weights(float(s))
        for ai, a in enumerate((-1, 0, 1, 2)):
            exact = _piece_value(rows[-a], s)
            dexact = _piece_deriv(rows[-a], s)
            assert abs(w[ai] - float(exact)) <= 4e-15 * max(1.0, abs(float(exact)))
            assert abs(dw[ai] - float(dexact)) <= 8e-15 * max(1.0, abs(float(dexact)))


def test_weights_interpolate_all_four_nodes(orc):
    for node, expect in ((-1, 0), (0, 1), (1, 2), (2, 3)):
        w, _ = orc.gd_weights(float(node))
        e = np.zeros(4)
        e[expect] = 1.0
        np.testing.assert_allclose(w, e, atol=1e-15)


def test_derivative_weights_are_appendix_central_differences(orc):
    eta = {}
    for line in open(os.path.join(GOLD, "fd_weights_appendix.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            eta[int(k)] = float(Fraction(v))
    # at s = 0 (node j): weights of nodes j-1, j, j+1, j+2
    _, dw0 = orc.gd_weights(0.0)
    np.testing.assert_allclose(dw0, [eta[-1], eta[0], eta[1], eta[2]], atol=1e-15)
    # at s = 1 (node j+1): weights of nodes j-1 .. j+2 are eta[-2], eta[-1], eta[0], eta[1]
    _, dw1 = orc.gd_weights(1.0)
    np.testing.assert_allclose(dw1, [eta[-2], eta[-1], eta[0], eta[1]], atol=1e-15)


@pytest.mark.parametrize("s", np.linspace(-1.0, 2.0, 31))
def test_partition_of_unity(orc, s):
    w, dw = orc.gd_weights(s)
    assert abs(w.sum() - 1.0) < 1e-14
    assert abs(dw.sum()) < 1e-14


def test_second_derivative_jumps_so_only_c1():
    """The global basis is C1 but not C2: psi'' jumps by -5/3 at xi = 1 (and
    by +5/3 at xi = -1; the jumps at xi = 0 cancel by symmetry)."""
    rows = _pieces()

    def d2(coefs, t):
        deg = len(coefs) - 1
        v = Fraction(0)
        for i, c in enumerate(coefs[:-2]):
            p = deg - i
            v = v * t + c * p * (p - 1)
        return v
    # xi = 1: end of piece k=0 (t=1) vs start of piece k=1 (t=0)
    jump = d2(rows[1], Fraction(0)) - d2(rows[0], Fraction(1))
    assert jump == Fraction(-5, 3)
    jump_m1 = d2(rows[-1], Fraction(0)) - d2(rows[-2], Fraction(1))
    assert jump_m1 == Fraction(5, 3)


def _grid(n, lat0, dlat, lon0, dlon, h0, dh, fn):
    from paper_2506_18579_amd.synth import Grid, GridGeom
    g = GridGeom(n[0], n[1], n[2], lat0, dlat, lon0, dlon, h0, dh)
    LA, LO, H = np.meshgrid(g.lats(), g.lons(), g.heights(), indexing="ij")
    return Grid(g, np.ascontiguousarray(fn(LA, LO, H)))


R = 6371.0
DEG = math.pi / 180.0


def _eval_geo(orc, med, lat, lon, h):
    return med.eval(R, R + h, (90.0 - lat) * DEG, lon * DEG)


@pytest.mark.parametrize("pa,pb,pc", [(a, b, c) for a in range(3) for b in range(3)
                                      for c in range(3)])
def test_3d_reproduces_quadratics_exactly(orc, pa, pb, pc):
    """u = lat^a lon^b h^c with a, b, c <= 2: value and gradient exact."""
    lat_c, lon_c, h_c = 30.0, 110.0, 200.0

    def fn(la, lo, h):
        return ((la - lat_c) ** pa) * ((lo - lon_c) ** pb) * ((h - h_c) ** pc) + 1e3

    grid = _grid((9, 10, 12), 28.0, 0.5, 108.0, 0.4, 190.0, 2.0, fn)
    med = orc.OracleMedium.from_grid(grid)
    rng = np.random.default_rng(pa * 9 + pb * 3 + pc)
    for _ in range(40):
        # include points in edge cells (s in [-1, 0) and [1, 2])
        la = rng.uniform(28.0, 32.0)
        lo = rng.uniform(108.0, 111.6)
        h = rng.uniform(190.0, 212.0)
        v = _eval_geo(orc, med, la, lo, h)
        x, y, z = la - lat_c, lo - lon_c, h - h_c
        val = x ** pa * y ** pb * z ** pc + 1e3
        d_la = pa * x ** max(pa - 1, 0) * y ** pb * z ** pc
        d_lo = pb * x ** pa * y ** max(pb - 1, 0) * z ** pc
        d_h = pc * x ** pa * y ** pb * z ** max(pc - 1, 0)
        assert abs(v[0] - val) <= 1e-11 * max(1.0, abs(val))
        # physical partials: d/dr = d/dh, d/dtheta = -(180/pi) d/dlat, d/dphi = (180/pi) d/dlon
        assert abs(v[1] - d_h) <= 1e-10
        assert abs(v[2] - (-d_la / DEG)) <= 1e-8
        assert abs(v[3] - (d_lo / DEG)) <= 1e-8


def test_3d_does_not_reproduce_cubics(orc):
    grid = _grid((8, 8, 8), 28.0, 1.0, 108.0, 1.0, 190.0, 2.0,
                 lambda la, lo, h: (h - 195.0) ** 3)
    med = orc.OracleMedium.from_grid(grid)
    v = _eval_geo(orc, med, 31.3, 111.2, 195.7)
    assert abs(v[0] - 0.7 ** 3) > 1e-3


def test_c1_across_cell_faces(orc):
    rng = np.random.default_rng(7)
    from paper_2506_18579_amd.synth import Grid, GridGeom
    g = GridGeom(8, 8, 10, 28.0, 0.5, 108.0, 0.5, 100.0, 3.0)
    grid = Grid(g, rng.uniform(1e10, 2e11, (8, 8, 10)))
    med = orc.OracleMedium.from_grid(grid)
    eps = 1e-9
    base = (29.6, 109.7, 113.3)
    for axis, face in ((0, 29.5), (1, 109.5), (2, 112.0)):
        lo_p = list(base)
        hi_p = list(base)
        lo_p[axis] = face - eps
        hi_p[axis] = face + eps
        a = _eval_geo(orc, med, *lo_p)
        b = _eval_geo(orc, med, *hi_p)
        scale = np.abs(a).max()
        # value and all partials continuous to O(eps)
        assert np.abs(a - b).max() <= 1e-6 * scale


def test_outside_box_is_clamped_and_vacuum_below(orc):
    from paper_2506_18579_amd.synth import Grid, GridGeom
    g = GridGeom(6, 6, 8, 28.0, 0.5, 108.0, 0.5, 100.0, 3.0)
    rng = np.random.default_rng(3)
    grid = Grid(g, rng.uniform(1e10, 2e11, (6, 6, 8)))
    med = orc.OracleMedium.from_grid(grid)
    below = _eval_geo(orc, med, 29.0, 109.0, 99.999)
    assert np.all(below == 0.0)
    # west of the box: equals the value on the west face, d/dphi = 0
    out = _eval_geo(orc, med, 29.1, 100.0, 110.0)
    face = _eval_geo(orc, med, 29.1, 108.0, 110.0)
    assert out[3] == 0.0
    assert abs(out[0] - face[0]) <= 1e-12 * abs(face[0])
    # above the top: constant continuation, d/dr = 0
    top = _eval_geo(orc, med, 29.1, 109.1, 130.0)
    assert top[1] == 0.0
    # north and south of the box: the value of the north / south face,
    # d/dtheta = 0, while the other partials are those of the face
    for lat_out, lat_face in ((35.0, 30.5), (20.0, 28.0)):
        out = _eval_geo(orc, med, lat_out, 109.3, 110.0)
        face = _eval_geo(orc, med, lat_face, 109.3, 110.0)
        assert out[2] == 0.0 and face[2] != 0.0
        assert abs(out[0] - face[0]) <= 1e-12 * abs(face[0])
        assert abs(out[3] - face[3]) <= 1e-12 * abs(face[3])


def test_convergence_orders_value3_gradient2(orc):
    """Sec. III-A-2 bounds: value O(h^p), gradient O(h^(p-1)), p = 3."""
    from paper_2506_18579_amd.synth import Grid, GridGeom, chapman
    errs_v, errs_g = [], []
    hs = [8.0, 4.0, 2.0, 1.0]
    zq = np.linspace(150.0, 400.0, 1201)
    exact = chapman(zq, 8.0, 300.0, 50.0)
    # analytic derivative of the Chapman profile
    z = (zq - 300.0) / 50.0
    dexact = exact * 0.5 * (np.exp(-z) - 1.0) / 50.0
    for dh in hs:
        n_h = int(round((450.0 - 100.0) / dh)) + 1
        g = GridGeom(4, 4, n_h, 29.0, 1.0, 109.0, 1.0, 100.0, dh)
        vals = np.broadcast_to(chapman(g.heights(), 8.0, 300.0, 50.0), (4, 4, n_h)).copy()
        med = orc.OracleMedium.from_grid(Grid(g, vals))
        ev = np.array([_eval_geo(orc, med, 30.0, 110.0, h) for h in zq])
        errs_v.append(np.abs(ev[:, 0] - exact).max() / exact.max())
        errs_g.append(np.abs(ev[:, 1] - dexact).max() / np.abs(dexact).max())
    ov = [math.log2(errs_v[i] / errs_v[i + 1]) for i in range(len(hs) - 1)]
    og = [math.log2(errs_g[i] / errs_g[i + 1]) for i in range(len(hs) - 1)]
    assert abs(ov[-1] - 3.0) < 0.15, ov
    assert abs(og[-1] - 2.0) < 0.15, og


def test_cr_basis_matches_printed_matrix(orc):
    """Catmull-Rom basis, eq. (cr_basis), and its interpolation property."""
    for t in np.linspace(0.0, 1.0, 11):
        w, dw = orc.cr_weights(t)
        ref = 0.5 * np.array([-t ** 3 + 2 * t ** 2 - t, 3 * t ** 3 - 5 * t ** 2 + 2,
                              -3 * t ** 3 + 4 * t ** 2 + t, t ** 3 - t ** 2])
        np.testing.assert_allclose(w, ref, atol=1e-15)
        assert abs(w.sum() - 1) < 1e-15 and abs(dw.sum()) < 1e-14
    w0, d0 = orc.cr_weights(0.0)
    np.testing.assert_allclose(w0, [0, 1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(d0, [-0.5, 0, 0.5, 0], atol=1e-15)
