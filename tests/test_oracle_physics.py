"""Pins of the oracle's refractive index, field, Hamiltonian and ray equations.

Appleton-Hartree (Sec. II-A, eq. appleton): textbook special cases and the
partial derivatives against high-precision numerical differentiation of the
formula exactly as printed.  Dipole: |B| at equator and pole, zero
divergence and curl.  Hamiltonian partials: finite differences of H.  Ray
equations (eq. 1a-1f with the sin(theta) frame term in 1d): the identity
dH/dP' = 0 at arbitrary states, and |dx/dP'| = mu in isotropic media.
"""
import math

import mpmath as mp
import numpy as np
import pytest

R = 6371.0
KB = 2.799248983422872e10


def ah_printed(X, a, b, sigma):
    """mu^2 from eq. (appleton) as printed, in mpmath (a = Y_T^2, b = Y_L^2)."""
    X, a, b = mp.mpf(X), mp.mpf(a), mp.mpf(b)
    D = 2 * (1 - X) - a + sigma * mp.sqrt(a ** 2 + 4 * b * (1 - X) ** 2)
    return 1 - 2 * X * (1 - X) / D


@pytest.mark.parametrize("mode", [1, -1])
def test_appleton_no_field_limit(orc, mode):
    for X in (0.1, 0.5, 0.9):
        out, ok = orc.appleton(X, 1e-24, 1e-24, mode)   # Y ~ 1e-12
        assert ok and abs(out[0] - (1 - X)) < 1e-10


def test_appleton_transverse_and_longitudinal(orc):
    for X in (0.2, 0.6):
        for Y in (0.05, 0.3):
            o, _ = orc.appleton(X, Y * Y, 0.0, 1)      # theta = 90 deg
            x, _ = orc.appleton(X, Y * Y, 0.0, -1)
            assert abs(o[0] - (1 - X)) < 1e-14
            assert abs(x[0] - (1 - X * (1 - X) / (1 - X - Y * Y))) < 1e-13
            o, _ = orc.appleton(X, 0.0, Y * Y, 1)      # theta = 0
            x, _ = orc.appleton(X, 0.0, Y * Y, -1)
            assert abs(o[0] - (1 - X / (1 + Y))) < 1e-14
            assert abs(x[0] - (1 - X / (1 - Y))) < 1e-13


def test_appleton_reflection_points(orc):
    """Vertical-incidence reflection: O at X = 1, X mode at X = 1 - Y."""
    Y = 0.2
    for th in (0.3, 1.0):
        a, b = (Y * math.sin(th)) ** 2, (Y * math.cos(th)) ** 2
        o, _ = orc.appleton(1.0 - 1e-12, a, b, 1)
        assert abs(o[0]) < 1e-10
        x, _ = orc.appleton(1.0 - Y, a, b, -1)
        assert abs(x[0]) < 1e-12


@pytest.mark.parametrize("mode", [1, -1])
def test_appleton_matches_printed_formula_and_partials(orc, mode):
    mp.mp.dps = 40
    rng = np.random.default_rng(11 if mode > 0 else 12)
    for _ in range(60):
        X = rng.uniform(0.0, 0.95)
        Y = rng.uniform(0.02, 0.6)
        th = rng.uniform(0.05, math.pi - 0.05)
        a, b = (Y * math.sin(th)) ** 2, (Y * math.cos(th)) ** 2
        if mode < 0 and 1 - X - Y * Y < 0.05:      # stay off the X-mode resonance
            continue
        out, ok = orc.appleton(X, a, b, mode)
        assert ok
        ref = ah_printed(X, a, b, mode)
        dX = mp.diff(lambda v: ah_printed(v, a, b, mode), X)
        da = mp.diff(lambda v: ah_printed(X, v, b, mode), a)
        db = mp.diff(lambda v: ah_printed(X, a, v, mode), b)
        for got, want in zip(out, (ref, dX, da, db)):
            want = float(want)
            assert abs(got - want) <= 1e-11 * max(1.0, abs(want)), (X, Y, th, got, want)


def test_appleton_o_mode_no_cancellation_near_reflection(orc):
    mp.mp.dps = 60
    a, b = 0.01, 0.04
    for eps in (1e-4, 1e-8, 1e-12):
        X = 1.0 - eps
        out, _ = orc.appleton(X, a, b, 1)
        ref = float(ah_printed(X, a, b, 1))        # same binary X, 60 digits
        assert abs(out[0] - ref) <= 1e-13 * abs(ref)


def test_dipole_magnitude_and_direction(orc):
    B0, f = 3.12e-5, 10.0
    Y, _, _ = orc.dipole(B0, R, f, R, math.pi / 2)
    assert abs(np.linalg.norm(Y) * f * 1e6 / KB - B0) < 1e-18
    Y, _, _ = orc.dipole(B0, R, f, R, 0.0)
    assert abs(np.linalg.norm(Y) * f * 1e6 / KB - 2 * B0) < 1e-18
    Y, _, _ = orc.dipole(B0, R, f, R, math.radians(60.0))    # 30N
    assert Y[0] < 0 and Y[1] < 0      # points down and north (-theta-hat)
    # f_H(equator) = 0.8734 MHz, f_H(pole) = 1.7467 MHz
    assert abs(KB * B0 / 1e6 - 0.87337) < 1e-4


def test_dipole_divergence_and_curl_free(orc):
    B0, f = 3.12e-5, 10.0
    h = 1e-4

    def Yv(r, th):
        return orc.dipole(B0, R, f, r, th)[0]
    for r, th in ((R + 100, 1.0), (R + 400, 0.5), (R + 250, 2.0)):
        # div B = (1/r^2) d(r^2 B_r)/dr + (1/(r sin th)) d(sin th B_th)/dth
        d1 = ((r + h) ** 2 * Yv(r + h, th)[0] - (r - h) ** 2 * Yv(r - h, th)[0]) / (2 * h) / r ** 2
        d2 = (math.sin(th + h) * Yv(r, th + h)[1] - math.sin(th - h) * Yv(r, th - h)[1]) / (2 * h)
        d2 /= r * math.sin(th)
        scale = np.abs(Yv(r, th)).max() / r
        assert abs(d1 + d2) < 1e-7 * scale
        # curl_phi = (1/r)(d(r B_th)/dr - dB_r/dth)
        c1 = ((r + h) * Yv(r + h, th)[1] - (r - h) * Yv(r - h, th)[1]) / (2 * h)
        c2 = (Yv(r, th + h)[0] - Yv(r, th - h)[0]) / (2 * h)
        assert abs((c1 - c2) / r) < 1e-7 * scale
        # analytic derivatives
        _, Yr, Yt = orc.dipole(B0, R, f, r, th)
        np.testing.assert_allclose(Yr, (Yv(r + h, th) - Yv(r - h, th)) / (2 * h),
                                   atol=1e-9 * scale * r)
        np.testing.assert_allclose(Yt, (Yv(r, th + h) - Yv(r, th - h)) / (2 * h),
                                   atol=1e-9 * scale * r)


def _aniso_grid(seed=5):
    from paper_2506_18579_amd.synth import GridGeom, ionosphere_grid
    g = GridGeom(21, 21, 80, 25.0, 0.5, 105.0, 0.5, 60.0, 6.0)
    return ionosphere_grid(g, seed)


def _random_state(rng, f_mhz, grid, med, orc, mode, B0):
    """A state inside the grid with |n| on the mode's dispersion surface."""
    r = R + rng.uniform(150.0, 400.0)
    th = math.radians(90.0 - rng.uniform(27.0, 33.0))
    ph = math.radians(rng.uniform(107.0, 113.0))
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    y = np.array([r, th, ph, *d, 0.0])
    hm = orc.hamiltonian(med, B0, R, f_mhz, mode, y)
    if not hm["ok"] or hm["mu2"] <= 0.05:
        return None
    y[3:6] = d * math.sqrt(hm["mu2"])
    return y


@pytest.mark.parametrize("mode,B0", [(1, 3.12e-5), (-1, 3.12e-5), (1, 0.0)])
def test_hamiltonian_partials_by_finite_differences(orc, mode, B0):
    grid = _aniso_grid()
    med = orc.OracleMedium.from_grid(grid)
    rng = np.random.default_rng(21)
    f = 9.0
    done = 0
    while done < 20:
        y = _random_state(rng, f, grid, med, orc, mode, B0)
        if y is None:
            continue
        hm = orc.hamiltonian(med, B0, R, f, mode, y)

        def H(yy, ff=f):
            return orc.hamiltonian(med, B0, R, ff, mode, yy)["H"]
        for i in range(3):
            e = np.zeros(7)
            e[3 + i] = 1e-6
            fd = (H(y + e) - H(y - e)) / 2e-6
            assert abs(fd - hm["Hn"][i]) < 1e-7
        steps = (1e-4, 1e-7, 1e-7)
        for i in range(3):
            e = np.zeros(7)
            e[i] = steps[i]
            fd = (H(y + e) - H(y - e)) / (2 * steps[i])
            assert abs(fd - hm["Hq"][i]) < 1e-5 * max(1.0, abs(hm["Hq"][i])), (i, fd, hm["Hq"][i])
        # G = omega dH/domega at fixed k: n scales as 1/omega
        eps = 1e-6
        yp, ym = y.copy(), y.copy()
        yp[3:6] = y[3:6] / (1 + eps)
        ym[3:6] = y[3:6] / (1 - eps)
        G_fd = (H(yp, f * (1 + eps)) - H(ym, f * (1 - eps))) / (2 * eps)
        assert abs(G_fd - hm["G"]) < 1e-6 * abs(hm["G"]), (G_fd, hm["G"])
        done += 1


@pytest.mark.parametrize("mode,B0", [(1, 3.12e-5), (-1, 3.12e-5), (1, 0.0)])
def test_ray_equations_conserve_hamiltonian(orc, mode, B0):
    """dH/dP' = sum_q H_q dq/dP' + sum_i H_ni dn_i/dP' vanishes identically
    for eq. (1a)-(1f) with the sin(theta) factor in the k_r equation."""
    grid = _aniso_grid()
    med = orc.OracleMedium.from_grid(grid)
    rng = np.random.default_rng(5)
    f = 11.0
    done = 0
    while done < 30:
        y = _random_state(rng, f, grid, med, orc, mode, B0)
        if y is None:
            continue
        # off the dispersion surface too: the identity holds for any state
        y[3:6] *= rng.uniform(0.8, 1.2)
        hm = orc.hamiltonian(med, B0, R, f, mode, y)
        dy = orc.rhs(med, B0, R, f, mode, y)
        terms = np.concatenate([hm["Hq"] * dy[:3], hm["Hn"] * dy[3:6]])
        dH = terms.sum()
        assert abs(dH) <= 1e-13 * np.abs(terms).max(), (dH, terms)
        done += 1


def test_dropping_sin_theta_in_kr_equation_breaks_conservation(orc):
    """The paper's (1d) printed without sin(theta) gives dH/dP' != 0."""
    grid = _aniso_grid()
    med = orc.OracleMedium.from_grid(grid)
    rng = np.random.default_rng(9)
    y = None
    while y is None:
        y = _random_state(rng, 11.0, grid, med, orc, 1, 3.12e-5)
    y[5] = 0.3              # a sizeable n_phi
    hm = orc.hamiltonian(med, 3.12e-5, R, 11.0, 1, y)
    dy = orc.rhs(med, 3.12e-5, R, 11.0, 1, y)
    st = math.sin(y[1])
    dy_lit = dy.copy()
    dy_lit[3] = dy[3] - y[5] * st * dy[2] + y[5] * dy[2]
    terms = np.concatenate([hm["Hq"] * dy_lit[:3], hm["Hn"] * dy_lit[3:6]])
    # the correct equations cancel to ~1e-16 of the largest term; the
    # printed (1d) leaves a residual many orders of magnitude larger
    assert abs(terms.sum()) > 1e-6 * np.abs(terms).max()


def test_isotropic_group_speed_is_mu(orc):
    from paper_2506_18579_amd.synth import GridGeom, chapman_grid
    grid = chapman_grid(GridGeom(6, 6, 150, 25.0, 2.0, 105.0, 2.0, 60.0, 3.0))
    med = orc.OracleMedium.from_grid(grid)
    rng = np.random.default_rng(2)
    for _ in range(10):
        y = _random_state(rng, 10.0, grid, med, orc, 1, 0.0)
        if y is None:
            continue
        dy = orc.rhs(med, 0.0, R, 10.0, 1, y)
        speed = math.sqrt(dy[0] ** 2 + (y[0] * dy[1]) ** 2 + (y[0] * math.sin(y[1]) * dy[2]) ** 2)
        mu = math.sqrt(orc.hamiltonian(med, 0.0, R, 10.0, 1, y)["mu2"])
        assert abs(speed - mu) < 1e-13
        # phase-path rate = mu^2 / (group rate 1) in isotropic media
        assert abs(dy[6] - mu * mu) < 1e-13


@pytest.mark.parametrize("elev,az", [(1.0, 0.0), (15.0, 30.0), (45.0, -120.0), (89.0, 200.0)])
def test_launch_vacuum_segment_geometry(orc, elev, az):
    """Straight line from the ground at elevation beta0 to radius r_b:
    r_b cos(beta_b) = R cos(beta0) and central angle beta_b - beta0."""
    opts = orc.make_opts(R=R, tx=(30.0, 110.0, 0.0))
    y, s = orc.launch(opts, 60.0, elev, az)
    rb = R + 60.0
    assert abs(y[0] - rb) < 1e-9
    n = y[3:6]
    assert abs(np.linalg.norm(n) - 1.0) < 1e-14
    beta_b = math.acos(R * math.cos(math.radians(elev)) / rb)
    assert abs(math.asin(n[0]) - beta_b) < 1e-12
    la2 = math.pi / 2 - y[1]
    la1 = math.radians(30.0)
    dl = y[2] - math.radians(110.0)
    gam = math.acos(min(1.0, math.sin(la1) * math.sin(la2) +
                        math.cos(la1) * math.cos(la2) * math.cos(dl)))
    assert abs(gam - (beta_b - math.radians(elev))) < 1e-12
    assert abs(s - (rb * math.sin(beta_b) - R * math.sin(math.radians(elev)))) < 1e-9
    # horizontal direction of n keeps the launch azimuth (great-circle bearing at Tx)
    if elev < 89.0:
        bearing = math.degrees(math.atan2(y[5], -y[4]))
        # the local bearing at the end point differs from az by the
        # convergence of meridians; for small arcs it is close
        assert abs(((bearing - az + 180) % 360) - 180) < 6.0
