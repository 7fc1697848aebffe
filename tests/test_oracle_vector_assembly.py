"""Pins of the oracle's Hamiltonian vector assembly (Sec. II-A, eq. appleton
and eq. hamiltonian) at real states, with |n| != 1.

or_hamiltonian builds Y_L^2 = (Y.n)^2 / n.n and Y_T^2 = Y^2 - Y_L^2 from the
dipole vector Y and the wave-normal vector n before it calls the scalar
Appleton-Hartree routine.  At a state where n is parallel or perpendicular
to Y the refractive index and G = omega dH/domega have textbook closed forms
in (X, |Y|, n.n) alone:

* n || Y (Theta = 0):  mu^2 = 1 - X/(1 + s Y) (s = +1 O, -1 X), and with
  X ~ omega^-2, Y ~ omega^-1, n ~ omega^-1 at fixed k and fixed Theta,
  G = -n.n - X/(1 + s Y) + (s/2) X Y/(1 + s Y)^2;
* n _|_ Y (Theta = 90 deg): O mode mu^2 = 1 - X, G = -n.n - X; X mode
  mu^2 = 1 - N/D with N = X(1-X), D = 1 - X - Y^2 and
  G = -n.n - X((1-2X)D + N)/D^2 - Y^2 N/D^2;
* in both, d(Y_L^2)/dn = 0, so dH/dn = n exactly.

The checks run on the oracle and on a copy of it built with one planted
slip (Y_L^2 without the division by n.n), which they must catch.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

R = 6371.0
B0 = 3.12e-5


def _states(orc, lib):
    """(med, y, mode, Y) at a few points inside a Chapman layer: n along or
    across the local dipole vector, |n| in {0.55, 1.3}."""
    med = orc.OracleMedium.chapman(8.0, 300.0, 50.0, floor_km=60.0)
    out = []
    for h, th_deg in ((240.0, 60.0), (290.0, 40.0), (330.0, 75.0)):
        r, th = R + h, math.radians(th_deg)
        Y = np.zeros(3)
        Yr, Yt = np.zeros(3), np.zeros(3)
        lib.or_dipole(B0, R, 9.0, r, th, Y.ctypes.data_as(orc._DP), Yr.ctypes.data_as(orc._DP),
                      Yt.ctypes.data_as(orc._DP))
        yhat = Y / np.linalg.norm(Y)
        perp = np.array([yhat[1], -yhat[0], 0.0])      # in the r-theta plane, across Y
        for kind, d in (("par", yhat), ("par", -yhat), ("perp", perp),
                        ("perp", np.array([0.0, 0.0, 1.0]))):
            for s in (0.55, 1.3):
                y = np.array([r, th, 0.3, *(s * d), 0.0])
                out.append((med, y, kind, np.linalg.norm(Y)))
    return out


def _ham(orc, lib, med, mode, y):
    h = orc.Ham()
    fld = orc.Field(B0)
    yy = np.ascontiguousarray(y[:6])
    ok = lib.or_hamiltonian(ctypes.byref(med.m), ctypes.byref(fld), R, 9.0, mode,
                            yy.ctypes.data_as(orc._DP), ctypes.byref(h))
    return h, bool(ok)


def _max_error(orc, lib):
    """Largest relative error of mu^2, G and dH/dn against the closed forms."""
    worst = 0.0
    for med, y, kind, Y in _states(orc, lib):
        n2 = float(y[3:6] @ y[3:6])
        for mode in (1, -1):
            h, ok = _ham(orc, lib, med, mode, y)
            assert ok
            X = h.X
            assert 0.2 < X < 0.9
            if kind == "par":
                mu2 = 1.0 - X / (1.0 + mode * Y)
                G = -n2 - X / (1.0 + mode * Y) + 0.5 * mode * X * Y / (1.0 + mode * Y) ** 2
            elif mode == 1:
                mu2, G = 1.0 - X, -n2 - X
            else:
                N, D = X * (1.0 - X), 1.0 - X - Y * Y
                mu2 = 1.0 - N / D
                G = -n2 - X * ((1.0 - 2.0 * X) * D + N) / D ** 2 - Y * Y * N / D ** 2
            worst = max(worst, abs(h.mu2 - mu2) / abs(mu2), abs(h.G - G) / abs(G),
                        float(np.abs(np.array(h.Hn[:]) - y[3:6]).max()) / math.sqrt(n2))
    return worst


def test_vector_assembly_matches_closed_forms(orc):
    assert _max_error(orc, orc.lib()) < 1e-13


def _mutant(tmp_path, orc):
    src = open(orc.SRC).read()
    good = "double b = Yn * Yn / n2;"
    assert src.count(good) == 1
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(good, "double b = Yn * Yn;"))
    lib = str(tmp_path / "libmutant.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-I",
                    os.path.dirname(orc.SRC), "-o", lib, str(path), "-lm"], check=True)
    L = ctypes.CDLL(lib)
    L.or_dipole.argtypes = [ctypes.c_double] * 5 + [orc._DP] * 3
    L.or_hamiltonian.argtypes = [ctypes.POINTER(orc.Medium), ctypes.POINTER(orc.Field),
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, orc._DP,
                                 ctypes.POINTER(orc.Ham)]
    L.or_hamiltonian.restype = ctypes.c_int
    return L


def test_planted_slip_in_vector_assembly_is_caught(orc, tmp_path):
    """Y_L^2 = (Y.n)^2 without / n.n: the same closed forms reject it."""
    assert _max_error(orc, _mutant(tmp_path, orc)) > 1e-3
