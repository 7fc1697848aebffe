"""The oracle's pins against planted mistakes (mutation check, CPU only).

Each mutant is the oracle's source with one plausible slip planted: a
dropped term, a wrong sign, factor or index, a transposed operand, a wrong
coefficient.  It is compiled like the oracle, and the oracle's pin tests
(closed forms, invariants, Appendix A, brute force, finite differences) run
against it in a subprocess.  They must fail: a mutant they pass would be a
mistake the pins cannot see.  The unmutated source, built the same way, must
pass them (the control).  The operation-count tests are left out: they
compare against a separate counting build of the unmutated source.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rtgd_oracle.c")
PIN_TESTS = ["tests/test_oracle_gd.py", "tests/test_oracle_physics.py", "tests/test_oracle_rays.py",
             "tests/test_oracle_vector_assembly.py"]

# (what the slip is, where it is in the method, text of the oracle, mutated text)
MUTANTS = [
    ("Y_L^2 without the division by n.n", "eq. hamiltonian",
     "double b = Yn * Yn / n2;", "double b = Yn * Yn;"),
    ("sign of the sin(theta) frame term of dn_r/dP'", "eq. 1d",
     "dy[3] = hm.Hq[0] / G + nth * thdot + nph * st * phdot;",
     "dy[3] = hm.Hq[0] / G + nth * thdot - nph * st * phdot;"),
    ("GD coefficient 11/12 read as 1/12", "Appendix A",
     "{0.0, -1.0 / 2.0, 11.0 / 12.0, -1.0 / 6.0, -5.0 / 12.0, 1.0 / 6.0}",
     "{0.0, -1.0 / 2.0, 1.0 / 12.0, -1.0 / 6.0, -5.0 / 12.0, 1.0 / 6.0}"),
    ("sign of the latitude -> colatitude derivative", "eq. 3dinterp_gd",
     "out[2] = -g_lat / (DEG * m->dlat_deg);", "out[2] = g_lat / (DEG * m->dlat_deg);"),
    ("O and X modes swapped", "eq. appleton",
     "if (mode > 0) {", "if (mode < 0) {"),
    ("dipole radial component without the factor 2", "Sec. II-C, dipole",
     "Y[0] = -2.0 * Y0 * q3 * ct;", "Y[0] = -Y0 * q3 * ct;"),
    ("last cell clamped one node early", "Sec. II-B, cell location",
     "if (k > n - 3) k = n - 3;", "if (k > n - 4) k = n - 4;"),
    ("phase path without its phi term", "Sec. II-C outputs",
     "dy[6] = nr * rdot + nth * r * thdot + nph * r * st * phdot;",
     "dy[6] = nr * rdot + nth * r * thdot;"),
    ("latitude and longitude weights transposed", "eq. 3dinterp_gd",
     "v += u * wl[a] * wo[b] * wh[c];", "v += u * wo[a] * wl[b] * wh[c];"),
    ("sign of dH/dtheta", "eq. hamiltonian",
     "out->Hq[1] = -0.5 * (mX * Xq[1] + mY2 * dY2 + mb * db);",
     "out->Hq[1] = 0.5 * (mX * Xq[1] + mY2 * dY2 + mb * db);"),
    ("sign of dY_r/dtheta", "Sec. II-C, dipole",
     "dYdth[0] = 2.0 * Y0 * q3 * st;", "dYdth[0] = -2.0 * Y0 * q3 * st;"),
    ("sign of the second term of d(Y_L^2)/dn", "eq. hamiltonian",
     "double dbdn = 2.0 * Yn * Y[i] / n2 - 2.0 * Yn * Yn * n[i] / (n2 * n2);",
     "double dbdn = 2.0 * Yn * Y[i] / n2 + 2.0 * Yn * Yn * n[i] / (n2 * n2);"),
    ("G without its Y_L^2 term", "eq. hamiltonian",
     "out->G = -n2 + X * mX + Y2 * mY2 + b * mb;", "out->G = -n2 + X * mX + Y2 * mY2;"),
    ("height derivative multiplied by the spacing", "eq. 3dinterp_gd",
     "out[1] = g_h / m->dh_km;", "out[1] = g_h * m->dh_km;"),
    ("phase path without the landing chord", "Sec. II-C outputs",
     "            y[6] += s;\n            y[0] = sqrt(dot3(x, x));",
     "            y[0] = sqrt(dot3(x, x));"),
    ("sign of the Chapman layer's gradient", "analytic test medium",
     "out[1] = ne * 0.5 * (ez - 1.0) / m->thick_km;", "out[1] = ne * 0.5 * (1.0 - ez) / m->thick_km;"),
    ("QP layer gradient without its 1/r term", "analytic test medium",
     "out[1] = -Nm * (2.0 * q * p * p / ym - 2.0 * q * q * p * p / r);",
     "out[1] = -Nm * (2.0 * q * p * p / ym);"),
    ("RK4 fourth stage taken at half the step", "Sec. II-C, RK4",
     "for (int i = 0; i < 7; ++i) t[i] = y[i] + h * k3[i];",
     "for (int i = 0; i < 7; ++i) t[i] = y[i] + 0.5 * h * k3[i];"),
    ("RK4 combination without the weight of k3", "Sec. II-C, RK4",
     "y[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);",
     "y[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + k3[i] + k4[i]);"),
    ("azimuth counted counterclockwise", "Sec. II-C, launch",
     "d[i] = sin(be) * up[i] + cos(be) * (cos(al) * north[i] + sin(al) * east[i]);",
     "d[i] = sin(be) * up[i] + cos(be) * (cos(al) * north[i] - sin(al) * east[i]);"),
    ("sign of the n_theta dr/dP' term of dn_theta/dP'", "eq. 1e",
     "dy[4] = (hm.Hq[1] / G - nth * rdot + nph * r * ct * phdot) / r;",
     "dy[4] = (hm.Hq[1] / G + nth * rdot + nph * r * ct * phdot) / r;"),
    ("dn_phi/dP' divided by r only", "eq. 1f",
     "dy[5] = (hm.Hq[2] / G - nph * st * rdot - nph * r * ct * thdot) / (r * st);",
     "dy[5] = (hm.Hq[2] / G - nph * st * rdot - nph * r * ct * thdot) / r;"),
    ("d mu^2/d Y_L^2 taken at fixed Y_T^2 instead of fixed Y^2", "eq. hamiltonian",
     "double mb = ah[3] - ah[2];", "double mb = ah[3];"),
    ("dH/dn with mu2_b instead of mu2_b / 2", "eq. hamiltonian",
     "out->Hn[i] = n[i] - 0.5 * mb * dbdn;", "out->Hn[i] = n[i] - mb * dbdn;"),
    ("azimuth deviation with its sign reversed", "Sec. II-C outputs",
     "double x = bear - az;", "double x = az - bear;"),
    ("GD derivative coefficients without the power factor", "Appendix A",
     "if (k < 5) d += (k + 1) * GD_COEF[a][k + 1] * p;", "if (k < 5) d += GD_COEF[a][k + 1] * p;"),
    ("Catmull-Rom weight of node 0 with -4 t^2", "eq. cr_basis",
     "w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);", "w[1] = 0.5 * (3.0 * t3 - 4.0 * t2 + 2.0);"),
    ("latitude derivative kept outside the box", "Sec. II-B, box edges",
     "if (c_lat) g_lat = 0.0;", "if (c_lat) g_lat = g_lat;"),
    ("landing chord root with the wrong sign", "Sec. II-C, landing",
     "s = c / (-xd + sqrt(disc));", "s = c / (xd + sqrt(disc));"),
    ("apogee never updated", "Sec. II-C outputs",
     "if (status != OR_NUMERIC && h > apogee) apogee = h;", "if (status != OR_NUMERIC && h > 1e300) apogee = h;"),
    ("O-mode E with b u^2 for b u", "eq. appleton",
     "double E = 1.0 + 2.0 * b * u / T;", "double E = 1.0 + 2.0 * b * u * u / T;"),
    ("X-mode dD/db with the wrong sign", "eq. appleton",
     "double Db = -2.0 * u * u / S;", "double Db = 2.0 * u * u / S;"),
    ("d(Y^2)/dr without the factor 2", "eq. hamiltonian",
     "double dY2 = 2.0 * (Y[0] * Yr[0] + Y[1] * Yr[1] + Y[2] * Yr[2]);",
     "double dY2 = (Y[0] * Yr[0] + Y[1] * Yr[1] + Y[2] * Yr[2]);"),
    ("dtheta/dP' without the division by r", "eq. 1b",
     "double thdot = -hm.Hn[1] / (r * G);", "double thdot = -hm.Hn[1] / G;"),
    ("launch chord root taken as the negative one", "Sec. II-C, launch",
     "double s = c / (p + sqrt(p * p + c));", "double s = -(p + sqrt(p * p + c));"),
    ("longitude derivative with the latitude spacing", "eq. 3dinterp_gd",
     "out[3] = g_lon / (DEG * m->dlon_deg);", "out[3] = g_lon / (DEG * m->dlat_deg);"),
    ("ground range on the sphere of the grid bottom", "Sec. II-C outputs",
     "out[2] = R * gam;", "out[2] = (R + hb) * gam;"),
    ("landing latitude as the colatitude", "Sec. II-C outputs",
     "out[5] = 90.0 - y[1] / DEG;", "out[5] = y[1] / DEG;"),
    ("launch chord with cos(elevation)", "Sec. II-C, launch",
     "double p = r0 * sin(be);", "double p = r0 * cos(be);"),
    ("GD coefficient 5/12 of psi_-2 read as 7/12", "Appendix A",
     "/* a = +2 : psi_-2 */ {0.0, 0.0, -5.0 / 12.0, 1.0 / 6.0, 5.0 / 12.0, -1.0 / 6.0},",
     "/* a = +2 : psi_-2 */ {0.0, 0.0, -5.0 / 12.0, 1.0 / 6.0, 7.0 / 12.0, -1.0 / 6.0},"),
    ("X-mode denominator with +S", "eq. appleton",
     "double D = 2.0 * u - T;", "double D = 2.0 * u - a + S;"),
    ("sign of dH/dphi", "eq. hamiltonian",
     "out->Hq[2] = -0.5 * mX * Xq[2];", "out->Hq[2] = 0.5 * mX * Xq[2];"),
    ("X = f_N^2 / f instead of f_N^2 / f^2", "eq. appleton",
     "double xs = KN / (fhz * fhz);", "double xs = KN / (fhz * 1e6);"),
    ("grazing chord followed back to the ground, not to the grid bottom", "Sec. II-C, landing",
     "double rb = R + hb;", "double rb = R;"),
    ("dphi/dP' without sin(theta)", "eq. 1c",
     "double phdot = -hm.Hn[2] / (r * st * G);", "double phdot = -hm.Hn[2] / (r * G);"),
    ("O-mode dE/dX without its 4 b u^2 / S term", "eq. appleton",
     "double EX = 2.0 * b * (-T + 4.0 * b * u * u / S) / (T * T);", "double EX = 2.0 * b * (-T) / (T * T);"),
    ("X-mode dmu^2/dX with 1 - X for 1 - 2X", "eq. appleton",
     "out[1] = -(2.0 * (1.0 - 2.0 * X) * D - N * DX) / (D * D);",
     "out[1] = -(2.0 * (1.0 - X) * D - N * DX) / (D * D);"),
    ("gyrofrequency ratio with f in MHz", "eq. appleton, Y",
     "double Y0 = KB * B0_T / (f_mhz * 1e6);", "double Y0 = KB * B0_T / (f_mhz * 1e5);"),
    ("Chapman height variable without the scale height", "analytic test medium",
     "double z = (h - m->hm_km) / m->thick_km;", "double z = (h - m->hm_km) / (2.0 * m->thick_km);"),
    ("RK4 third stage from y + h k2", "Sec. II-C, RK4",
     "for (int i = 0; i < 7; ++i) t[i] = y[i] + 0.5 * h * k2[i];",
     "for (int i = 0; i < 7; ++i) t[i] = y[i] + h * k2[i];"),
    ("local coordinate measured from the next node", "Sec. II-B, cell location",
     "*s = t - (double)k;", "*s = t - (double)(k + 1);"),
    ("dY_theta/dtheta with the sign of Y_theta", "Sec. II-C, dipole",
     "dYdth[1] = -Y0 * q3 * ct;", "dYdth[1] = Y0 * q3 * ct;"),
]


def _build(src_text, tag, d):
    c = os.path.join(d, f"{tag}.c")
    so = os.path.join(d, f"{tag}.so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-I", os.path.dirname(SRC), "-o", so, c, "-lm"],
                   check=True, capture_output=True)
    return so


def _pins(so):
    env = dict(os.environ, RTGD_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *PIN_TESTS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("mutants"))
    with open(SRC) as f:
        src = f.read()
    jobs = [("control", src)]
    for k, (_, _, a, b) in enumerate(MUTANTS):
        assert src.count(a) == 1, MUTANTS[k][0]
        jobs.append((f"m{k:02d}", src.replace(a, b)))
    sos = [_build(text, tag, d) for tag, text in jobs]
    with ThreadPoolExecutor(max_workers=4) as ex:
        return list(ex.map(_pins, sos))


def test_control_passes_the_pins(outcomes):
    code, out = outcomes[0]
    assert code == 0, out


@pytest.mark.parametrize("k", range(len(MUTANTS)), ids=[f"m{k:02d}" for k in range(len(MUTANTS))])
def test_pins_catch_the_mutant(outcomes, k):
    code, out = outcomes[k + 1]
    what, where, _, _ = MUTANTS[k]
    # 1: a pin failed; a negative code: the mutant crashed the process
    assert code == 1 or code < 0, f"the pins pass with a planted mistake: {what} ({where})\n{out}"
