/*
 * rtgd_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Straight scalar C, compiled without fast-math and without FMA contraction.
 * Each function states the passage of the paper it follows.  No blocking,
 * fusion or reordering beyond what the definitions state.  Rays are
 * independent; OpenMP only distributes whole rays over threads.
 *
 * Pins (tests/test_oracle_*.py, tests/test_ionogram.py): every function is
 * checked against closed forms, high-precision quadrature, invariants or
 * finite differences.  Anisotropic whole rays have no closed form and the
 * paper prints no worked example for them: they are pinned by invariants
 * only (H = 0 along the ray, O = X as the field vanishes, the partials
 * against finite differences of H).
 */
#include "rtgd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define DEG (OR_PI / 180.0)

/* CODATA 2022: f_N^2 = KN * N_e (Hz^2, N_e in m^-3), f_H = KB * |B| (Hz, T). */
static const double KN = 80.61638587963628;
static const double KB = 2.799248983422872e10;

/* ------------------------------------------------------------------------
 * 1-D GD p = 3 basis (Appendix A).  The appendix gives the global basis of
 * one node as four quintic pieces psi_k, k = -2..1, each written in its own
 * local variable (xi - k) in [0, 1].  For a point at local coordinate
 * s in [0, 1) of cell [x_j, x_j+1], node j+a contributes psi_{-a} evaluated
 * at local variable s.  Row a below is therefore the coefficient list of
 * psi_{-a} (powers s^0 .. s^5) exactly as printed in Appendix A.
 * ---------------------------------------------------------------------- */
static const double GD_COEF[4][6] = {
    /* a = -1 : psi_1  */ {0.0, -1.0 / 2.0, 11.0 / 12.0, -1.0 / 6.0, -5.0 / 12.0, 1.0 / 6.0},
    /* a =  0 : psi_0  */ {1.0, 0.0, -9.0 / 4.0, 1.0 / 2.0, 5.0 / 4.0, -1.0 / 2.0},
    /* a = +1 : psi_-1 */ {0.0, 1.0 / 2.0, 7.0 / 4.0, -1.0 / 2.0, -5.0 / 4.0, 1.0 / 2.0},
    /* a = +2 : psi_-2 */ {0.0, 0.0, -5.0 / 12.0, 1.0 / 6.0, 5.0 / 12.0, -1.0 / 6.0},
};

void or_gd_weights(double s, double w[4], double dw[4])
{
    for (int a = 0; a < 4; ++a) {
        double v = 0.0, d = 0.0, p = 1.0;
        for (int k = 0; k <= 5; ++k) {
            v += GD_COEF[a][k] * p;               /* c_k s^k          */
            if (k < 5) d += (k + 1) * GD_COEF[a][k + 1] * p; /* (k+1) c_{k+1} s^k */
            p *= s;
        }
        w[a] = v;
        dw[a] = d;
    }
}

/* Catmull-Rom cubic basis, eq. (cr_basis): node offsets -1, 0, 1, 2. */
void or_cr_weights(double t, double w[4], double dw[4])
{
    double t2 = t * t, t3 = t2 * t;
    w[0] = 0.5 * (-t3 + 2.0 * t2 - t);
    w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
    w[2] = 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
    w[3] = 0.5 * (t3 - t2);
    dw[0] = 0.5 * (-3.0 * t2 + 4.0 * t - 1.0);
    dw[1] = 0.5 * (9.0 * t2 - 10.0 * t);
    dw[2] = 0.5 * (-9.0 * t2 + 8.0 * t + 1.0);
    dw[3] = 0.5 * (3.0 * t2 - 2.0 * t);
}

/* Locate one axis: t = (c - c0)/dc, cell i = clamp(floor(t), 1, n-3),
 * s = t - i.  The clamp keeps the 4-node stencil i-1..i+2 inside the grid;
 * near the first/last node s runs over [-1, 0) or [1, 2] of the edge cell's
 * polynomial, which still interpolates those nodes. */
static void locate(double c, double c0, double dc, int n, int *i, double *s)
{
    double t = (c - c0) / dc;
    double f = floor(t);
    int k = (int)f;
    if (k < 1) k = 1;
    if (k > n - 3) k = n - 3;
    *i = k;
    *s = t - (double)k;
}

/* Clamp a coordinate into [lo, hi]; returns 1 if it was outside (the
 * derivative along a clamped axis is zero: constant continuation). */
static int clampc(double *c, double lo, double hi)
{
    if (*c < lo) { *c = lo; return 1; }
    if (*c > hi) { *c = hi; return 1; }
    return 0;
}

/* Tensor-product interpolation, eq. (3dinterp_gd) (or (3dinterp_cr) for
 * the CR kind): value and the three index-space partials. */
static void grid_eval(const or_medium *m, double R, double r, double th,
                      double ph, double out[4])
{
    double h = r - R;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (h < m->h0_km) return;                 /* vacuum below the grid */

    double lat = 90.0 - th / DEG;
    double lon = ph / DEG;
    double lat_hi = m->lat0_deg + (m->n_lat - 1) * m->dlat_deg;
    double lon_hi = m->lon0_deg + (m->n_lon - 1) * m->dlon_deg;
    double h_hi = m->h0_km + (m->n_h - 1) * m->dh_km;
    int c_lat = clampc(&lat, m->lat0_deg, lat_hi);
    int c_lon = clampc(&lon, m->lon0_deg, lon_hi);
    int c_h = clampc(&h, m->h0_km, h_hi);

    int il, jl, kh;
    double sl, so, sh;
    locate(lat, m->lat0_deg, m->dlat_deg, m->n_lat, &il, &sl);
    locate(lon, m->lon0_deg, m->dlon_deg, m->n_lon, &jl, &so);
    locate(h, m->h0_km, m->dh_km, m->n_h, &kh, &sh);

    double wl[4], dwl[4], wo[4], dwo[4], wh[4], dwh[4];
    if (m->kind == OR_GRID_CR) {
        or_cr_weights(sl, wl, dwl);
        or_cr_weights(so, wo, dwo);
        or_cr_weights(sh, wh, dwh);
    } else {
        or_gd_weights(sl, wl, dwl);
        or_gd_weights(so, wo, dwo);
        or_gd_weights(sh, wh, dwh);
    }

    double v = 0.0, g_lat = 0.0, g_lon = 0.0, g_h = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                long idx = ((long)(il - 1 + a) * m->n_lon + (jl - 1 + b)) * m->n_h + (kh - 1 + c);
                double u = m->ne[idx];
                v += u * wl[a] * wo[b] * wh[c];
                g_lat += u * dwl[a] * wo[b] * wh[c];
                g_lon += u * wl[a] * dwo[b] * wh[c];
                g_h += u * wl[a] * wo[b] * dwh[c];
            }
    if (c_lat) g_lat = 0.0;
    if (c_lon) g_lon = 0.0;
    if (c_h) g_h = 0.0;

    /* index-space -> physical partials: t_h = (r - R - h0)/dh,
     * t_lat = (90 - theta/DEG - lat0)/dlat, t_lon = (phi/DEG - lon0)/dlon */
    out[0] = v;
    out[1] = g_h / m->dh_km;
    out[2] = -g_lat / (DEG * m->dlat_deg);
    out[3] = g_lon / (DEG * m->dlon_deg);
}

/* Analytic alpha-Chapman layer (synthetic stand-in for gridded models):
 * N_e = Nm exp(0.5 (1 - z - exp(-z))), z = (h - hm)/H, Nm from fc. */
static void chapman_eval(const or_medium *m, double R, double r, double out[4])
{
    double h = r - R;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (h < m->floor_km) return;
    double fc = m->fc_mhz * 1e6;
    double Nm = fc * fc / KN;
    double z = (h - m->hm_km) / m->thick_km;
    double ez = exp(-z);
    double ne = Nm * exp(0.5 * (1.0 - z - ez));
    out[0] = ne;
    out[1] = ne * 0.5 * (ez - 1.0) / m->thick_km;
}

/* Analytic quasi-parabolic layer: N_e = Nm [1 - ((r - rm)/ym)^2 (rb/r)^2]
 * for rb < r < rm rb/(rb - ym), rb = rm - ym, zero elsewhere. */
static void qp_eval(const or_medium *m, double R, double r, double out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    double rm = R + m->hm_km, ym = m->thick_km, rb = rm - ym;
    double rt = rm * rb / (rb - ym);
    if (r <= rb || r >= rt) return;
    double fc = m->fc_mhz * 1e6;
    double Nm = fc * fc / KN;
    double q = (r - rm) / ym, p = rb / r;
    out[0] = Nm * (1.0 - q * q * p * p);
    /* d/dr of q^2 p^2 = 2 q p^2 / ym - 2 q^2 p^2 / r */
    out[1] = -Nm * (2.0 * q * p * p / ym - 2.0 * q * q * p * p / r);
}

void or_medium_eval(const or_medium *m, double R_km, double r, double th,
                    double ph, double out[4])
{
    switch (m->kind) {
    case OR_CHAPMAN: chapman_eval(m, R_km, r, out); break;
    case OR_QP: qp_eval(m, R_km, r, out); break;
    default: grid_eval(m, R_km, r, th, ph, out); break;
    }
}

/* Axial centred dipole: B_r = -2 B0 (R/r)^3 cos(th), B_th = -B0 (R/r)^3
 * sin(th), B_ph = 0 (field points down in the northern hemisphere).
 * Y = f_H / f = KB B / f, per component. */
void or_dipole(double B0_T, double R_km, double f_mhz, double r, double th,
               double Y[3], double dYdr[3], double dYdth[3])
{
    double Y0 = KB * B0_T / (f_mhz * 1e6);
    double q = R_km / r;
    double q3 = q * q * q;
    double st = sin(th), ct = cos(th);
    Y[0] = -2.0 * Y0 * q3 * ct;
    Y[1] = -Y0 * q3 * st;
    Y[2] = 0.0;
    for (int i = 0; i < 3; ++i) dYdr[i] = -3.0 * Y[i] / r;
    dYdth[0] = 2.0 * Y0 * q3 * st;
    dYdth[1] = -Y0 * q3 * ct;
    dYdth[2] = 0.0;
}

/* Appleton-Hartree, eq. (appleton): mu^2 = 1 - 2X(1-X)/D,
 * D = 2(1-X) - a + sigma sqrt(a^2 + 4 b (1-X)^2), a = Y_T^2, b = Y_L^2,
 * sigma = +1 (O), -1 (X).  out = {mu^2, dmu2/dX, dmu2/da, dmu2/db} with
 * X, a, b independent.
 *
 * O mode: S - a = 4 b (1-X)^2 / (S + a), so D = 2(1-X) E with
 * E = 1 + 2 b (1-X)/(S + a); the common factor 1-X cancels and
 * mu^2 = 1 - X/E = (1-X)(T + 2b)/(T + 2b(1-X)), T = S + a: the same value,
 * with no cancellation as X -> 1 or mu^2 -> 0 (reflection).
 * X mode: D used as printed. */
int or_appleton(double X, double a, double b, int mode, double out[4])
{
    double u = 1.0 - X;
    double S = sqrt(a * a + 4.0 * b * u * u);
    double T = S + a;
    if (mode > 0) {
        double E = 1.0 + 2.0 * b * u / T;
        double EX = 2.0 * b * (-T + 4.0 * b * u * u / S) / (T * T);
        double Ea = -2.0 * b * u / (S * T);
        double Eb = 2.0 * u / T - 4.0 * b * u * u * u / (S * T * T);
        out[0] = u * (T + 2.0 * b) / (T + 2.0 * b * u);
        out[1] = -1.0 / E + X * EX / (E * E);
        out[2] = X * Ea / (E * E);
        out[3] = X * Eb / (E * E);
    } else {
        double D = 2.0 * u - T;
        double N = 2.0 * X * u;
        double DX = -2.0 + 4.0 * b * u / S;
        double Da = -T / S;
        double Db = -2.0 * u * u / S;
        out[0] = 1.0 - N / D;
        out[1] = -(2.0 * (1.0 - 2.0 * X) * D - N * DX) / (D * D);
        out[2] = N * Da / (D * D);
        out[3] = N * Db / (D * D);
    }
    return isfinite(out[0]) && isfinite(out[1]) && isfinite(out[2]) && isfinite(out[3]);
}

/* H = 0.5 (n.n - mu^2), eq. (hamiltonian) with n = c k / omega.
 * Independent variables of mu^2: X, Y^2 = Y.Y and b = (Y.n)^2 / n.n.
 *   G = omega dH/domega |k = -n.n + X mu2_X + Y^2 mu2_Y2 + b mu2_b
 *   (X ~ omega^-2, Y ~ omega^-1, n ~ omega^-1 at fixed k)
 *   dH/dn = n - 0.5 mu2_b db/dn
 *   dH/dq = -0.5 (mu2_X dX/dq + mu2_Y2 dY^2/dq + mu2_b db/dq), local n fixed.
 * Without a field mu^2 = 1 - X exactly. */
int or_hamiltonian(const or_medium *m, const or_field *fld, double R_km,
                   double f_mhz, int mode, const double y[6], or_ham *out)
{
    double r = y[0], th = y[1], ph = y[2];
    const double *n = y + 3;
    double ne[4];
    or_medium_eval(m, R_km, r, th, ph, ne);
    double fhz = f_mhz * 1e6;
    double xs = KN / (fhz * fhz);
    double X = ne[0] * xs;
    double Xq[3] = {ne[1] * xs, ne[2] * xs, ne[3] * xs};
    double n2 = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];

    if (fld == NULL || fld->B0_T == 0.0) {
        out->X = X;
        out->mu2 = 1.0 - X;
        out->H = 0.5 * (n2 - out->mu2);
        out->G = -n2 - X;                  /* mu2_X = -1 */
        for (int i = 0; i < 3; ++i) {
            out->Hn[i] = n[i];
            out->Hq[i] = 0.5 * Xq[i];
        }
        return isfinite(out->H) && isfinite(out->G);
    }

    double Y[3], Yr[3], Yth[3];
    or_dipole(fld->B0_T, R_km, f_mhz, r, th, Y, Yr, Yth);
    double Y2 = Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2];
    double Yn = Y[0] * n[0] + Y[1] * n[1] + Y[2] * n[2];
    double b = Yn * Yn / n2;
    double a = Y2 - b;
    double ah[4];
    int ok = or_appleton(X, a, b, mode, ah);
    double mu2 = ah[0], mX = ah[1];
    double mY2 = ah[2];              /* d/dY^2 at fixed b  = d/da        */
    double mb = ah[3] - ah[2];       /* d/db at fixed Y^2 = d/db - d/da  */

    out->X = X;
    out->mu2 = mu2;
    out->H = 0.5 * (n2 - mu2);
    out->G = -n2 + X * mX + Y2 * mY2 + b * mb;
    for (int i = 0; i < 3; ++i) {
        double dbdn = 2.0 * Yn * Y[i] / n2 - 2.0 * Yn * Yn * n[i] / (n2 * n2);
        out->Hn[i] = n[i] - 0.5 * mb * dbdn;
    }
    /* q = r */
    {
        double dY2 = 2.0 * (Y[0] * Yr[0] + Y[1] * Yr[1] + Y[2] * Yr[2]);
        double db = 2.0 * Yn * (Yr[0] * n[0] + Yr[1] * n[1] + Yr[2] * n[2]) / n2;
        out->Hq[0] = -0.5 * (mX * Xq[0] + mY2 * dY2 + mb * db);
    }
    /* q = theta */
    {
        double dY2 = 2.0 * (Y[0] * Yth[0] + Y[1] * Yth[1] + Y[2] * Yth[2]);
        double db = 2.0 * Yn * (Yth[0] * n[0] + Yth[1] * n[1] + Yth[2] * n[2]) / n2;
        out->Hq[1] = -0.5 * (mX * Xq[1] + mY2 * dY2 + mb * db);
    }
    /* q = phi: the axial dipole does not depend on phi */
    out->Hq[2] = -0.5 * mX * Xq[2];
    return ok && isfinite(out->H) && isfinite(out->G);
}

/* Ray equations, Sec. II-A eq. (1a)-(1f), divided through by omega/c
 * (n = c k / omega) so that with G = omega dH/domega:
 *   dr/dP'   = -H_nr / G
 *   dth/dP'  = -H_nth / (r G)
 *   dph/dP'  = -H_nph / (r sin th G)
 *   dn_r/dP' =  H_r / G + n_th dth/dP' + n_ph sin th dph/dP'
 *   dn_th/dP'= (H_th / G - n_th dr/dP' + n_ph r cos th dph/dP') / r
 *   dn_ph/dP'= (H_ph / G - n_ph sin th dr/dP' - n_ph r cos th dth/dP') / (r sin th)
 * plus the phase path dP/dP' = n . dx/dP'. */
int or_rhs(const or_medium *m, const or_field *fld, double R_km,
           double f_mhz, int mode, const double y[7], double dy[7])
{
    or_ham hm;
    int ok = or_hamiltonian(m, fld, R_km, f_mhz, mode, y, &hm);
    double r = y[0], th = y[1];
    double nr = y[3], nth = y[4], nph = y[5];
    double st = sin(th), ct = cos(th);
    double G = hm.G;
    double rdot = -hm.Hn[0] / G;
    double thdot = -hm.Hn[1] / (r * G);
    double phdot = -hm.Hn[2] / (r * st * G);
    dy[0] = rdot;
    dy[1] = thdot;
    dy[2] = phdot;
    dy[3] = hm.Hq[0] / G + nth * thdot + nph * st * phdot;
    dy[4] = (hm.Hq[1] / G - nth * rdot + nph * r * ct * phdot) / r;
    dy[5] = (hm.Hq[2] / G - nph * st * rdot - nph * r * ct * thdot) / (r * st);
    dy[6] = nr * rdot + nth * r * thdot + nph * r * st * phdot;
    return ok;
}

/* ------------------------------------------------------------------------
 * Geometry helpers (spherical Earth, Cartesian frame with z to the north
 * pole and x through longitude 0).
 * ---------------------------------------------------------------------- */
static void sph_basis(double th, double ph, double rh[3], double thh[3], double phh[3])
{
    double st = sin(th), ct = cos(th), sp = sin(ph), cp = cos(ph);
    rh[0] = st * cp; rh[1] = st * sp; rh[2] = ct;
    thh[0] = ct * cp; thh[1] = ct * sp; thh[2] = -st;
    phh[0] = -sp; phh[1] = cp; phh[2] = 0.0;
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Longitude (rad) of Cartesian point, unwrapped to within pi of ref. */
static double lon_near(double x, double y, double ref)
{
    double p = atan2(y, x);
    return p + 2.0 * OR_PI * floor((ref - p) / (2.0 * OR_PI) + 0.5);
}

/* Cartesian point -> spherical state; direction d (Cartesian) -> local
 * wave-normal components scaled by nmag. */
static void cart_to_state(const double x[3], const double d[3], double nmag,
                          double ref_lon, double y[6])
{
    double r = sqrt(dot3(x, x));
    double th = atan2(sqrt(x[0] * x[0] + x[1] * x[1]), x[2]);
    double ph = lon_near(x[0], x[1], ref_lon);
    double rh[3], thh[3], phh[3];
    sph_basis(th, ph, rh, thh, phh);
    y[0] = r; y[1] = th; y[2] = ph;
    y[3] = nmag * dot3(d, rh);
    y[4] = nmag * dot3(d, thh);
    y[5] = nmag * dot3(d, phh);
}

static void state_to_cart(const double y[6], double x[3], double d[3])
{
    double rh[3], thh[3], phh[3];
    sph_basis(y[1], y[2], rh, thh, phh);
    double nm = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
    for (int i = 0; i < 3; ++i) {
        x[i] = y[0] * rh[i];
        d[i] = (y[3] * rh[i] + y[4] * thh[i] + y[5] * phh[i]) / nm;
    }
}

/* Ray initialisation (Sec. II-C): from the transmitter at (lat, lon, h)
 * with elevation beta and azimuth alpha (clockwise from north) the ray
 * runs as a straight line through the N_e-free region to the height
 * floor_km, where the state is handed to the integrator with |n| = 1. */
double or_launch(const or_opts *o, double floor_km, double elev_deg,
                 double az_deg, double y[7])
{
    double R = o->R_km;
    double la = o->tx_lat_deg * DEG, lo = o->tx_lon_deg * DEG;
    double be = elev_deg * DEG, al = az_deg * DEG;
    double up[3] = {cos(la) * cos(lo), cos(la) * sin(lo), sin(la)};
    double north[3] = {-sin(la) * cos(lo), -sin(la) * sin(lo), cos(la)};
    double east[3] = {-sin(lo), cos(lo), 0.0};
    double r0 = R + o->tx_h_km, rb = R + floor_km;
    double d[3], x[3];
    for (int i = 0; i < 3; ++i)
        d[i] = sin(be) * up[i] + cos(be) * (cos(al) * north[i] + sin(al) * east[i]);
    /* |x0 + s d| = rb, x0.d = r0 sin(beta); positive root in the form
     * without cancellation */
    double p = r0 * sin(be);
    double c = rb * rb - r0 * r0;
    double s = c / (p + sqrt(p * p + c));
    for (int i = 0; i < 3; ++i) x[i] = r0 * up[i] + s * d[i];
    cart_to_state(x, d, 1.0, lo, y);
    y[6] = s;
    return s;
}

/* One fixed RK4 step of size h on the 7-component state. */
static int rk4(const or_medium *m, const or_field *fld, double R, double f,
               int mode, double y[7], double h)
{
    double k1[7], k2[7], k3[7], k4[7], t[7];
    int ok = or_rhs(m, fld, R, f, mode, y, k1);
    for (int i = 0; i < 7; ++i) t[i] = y[i] + 0.5 * h * k1[i];
    ok &= or_rhs(m, fld, R, f, mode, t, k2);
    for (int i = 0; i < 7; ++i) t[i] = y[i] + 0.5 * h * k2[i];
    ok &= or_rhs(m, fld, R, f, mode, t, k3);
    for (int i = 0; i < 7; ++i) t[i] = y[i] + h * k3[i];
    ok &= or_rhs(m, fld, R, f, mode, t, k4);
    for (int i = 0; i < 7; ++i)
        y[i] = y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    return ok;
}

static int all_finite(const double y[7])
{
    for (int i = 0; i < 7; ++i)
        if (!isfinite(y[i])) return 0;
    return 1;
}

static void put_traj(double *rec, const double y[7], double gp)
{
    for (int i = 0; i < 6; ++i) rec[i] = y[i];
    rec[6] = gp;
    rec[7] = y[6];
}

/* Trace one ray: launch, RK4 until ground return / escape / max path /
 * non-finite state, then the ray outputs (Sec. II-C: group path, ground
 * distance, azimuth deviation, reflection height; plus phase path). */
static int trace_one(const or_medium *m, const or_field *fld, const or_opts *o,
                     double elev, double az, double f, int mode, double out[7],
                     int *n_steps, double *traj, int traj_cap, int *traj_n)
{
    double R = o->R_km;
    double hb = (m->kind == OR_GRID || m->kind == OR_GRID_CR) ? m->h0_km : m->floor_km;
    double y[7];
    double gp = or_launch(o, hb, elev, az, y);
    double apogee = y[0] - R;
    int steps = 0, status = -1, nt = 0;
    double lo = o->tx_lon_deg * DEG;

    if (traj && traj_cap > 0 && o->traj_stride > 0) put_traj(traj + 8 * nt++, y, gp);

    while (status < 0) {
        int ok = rk4(m, fld, R, f, mode, y, o->step_km);
        gp += o->step_km;
        ++steps;
        double h = y[0] - R;
        int graze = 0;
        double x[3], d[3], s = 0.0;
        /* termination tests; a non-finite state is tested first so that an
         * infinite height is not taken for an escape */
        if (!ok || !all_finite(y)) {
            status = OR_NUMERIC;
        } else if (h < hb && y[3] < 0.0) {
            /* below the floor and descending: straight vacuum line to r = R */
            state_to_cart(y, x, d);
            double xd = dot3(x, d);
            double c = dot3(x, x) - R * R;
            double disc = xd * xd - c;
            if (disc >= 0.0) {
                s = c / (-xd + sqrt(disc));
                status = OR_GROUND;
            } else {
                /* grazing line that misses the Earth: follow it back up to
                 * the floor and continue integrating there */
                double rb = R + hb;
                double c2 = dot3(x, x) - rb * rb;
                s = -xd + sqrt(xd * xd - c2);
                graze = 1;
            }
        } else if (h >= o->exit_h_km) {
            status = OR_ESCAPE;
        } else if (gp >= o->max_group_km) {
            status = OR_MAX_PATH;
        }
        if (status != OR_NUMERIC && h > apogee) apogee = h;
        /* trajectory: every stride-th step end and the last step end */
        if (traj && o->traj_stride > 0 && nt < traj_cap &&
            (steps % o->traj_stride == 0 || status >= 0))
            put_traj(traj + 8 * nt++, y, gp);

        if (status == OR_GROUND) {
            for (int i = 0; i < 3; ++i) x[i] += s * d[i];
            gp += s;
            y[6] += s;
            y[0] = sqrt(dot3(x, x));
            y[1] = atan2(sqrt(x[0] * x[0] + x[1] * x[1]), x[2]);
            y[2] = lon_near(x[0], x[1], lo);
        } else if (graze) {
            for (int i = 0; i < 3; ++i) x[i] += s * d[i];
            gp += s;
            double ph = y[6] + s;
            cart_to_state(x, d, 1.0, lo, y);
            y[6] = ph;
        }
    }
    if (traj_n) *traj_n = nt;

    /* landing (or sub-ray) point, ground range and azimuth deviation */
    double la = o->tx_lat_deg * DEG;
    double uT[3] = {cos(la) * cos(lo), cos(la) * sin(lo), sin(la)};
    double north[3] = {-sin(la) * cos(lo), -sin(la) * sin(lo), cos(la)};
    double east[3] = {-sin(lo), cos(lo), 0.0};
    double st = sin(y[1]);
    double uL[3] = {st * cos(y[2]), st * sin(y[2]), cos(y[1])};
    double cr[3] = {uT[1] * uL[2] - uT[2] * uL[1], uT[2] * uL[0] - uT[0] * uL[2],
                    uT[0] * uL[1] - uT[1] * uL[0]};
    double gam = atan2(sqrt(dot3(cr, cr)), dot3(uT, uL));
    double azd = 0.0;
    if (gam >= 1e-9) {
        double bear = atan2(dot3(uL, east), dot3(uL, north)) / DEG;
        double x = bear - az;
        azd = x - 360.0 * ceil((x - 180.0) / 360.0);   /* (-180, 180] */
    }
    out[0] = gp;
    out[1] = y[6];
    out[2] = R * gam;
    out[3] = azd;
    out[4] = apogee;
    out[5] = 90.0 - y[1] / DEG;
    out[6] = y[2] / DEG;
    *n_steps = steps;
    if (status == OR_NUMERIC) {
        for (int i = 0; i < 7; ++i) out[i] = NAN;
    }
    return status;
}

long long or_trace(const or_medium *m, const or_field *fld, const or_opts *o,
                   int n, const double *elev_deg, const double *az_deg,
                   const double *f_mhz, const int *mode, double *out7,
                   int *status, int *n_steps, double *traj, int traj_per_ray,
                   int *traj_count)
{
    long long total = 0;
#ifdef _OPENMP
    if (o->nthreads > 0) omp_set_num_threads(o->nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int i = 0; i < n; ++i) {
        int ns = 0, tn = 0;
        double *tr = traj ? traj + (size_t)i * traj_per_ray * 8 : NULL;
        status[i] = trace_one(m, fld, o, elev_deg[i], az_deg[i], f_mhz[i],
                              mode ? mode[i] : 1, out7 + 7 * (size_t)i, &ns,
                              tr, traj_per_ray, &tn);
        n_steps[i] = ns;
        if (traj_count) traj_count[i] = tn;
        total += ns;
    }
    return total;
}
