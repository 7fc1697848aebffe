// rtgd_device.h -- device-side arithmetic of one ray step (gfx950, HIP).
//
// Everything a lane needs to advance one ray: Galerkin-Difference p = 3
// interpolation of f_N^2 and its gradient (Sec. II-B-2, eq. 3dinterp_gd,
// Appendix A), the axial dipole, Appleton-Hartree partial derivatives
// (eq. appleton), the Hamiltonian ray equations (Sec. II-A, eq. 1a-1f with
// the k_phi sin(theta) dphi/dP' frame term in 1d) and the fixed-step RK4
// stage combination (Sec. II-C).
//
// Evaluation precision T is double (FP64 path) or float (mixed path: the
// interpolation, field and refractive-index work in FP32; the state, the
// step combination and the path accumulation stay FP64 in the caller).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// 1: issue the stencil loads one latitude row (16 nodes) at a time (fewer
// registers); 0: let the compiler hoist all 64 (more memory parallelism).
#ifndef RTGD_ROW_BATCH
#define RTGD_ROW_BATCH 0
#endif

namespace rtgd {

constexpr double kPi = 3.14159265358979323846;
constexpr double kRad2Deg = 180.0 / kPi;
constexpr double kDeg2Rad = kPi / 180.0;
// CODATA 2022: f_N^2 = kKN * N_e (Hz^2, m^-3); f_H = kKB * |B| (Hz, T)
constexpr double kKN = 80.61638587963628;
constexpr double kKB = 2.799248983422872e10;

enum RayStatus : int32_t { kGround = 0, kEscape = 1, kMaxPath = 2, kNumeric = 3 };

// Grid geometry and values as the kernels see them.  Values are f_N^2 in
// MHz^2 so that X = value / f_MHz^2.
template <typename T>
struct GridDev {
    const T *v;                 // [n_lat][n_lon][n_h], height fastest
    int32_t n_lat, n_lon, n_h;
    int32_t interp;             // 0 = GD, 1 = Catmull-Rom
    double lat0, lon0, h0;      // first node (deg, deg, km)
    double inv_dlat, inv_dlon, inv_dh;
    double lat_hi, lon_hi, h_hi;
    double R;                   // Earth radius, km
};

// Per-ray constants.
struct RayConst {
    double inv_f2;   // 1 / f_MHz^2
    double Y0;       // f_H at the equatorial surface / f (0: no field)
    int32_t sigma;   // +1 O, -1 X, 0 isotropic
};

// ---------------------------------------------------------------------------
// 1-D weights for node offsets a = -1, 0, 1, 2 of the cell containing s.
// GD p=3: the four Appendix A quintic pieces, node j+a taking piece -a in
// its shifted variable s (Horner form).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void gd_weights(T s, T w[4], T dw[4])
{
    const T c12 = T(1.0 / 12.0), c6 = T(1.0 / 6.0);
    w[0] = s * (T(-0.5) + s * (T(11) * c12 + s * (-c6 + s * (T(-5) * c12 + s * c6))));
    w[1] = T(1) + s * s * (T(-2.25) + s * (T(0.5) + s * (T(1.25) + s * T(-0.5))));
    w[2] = s * (T(0.5) + s * (T(1.75) + s * (T(-0.5) + s * (T(-1.25) + s * T(0.5)))));
    w[3] = s * s * (T(-5) * c12 + s * (c6 + s * (T(5) * c12 + s * (-c6))));
    dw[0] = T(-0.5) + s * (T(11) * c6 + s * (T(-0.5) + s * (T(-5) / T(3) + s * (T(5) * c6))));
    dw[1] = s * (T(-4.5) + s * (T(1.5) + s * (T(5) + s * T(-2.5))));
    dw[2] = T(0.5) + s * (T(3.5) + s * (T(-1.5) + s * (T(-5) + s * T(2.5))));
    dw[3] = s * (T(-5) * c6 + s * (T(0.5) + s * (T(5) / T(3) + s * (T(-5) * c6))));
}

// Catmull-Rom cubic weights (eq. cr_basis), the paper's comparison scheme.
template <typename T>
__device__ __forceinline__ void cr_weights(T t, T w[4], T dw[4])
{
    T t2 = t * t, t3 = t2 * t;
    w[0] = T(0.5) * (-t3 + T(2) * t2 - t);
    w[1] = T(0.5) * (T(3) * t3 - T(5) * t2 + T(2));
    w[2] = T(0.5) * (T(-3) * t3 + T(4) * t2 + t);
    w[3] = T(0.5) * (t3 - t2);
    dw[0] = T(0.5) * (T(-3) * t2 + T(4) * t - T(1));
    dw[1] = T(0.5) * (T(9) * t2 - T(10) * t);
    dw[2] = T(0.5) * (T(-9) * t2 + T(8) * t + T(1));
    dw[3] = T(0.5) * (T(3) * t2 - T(2) * t);
}

// Weight and derivative of one node offset (a = 0..3 for offsets -1..2).
template <typename T>
__device__ __forceinline__ void gd_weight1(T s, int a, T &w, T &dw)
{
    T w4[4], d4[4];
    gd_weights<T>(s, w4, d4);
    w = a == 0 ? w4[0] : a == 1 ? w4[1] : a == 2 ? w4[2] : w4[3];
    dw = a == 0 ? d4[0] : a == 1 ? d4[1] : a == 2 ? d4[2] : d4[3];
}

template <typename T>
__device__ __forceinline__ void cr_weight1(T s, int a, T &w, T &dw)
{
    T w4[4], d4[4];
    cr_weights<T>(s, w4, d4);
    w = a == 0 ? w4[0] : a == 1 ? w4[1] : a == 2 ? w4[2] : w4[3];
    dw = a == 0 ? d4[0] : a == 1 ? d4[1] : a == 2 ? d4[2] : d4[3];
}

// Cell of one axis: t in index units, cell k = clamp(floor(t), 1, n-3),
// local s = t - k (s in [-1, 2] at the edge cells).  fmax/fmin keep the
// index in range even for a NaN coordinate.
__device__ __forceinline__ int locate(double t, int n, double &s)
{
    double f = floor(t);
    f = fmin(fmax(f, 1.0), double(n - 3));
    s = t - f;
    return int(f);
}

// f_N^2 (MHz^2) and its partials d/dr, d/dtheta, d/dphi at a position.
// Below the grid bottom the medium is vacuum; outside the box laterally or
// above the top the value is continued as a constant.
template <typename T>
__device__ __forceinline__ void medium(const GridDev<T> &g, double r, double th, double ph,
                                       T &F, T &Fr, T &Fth, T &Fph)
{
    double h = r - g.R;
    if (h < g.h0) {
        F = Fr = Fth = Fph = T(0);
        return;
    }
    double lat = 90.0 - th * kRad2Deg;
    double lon = ph * kRad2Deg;
    bool cl = false, co = false, ch = false;
    if (lat < g.lat0) { lat = g.lat0; cl = true; }
    else if (lat > g.lat_hi) { lat = g.lat_hi; cl = true; }
    if (lon < g.lon0) { lon = g.lon0; co = true; }
    else if (lon > g.lon_hi) { lon = g.lon_hi; co = true; }
    if (h > g.h_hi) { h = g.h_hi; ch = true; }

    double sl_, so_, sh_;
    int il = locate((lat - g.lat0) * g.inv_dlat, g.n_lat, sl_);
    int jl = locate((lon - g.lon0) * g.inv_dlon, g.n_lon, so_);
    int kh = locate((h - g.h0) * g.inv_dh, g.n_h, sh_);

    T wo[4], dwo[4], wh[4], dwh[4];
    const bool cr = (g.interp == 1);
    if (cr) {
        cr_weights<T>(T(so_), wo, dwo);
        cr_weights<T>(T(sh_), wh, dwh);
    } else {
        gd_weights<T>(T(so_), wo, dwo);
        gd_weights<T>(T(sh_), wh, dwh);
    }

    const size_t nh = size_t(g.n_h);
    const size_t row = size_t(g.n_lon) * nh;
    const T *base = g.v + (size_t(il - 1) * size_t(g.n_lon) + size_t(jl - 1)) * nh + size_t(kh - 1);

    // contract height first (value and d/dh per column), then longitude,
    // then latitude: 128 + 48 + 16 FMAs for the value and three partials.
    // One latitude row (16 nodes) in flight at a time.
    T v = T(0), glat = T(0), glon = T(0), gh = T(0);
#if RTGD_ROW_BATCH
#pragma unroll 1
#else
#pragma unroll
#endif
    for (int a = 0; a < 4; ++a) {
        T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T *p = base + size_t(a) * row + size_t(b) * nh;
            T u0 = p[0], u1 = p[1], u2 = p[2], u3 = p[3];
            T c0 = u0 * wh[0] + u1 * wh[1] + u2 * wh[2] + u3 * wh[3];
            T c1 = u0 * dwh[0] + u1 * dwh[1] + u2 * dwh[2] + u3 * dwh[3];
            s0 += c0 * wo[b];
            s1 += c0 * dwo[b];
            s2 += c1 * wo[b];
        }
        T wl, dwl;
        if (cr) cr_weight1<T>(T(sl_), a, wl, dwl);
        else gd_weight1<T>(T(sl_), a, wl, dwl);
        v += s0 * wl;
        glat += s0 * dwl;
        glon += s1 * wl;
        gh += s2 * wl;
    }
    // index space -> physical: t_h = (r - R - h0)/dh,
    // t_lat = (90 - theta deg - lat0)/dlat, t_lon = (phi deg - lon0)/dlon
    F = v;
    Fr = ch ? T(0) : gh * T(g.inv_dh);
    Fth = cl ? T(0) : glat * T(-kRad2Deg * g.inv_dlat);
    Fph = co ? T(0) : glon * T(kRad2Deg * g.inv_dlon);
}

// Appleton-Hartree partial derivatives of mu^2 with respect to X,
// a = Y_T^2 and b = Y_L^2 (independent).  O mode from the factored
// D = 2(1-X) E, E = 1 + 2b(1-X)/(S+a) (exact rearrangement, no cancellation
// as X -> 1); X mode from D as printed.
template <typename T>
__device__ __forceinline__ void appleton_partials(T X, T a, T b, int sigma, T &mX, T &ma, T &mb)
{
    T u = T(1) - X;
    T S = sqrt(a * a + T(4) * b * u * u);
    T iS = T(1) / S;
    T Tt = S + a;
    if (sigma > 0) {
        T iT = T(1) / Tt;
        T E = T(1) + T(2) * b * u * iT;
        T iE = T(1) / E;
        T EX = T(2) * b * (T(4) * b * u * u * iS - Tt) * iT * iT;
        T Ea = T(-2) * b * u * iS * iT;
        T Eb = T(2) * u * iT - T(4) * b * u * u * u * iS * iT * iT;
        T XiE2 = X * iE * iE;
        mX = -iE + EX * XiE2;
        ma = Ea * XiE2;
        mb = Eb * XiE2;
    } else {
        T D = T(2) * u - Tt;
        T iD = T(1) / D;
        T N = T(2) * X * u;
        T DX = T(-2) + T(4) * b * u * iS;
        T Da = -Tt * iS;
        T Db = T(-2) * u * u * iS;
        T iD2 = iD * iD;
        mX = -(T(2) * (T(1) - T(2) * X) * D - N * DX) * iD2;
        ma = N * Da * iD2;
        mb = N * Db * iD2;
    }
}

// dy/dP' of the 7-component state (r, th, ph, n_r, n_th, n_ph, P).
// Returns false if G is not finite and non-zero.
template <typename T>
__device__ __forceinline__ bool ray_rhs(const GridDev<T> &g, const RayConst &rc,
                                        const double y[7], double dy[7])
{
    const double r = y[0], th = y[1], ph = y[2];
    T F, Fr, Fth, Fph;
    medium<T>(g, r, th, ph, F, Fr, Fth, Fph);
    const T inv_f2 = T(rc.inv_f2);
    const T X = F * inv_f2;
    const T Xr = Fr * inv_f2, Xth = Fth * inv_f2, Xph = Fph * inv_f2;

    T st, ct;
    if constexpr (sizeof(T) == 8) {
        sincos(th, &st, &ct);
    } else {
        sincosf(float(th), &st, &ct);
    }
    const T rr = T(r);
    const T nr = T(y[3]), nt = T(y[4]), np = T(y[5]);
    const T n2 = nr * nr + nt * nt + np * np;

    T G, Hn0, Hn1, Hn2, Hr, Hth, Hph;
    if (rc.sigma == 0) {
        // mu^2 = 1 - X: dH/dn = n, G = -n.n - X, dH/dq = X_q / 2
        G = -n2 - X;
        Hn0 = nr; Hn1 = nt; Hn2 = np;
        Hr = T(0.5) * Xr; Hth = T(0.5) * Xth; Hph = T(0.5) * Xph;
    } else {
        // axial dipole: Y_r = -2 Yc cos th, Y_th = -Yc sin th, Yc = Y0 (R/r)^3
        const T q = T(g.R) / rr;
        const T Yc = T(rc.Y0) * q * q * q;
        const T Y0 = T(-2) * Yc * ct, Y1 = -Yc * st;
        const T ir = T(1) / rr;
        const T Yr0 = T(-3) * Y0 * ir, Yr1 = T(-3) * Y1 * ir;   // dY/dr
        const T Yt0 = T(2) * Yc * st, Yt1 = -Yc * ct;           // dY/dth
        const T Y2 = Y0 * Y0 + Y1 * Y1;
        const T Yn = Y0 * nr + Y1 * nt;
        const T in2 = T(1) / n2;
        const T b = Yn * Yn * in2;
        const T a = Y2 - b;
        T mX, ma, mba;
        appleton_partials<T>(X, a, b, rc.sigma, mX, ma, mba);
        const T mY2 = ma;            // d mu^2 / d Y^2 at fixed b
        const T mb = mba - ma;       // d mu^2 / d b at fixed Y^2
        G = -n2 + X * mX + Y2 * mY2 + b * mb;
        // dH/dn = n - mb/2 db/dn, db/dn = 2 Yn Y/n2 - 2 Yn^2 n / n2^2
        const T c1 = mb * Yn * in2;
        const T c2 = mb * Yn * Yn * in2 * in2;
        Hn0 = nr - c1 * Y0 + c2 * nr;
        Hn1 = nt - c1 * Y1 + c2 * nt;
        Hn2 = np + c2 * np;
        const T dY2r = T(2) * (Y0 * Yr0 + Y1 * Yr1);
        const T dY2t = T(2) * (Y0 * Yt0 + Y1 * Yt1);
        const T dbr = T(2) * Yn * (Yr0 * nr + Yr1 * nt) * in2;
        const T dbt = T(2) * Yn * (Yt0 * nr + Yt1 * nt) * in2;
        Hr = T(-0.5) * (mX * Xr + mY2 * dY2r + mb * dbr);
        Hth = T(-0.5) * (mX * Xth + mY2 * dY2t + mb * dbt);
        Hph = T(-0.5) * (mX * Xph);
    }
    const T iG = T(1) / G;
    const T ir = T(1) / rr;
    const T irs = ir / st;
    const T rdot = -Hn0 * iG;
    const T thdot = -Hn1 * iG * ir;
    const T phdot = -Hn2 * iG * irs;
    dy[0] = double(rdot);
    dy[1] = double(thdot);
    dy[2] = double(phdot);
    dy[3] = double(Hr * iG + nt * thdot + np * st * phdot);
    dy[4] = double((Hth * iG - nt * rdot + np * rr * ct * phdot) * ir);
    dy[5] = double((Hph * iG - np * st * rdot - np * rr * ct * thdot) * irs);
    dy[6] = double(nr * rdot + nt * rr * thdot + np * rr * st * phdot);
    return isfinite(double(G)) && G != T(0);
}

// One fixed RK4 step of size h (always FP64 state and combination).  The
// four stages share one copy of the right-hand side (stage loop, not
// unrolled) to keep register pressure and code size down.
template <typename T>
__device__ __forceinline__ bool rk4_step(const GridDev<T> &g, const RayConst &rc, double y[7], double h)
{
    double k[7], acc[7], t[7];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 7; ++i) { t[i] = y[i]; acc[i] = 0.0; }
#pragma unroll 1
    for (int stage = 0; stage < 4; ++stage) {
        ok &= ray_rhs<T>(g, rc, t, k);
        // weights 1, 2, 2, 1 of the combination; next stage at y + c h k
        const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
        const double c = (stage == 2) ? h : 0.5 * h;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            acc[i] += wgt * k[i];
            t[i] = y[i] + c * k[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) y[i] = y[i] + h / 6.0 * acc[i];
    return ok;
}

}  // namespace rtgd
