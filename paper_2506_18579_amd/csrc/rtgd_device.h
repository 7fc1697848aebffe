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


namespace rtgd {

// Device code is compiled with FP contraction off: every fused multiply-add
// is written out, so that every kernel variant (one or four lanes per ray)
// performs the same rounded operations in the same order.
__device__ __forceinline__ double fm(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fm(float a, float b, float c) { return fmaf(a, b, c); }

constexpr double kPi = 3.14159265358979323846;
constexpr double kRad2Deg = 180.0 / kPi;
constexpr double kDeg2Rad = kPi / 180.0;
// CODATA 2022: f_N^2 = kKN * N_e (Hz^2, m^-3); f_H = kKB * |B| (Hz, T)
constexpr double kKN = 80.61638587963628;
constexpr double kKB = 2.799248983422872e10;

enum RayStatus : int32_t { kGround = 0, kEscape = 1, kMaxPath = 2, kNumeric = 3 };

// Grid geometry as the kernels see it.  The values (f_N^2 in MHz^2, so
// that X = value / f_MHz^2, laid out [n_lat][n_lon][n_h], height fastest)
// are reached through each ray's RayConst::v: rays of one launch may run
// through different grids of the same geometry.
template <typename T>
struct GridDev {
    int32_t n_lat, n_lon, n_h;
    double lat0, lon0, h0;      // first node (deg, deg, km)
    double inv_dlat, inv_dlon, inv_dh;
    double lat_hi, lon_hi, h_hi;
    double R;                   // Earth radius, km
};

// Per-ray constants.
struct RayConst {
    const void *v;   // grid values (T) of the ray's grid
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
    const T s2 = s * s;
    w[0] = s * fm(s, fm(s, fm(s, fm(s, c6, T(-5) * c12), -c6), T(11) * c12), T(-0.5));
    w[1] = fm(s2, fm(s, fm(s, fm(s, T(-0.5), T(1.25)), T(0.5)), T(-2.25)), T(1));
    w[2] = s * fm(s, fm(s, fm(s, fm(s, T(0.5), T(-1.25)), T(-0.5)), T(1.75)), T(0.5));
    w[3] = s2 * fm(s, fm(s, fm(s, -c6, T(5) * c12), c6), T(-5) * c12);
    dw[0] = fm(s, fm(s, fm(s, fm(s, T(5) * c6, T(-5) / T(3)), T(-0.5)), T(11) * c6), T(-0.5));
    dw[1] = s * fm(s, fm(s, fm(s, T(-2.5), T(5)), T(1.5)), T(-4.5));
    dw[2] = fm(s, fm(s, fm(s, fm(s, T(2.5), T(-5)), T(-1.5)), T(3.5)), T(0.5));
    dw[3] = s * fm(s, fm(s, fm(s, T(-5) * c6, T(5) / T(3)), T(0.5)), T(-5) * c6);
}

// Catmull-Rom cubic weights (eq. cr_basis), the paper's comparison scheme.
template <typename T>
__device__ __forceinline__ void cr_weights(T t, T w[4], T dw[4])
{
    w[0] = T(0.5) * t * fm(t, T(2) - t, T(-1));
    w[1] = T(0.5) * fm(t * t, fm(T(3), t, T(-5)), T(2));
    w[2] = T(0.5) * t * fm(t, fm(T(-3), t, T(4)), T(1));
    w[3] = T(0.5) * t * t * (t - T(1));
    dw[0] = T(0.5) * fm(t, fm(T(-3), t, T(4)), T(-1));
    dw[1] = T(0.5) * t * fm(T(9), t, T(-10));
    dw[2] = T(0.5) * fm(t, fm(T(-9), t, T(8)), T(1));
    dw[3] = T(0.5) * t * fm(T(3), t, T(-2));
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

// Reciprocal by Newton-Raphson: the hardware estimate refined twice
// (each step x' = x + x (1 - a x) doubles the correct bits), ~1 ulp.
__device__ __forceinline__ double rcp(double a)
{
    double x = __builtin_amdgcn_rcp(a);
    double e = fma(-a, x, 1.0);
    x = fma(x, e, x);
    e = fma(-a, x, 1.0);
    return fma(x, e, x);
}
__device__ __forceinline__ float rcp(float a)
{
    float x = __builtin_amdgcn_rcpf(a);
    float e = fmaf(-a, x, 1.0f);
    return fmaf(x, e, x);
}

// sin and cos of theta0 + d from those of theta0, for a small increment d
// (|d| <= 0.05 rad): Taylor series of sin d and cos d (error < d^9/9!) and
// the angle-addition formulas.
__device__ __forceinline__ void sincos_add(double s0, double c0, double d, double &s, double &c)
{
    double d2 = d * d;
    double sd = d * fm(-d2 * (1.0 / 6.0), fm(-d2 * (1.0 / 20.0), fm(-d2, 1.0 / 42.0, 1.0), 1.0), 1.0);
    double cd = fm(-d2 * 0.5,
                   fm(-d2 * (1.0 / 12.0), fm(-d2 * (1.0 / 30.0), fm(-d2, 1.0 / 56.0, 1.0), 1.0), 1.0), 1.0);
    s = fm(s0, cd, c0 * sd);
    c = fm(c0, cd, -(s0 * sd));
}

// Height-then-longitude contraction of one latitude row of the stencil
// (4 columns x 4 heights): s0 = value, s1 = d/dlon, s2 = d/dh, each still to
// be weighted by the latitude weight of the row.
// Exchange with the lane (lane ^ 1) or (lane ^ 2) of the same quad through
// a DPP quad permutation (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true); }
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v)
{
    int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v) { return __int_as_float(dpp_i<CTRL>(__float_as_int(v))); }
constexpr int kQuadXor1 = 0xB1;   // quad_perm(1, 0, 3, 2)
constexpr int kQuadXor2 = 0x4E;   // quad_perm(2, 3, 0, 1)

// The grid lives in global memory; saying so (address space 1) lets the
// compiler use global loads, which do not share a wait counter with the
// scalar loads of the parameter block the way generic (flat) loads do.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

// Load one latitude row of the stencil: 4 columns x 4 consecutive heights.
template <typename T>
__device__ __forceinline__ void row_load(gptr<T> p, size_t nh, T u[16])
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        gptr<T> q = p + size_t(b) * nh;
#pragma unroll
        for (int c = 0; c < 4; ++c) u[4 * b + c] = q[c];
    }
}

// Height-then-longitude contraction of one loaded latitude row: s0 = value,
// s1 = d/dlon, s2 = d/dh, each still to be weighted by the row's latitude
// weight.
template <typename T>
__device__ __forceinline__ void row_contract(const T u[16], const T wh[4], const T dwh[4],
                                             const T wo[4], const T dwo[4], T &s0, T &s1, T &s2)
{
    s0 = s1 = s2 = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const T *q = u + 4 * b;
        T c0 = fm(q[3], wh[3], fm(q[2], wh[2], fm(q[1], wh[1], q[0] * wh[0])));
        T c1 = fm(q[3], dwh[3], fm(q[2], dwh[2], fm(q[1], dwh[1], q[0] * dwh[0])));
        s0 = fm(c0, wo[b], s0);
        s1 = fm(c0, dwo[b], s1);
        s2 = fm(c1, wo[b], s2);
    }
}

// The stencil values a lane last loaded and the cell they belong to.  Rays
// move less than a cell per RK4 stage, so most evaluations reuse them and
// skip the gather (and its memory round trip).  il < 0: empty.
template <typename T, int LANES>
struct StencilCache {
    static constexpr int ROWS = (LANES == 1) ? 4 : 1;
    int il, jl, kh;
    T u[ROWS][16];
    __device__ void clear() { il = -1; jl = -1; kh = -1; }
};

// f_N^2 (MHz^2, returned in FP64) and its partials d/dr, d/dtheta, d/dphi
// at a position.
// Below the grid bottom the medium is vacuum; outside the box laterally or
// above the top the value is continued as a constant.
//
// LANES = 1: one lane does the whole 4x4x4 stencil.  LANES = 4: the four
// lanes of a quad each take one latitude row and the row results are
// combined across the quad.  Both combine the four weighted row results in
// the same order, ((row0 + row1) + (row2 + row3)), with the products
// rounded separately, so the two give bit-identical results.
template <typename T, int IP, int LANES>
__device__ __forceinline__ void medium(const GridDev<T> &g, const T *vals, double r, double th, double ph,
                                       StencilCache<T, LANES> &sc, double &F, T &Fr, T &Fth, T &Fph)
{
    double h = r - g.R;
    if (h < g.h0) {
        F = 0.0;
        Fr = Fth = Fph = T(0);
        return;
    }
    double lat = fm(-th, kRad2Deg, 90.0);
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

    const size_t nh = size_t(g.n_h);
    const size_t row = size_t(g.n_lon) * nh;
    gptr<T> base = (gptr<T>)(vals) + (size_t(il - 1) * size_t(g.n_lon) + size_t(jl - 1)) * nh + size_t(kh - 1);

    // On a cell change, issue every load of this lane's share of the stencil
    // before any use, so that the memory round trips overlap (one wait
    // instead of one per column); the weights are computed while the loads
    // are in flight.
    constexpr int ROWS = StencilCache<T, LANES>::ROWS;
    const int a0 = (LANES == 1) ? 0 : (int(__lane_id()) & 3);
    if (il != sc.il || jl != sc.jl || kh != sc.kh) {
#pragma unroll
        for (int k = 0; k < ROWS; ++k) row_load<T>(base + size_t(a0 + k) * row, nh, sc.u[k]);
        sc.il = il;
        sc.jl = jl;
        sc.kh = kh;
    }
    __builtin_amdgcn_sched_barrier(0);

    // FP32 (mixed path): contract the differences u - u_ref to the cell's
    // base node.  The weights sum to 1 and their derivatives to 0, so this is
    // the same interpolant, but the gradient no longer cancels between large
    // node values where the density varies little across the cell.
    T u[ROWS][16];
    T uref = T(0);
    if constexpr (sizeof(T) == 4) {
        if constexpr (LANES == 1) {
            uref = sc.u[1][4 * 1 + 1];               // node (a, b, c) = (1, 1, 1)
        } else {
            uref = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(sc.u[0][4 * 1 + 1]),
                                                              0x55, 0xF, 0xF, true));  // from lane a = 1
        }
    }
#pragma unroll
    for (int k = 0; k < ROWS; ++k)
#pragma unroll
        for (int j = 0; j < 16; ++j) u[k][j] = sc.u[k][j] - uref;

    // IP = 0: Galerkin-Difference p = 3 (the method); IP = 1: Catmull-Rom
    T wo[4], dwo[4], wh[4], dwh[4];
    if constexpr (IP == 1) {
        cr_weights<T>(T(so_), wo, dwo);
        cr_weights<T>(T(sh_), wh, dwh);
    } else {
        gd_weights<T>(T(so_), wo, dwo);
        gd_weights<T>(T(sh_), wh, dwh);
    }

    T v, glat, glon, gh;
    if constexpr (LANES == 1) {
        T wl[4], dwl[4];
        if constexpr (IP == 1) cr_weights<T>(T(sl_), wl, dwl);
        else gd_weights<T>(T(sl_), wl, dwl);
        T pv[4], pla[4], plo[4], phh[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T s0, s1, s2;
            row_contract<T>(u[a], wh, dwh, wo, dwo, s0, s1, s2);
            pv[a] = s0 * wl[a];
            pla[a] = s0 * dwl[a];
            plo[a] = s1 * wl[a];
            phh[a] = s2 * wl[a];
        }
        v = (pv[0] + pv[1]) + (pv[2] + pv[3]);
        glat = (pla[0] + pla[1]) + (pla[2] + pla[3]);
        glon = (plo[0] + plo[1]) + (plo[2] + plo[3]);
        gh = (phh[0] + phh[1]) + (phh[2] + phh[3]);
    } else {
        static_assert(LANES == 4, "LANES must be 1 or 4");
        const int a = a0;
        T s0, s1, s2, wl, dwl;
        row_contract<T>(u[0], wh, dwh, wo, dwo, s0, s1, s2);
        if constexpr (IP == 1) cr_weight1<T>(T(sl_), a, wl, dwl);
        else gd_weight1<T>(T(sl_), a, wl, dwl);
        T pv = s0 * wl, pla = s0 * dwl, plo = s1 * wl, phh = s2 * wl;
        // (row a + row a^1), then + the other pair: lanes 0,1 form
        // (p0+p1)+(p2+p3), lanes 2,3 (p2+p3)+(p0+p1) -- equal, + commutes
        pv = pv + quad_swap<kQuadXor1>(pv);
        pla = pla + quad_swap<kQuadXor1>(pla);
        plo = plo + quad_swap<kQuadXor1>(plo);
        phh = phh + quad_swap<kQuadXor1>(phh);
        v = pv + quad_swap<kQuadXor2>(pv);
        glat = pla + quad_swap<kQuadXor2>(pla);
        glon = plo + quad_swap<kQuadXor2>(plo);
        gh = phh + quad_swap<kQuadXor2>(phh);
    }
    // index space -> physical: t_h = (r - R - h0)/dh,
    // t_lat = (90 - theta deg - lat0)/dlat, t_lon = (phi deg - lon0)/dlon
    // FP32: the base node value plus the contracted differences, summed in
    // FP64 so that 1 - X keeps its relative accuracy where X -> 1
    if constexpr (sizeof(T) == 4) F = double(v) + double(uref);
    else F = v;
    Fr = ch ? T(0) : gh * T(g.inv_dh);
    Fth = cl ? T(0) : glat * T(-kRad2Deg * g.inv_dlat);
    Fph = co ? T(0) : glon * T(kRad2Deg * g.inv_dlon);
}

// Appleton-Hartree partial derivatives of mu^2 with respect to X,
// a = Y_T^2 and b = Y_L^2 (independent), given X and u = 1 - X (formed by
// the caller in FP64).  O mode from the factored D = 2(1-X) E,
// E = 1 + 2b(1-X)/(S+a) (exact rearrangement, no cancellation as X -> 1);
// X mode from D as printed.
template <typename T>
__device__ __forceinline__ void appleton_partials(T X, T u, T a, T b, int sigma, T &mX, T &ma, T &mb)
{
    T bu = b * u;
    T S = sqrt(fm(a, a, T(4) * bu * u));
    T iS = rcp(S);
    T Tt = S + a;
    if (sigma > 0) {
        T iT = rcp(Tt);
        T E = fm(T(2) * bu, iT, T(1));
        T iE = rcp(E);
        // dE/dX = 2b (4bu^2/S - T)/T^2; with S^2 = a^2 + 4bu^2 the bracket is
        // exactly -aT/S, so dE/dX = -2ab/(S T) (no cancellation when a << S)
        T EX = T(-2) * a * b * iS * iT;
        T Ea = T(-2) * bu * iS * iT;
        T Eb = fm(T(-4) * bu * u * u * iS, iT * iT, T(2) * u * iT);
        T XiE2 = X * iE * iE;
        mX = fm(EX, XiE2, -iE);
        ma = Ea * XiE2;
        mb = Eb * XiE2;
    } else {
        T D = fm(T(2), u, -Tt);
        T iD = rcp(D);
        T N = T(2) * X * u;
        T DX = fm(T(4) * bu, iS, T(-2));
        T Da = -Tt * iS;
        T Db = T(-2) * u * u * iS;
        T iD2 = iD * iD;
        mX = -fm(T(2) * fm(T(-2), X, T(1)), D, -(N * DX)) * iD2;
        ma = N * Da * iD2;
        mb = N * Db * iD2;
    }
}

// dy/dP' of the 7-component state (r, th, ph, n_r, n_th, n_ph, P), given
// st = sin(th), ct = cos(th).  Returns false if G is not finite and non-zero.
template <typename T, int IP, int LANES>
__device__ __forceinline__ bool ray_rhs(const GridDev<T> &g, const RayConst &rc,
                                        const double y[7], T st, T ct, StencilCache<T, LANES> &sc,
                                        double dy[7])
{
    const double r = y[0], th = y[1], ph = y[2];
    double F;
    T Fr, Fth, Fph;
    medium<T, IP, LANES>(g, static_cast<const T *>(rc.v), r, th, ph, sc, F, Fr, Fth, Fph);
    const T inv_f2 = T(rc.inv_f2);
    const double Xd = F * rc.inv_f2;
    const T X = T(Xd);
    const T u = T(1.0 - Xd);
    const T Xr = Fr * inv_f2, Xth = Fth * inv_f2, Xph = Fph * inv_f2;

    const T rr = T(r);
    const T ir = rcp(rr);
    const T nr = T(y[3]), nt = T(y[4]), np = T(y[5]);
    const T n2 = fm(nr, nr, fm(nt, nt, np * np));

    T G, Hn0, Hn1, Hn2, Hr, Hth, Hph;
    if (rc.sigma == 0) {
        // mu^2 = 1 - X: dH/dn = n, G = -n.n - X, dH/dq = X_q / 2
        G = -n2 - X;
        Hn0 = nr; Hn1 = nt; Hn2 = np;
        Hr = T(0.5) * Xr; Hth = T(0.5) * Xth; Hph = T(0.5) * Xph;
    } else {
        // axial dipole: Y_r = -2 Yc cos th, Y_th = -Yc sin th, Yc = Y0 (R/r)^3
        const T q = T(g.R) * ir;
        const T Yc = T(rc.Y0) * (q * q * q);
        const T Y0 = T(-2) * Yc * ct, Y1 = -Yc * st;
        const T Yr0 = T(-3) * Y0 * ir, Yr1 = T(-3) * Y1 * ir;   // dY/dr
        const T Yt0 = T(2) * Yc * st, Yt1 = -Yc * ct;           // dY/dth
        const T Y2 = fm(Y0, Y0, Y1 * Y1);
        const T Yn = fm(Y0, nr, Y1 * nt);
        const T in2 = rcp(n2);
        const T b = Yn * Yn * in2;
        // Y_T^2 = |Y x n|^2 / n^2 directly, rather than Y^2 - Y_L^2, which
        // cancels for near-longitudinal propagation
        const T cz = fm(Y0, nt, -(Y1 * nr));
        const T a = fm(cz, cz, np * np * Y2) * in2;
        T mX, ma, mba;
        appleton_partials<T>(X, u, a, b, rc.sigma, mX, ma, mba);
        const T mY2 = ma;            // d mu^2 / d Y^2 at fixed b
        const T mb = mba - ma;       // d mu^2 / d b at fixed Y^2
        G = fm(X, mX, fm(Y2, mY2, fm(b, mb, -n2)));
        // dH/dn = n - mb/2 db/dn, db/dn = 2 Yn Y/n2 - 2 Yn^2 n / n2^2
        const T c1 = mb * Yn * in2;
        const T c2p = T(1) + mb * Yn * Yn * in2 * in2;
        Hn0 = fm(nr, c2p, -(c1 * Y0));
        Hn1 = fm(nt, c2p, -(c1 * Y1));
        Hn2 = np * c2p;
        const T dY2r = T(2) * fm(Y0, Yr0, Y1 * Yr1);
        const T dY2t = T(2) * fm(Y0, Yt0, Y1 * Yt1);
        const T tYn = T(2) * Yn * in2;
        const T dbr = tYn * fm(Yr0, nr, Yr1 * nt);
        const T dbt = tYn * fm(Yt0, nr, Yt1 * nt);
        Hr = T(-0.5) * fm(mX, Xr, fm(mY2, dY2r, mb * dbr));
        Hth = T(-0.5) * fm(mX, Xth, fm(mY2, dY2t, mb * dbt));
        Hph = T(-0.5) * (mX * Xph);
    }
    const T iG = rcp(G);
    const T irs = ir * rcp(st);
    const T rdot = -Hn0 * iG;
    const T thdot = -Hn1 * iG * ir;
    const T phdot = -Hn2 * iG * irs;
    const T stp = st * phdot, rtd = rr * thdot, rctp = rr * ct * phdot;
    dy[0] = double(rdot);
    dy[1] = double(thdot);
    dy[2] = double(phdot);
    dy[3] = double(fm(Hr, iG, fm(nt, thdot, np * stp)));
    dy[4] = double(fm(Hth, iG, fm(-nt, rdot, np * rctp)) * ir);
    dy[5] = double(fm(Hph, iG, fm(-np * st, rdot, -(np * rr * ct * thdot))) * irs);
    dy[6] = double(fm(nr, rdot, fm(nt, rtd, np * rr * stp)));
    return isfinite(double(G)) && G != T(0);
}

// One fixed RK4 step of size h (always FP64 state and combination).  The
// four stages share one copy of the right-hand side (stage loop, not
// unrolled) to keep register pressure and code size down.  sin and cos of
// the colatitude are evaluated once per step; the later stages, whose
// colatitude differs by a small increment, use sincos_add.
template <typename T, int IP, int LANES>
__device__ __forceinline__ bool rk4_step(const GridDev<T> &g, const RayConst &rc, double y[7], double h,
                                         StencilCache<T, LANES> &sc)
{
    double k[7], acc[7], t[7];
    bool ok = true;
    double s0, c0;
    sincos(y[1], &s0, &c0);
#pragma unroll
    for (int i = 0; i < 7; ++i) { t[i] = y[i]; acc[i] = 0.0; }
#pragma unroll 1
    for (int stage = 0; stage < 4; ++stage) {
        double st = s0, ct = c0;
        const double d = t[1] - y[1];
        if (stage > 0) {
            if (fabs(d) <= 0.05) sincos_add(s0, c0, d, st, ct);
            else sincos(t[1], &st, &ct);
        }
        ok &= ray_rhs<T, IP, LANES>(g, rc, t, T(st), T(ct), sc, k);
        // weights 1, 2, 2, 1 of the combination; next stage at y + c h k
        const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
        const double c = (stage == 2) ? h : 0.5 * h;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            acc[i] = fm(wgt, k[i], acc[i]);
            t[i] = fm(c, k[i], y[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) y[i] = fm(h / 6.0, acc[i], y[i]);
    return ok;
}

}  // namespace rtgd
