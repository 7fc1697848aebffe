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
// is written out, so that every kernel variant (one or sixteen lanes per ray)
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
    double h0;                  // grid bottom (km)
    // index coordinates as affine maps: t_lat = lat_a th + lat_b (th the
    // colatitude, rad), t_lon = lon_a ph + lon_b (ph the longitude, rad),
    // t_h = inv_dh h + h_b (h the height, km)
    double lat_a, lat_b, lon_a, lon_b, inv_dh, h_b;
    double kmax_lat, kmax_lon, kmax_h;   // last cell of each axis: n - 3
    double R;                   // Earth radius, km
};

// Per-ray constants.
struct RayConst {
    const void *v;   // grid values (T) of the ray's grid
    double inv_f2;   // 1 / f_MHz^2
    double YR3;      // (f_H at the equatorial surface / f) R^3, km^3 (0: no field)
    int32_t sigma;   // +1 O, -1 X, 0 isotropic
};

// ---------------------------------------------------------------------------
// 1-D weights for node offsets a = -1, 0, 1, 2 (index 0..3) of the cell
// containing s.  GD p = 3: node j+a takes the Appendix A piece psi_{-a} in
// its shifted variable, a quintic in s; Catmull-Rom (eq. cr_basis): a cubic.
// Every weight is evaluated in the same full Horner form from its monomial
// coefficients (w = ((c5 s + c4) s + ...) s + c0, w' from 5 c5, 4 c4, ...),
// so a lane that evaluates a single node's piece from coefficients held in
// registers rounds exactly as a lane that evaluates all four with
// compile-time constants.
// ---------------------------------------------------------------------------
template <int IP>
struct Basis;
template <>
struct Basis<0> {                      // GD p = 3, coefficients of s^0..s^5
    static constexpr int DEG = 5;
    static constexpr double c[4][6] = {
        {0.0, -0.5, 11.0 / 12.0, -1.0 / 6.0, -5.0 / 12.0, 1.0 / 6.0},
        {1.0, 0.0, -2.25, 0.5, 1.25, -0.5},
        {0.0, 0.5, 1.75, -0.5, -1.25, 0.5},
        {0.0, 0.0, -5.0 / 12.0, 1.0 / 6.0, 5.0 / 12.0, -1.0 / 6.0}};
};
template <>
struct Basis<1> {                      // Catmull-Rom, coefficients of t^0..t^3
    static constexpr int DEG = 3;
    static constexpr double c[4][6] = {
        {0.0, -0.5, 1.0, -0.5, 0.0, 0.0},
        {1.0, 0.0, -2.5, 1.5, 0.0, 0.0},
        {0.0, 0.5, 2.0, -1.5, 0.0, 0.0},
        {0.0, 0.0, -0.5, 0.5, 0.0, 0.0}};
};

// Monomial coefficients of one node's weight and derivative, as values (a
// lane keeps those of its own node offset in registers).
template <typename T>
struct Piece {
    T c[6];   // w  = sum c[k] s^k
    T d[5];   // w' = sum d[k] s^k, d[k] = (k + 1) c[k + 1]
};

// Kernel variant: bit 0 is the interpolation (0 GD, 1 Catmull-Rom), bit 1
// says that every ray of the launch is anisotropic (a field is set), so the
// isotropic branch of the right-hand side is compiled out.
constexpr int interp_of(int V) { return V & 1; }
constexpr bool aniso_only(int V) { return (V & 2) != 0; }

template <typename T, int IP>
__device__ __forceinline__ Piece<T> piece(int a)
{
    using B = Basis<interp_of(IP)>;
    Piece<T> p;
#pragma unroll
    for (int k = 0; k <= B::DEG; ++k) {
        double v = a == 0 ? B::c[0][k] : a == 1 ? B::c[1][k] : a == 2 ? B::c[2][k] : B::c[3][k];
        p.c[k] = T(v);
    }
#pragma unroll
    for (int k = 0; k < B::DEG; ++k) {
        double v = a == 0 ? B::c[0][k + 1] : a == 1 ? B::c[1][k + 1] : a == 2 ? B::c[2][k + 1] : B::c[3][k + 1];
        p.d[k] = T(v * double(k + 1));
    }
    return p;
}

template <typename T, int IP>
__device__ __forceinline__ void eval_piece(const Piece<T> &p, T s, T &w, T &dw)
{
    constexpr int D = Basis<interp_of(IP)>::DEG;
    T x = p.c[D];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) x = fm(x, s, p.c[k]);
    T y = p.d[D - 1];
#pragma unroll
    for (int k = D - 2; k >= 0; --k) y = fm(y, s, p.d[k]);
    w = x;
    dw = y;
}

// All four weights of one axis with compile-time coefficients.
template <typename T, int IP>
__device__ __forceinline__ void weights4(T s, T w[4], T dw[4])
{
#pragma unroll
    for (int a = 0; a < 4; ++a) eval_piece<T, IP>(piece<T, IP>(a), s, w[a], dw[a]);
}

// Cell of one axis from the index coordinate t = (c - c0) / dc: cell
// k = clamp(floor(t), 1, kmax) with kmax = n - 3, and local s = t - k,
// clamped to [-1, 2] (the edge cells' range), which is t clamped to the box
// [0, n - 1].  A clamped axis has a zero partial derivative.  The cell is
// clamped before the conversion to int, so it is in range for any t, NaN
// included (s is then clamped to -1).
__device__ __forceinline__ int locate(double t, double kmax, double &s, bool &clamped)
{
    const double f = fmin(fmax(floor(t), 1.0), kmax);
    const double su = t - f;
    s = fmin(fmax(su, -1.0), 2.0);
    clamped = s != su;
    return int(f);
}

// Reciprocal and reciprocal square root from the hardware estimates.  On
// gfx950 v_rcp_f64 / v_rsq_f64 are good to about 24 bits (max relative error
// 4.6e-8 / 5.2e-8 measured over 2^20 arguments), so one Newton step each,
// x' = x + x (1 - a x) for the reciprocal (relative error ~ e^2 ~ 2.1e-15)
// and x' = x + x (1/2 - (a/2) x^2) for the reciprocal square root
// (~ 1.5 e^2 ~ 4.1e-15), brings them to within a few times 1e-15, six
// orders below the 1e-9 agreement asked of the FP64 path.  The FP32
// estimates are within 1.5 ulp of FP32 (9.0e-8 / 9.3e-8) and are used as
// they are.
__device__ __forceinline__ double rcp(double a)
{
    double x = __builtin_amdgcn_rcp(a);
    double e = fma(-a, x, 1.0);
    return fma(x, e, x);
}
__device__ __forceinline__ float rcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ double rsqrt(double a)
{
    const double h = 0.5 * a;
    const double x = __builtin_amdgcn_rsq(a);
    const double e = fma(-h, x * x, 0.5);
    return fma(x, e, x);
}
__device__ __forceinline__ float rsqrt(float a) { return __builtin_amdgcn_rsqf(a); }

// sin and cos of theta0 + d from those of theta0, for |d| <= 0.05 rad: the
// Taylor series of sin d (to d^7) and cos d (to d^8), whose first omitted
// terms are below 6e-18 and 3e-20, and the angle-addition formulas.
__device__ __forceinline__ void sincos_add(double s0, double c0, double d, double &s, double &c)
{
    double d2 = d * d;
    double sd = d * fm(-d2 * (1.0 / 6.0), fm(-d2 * (1.0 / 20.0), fm(-d2, 1.0 / 42.0, 1.0), 1.0), 1.0);
    double cd = fm(-d2 * 0.5,
                   fm(-d2 * (1.0 / 12.0), fm(-d2 * (1.0 / 30.0), fm(-d2, 1.0 / 56.0, 1.0), 1.0), 1.0), 1.0);
    s = fm(s0, cd, c0 * sd);
    c = fm(c0, cd, -(s0 * sd));
}

// The library's sin and cos, kept out of line: it runs rarely (a new
// anchor, below), and inlined its many constants would hold registers for
// the whole trace loop.
struct SinCos {
    double s, c;
};
__device__ __attribute__((noinline)) SinCos sincos_ref(double x)
{
    SinCos r;
    sincos(x, &r.s, &r.c);
    return r;
}

// Cross-lane exchange through DPP (no LDS round trip), on the two 32-bit
// halves of a double: quad permutations within groups of 4 lanes and the
// 16-lane row mirrors.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true); }
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) { return __int_as_float(dpp_i<CTRL>(__float_as_int(v))); }
// Broadcast of lane N of each 16-lane row to the whole row (row_newbcast);
// gfx950 moves a 64-bit value this way in one instruction.
template <int N>
__device__ __forceinline__ double row_bcast(double v)
{
    const long long x = __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x150 + N, 0xF, 0xF, true);
    return __longlong_as_double(x);
}
template <int N>
__device__ __forceinline__ float row_bcast(float v) { return dpp<0x150 + N>(v); }
constexpr int kQuadXor1 = 0xB1;          // quad_perm(1, 0, 3, 2): lane ^ 1
constexpr int kQuadXor2 = 0x4E;          // quad_perm(2, 3, 0, 1): lane ^ 2
// Per-lane choice between two values by a lane mask m (all ones or all
// zeros) held in a VGPR: bitwise (b & m) | (a & ~m), one v_bfi_b32 per 32
// bits, so that lane-dependent choices need no SGPR lane masks.
__device__ __forceinline__ unsigned bfi(unsigned m, unsigned b, unsigned a)
{
    unsigned d;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(d) : "v"(m), "v"(b), "v"(a));
    return d;
}
__device__ __forceinline__ double pick(unsigned m, double a, double b)
{
    const unsigned lo = bfi(m, unsigned(__double2loint(b)), unsigned(__double2loint(a)));
    const unsigned hi = bfi(m, unsigned(__double2hiint(b)), unsigned(__double2hiint(a)));
    return __hiloint2double(int(hi), int(lo));
}
__device__ __forceinline__ float pick(unsigned m, float a, float b)
{
    return __uint_as_float(bfi(m, __float_as_uint(b), __float_as_uint(a)));
}
constexpr int kRowRor8 = 0x128;          // lane i <- lane (i + 8) mod 16 within 16
constexpr int kRowShr4 = 0x114;          // lane i <- lane i - 4 within 16 (0 for i < 4)
constexpr int kQuadEven = 0xA0;          // quad_perm(0, 0, 2, 2): odd lanes read lane - 1
constexpr int kQuadOdd = 0xF5;           // quad_perm(1, 1, 3, 3): even lanes read lane + 1

// The grid lives in global memory; saying so (address space 1) lets the
// compiler use global loads, which do not share a wait counter with the
// scalar loads of the parameter block the way generic (flat) loads do.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

// Load one column of the stencil: 4 consecutive heights.
template <typename T>
__device__ __forceinline__ void col_load(gptr<T> p, T u[4])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = p[c];
}

// Contraction order, shared by every kernel variant so that all give the
// same rounded result: per column, heights in a fused chain (value and
// d/dh); per latitude row, the weighted columns in pairs,
// fma(col1, w1, col0 w0) + fma(col3, w3, col2 w2); over rows, the same
// pairing of rows (0, 1) and (2, 3).
template <typename T>
__device__ __forceinline__ void col_contract(const T u[4], const T wh[4], const T dwh[4], T &cv, T &dcv)
{
    cv = fm(u[3], wh[3], fm(u[2], wh[2], fm(u[1], wh[1], u[0] * wh[0])));
    dcv = fm(u[3], dwh[3], fm(u[2], dwh[2], fm(u[1], dwh[1], u[0] * dwh[0])));
}

// The stencil values a lane last loaded and the cell they belong to.  Rays
// move less than a cell per RK4 stage, so most evaluations reuse them and
// skip the gather (and its memory round trip).  il < 0: empty.
//   LANES = 1:  the lane holds all 4 x 4 x 4 nodes, u[a][b][c].
//   LANES = 16: each lane of a 16-lane row holds one column (lat offset
//               a = (lane >> 2) & 3, lon offset b = lane & 3), u[0][0][c],
//               and the coefficients of its own lat and lon weights.
template <typename T, int LANES>
struct StencilCache {
    static constexpr int NA = (LANES == 1) ? 4 : 1;
    int il, jl, kh;
    T u[NA][NA][4];
    T uref;                   // node (1, 1, 1), the mixed path's reference
    Piece<T> pa, pb;          // LANES = 16: weights of this lane's a and b
    unsigned m1, m3;          // LANES = 16: all ones where lane & 3 is 1, 3
    __device__ void clear() { il = -1; jl = -1; kh = -1; }
    __device__ void set_masks(int lane)
    {
        m1 = (lane & 3) == 1 ? ~0u : 0u;
        m3 = (lane & 3) == 3 ? ~0u : 0u;
        // opaque to the compiler from here on: it would turn pick() back
        // into selects on SGPR lane masks, which crowd the SGPRs
        asm volatile("" : "+v"(m1), "+v"(m3));
    }
};

// f_N^2 (MHz^2, returned in FP64) and its partials d/dr, d/dtheta, d/dphi
// at a position.  Below the grid bottom the medium is vacuum; outside the
// box laterally or above the top the value is continued as a constant.
//
// LANES = 1: one lane does the whole 4x4x4 stencil.  LANES = 16: the 16
// lanes of a row each contract one column; the row sums are formed within
// quads and the lat sum across the row with DPP, in the order described at
// col_contract, so the two variants give bit-identical results and every
// lane of the row ends with the same values.
template <typename T, int IP, int LANES>
__device__ __forceinline__ void medium(const GridDev<T> &g, const T *vals, double r, double th, double ph,
                                       StencilCache<T, LANES> &sc, double &F, T &Fr, T &Fth, T &Fph)
{
    static_assert(LANES == 1 || LANES == 16, "LANES must be 1 or 16");
    double h = r - g.R;
    if (h < g.h0) {
        F = 0.0;
        Fr = Fth = Fph = T(0);
        return;
    }
    // index coordinates, clamped to the box through the local coordinates
    // (selects, no branches)
    double sl_, so_, sh_;
    bool cl, co, ch;
    const int il = locate(fm(th, g.lat_a, g.lat_b), g.kmax_lat, sl_, cl);
    const int jl = locate(fm(ph, g.lon_a, g.lon_b), g.kmax_lon, so_, co);
    const int kh = locate(fm(h, g.inv_dh, g.h_b), g.kmax_h, sh_, ch);

    const size_t nh = size_t(g.n_h);
    const size_t row = size_t(g.n_lon) * nh;
    gptr<T> base = (gptr<T>)(vals) + (size_t(il - 1) * size_t(g.n_lon) + size_t(jl - 1)) * nh + size_t(kh - 1);

    // On a cell change, issue every load of this lane's share of the stencil
    // before any use, so that the memory round trips overlap (one wait
    // instead of one per column); the weights are computed while the loads
    // are in flight.
    const int lane = int(__lane_id());
    const int a16 = (lane >> 2) & 3, b16 = lane & 3;
    if (il != sc.il || jl != sc.jl || kh != sc.kh) {
        if constexpr (LANES == 1) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) col_load<T>(base + size_t(a) * row + size_t(b) * nh, sc.u[a][b]);
        } else {
            col_load<T>(base + size_t(a16) * row + size_t(b16) * nh, sc.u[0][0]);
            if constexpr (sizeof(T) == 4) sc.uref = base[row + nh + 1];
        }
        sc.il = il;
        sc.jl = jl;
        sc.kh = kh;
    }
    __builtin_amdgcn_sched_barrier(0);

    // FP32 (mixed path): contract the differences u - u_ref to the cell's
    // node (1, 1, 1).  The weights sum to 1 and their derivatives to 0, so
    // this is the same interpolant, but the gradient no longer cancels
    // between large node values where the density varies little across the
    // cell.
    T uref = T(0);
    if constexpr (sizeof(T) == 4) {
        if constexpr (LANES == 1) uref = sc.u[1][1][1];
        else uref = sc.uref;
    }

    T v, glat, glon, gh;
    if constexpr (LANES == 1) {
        T wh[4], dwh[4];
        weights4<T, IP>(T(sh_), wh, dwh);
        T wo[4], dwo[4], wl[4], dwl[4];
        weights4<T, IP>(T(so_), wo, dwo);
        weights4<T, IP>(T(sl_), wl, dwl);
        T s0[4], s1[4], s2[4];   // per lat offset a: sums over the lon offsets b
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            T cv[4], dcv[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                T uu[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) uu[c] = sc.u[a][b][c] - uref;
                col_contract<T>(uu, wh, dwh, cv[b], dcv[b]);
            }
            s0[a] = fm(cv[1], wo[1], cv[0] * wo[0]) + fm(cv[3], wo[3], cv[2] * wo[2]);
            s1[a] = fm(cv[1], dwo[1], cv[0] * dwo[0]) + fm(cv[3], dwo[3], cv[2] * dwo[2]);
            s2[a] = fm(dcv[1], wo[1], dcv[0] * wo[0]) + fm(dcv[3], wo[3], dcv[2] * wo[2]);
        }
        v = fm(s0[1], wl[1], s0[0] * wl[0]) + fm(s0[3], wl[3], s0[2] * wl[2]);
        glat = fm(s0[1], dwl[1], s0[0] * dwl[0]) + fm(s0[3], dwl[3], s0[2] * dwl[2]);
        glon = fm(s1[1], wl[1], s1[0] * wl[0]) + fm(s1[3], wl[3], s1[2] * wl[2]);
        gh = fm(s2[1], wl[1], s2[0] * wl[0]) + fm(s2[3], wl[3], s2[2] * wl[2]);
    } else {
        T wo, dwo, wl, dwl, w1, dw1;
        eval_piece<T, IP>(sc.pb, T(so_), wo, dwo);
        eval_piece<T, IP>(sc.pa, T(sl_), wl, dwl);
        // height weights: lane b of each quad evaluates node b's piece (the
        // same piece as its longitude weight); lanes 0..3 of the row hold
        // pieces 0..3, which the row broadcasts
        eval_piece<T, IP>(sc.pb, T(sh_), w1, dw1);
        T wh[4], dwh[4];
        wh[0] = row_bcast<0>(w1); dwh[0] = row_bcast<0>(dw1);
        wh[1] = row_bcast<1>(w1); dwh[1] = row_bcast<1>(dw1);
        wh[2] = row_bcast<2>(w1); dwh[2] = row_bcast<2>(dw1);
        wh[3] = row_bcast<3>(w1); dwh[3] = row_bcast<3>(dw1);
        T uu[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) uu[c] = sc.u[0][0][c] - uref;
        T cv, dcv;
        col_contract<T>(uu, wh, dwh, cv, dcv);
        // within the quad (lon offsets b): the odd lane of each pair adds
        // its weighted column to the even lane's product by one FMA, then
        // lanes 1 and 3 add the two pairs (equal on both)
        T t0 = cv * wo, t1 = cv * dwo, t2 = dcv * wo;
        t0 = fm(cv, wo, dpp<kQuadEven>(t0));
        t1 = fm(cv, dwo, dpp<kQuadEven>(t1));
        t2 = fm(dcv, wo, dpp<kQuadEven>(t2));
        const T s0 = t0 + dpp<kQuadXor2>(t0);
        const T s1 = t1 + dpp<kQuadXor2>(t1);
        const T s2 = t2 + dpp<kQuadXor2>(t2);
        // Only the odd lanes of a quad hold the sums.  Lane b of each quad
        // takes one of the four row products, q = b: the value s0 wl, d/dlat
        // s0 dwl, d/dlon s1 wl, d/dh s2 wl; lanes 0 and 2 receive their sum
        // (s0, s1) from lanes 1 and 3.
        const T lhs = pick(sc.m3, dpp<kQuadOdd>(pick(sc.m3, s0, s1)), s2);
        const T rhs = pick(sc.m1, wl, dwl);
        // over the lat offsets a (quads of the row), paired the same way:
        // quads 1 and 3 hold the pairs, then each adds the other's
        T p = lhs * rhs;
        p = fm(lhs, rhs, dpp<kRowShr4>(p));
        p = p + dpp<kRowRor8>(p);
        // lane 4 + q of the row holds quantity q, which the row broadcasts
        v = row_bcast<4>(p);
        glat = row_bcast<5>(p);
        glon = row_bcast<6>(p);
        gh = row_bcast<7>(p);
    }
    // index space -> physical: dt_h/dr = 1/dh, dt_lat/dth = lat_a,
    // dt_lon/dph = lon_a
    // FP32: the base node value plus the contracted differences, summed in
    // FP64 so that 1 - X keeps its relative accuracy where X -> 1
    if constexpr (sizeof(T) == 4) F = double(v) + double(uref);
    else F = v;
    Fr = ch ? T(0) : gh * T(g.inv_dh);
    Fth = cl ? T(0) : glat * T(g.lat_a);
    Fph = co ? T(0) : glon * T(g.lon_a);
}

// Appleton-Hartree partial derivatives of mu^2 with respect to X,
// a = Y_T^2 and b = Y_L^2 (independent), given X and u = 1 - X (formed by
// the caller in FP64), for the O mode (sigma > 0) and the X mode in one
// instruction stream, so that rays of both modes in one wave (or on the rows
// of one wave) run no divergent branch.  Both modes are written as
// mu^2 = 1 - X / E, an exact rearrangement of eq. appleton with
// D = 2u - a + sigma S = 2u E, S = sqrt(a^2 + 4 b u^2), T = S + a:
//   O:  E = 1 + 2 b u / T   (S - a = 4 b u^2 / T: no cancellation as X -> 1)
//   X:  E = 1 - T / (2 u)   (u >= Y > 0 where the X mode propagates)
// With k = (E - 1) / u (O: 2b/T, X: -T/(2u^2)) and m = -sigma k / S:
//   dE/dX = a m,  dE/da = u m,
//   dE/db = O: 2u/T - 4 b u^3 / (S T^2),  X: -u / S,
// and mu^2_X = -1/E + X E_X / E^2, mu^2_a = X E_a / E^2, mu^2_b = X E_b / E^2.
// The mode-specific terms are selects: a candidate that is infinite for the
// other mode (1/u where the O mode reflects) is never used.
template <typename T>
__device__ __forceinline__ void appleton_partials(T X, T u, T a, T b, int sigma, T &mX, T &ma, T &mb)
{
    const bool o_mode = sigma > 0;
    const T w4 = T(4) * (b * u) * u;      // 4 b u^2
    const T S2 = fm(a, a, w4);
    const T iS = rsqrt(S2);
    const T S = S2 * iS;
    const T Tt = S + a;
    const T x = rcp(o_mode ? Tt : u);     // O: 1/T, X: 1/u (the one each mode needs)
    const T xx = x * x;
    const T k = o_mode ? T(2) * b * x : T(-0.5) * Tt * xx;
    const T E = fm(k, u, T(1));
    const T iE = rcp(E);
    const T m = (o_mode ? -k : k) * iS;
    const T ui = u * iS;
    // O: 2u/T - 4 b u^3 / (S T^2) = 2 u x - 4 b u^2 (u / S) x^2
    const T Eb = o_mode ? fm(-w4 * ui, xx, T(2) * u * x) : -ui;
    const T XiE2 = (X * iE) * iE;
    mX = fm(a * m, XiE2, -iE);
    ma = (u * m) * XiE2;
    mb = Eb * XiE2;
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

    const T rr = T(r);
    const T rst = rr * st;
    const T irs = rcp(rst);       // 1 / (r sin th)
    const T ir = irs * st;
    const T nr = T(y[3]), nt = T(y[4]), np = T(y[5]);
    const T n2 = fm(nr, nr, fm(nt, nt, np * np));

    // The medium enters dH/dq (q = r, th, ph) only as -1/2 mu^2_X dX/dq
    // = sX F_q, with sX = -mu^2_X / (2 f^2).
    T G, Hn0, Hn1, Hn2, Hr, Hth, Hph;
    if (!aniso_only(IP) && rc.sigma == 0) {
        // mu^2 = 1 - X: dH/dn = n, G = -n.n - X, dH/dq = X_q / 2
        G = -n2 - X;
        Hn0 = nr; Hn1 = nt; Hn2 = np;
        const T sX = T(0.5) * inv_f2;
        Hr = sX * Fr; Hth = sX * Fth; Hph = sX * Fph;
    } else {
        // axial dipole: Y_r = -2 Yc cos th, Y_th = -Yc sin th, Yc = Y0 (R/r)^3,
        // so dY_th/dth = -Yc cos th = Y_r / 2 and dY_r/dth = -2 Y_th;
        // dY/dr = -3 Y / r (used below in closed form)
        const T Yc = T(rc.YR3) * (ir * ir * ir);
        const T Y1 = -(Yc * st);
        const T Yt1 = -(Yc * ct);    // dY_th/dth
        const T Y0 = Yt1 + Yt1;
        const T Y2 = fm(Y0, Y0, Y1 * Y1);
        const T Yn = fm(Y0, nr, Y1 * nt);
        const T in2 = rcp(n2);
        const T Yni = Yn * in2;
        const T b = Yn * Yni;
        // Y_T^2 = |Y x n|^2 / n^2 directly, rather than Y^2 - Y_L^2, which
        // cancels for near-longitudinal propagation
        const T cz = fm(Y0, nt, -(Y1 * nr));
        const T a = fm(cz, cz, np * np * Y2) * in2;
        T mX, ma, mba;
        appleton_partials<T>(X, u, a, b, rc.sigma, mX, ma, mba);
        const T mY2 = ma;            // d mu^2 / d Y^2 at fixed b
        const T mb = mba - ma;       // d mu^2 / d b at fixed Y^2
        G = fm(X, mX, fm(Y2, mY2, fm(b, mb, -n2)));
        // dH/dn = n - mb/2 db/dn, db/dn = 2 Yn Y/n2 - 2 Yn^2 n / n2^2:
        // n (1 + mb Yn^2 / n2^2) - mb (Yn / n2) Y
        const T c1 = mb * Yni;
        const T c2p = fm(c1, Yni, T(1));
        Hn0 = fm(nr, c2p, -(c1 * Y0));
        Hn1 = fm(nt, c2p, -(c1 * Y1));
        Hn2 = np * c2p;
        // dH/dq = -1/2 (mX dX/dq + mY2 dY^2/dq + mb db/dq); with dY/dr = -3Y/r,
        // dY^2/dr = -6 Y^2 / r and db/dr = -6 b / r.  Along th:
        // -1/2 dY^2/dth = -(Y_r (-2 Y_th) + Y_th Y_r / 2) = 3 Y_th dY_th/dth,
        // -1/2 db/dth = -(Yn / n2) (-2 Y_th n_r + dY_th/dth n_th)
        const T sX = T(-0.5) * mX * inv_f2;
        const T hY2t = T(3) * (Y1 * Yt1);
        const T hbt = -Yni * fm(T(-2) * Y1, nr, Yt1 * nt);
        Hr = fm(sX, Fr, T(3) * ir * fm(mY2, Y2, mb * b));
        Hth = fm(sX, Fth, fm(mY2, hY2t, mb * hbt));
        Hph = sX * Fph;
    }
    // eq. (1): dx/dP' = -(dH/dn) / G and dn/dP' = (dH/dx) / G in the
    // spherical frame, with the frame terms of n
    const T iG = rcp(G);
    const T miG = -iG;
    const T rdot = Hn0 * miG;
    const T thdot = Hn1 * (miG * ir);
    const T phdot = Hn2 * (miG * irs);
    const T A = np * phdot;          // n_ph dph/dP'
    const T B = rr * thdot;          // r dth/dP'
    dy[0] = double(rdot);
    dy[1] = double(thdot);
    dy[2] = double(phdot);
    dy[3] = double(fm(Hr, iG, fm(nt, thdot, A * st)));
    dy[4] = double(fm(Hth, iG, fm(-nt, rdot, A * (rr * ct))) * ir);
    dy[5] = double(fm(Hph, iG, -(np * fm(st, rdot, ct * B))) * irs);
    dy[6] = double(fm(nr, rdot, fm(nt, B, A * rst)));
    return isfinite(double(G)) && G != T(0);
}

// Anchor of a ray's colatitude: th and its sin and cos from the library.
// Every stage takes sin and cos of its colatitude from the anchor with
// sincos_add, so that the library is needed only when the ray has moved
// far from the anchor (see rk4_step).
struct Anchor {
    double th, s, c;
};
constexpr double kAnchorMove = 0.025;   // re-anchor beyond this (rad)
constexpr double kSeriesMax = 0.05;     // range of sincos_add (rad)

__device__ __forceinline__ Anchor make_anchor(double th)
{
    const SinCos q = sincos_ref(th);
    return Anchor{th, q.s, q.c};
}

// Steps for which every RK4 stage stays within kSeriesMax of the anchor: the
// step starts within kAnchorMove of it, and a stage lies at most h |dth/dP'|
// further, with |dth/dP'| <= |dx/dP'| / r <= 1 / R (the group speed is at
// most c) -- h <= R / 60 leaves a margin of 50 % on that slope.
__host__ __device__ inline bool series_covers_step(double h_km, double R_km) { return h_km <= R_km / 60.0; }

// One fixed RK4 step of size h (always FP64 state and combination); h6 is
// h / 6, rounded once by the caller.  UNROLL = false: the four stages share
// one copy of the right-hand side (a stage loop), which keeps register
// pressure and code size down where many rays share a wave; UNROLL = true
// (the sixteen-lane tail, bound by the latency of one ray) drops the loop's
// per-stage selects and copies.  The arithmetic is the same either way.
// The anchor moves to the step's starting colatitude when that is more than
// kAnchorMove from it (every 160 km or more of north-south travel), so that
// every stage is within kSeriesMax of it for steps up to about 150 km; a
// stage beyond that uses the library.
template <typename T, int IP, int LANES, bool UNROLL = false>
__device__ __forceinline__ bool rk4_step(const GridDev<T> &g, const RayConst &rc, double y[7], double h,
                                         double h6, bool short_step, Anchor &an, StencilCache<T, LANES> &sc)
{
    double k[7], acc[7], t[7];
    bool ok = true;
    if (!(fabs(y[1] - an.th) <= kAnchorMove)) an = make_anchor(y[1]);
#pragma unroll
    // acc starts at -0: 1 * k + (-0) is k exactly (also for k = +-0), so
    // the unrolled form may take k itself at the first stage
    for (int i = 0; i < 7; ++i) { t[i] = y[i]; acc[i] = -0.0; }
    auto stage_body = [&](int stage) {
        const double d = t[1] - an.th;
        double st, ct;
        sincos_add(an.s, an.c, d, st, ct);
        // short_step (uniform over the launch): every stage is within
        // kSeriesMax of the anchor, so no lane needs the library
        if (!short_step) {
            if (!(fabs(d) <= kSeriesMax)) {
                const SinCos q = sincos_ref(t[1]);
                st = q.s;
                ct = q.c;
            }
        }
        ok &= ray_rhs<T, IP, LANES>(g, rc, t, T(st), T(ct), sc, k);
        // weights 1, 2, 2, 1 of the combination; next stage at y + c h k
        const double wgt = (stage == 0 || stage == 3) ? 1.0 : 2.0;
        const double c = (stage == 2) ? h : 0.5 * h;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            acc[i] = (UNROLL && stage == 0) ? k[i] : fm(wgt, k[i], acc[i]);
            t[i] = fm(c, k[i], y[i]);
        }
    };
    if constexpr (UNROLL) {
#pragma unroll
        for (int stage = 0; stage < 4; ++stage) stage_body(stage);
    } else {
#pragma unroll 1
        for (int stage = 0; stage < 4; ++stage) stage_body(stage);
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) y[i] = fm(h6, acc[i], y[i]);
    return ok;
}

}  // namespace rtgd
