// rtgd_kernels.h -- the trace kernels of librtgd (gfx950): per-launch
// parameter block, ray set-up and termination, the persistent one-lane
// kernel, the sixteen-lanes-per-ray row phase and tail kernel, and the
// ionogram extraction kernel.  Included once, by rtgd.hip.
//
// Design (one MI355X):
//   * one lane integrates one ray; its state (position, wave normal, phase
//     and group path) lives in registers for the ray's whole life;
//   * a persistent grid of single-wave workgroups pulls rays from a device
//     queue: when a lane's ray terminates the wave refills every idle lane
//     with one atomic (ballot + popcount), so waves stay full while rays of
//     very different lengths retire at different times;
//   * the last live rays finish on sixteen lanes each, which splits the
//     stencil work of a step and shortens its dependent chain;
//   * the density grid stays resident in HBM and is re-read through the L2
//     and Infinity Cache; nothing on the path is a dense contraction, so
//     all arithmetic is VALU (no MFMA).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtgd_device.h"

using namespace rtgd;

namespace {

// ---------------------------------------------------------------------------
// Kernel parameters (one block in device memory per launch)
// ---------------------------------------------------------------------------

// One request of a launch: launch rays [start, start + n) are its fan, in
// the order ((i_f * n_mode + i_m) * n_elev + i_e) * n_az + i_a.  A launch
// holds one segment (rt_trace) or a batch of requests (the server) that
// share the grid geometry, the transmitter and the step options.
struct Segment {
    const double *elev, *az, *freq;  // device copies of the fan axes
    const void *v;                   // grid values (T) of the request's grid
    double B0;                       // 0: isotropic
    double *out[7];                  // group, phase, range, az_dev, apogee, land_lat, land_lon
    int32_t *status, *nsteps;
    unsigned long long *steps;       // RK4 steps of the request (accumulated)
    int32_t n_elev, n_az, n_mode;
    int32_t mode_first;              // +1 if the first mode is O, -1 if X
    int32_t start, n;
    int32_t bin_pos[2];              // mode-sorted queue: where this segment's O (or isotropic)
                                     // rays and its X rays begin
};

template <typename T>
struct TraceParams {
    GridDev<T> g;
    const Segment *seg;
    int32_t n_seg;
    int32_t n_rays;            // over all segments
    double tx_lon;             // rad
    double up[3], north[3], east[3];   // transmitter frame (Cartesian)
    double r0;                 // R + tx height
    double step, step6;        // step and step / 6 (km)
    int32_t short_step;        // every RK4 stage within the anchor series (series_covers_step)
    double max_group, exit_h, floor_h;
    int32_t max_steps;         // hard cap (never reached before max_group)
    int32_t traj_stride;
    int64_t traj_per_ray;
    struct RayRec *rec;        // per launch ray: starting, then final state
    double *traj;              // trajectories, indexed by launch ray (one segment only)
    int32_t *traj_count;
    // scheduling
    int32_t *queue_head;
    int32_t *truncated;
    // hand-off of the last live rays to the 16-lanes-per-ray tail kernel
    int32_t *live;             // rays neither finished nor handed off
    int32_t *n_handoff;        // records written
    struct Handoff *handoff;   // capacity handoff_threshold
    int32_t handoff_threshold; // hand off once at most this many rays are live (0: never);
                               // also the hand-off buffer capacity
    int32_t inwave;            // a drained wave with <= 4 live rays finishes them 16 lanes each
    int64_t perm_stride;       // launch ray q is visited as (q * perm_stride) mod n_rays
    int32_t *order;            // if set: queue entry q holds launch ray order[q] (mode-sorted)
    // promotion: waves with block index >= n_producers run promoted rays
    // sixteen lanes each while the other waves still run one lane per ray
    int32_t n_producers;       // one-lane waves (all waves when promotion is off)
    int32_t promote_cap;       // promoted rays running or queued at most (4 per promotion wave; 0: off)
    int32_t promote_age;       // also promote rays of at least this many steps (0: trapped and grazing rays only)
    int32_t *promo_push;       // tickets issued (promoted rays)
    int32_t *promo_pop;        // tickets claimed by promotion waves
    int32_t *promo_live;       // promoted rays not yet finished or handed off
    int32_t *producers_alive;  // one-lane waves still running
    int32_t *promo_err;        // waits that timed out (reported as a launch error)
    int32_t *unfinished;       // rays k_finish found without a final status (a launch error)
    unsigned long long *phase_steps;
    unsigned long long *wave_iters;  // one-lane wave iterations that stepped a ray   // RK4 ray-steps run one lane per ray, on promotion
                                       // rows, on 16-lane rows after the hand-off (or the
                                       // in-wave switch)
    int64_t idle_ticks;        // wall-clock bound of an idle promotion wave's wait
    int32_t *promo_ids;        // ray of each ticket, -1 until published (n_rays entries)
};

// State of a ray moved from the one-lane to the sixteen-lane kernel.
struct Handoff {
    double y[7];
    double gp, apogee;
    Anchor an;
    int32_t ray, steps, ntraj, pad;
};

__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// longitude of (x, y) unwrapped to within pi of ref
__device__ __forceinline__ double lon_near(double x, double y, double ref)
{
    double p = atan2(y, x);
    return p + 2.0 * kPi * floor((ref - p) / (2.0 * kPi) + 0.5);
}

__device__ __forceinline__ void sph_basis(double th, double ph, double rh[3], double thh[3],
                                          double phh[3])
{
    double st, ct, sp, cp;
    sincos(th, &st, &ct);
    sincos(ph, &sp, &cp);
    rh[0] = st * cp; rh[1] = st * sp; rh[2] = ct;
    thh[0] = ct * cp; thh[1] = ct * sp; thh[2] = -st;
    phh[0] = -sp; phh[1] = cp; phh[2] = 0.0;
}

__device__ __forceinline__ void cart_to_state(const double x[3], const double d[3], double ref_lon,
                                              double y[7])
{
    double r = sqrt(dot3(x, x));
    double th = atan2(sqrt(x[0] * x[0] + x[1] * x[1]), x[2]);
    double ph = lon_near(x[0], x[1], ref_lon);
    double rh[3], thh[3], phh[3];
    sph_basis(th, ph, rh, thh, phh);
    y[0] = r; y[1] = th; y[2] = ph;
    y[3] = dot3(d, rh);
    y[4] = dot3(d, thh);
    y[5] = dot3(d, phh);
}

__device__ __forceinline__ void state_to_cart(const double y[7], double x[3], double d[3])
{
    double rh[3], thh[3], phh[3];
    sph_basis(y[1], y[2], rh, thh, phh);
    double inv = 1.0 / sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        x[i] = y[0] * rh[i];
        d[i] = (y[3] * rh[i] + y[4] * thh[i] + y[5] * phh[i]) * inv;
    }
}

// Per-lane ray bookkeeping.
struct Lane {
    double y[7];          // r, th, ph, n_r, n_th, n_ph, P
    double gp;            // group path P'
    double apogee;
    double az0;           // launch azimuth (deg)
    RayConst rc;
    Anchor an;            // colatitude anchor (sin and cos of the stages)
    int32_t steps;
    int32_t ntraj;
    int32_t seg;          // segment of the ray
    int32_t local;        // ray index within the segment
    int32_t trapped;      // 1: turned upward inside the ionosphere (a duct);
                          // 2: grazed a layer peak on the first ascent
    float nr_lo;          // smallest n_r so far on the first ascent (one-lane
                          // kernels, promotion on); negative once it ended
};

// Per launch ray, in device memory: the starting state, written by k_start
// before the trace kernels run, and, once the ray has terminated, its final
// state and status, written by the trace kernels and turned into the ray's
// outputs by k_finish.  Keeping launch and landing geometry (library
// sin, cos, atan2, sqrt) out of the trace loop keeps that loop's registers
// for the step itself.
struct RayRec {
    Lane L;
    int32_t status, pad;
};

template <typename T>
__device__ __forceinline__ void put_traj(const TraceParams<T> &P, int ray, Lane &L)
{
    if (L.ntraj < P.traj_per_ray) {
        double *rec = P.traj + (size_t(ray) * size_t(P.traj_per_ray) + size_t(L.ntraj)) * 8;
#pragma unroll
        for (int i = 0; i < 6; ++i) rec[i] = L.y[i];
        rec[6] = L.gp;
        rec[7] = L.y[6];
        ++L.ntraj;
    } else {
        *P.truncated = 1;
    }
}

// Per-ray constants from the launch ray index: find the segment (binary
// search over the segment starts), then decode its fan.
template <typename T>
__device__ __forceinline__ void ray_const(const TraceParams<T> &P, int ray, Lane &L, double &elev)
{
    int lo = 0, hi = P.n_seg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (P.seg[mid].start <= ray) lo = mid;
        else hi = mid - 1;
    }
    const Segment &S = P.seg[lo];
    int i = ray - S.start;
    L.seg = lo;
    L.local = i;
    int ia = i % S.n_az; i /= S.n_az;
    int ie = i % S.n_elev; i /= S.n_elev;
    int im = i % S.n_mode; i /= S.n_mode;
    int jf = i;
    elev = S.elev[ie];
    double f = S.freq[jf];
    int sigma = (im == 0) ? S.mode_first : -1;
    L.rc.v = S.v;
    L.rc.inv_f2 = 1.0 / (f * f);
    L.rc.YR3 = kKB * S.B0 / (f * 1e6) * (P.g.R * P.g.R * P.g.R);
    L.rc.sigma = (S.B0 == 0.0) ? 0 : sigma;
    L.az0 = S.az[ia];
}

// Ray initialisation (Sec. II-C): straight vacuum line from the transmitter
// to the grid bottom, |n| = 1 there.
template <typename T>
__device__ __forceinline__ void init_ray(const TraceParams<T> &P, int ray, Lane &L, bool write)
{
    double elev_deg;
    ray_const(P, ray, L, elev_deg);
    double sb, cb, sa, ca;
    sincos(elev_deg * kDeg2Rad, &sb, &cb);
    sincos(L.az0 * kDeg2Rad, &sa, &ca);
    double d[3], x[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = sb * P.up[k] + cb * (ca * P.north[k] + sa * P.east[k]);
    double rb = P.g.R + P.floor_h;
    double p = P.r0 * sb;
    double c = rb * rb - P.r0 * P.r0;
    double s = c / (p + sqrt(p * p + c));
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = P.r0 * P.up[k] + s * d[k];
    cart_to_state(x, d, P.tx_lon, L.y);
    L.y[6] = s;
    L.gp = s;
    L.apogee = L.y[0] - P.g.R;
    L.an = make_anchor(L.y[1]);
    L.steps = 0;
    L.ntraj = 0;
    L.trapped = 0;
    L.nr_lo = 3.0e38f;
    if (P.traj_stride > 0 && write) put_traj(P, ray, L);
}

// Below the grid bottom and descending, a ray leaves along the straight
// vacuum line through its point.  In spherical terms (x.d = r n_r / |n|,
// |x|^2 = r^2) the line reaches r = R if disc = (x.d)^2 - (r^2 - R^2) >= 0,
// after a distance s = (r^2 - R^2) / (-x.d + sqrt(disc)).
__device__ __forceinline__ double vacuum_disc(const double y[7], double R, double &xd, double &c)
{
    xd = y[0] * y[3] * rtgd::rsqrt(fm(y[3], y[3], fm(y[4], y[4], y[5] * y[5])));
    c = fm(y[0], y[0], -R * R);
    return fm(xd, xd, -c);
}

// Outputs of a terminated ray (one thread per launch ray, from its final
// state): a ground return first follows the vacuum line to the ground; then
// the landing (or sub-ray) point, ground range and azimuth deviation
// (Sec. II-C outputs, plus the phase path).
template <typename T>
__device__ __forceinline__ void finish_ray(const TraceParams<T> &P, int ray)
{
    const RayRec &rec = P.rec[ray];
    Lane L = rec.L;
    const int status = rec.status;
    if (status == kGround) {
        double xd, c, x[3], d[3];
        const double disc = vacuum_disc(L.y, P.g.R, xd, c);
        const double s = c / (-xd + sqrt(fmax(disc, 0.0)));
        state_to_cart(L.y, x, d);
#pragma unroll
        for (int i = 0; i < 3; ++i) x[i] += s * d[i];
        L.gp += s;
        L.y[6] += s;
        L.y[0] = sqrt(dot3(x, x));
        L.y[1] = atan2(sqrt(x[0] * x[0] + x[1] * x[1]), x[2]);
        L.y[2] = lon_near(x[0], x[1], P.tx_lon);
    }
    double st, ct, sp, cp;
    sincos(L.y[1], &st, &ct);
    sincos(L.y[2], &sp, &cp);
    double uL[3] = {st * cp, st * sp, ct};
    const double *uT = P.up;
    double cr[3] = {uT[1] * uL[2] - uT[2] * uL[1], uT[2] * uL[0] - uT[0] * uL[2],
                    uT[0] * uL[1] - uT[1] * uL[0]};
    double gam = atan2(sqrt(dot3(cr, cr)), dot3(uT, uL));
    double azd = 0.0;
    if (gam >= 1e-9) {
        double bear = atan2(dot3(uL, P.east), dot3(uL, P.north)) * kRad2Deg;
        double x = bear - L.az0;
        azd = x - 360.0 * ceil((x - 180.0) / 360.0);
    }
    double o[7] = {L.gp, L.y[6], P.g.R * gam, azd, L.apogee, 90.0 - L.y[1] * kRad2Deg,
                   L.y[2] * kRad2Deg};
    if (status == kNumeric || status < 0) {
#pragma unroll
        for (int k = 0; k < 7; ++k) o[k] = __builtin_nan("");
    }
    const Segment &S = P.seg[L.seg];
    const int i = L.local;
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if (S.out[k]) S.out[k][i] = o[k];
    if (S.status) S.status[i] = status;
    if (S.nsteps) S.nsteps[i] = L.steps;
    if (P.traj_count) P.traj_count[ray] = L.ntraj;
}

// A terminated ray's final state into its record (the fields a step changes).
template <typename T>
__device__ __forceinline__ void retire(const TraceParams<T> &P, int ray, const Lane &L, int status)
{
    RayRec &rec = P.rec[ray];
#pragma unroll
    for (int i = 0; i < 7; ++i) rec.L.y[i] = L.y[i];
    rec.L.gp = L.gp;
    rec.L.apogee = L.apogee;
    rec.L.steps = L.steps;
    rec.L.ntraj = L.ntraj;
    rec.status = status;
}

// A ray below the grid bottom whose vacuum line misses the Earth: it is
// followed back up to the grid bottom and the ray goes on.  The trajectory
// point of the step is recorded first, as for any other step.  Out of line
// (rare).
template <typename T>
__device__ __attribute__((noinline)) Lane graze_back(const TraceParams<T> *Pp, int ray, Lane L, bool write)
{
    const TraceParams<T> &P = *Pp;
    double x[3], d[3];
    state_to_cart(L.y, x, d);
    const double xd = dot3(x, d);
    const double rb = P.g.R + P.floor_h;
    const double c2 = dot3(x, x) - rb * rb;
    const double s = -xd + sqrt(xd * xd - c2);
    if (P.traj_stride > 0 && write && L.steps % P.traj_stride == 0) put_traj(P, ray, L);
#pragma unroll
    for (int i = 0; i < 3; ++i) x[i] += s * d[i];
    L.gp += s;
    const double ph = L.y[6] + s;
    cart_to_state(x, d, P.tx_lon, L.y);
    L.y[6] = ph;
    return L;
}

// n_r / |n| below which a turning point passed on the first ascent counts
// as grazing (for promotion only).
constexpr double kGrazeQ = 0.02;

// One RK4 step plus the termination tests.  Returns the ray status, or -1
// if the ray goes on.  `write` is false on the lanes of a row that only
// shadow the row's leader (no memory writes).  P is the caller's copy of
// the parameter block (in registers), Pp the block itself (for the
// out-of-line calls).
template <typename T, int IP, int LANES, bool UNROLL = false>
__device__ __forceinline__ int advance(const TraceParams<T> &P, const TraceParams<T> *Pp, int ray, Lane &L,
                                       bool write, StencilCache<T, LANES> &sc)
{
    const double nr0 = L.y[3];
    bool ok = rk4_step<T, IP, LANES, UNROLL>(P.g, L.rc, L.y, P.step, P.step6, P.short_step != 0, L.an, sc);
    L.gp += P.step;
    ++L.steps;
    const double h = L.y[0] - P.g.R;
    // a ray whose wave normal turns from downward to upward well above the
    // grid bottom is trapped between layers: such rays run to the maximum
    // group path (used to pick rays for promotion only)
    if (nr0 < 0.0 && L.y[3] >= 0.0 && h > P.floor_h + 5.0) L.trapped = 1;
    // a ray whose n_r, on its first ascent, falls to a positive local minimum
    // below kGrazeQ |n| and then grows again has crossed a layer peak at
    // grazing incidence: on the way down such rays are often turned back up
    // by the same layer (trapped above it) or run far along a layer, and they
    // are recognised here hundreds of steps before their first upward turn
    if constexpr (LANES == 1) {
        if (P.promote_cap > 0 && L.nr_lo >= 0.0f) {
            const double nr = L.y[3], lo = double(L.nr_lo);
            if (nr < 0.0) {
                L.nr_lo = -1.0f;
            } else if (nr < lo) {
                L.nr_lo = float(nr);
            } else if (nr > lo && lo * lo < kGrazeQ * kGrazeQ * fm(nr, nr, fm(L.y[4], L.y[4], L.y[5] * L.y[5]))) {
                if (L.trapped == 0) L.trapped = 2;
                L.nr_lo = -1.0f;
            }
        }
    }
    // y[i] * 0 is NaN exactly when y[i] is infinite or NaN, else +-0
    double z = L.y[0] * 0.0;
#pragma unroll
    for (int i = 1; i < 7; ++i) z = fm(L.y[i], 0.0, z);
    const bool finite = ok && z == 0.0;
    const bool below = h < P.floor_h && L.y[3] < 0.0;
    // in order of precedence: NUMERIC, below the grid bottom, ESCAPE,
    // MAX_PATH; the common outcome (-1) by selects, without branches
    int status = (L.gp >= P.max_group || L.steps >= P.max_steps) ? kMaxPath : -1;
    status = h >= P.exit_h ? kEscape : status;
    status = finite ? status : kNumeric;
    if (finite && below) {
        // below the grid bottom and descending: a ground return (k_finish
        // follows the vacuum line) unless the line misses the Earth
        double xd, c;
        if (vacuum_disc(L.y, P.g.R, xd, c) >= 0.0) {
            status = kGround;
        } else {
            if (h > L.apogee) L.apogee = h;
            L = graze_back(Pp, ray, L, write);
            return -1;
        }
    }
    L.apogee = (status != kNumeric && h > L.apogee) ? h : L.apogee;
    if (P.traj_stride > 0 && write && (L.steps % P.traj_stride == 0 || status >= 0)) put_traj(P, ray, L);
    return status;
}

// Add the per-lane step counts of a wave to a launch-wide counter (one
// atomic per wave).
__device__ __forceinline__ void add_wave_steps(unsigned long long *ctr, unsigned long long mine)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    if (__lane_id() == 0 && mine) atomicAdd(ctr, mine);
}

// wave-aggregated atomic add (lanes with pred), returns each lane's slot
__device__ __forceinline__ int wave_append(int32_t *counter, bool pred, int lane)
{
    unsigned long long mask = __ballot(pred);
    int base = 0;
    if (mask) {
        int leader = __ffsll((long long)mask) - 1;
        if (lane == leader) base = atomicAdd(counter, __popcll(mask));
        base = __shfl(base, leader);
    }
    return base + __popcll(mask & ((1ull << lane) - 1ull));
}

// Sixteen lanes (a DPP row) per ray until every ray of the wave has
// terminated; rows with ray < 0 idle.  The row's lanes hold identical state
// and run identical arithmetic; only the stencil contraction is split (one
// column per lane, see medium<T, IP, 16>), so the results equal the
// one-lane kernel's bit for bit.  Lane 0 of the row writes.
template <typename T, int IP, bool UNROLL>
__device__ __forceinline__ void run_rows(const TraceParams<T> &P, const TraceParams<T> *Pp, int ray, Lane &L)
{
    const int lane = int(__lane_id());
    const bool lead = (lane & 15) == 0;
    StencilCache<T, 16> sc;
    sc.clear();
    sc.pa = piece<T, IP>((lane >> 2) & 3);
    sc.pb = piece<T, IP>(lane & 3);
    sc.set_masks(lane);
    unsigned long long nsteps = 0;
    for (;;) {
        if (__ballot(ray >= 0) == 0ull) break;
        if (ray >= 0) {
            nsteps += lead ? 1u : 0u;
            int st = advance<T, IP, 16, UNROLL>(P, Pp, ray, L, lead, sc);
            if (st >= 0) {
                if (lead) retire(P, ray, L, st);
                ray = -1;
            }
        }
    }
    add_wave_steps(P.phase_steps + 2, nsteps);
}

// Move the (at most four) live rays of the wave, marked in `live`, onto
// the wave's four 16-lane rows, in lane order; rows without a ray get -1.
__device__ __forceinline__ void gather_rows(unsigned long long live, int &ray, Lane &L)
{
    const int row = int(__lane_id()) >> 4;
    int src = -1;
    unsigned long long m = live;
    for (int i = 0; i < 4 && m; ++i) {
        const int b = __ffsll((long long)m) - 1;
        if (i == row) src = b;
        m &= m - 1ull;
    }
    const int s = src < 0 ? 0 : src;
    Lane M;
#pragma unroll
    for (int i = 0; i < 7; ++i) M.y[i] = __shfl(L.y[i], s);
    M.gp = __shfl(L.gp, s);
    M.apogee = __shfl(L.apogee, s);
    M.an.th = __shfl(L.an.th, s);
    M.an.s = __shfl(L.an.s, s);
    M.an.c = __shfl(L.an.c, s);
    M.az0 = __shfl(L.az0, s);
    M.rc.v = reinterpret_cast<const void *>(
        __shfl((unsigned long long)reinterpret_cast<uintptr_t>(L.rc.v), s));
    M.rc.inv_f2 = __shfl(L.rc.inv_f2, s);
    M.rc.YR3 = __shfl(L.rc.YR3, s);
    M.rc.sigma = __shfl(L.rc.sigma, s);
    M.steps = __shfl(L.steps, s);
    M.ntraj = __shfl(L.ntraj, s);
    M.seg = __shfl(L.seg, s);
    M.local = __shfl(L.local, s);
    M.trapped = __shfl(L.trapped, s);
    M.nr_lo = -1.0f;
    const int r = __shfl(ray, s);
    L = M;
    ray = src < 0 ? -1 : r;
}

// Promotion, producer side (a one-lane wave, every 32nd iteration): lanes
// whose ray is trapped in a duct or grazed a layer peak (see advance), or is
// at least promote_age steps old, move the ray to the promotion queue while
// there is room: trapped and grazing rays may fill all promote_cap places,
// old rays three quarters of them, so that the former (the longest rays)
// always find room.  The state goes to the ray's
// record, a ticket is taken, and the ray index is published under the
// ticket (release).  The lane then idles and refills from the launch queue.
// A member of the parameter block read from its device copy where it is
// used (a volatile load the compiler cannot hoist), so that members a loop
// needs only now and then hold no scalar registers across it.  The
// promotion waves read their queue and counter addresses this way: kept in
// scalar registers they spilled into vector lanes, a `v_readlane` each time
// the stepping loop touched them.
template <typename X>
__device__ __forceinline__ X fresh(const X &v) { return *reinterpret_cast<const volatile X *>(&v); }

template <typename T>
__device__ __forceinline__ int promote_room(const TraceParams<T> &P, unsigned long long cm, int cap, int lane)
{
    const int k = __popcll(cm);
    int room = 0;
    if (lane == 0 && k > 0) {
        const int old = atomicAdd(P.promo_live, k);
        room = min(k, max(0, cap - old));
        if (room < k) atomicSub(P.promo_live, k - room);
    }
    return __shfl(room, 0);
}

template <typename T>
__device__ __forceinline__ void promote(const TraceParams<T> &P, int &ray, const Lane &L, int lane)
{
    const unsigned long long below = (1ull << lane) - 1ull;
    const bool trap = ray >= 0 && L.trapped != 0;
    const bool aged = ray >= 0 && L.trapped == 0 && P.promote_age > 0 && L.steps >= P.promote_age;
    const unsigned long long tm = __ballot(trap), am = __ballot(aged);
    if ((tm | am) == 0ull) return;
    const int rt = promote_room(P, tm, P.promote_cap, lane);
    const int ra = promote_room(P, am, P.promote_cap - P.promote_cap / 4, lane);
    const bool go = (trap && __popcll(tm & below) < rt) || (aged && __popcll(am & below) < ra);
    if (__ballot(go) == 0ull) return;
    if (go) P.rec[ray].L = L;
    const int t = wave_append(P.promo_push, go, lane);
    if (go) {
        __hip_atomic_store(&P.promo_ids[t], ray, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        ray = -1;
    }
}

// Promotion, consumer side (one lane of a promotion wave's row): claim the
// next ticket if one is issued and not yet claimed, and wait for its ray
// index (the producer publishes it right after taking the ticket).  Returns
// the ray, or -1 if there is nothing to claim.  Both waits are bounded; a
// publication that does not arrive is counted in promo_err.
template <typename T>
__device__ __forceinline__ int claim_promoted(const TraceParams<T> &P)
{
    int p = __hip_atomic_load(P.promo_pop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int k = 0; k < 64; ++k) {
        const int q = __hip_atomic_load(P.promo_push, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p >= q) return -1;
        const int seen = atomicCAS(P.promo_pop, p, p + 1);
        if (seen == p) {
            for (int w = 0; w < (1 << 22); ++w) {
                const int r = __hip_atomic_load(&P.promo_ids[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (r >= 0) return r;
                __builtin_amdgcn_s_sleep(1);
            }
            atomicAdd(P.promo_err, 1);
            return -1;
        }
        p = seen;
    }
    return -1;
}

// Persistent one-lane-per-ray kernel.  Each 64-lane wave loops { refill
// idle lanes from the queue; one RK4 step on every live lane } until the
// queue is drained and every lane is idle.  Rays are visited in index order,
// in the order (q * perm_stride) mod n_rays, which spreads runs of
// neighbouring (and similarly long) rays over many waves, or sorted by wave
// mode (order, written by k_start).  Once the queue is drained, either
//   * (inwave) a wave left with at most four live rays moves them onto its
//     four 16-lane rows and finishes them there, or
//   * (handoff_threshold > 0) once at most handoff_threshold rays are live
//     in the whole launch, each remaining ray's state is written to the
//     hand-off buffer and the lane retires (the tail kernel finishes it with
//     sixteen lanes per ray).
// Every ray terminates (the group path grows by one step per iteration up
// to max_group), so every wave exits.
template <typename T, int IP>
__device__ __forceinline__ void trace_body(const TraceParams<T> &P, const TraceParams<T> *__restrict__ Pp)
{
    const int lane = int(__lane_id());
    int ray = -1;            // -1 idle, -2 queue drained, >= 0 live ray
    bool drained = false;
    unsigned long long to_rows = 0ull;   // live rays moving to 16-lane rows
    Lane L;
    StencilCache<T, 1> sc;
    sc.clear();
    unsigned long long nsteps = 0, iters = 0;
    for (int iter = 0;; ++iter) {
        bool need = (ray == -1);
        if (__ballot(need)) {
            int q = wave_append(P.queue_head, need, lane);
            if (need) {
                if (q < P.n_rays) {
                    ray = P.order ? P.order[q]
                                  : int((unsigned long long)q * (unsigned long long)P.perm_stride %
                                        (unsigned long long)P.n_rays);
                    L = P.rec[ray].L;
                } else {
                    ray = -2;
                }
            }
            drained = drained || __ballot(ray == -2) != 0ull;
        }
        const unsigned long long livem = __ballot(ray >= 0);
        if (livem == 0ull) break;
        if (P.inwave && drained && __popcll(livem) <= 4) {
            to_rows = livem;
            break;
        }
        if (P.handoff_threshold > 0 && (iter & 7) == 0) {
            int live = 0, head = 0;
            if (lane == 0) {
                live = __hip_atomic_load(P.live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                head = __hip_atomic_load(P.queue_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            live = __shfl(live, 0);
            head = __shfl(head, 0);
            if (head >= P.n_rays && live <= P.handoff_threshold) {
                bool hand = ray >= 0;
                int slot = wave_append(P.n_handoff, hand, lane);
                if (hand) {
                    Handoff &H = P.handoff[slot];
#pragma unroll
                    for (int i = 0; i < 7; ++i) H.y[i] = L.y[i];
                    H.gp = L.gp;
                    H.apogee = L.apogee;
                    H.an = L.an;
                    H.ray = ray;
                    H.steps = L.steps;
                    H.ntraj = L.ntraj;
                    H.pad = 0;
                    ray = -2;
                }
                unsigned long long hm = __ballot(hand);
                if (lane == 0 && hm) atomicSub(P.live, __popcll(hm));
                break;
            }
        }
        // every 32nd iteration: an attempt costs atomics on shared counters
        if (P.promote_cap > 0 && (iter & 31) == 0) promote(P, ray, L, lane);
        iters += __ballot(ray >= 0) != 0ull ? 1u : 0u;
        int st = -1;
        if (ray >= 0) {
            ++nsteps;
            st = advance<T, IP, 1>(P, Pp, ray, L, true, sc);
            if (st >= 0) {
                retire(P, ray, L, st);
                ray = -1;
            }
        }
        unsigned long long fin = __ballot(st >= 0);
        if (lane == 0 && fin && P.handoff_threshold > 0) atomicSub(P.live, __popcll(fin));
    }
    add_wave_steps(P.phase_steps, nsteps);
    if (lane == 0 && iters) atomicAdd(P.wave_iters, iters);
    // Release: the wave's earlier tickets (promo_push) and records are
    // visible to any promotion wave that reads the decremented count with
    // acquire.  The fence covers every lane's operations (a wave waits on
    // its own memory counters), then one lane decrements.
    if (P.promote_cap > 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0)
            __hip_atomic_fetch_add(P.producers_alive, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // after the one-lane loop, so that its stencil cache is dead here
    if (to_rows) {
        gather_rows(to_rows, ray, L);
        run_rows<T, IP, false>(P, Pp, ray, L);
    }
}

// Tail kernel: sixteen lanes (a DPP row) per handed-off ray, four rays per
// wave.  The row's lanes hold identical state and run identical arithmetic;
// only the stencil contraction is split (one column per lane, see
// medium<T, IP, 16>), so the results equal the one-lane kernel's bit for
// bit.  Lane 0 of the row writes.  Launched with enough rows for the
// hand-off capacity; rows past the number of records exit at once.
template <typename T, int IP>
__device__ __forceinline__ void tail_body(const TraceParams<T> &P, const TraceParams<T> *__restrict__ Pp)
{
    const int lane = int(__lane_id());
    const int slot = int(blockIdx.x) * 4 + (lane >> 4);
    const int n = *P.n_handoff;
    int ray = -1;
    Lane L;
    if (slot < n) {
        const Handoff &H = P.handoff[slot];
        ray = H.ray;
        L = P.rec[ray].L;   // per-ray constants
#pragma unroll
        for (int i = 0; i < 7; ++i) L.y[i] = H.y[i];
        L.gp = H.gp;
        L.apogee = H.apogee;
        L.an = H.an;
        L.steps = H.steps;
        L.ntraj = H.ntraj;
    }
    run_rows<T, IP, true>(P, Pp, ray, L);
}

// Hand the rays of the rows marked `pred` (row leaders) to the tail kernel;
// returns how many (the same on every lane).
__device__ __forceinline__ int handoff_rows(bool pred, int ray, const Lane &L, int32_t *n_handoff, Handoff *buf,
                                            int lane)
{
    const int slot = wave_append(n_handoff, pred, lane);
    if (pred) {
        Handoff &H = buf[slot];
#pragma unroll
        for (int i = 0; i < 7; ++i) H.y[i] = L.y[i];
        H.gp = L.gp;
        H.apogee = L.apogee;
        H.an = L.an;
        H.ray = ray;
        H.steps = L.steps;
        H.ntraj = L.ntraj;
        H.pad = 0;
    }
    return __popcll(__ballot(pred));
}

// Promotion wave: four 16-lane rows (as in the tail kernel) run promoted
// rays, each row claiming the next ticket when it is idle.  When the
// launch-wide hand-off condition holds, the rows' rays, and any ray claimed
// after that, go to the tail kernel instead.  The wave exits once no
// one-lane wave is left and every ticket is claimed (one-lane waves always
// finish, so this is reached); an idle wait with work still possible is
// bounded in wall-clock time (idle_ticks, far above any launch's one-lane
// phase) and counted in promo_err if it runs out.
template <typename T, int IP>
__device__ __forceinline__ void promote_body(const TraceParams<T> &P, const TraceParams<T> *Pp)
{
    const int lane = int(__lane_id());
    const int lead_lane = lane & ~15;
    const bool lead = lane == lead_lane;
    StencilCache<T, 16> sc;
    sc.clear();
    sc.pa = piece<T, IP>((lane >> 2) & 3);
    sc.pb = piece<T, IP>(lane & 3);
    sc.set_masks(lane);
    int ray = -1;
    Lane L;
    bool closing = false;
    bool idling = false;
    long long idle_t0 = 0;
    unsigned long long nsteps = 0;
    for (;;) {
        // The shared counters are polled once per pass of this loop: every
        // pass while the whole wave is idle, and after at most 32 steps (or
        // as soon as a row's ray ends) while rows run.  A poll is a memory
        // round trip, and the running rows (the longest rays of the launch)
        // stall for it.
        if (!closing && fresh(Pp->handoff_threshold) > 0) {
            int live = 0, head = 0;
            if (lane == 0) {
                live = __hip_atomic_load(fresh(Pp->live), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                head = __hip_atomic_load(fresh(Pp->queue_head), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            live = __shfl(live, 0);
            head = __shfl(head, 0);
            closing = head >= fresh(Pp->n_rays) && live <= fresh(Pp->handoff_threshold);
        }
        // idle rows claim promoted rays
        if (__ballot(ray < 0) != 0ull) {
            int r = -1;
            if (lead && ray < 0) r = claim_promoted(*Pp);
            r = __shfl(r, lead_lane);
            if (r >= 0) {
                ray = r;
                L = fresh(Pp->rec)[ray].L;
                sc.clear();
            }
        }
        if (closing) {
            const int n = handoff_rows(lead && ray >= 0, ray, L, fresh(Pp->n_handoff), fresh(Pp->handoff), lane);
            if (lane == 0 && n > 0) {
                atomicSub(fresh(Pp->live), n);
                atomicSub(fresh(Pp->promo_live), n);
            }
            ray = -1;
        }
        if (__ballot(ray >= 0) != 0ull) {
            // The rows step in a loop of their own, which holds nothing of the
            // bookkeeping above: compiled inside this loop's body, the step
            // kept the ray state partly in AGPRs and issued about 15 % more
            // instructions than the tail kernel's.  It ends after 32 steps or
            // once a row's ray ends (that row then claims the next ticket).
            int n = 0;
            for (int k = 0; k < 32; ++k) {
                int st = -1;
                if (ray >= 0) {
                    nsteps += lead ? 1u : 0u;
                    st = advance<T, IP, 16, true>(P, Pp, ray, L, lead, sc);
                    if (st >= 0) {
                        if (lead) retire(P, ray, L, st);
                        ray = -1;
                    }
                }
                const unsigned long long fin = __ballot(lead && st >= 0);
                if (fin) {
                    n = __popcll(fin);
                    break;
                }
            }
            if (lane == 0 && n > 0) {
                if (fresh(Pp->handoff_threshold) > 0) atomicSub(fresh(Pp->live), n);
                atomicSub(fresh(Pp->promo_live), n);
            }
            idling = false;
        } else {
            // Exit check, ordered: the count of running one-lane waves is read
            // with acquire first.  Once it reads 0, every producer's tickets
            // were pushed before its release decrement, so the push count read
            // after it is final and no ticket can be left unclaimed.
            int alive = 0, popped = 0, pushed = 0;
            if (lane == 0) {
                alive = __hip_atomic_load(fresh(Pp->producers_alive), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                pushed = __hip_atomic_load(fresh(Pp->promo_push), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                popped = __hip_atomic_load(fresh(Pp->promo_pop), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            alive = __shfl(alive, 0);
            popped = __shfl(popped, 0);
            pushed = __shfl(pushed, 0);
            if (alive == 0 && popped >= pushed) break;
            const long long now = wall_clock64();
            if (!idling) {
                idling = true;
                idle_t0 = now;
            } else if (now - idle_t0 > fresh(Pp->idle_ticks)) {
                if (lane == 0) atomicAdd(fresh(Pp->promo_err), 1);
                break;
            }
            __builtin_amdgcn_s_sleep(32);
        }
    }
    add_wave_steps(P.phase_steps + 1, nsteps);
}

// Starting state of every launch ray (one thread per ray).
template <typename T>
__device__ __forceinline__ void start_body(const TraceParams<T> &P)
{
    const int ray = int(blockIdx.x) * 64 + int(threadIdx.x);
    if (ray >= P.n_rays) return;
    Lane L;
    init_ray(P, ray, L, true);
    RayRec &rec = P.rec[ray];
    rec.L = L;
    rec.status = -1;
    if (P.promo_ids) P.promo_ids[ray] = -1;
    if (P.order) {
        // Counting sort of the queue by wave mode, stable in ray index: O and
        // isotropic rays first, then X rays.  The counts follow from the fans'
        // shapes, so each ray's place is computed, not counted: within a
        // segment with both modes, mode m of frequency i_f holds rays
        // i_f * n_elev * n_az + j of its group; otherwise the segment's rays
        // keep their order.
        const Segment &S = P.seg[L.seg];
        const int ea = S.n_elev * S.n_az;
        const int i = L.local;
        const int grp = L.rc.sigma < 0 ? 1 : 0;
        const int pos = (S.n_mode == 2 && L.rc.sigma != 0) ? (i / (2 * ea)) * ea + i % ea : i;
        P.order[S.bin_pos[grp] + pos] = ray;
    }
}

// Outputs of every launch ray (one thread per ray), after the trace kernels,
// and the RK4 step counts per segment: summed over the wave's lanes of each
// segment first, so that there is one atomic per wave and segment rather
// than one per ray on a single address.
template <typename T>
__device__ __forceinline__ void finish_body(const TraceParams<T> &P)
{
    const int ray = int(blockIdx.x) * 64 + int(threadIdx.x);
    const bool valid = ray < P.n_rays;
    int seg = 0;
    unsigned long long steps = 0;
    bool lost = false;
    if (valid) {
        lost = P.rec[ray].status < 0;
        finish_ray(P, ray);
        seg = P.rec[ray].L.seg;
        steps = (unsigned long long)P.rec[ray].L.steps;
    }
    // A ray still without a final status was never finished by a trace
    // kernel: its outputs are not valid, and the launch reports an error.
    const unsigned long long lm = __ballot(lost);
    if (lm && int(threadIdx.x) == __ffsll((long long)lm) - 1) atomicAdd(P.unfinished, __popcll(lm));
    unsigned long long todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int s0 = __shfl(seg, leader);
        const bool mine = valid && seg == s0;
        unsigned long long part = mine ? steps : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
        if (int(threadIdx.x) == leader) atomicAdd(P.seg[s0].steps, part);
        todo &= ~__ballot(mine);
    }
}

// Oblique-ionogram extraction: one thread per (frequency, mode) trace scans
// its elevations for ground-range crossings of the receiver distance.
__global__ __launch_bounds__(64) void k_ionogram(const double *__restrict__ elev, int n_elev,
                                                 int n_trace, const double *__restrict__ group,
                                                 const double *__restrict__ phase,
                                                 const double *__restrict__ range,
                                                 const double *__restrict__ apogee,
                                                 const int32_t *__restrict__ status, double D,
                                                 int max_points, double *__restrict__ out,
                                                 int32_t *__restrict__ counts)
{
    int t = int(blockIdx.x) * 64 + int(threadIdx.x);
    if (t >= n_trace) return;
    int found = 0;
    const size_t base = size_t(t) * size_t(n_elev);
    for (int e = 0; e + 1 < n_elev; ++e) {
        size_t i0 = base + e, i1 = i0 + 1;
        if (status[i0] != kGround || status[i1] != kGround) continue;
        double d0 = range[i0] - D, d1 = range[i1] - D;
        if ((d0 < 0.0) == (d1 < 0.0)) continue;
        if (found < max_points) {
            double w = d0 / (d0 - d1);
            double *o = out + (size_t(t) * size_t(max_points) + size_t(found)) * 4;
            o[0] = fm(w, elev[e + 1] - elev[e], elev[e]);
            o[1] = fm(w, group[i1] - group[i0], group[i0]);
            o[2] = fm(w, phase[i1] - phase[i0], phase[i0]);
            o[3] = fm(w, apogee[i1] - apogee[i0], apogee[i0]);
        }
        ++found;
    }
    // unused slots are defined (zero), never stale memory
    for (int k = found; k < max_points; ++k) {
        double *o = out + (size_t(t) * size_t(max_points) + size_t(k)) * 4;
        o[0] = o[1] = o[2] = o[3] = 0.0;
    }
    counts[t] = found;
}

// Waves [0, n_producers) of the launch run one lane per ray, the others are
// promotion waves.  A work-group holds one wave (k_trace, k_trace_w2) or four
// (k_trace_g), and a wave's index is its place in the launch.
template <typename T, int IP>
__device__ __forceinline__ void trace_entry(const TraceParams<T> &P, const TraceParams<T> *Pp)
{
    const int wave = int(blockIdx.x) * int(blockDim.x >> 6) + int(threadIdx.x >> 6);
    if (wave >= P.n_producers) promote_body<T, IP>(P, Pp);
    else trace_body<T, IP>(P, Pp);
}

// Launch wrappers.  The *_w2 variants ask the compiler to fit two waves per
// SIMD (at most 256 VGPRs, spilling if needed); the plain ones let it use
// the whole register file (one wave per SIMD for the FP64 path).  k_trace_g
// runs four waves per work-group and is launched with an LDS reservation
// above half of a CU's LDS, so that each CU holds exactly one work-group:
// the promotion waves (the last work-groups) then have CUs to themselves.
template <typename T, int IP>
__global__ __launch_bounds__(64) void k_trace(const TraceParams<T> P, const TraceParams<T> *__restrict__ Pp)
{
    trace_entry<T, IP>(P, Pp);
}
template <typename T, int IP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void k_trace_w2(const TraceParams<T> P, const TraceParams<T> *__restrict__ Pp)
{
    trace_entry<T, IP>(P, Pp);
}
template <typename T, int IP>
__global__ __launch_bounds__(256) void k_trace_g(const TraceParams<T> P, const TraceParams<T> *__restrict__ Pp)
{
    trace_entry<T, IP>(P, Pp);
}
template <typename T, int IP>
__global__ __launch_bounds__(64) void k_tail(const TraceParams<T> P, const TraceParams<T> *__restrict__ Pp)
{
    tail_body<T, IP>(P, Pp);
}
template <typename T, int IP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void k_tail_w2(const TraceParams<T> P, const TraceParams<T> *__restrict__ Pp)
{
    tail_body<T, IP>(P, Pp);
}

template <typename T>
__global__ __launch_bounds__(64) void k_start(const TraceParams<T> P) { start_body<T>(P); }
template <typename T>
__global__ __launch_bounds__(64) void k_finish(const TraceParams<T> P) { finish_body<T>(P); }

}  // namespace

