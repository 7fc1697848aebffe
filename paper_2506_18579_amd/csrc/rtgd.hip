// rtgd.hip -- librtgd: persistent ray-tracing kernel for gfx950 and the
// C-ABI host side (contexts, grids, fields, traces).
//
// Design (one MI355X):
//   * one lane integrates one ray; its state (position, wave normal, phase
//     and group path) lives in registers for the ray's whole life;
//   * a persistent grid of single-wave workgroups pulls rays from a device
//     queue: when a lane's ray terminates the wave refills every idle lane
//     with one atomic (ballot + popcount), so waves stay full while rays of
//     very different lengths retire at different times;
//   * the density grid stays resident in HBM and is re-read through the L2
//     and Infinity Cache; nothing on the path is a dense contraction, so
//     all arithmetic is VALU (no MFMA).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rtgd.h"
#include "rtgd_device.h"

using namespace rtgd;

namespace {

// ---------------------------------------------------------------------------
// Kernel parameters (passed by value)
// ---------------------------------------------------------------------------
template <typename T>
struct TraceParams {
    GridDev<T> g;
    double B0;                 // 0: isotropic
    // fan: ray index = ((i_f * n_mode + i_m) * n_elev + i_e) * n_az + i_a
    const double *elev, *az, *freq;
    int32_t n_elev, n_az, n_freq, n_mode;
    int32_t mode_first;        // +1 if the first mode is O, -1 if X
    int32_t n_rays;
    double tx_lon;             // rad
    double up[3], north[3], east[3];   // transmitter frame (Cartesian)
    double r0;                 // R + tx height
    double step, max_group, exit_h, floor_h;
    int32_t max_steps;         // hard cap (never reached before max_group)
    int32_t traj_stride;
    int64_t traj_per_ray;
    // outputs (device)
    double *group, *phase, *range, *azdev, *apogee, *land_lat, *land_lon;
    int32_t *status, *nsteps;
    double *traj;
    int32_t *traj_count;
    // scheduling
    const int32_t *order;      // ray visiting order (NULL: identity)
    int32_t *queue_head;
    unsigned long long *total_steps;
    int32_t *truncated;
    // hand-off of the last live rays to the 4-lanes-per-ray tail kernel
    int32_t *live;             // rays neither finished nor handed off
    int32_t *n_handoff;        // records written
    struct Handoff *handoff;   // capacity handoff_threshold
    int32_t handoff_threshold; // hand off once fewer rays than this are live (0: never)
};

// State of a ray moved from the one-lane to the four-lane kernel.
struct Handoff {
    double y[7];
    double gp, apogee;
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
    int32_t steps;
    int32_t ntraj;
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

// Per-ray constants from the ray index (fan decode).
template <typename T>
__device__ __forceinline__ void ray_const(const TraceParams<T> &P, int ray, Lane &L, double &elev)
{
    int i = ray;
    int ia = i % P.n_az; i /= P.n_az;
    int ie = i % P.n_elev; i /= P.n_elev;
    int im = i % P.n_mode; i /= P.n_mode;
    int jf = i;
    elev = P.elev[ie];
    double f = P.freq[jf];
    int sigma = (im == 0) ? P.mode_first : -1;
    L.rc.inv_f2 = 1.0 / (f * f);
    L.rc.Y0 = kKB * P.B0 / (f * 1e6);
    L.rc.sigma = (P.B0 == 0.0) ? 0 : sigma;
    L.az0 = P.az[ia];
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
    L.steps = 0;
    L.ntraj = 0;
    if (P.traj_stride > 0 && write) put_traj(P, ray, L);
}

// Outputs of a terminated ray: landing (or sub-ray) point, ground range,
// azimuth deviation (Sec. II-C outputs, plus the phase path).
template <typename T>
__device__ __forceinline__ void finish_ray(const TraceParams<T> &P, int ray, Lane &L, int status)
{
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
    if (status == kNumeric) {
#pragma unroll
        for (int k = 0; k < 7; ++k) o[k] = __builtin_nan("");
    }
    if (P.group) P.group[ray] = o[0];
    if (P.phase) P.phase[ray] = o[1];
    if (P.range) P.range[ray] = o[2];
    if (P.azdev) P.azdev[ray] = o[3];
    if (P.apogee) P.apogee[ray] = o[4];
    if (P.land_lat) P.land_lat[ray] = o[5];
    if (P.land_lon) P.land_lon[ray] = o[6];
    if (P.status) P.status[ray] = status;
    if (P.nsteps) P.nsteps[ray] = L.steps;
    if (P.traj_count) P.traj_count[ray] = L.ntraj;
}

// One RK4 step plus the termination tests.  Returns the ray status, or -1
// if the ray goes on.  `write` is false on the lanes of a quad that only
// shadow the quad's leader (no memory writes).
template <typename T, int IP, int LANES>
__device__ __forceinline__ int advance(const TraceParams<T> &P, int ray, Lane &L, bool write,
                                       StencilCache<T, LANES> &sc)
{
    bool ok = rk4_step<T, IP, LANES>(P.g, L.rc, L.y, P.step, sc);
    L.gp += P.step;
    ++L.steps;
    double h = L.y[0] - P.g.R;
    int status = -1;
    int graze = 0;
    double x[3], d[3], s = 0.0;
    bool finite = ok;
#pragma unroll
    for (int i = 0; i < 7; ++i) finite = finite && isfinite(L.y[i]);
    if (!finite) {
        status = kNumeric;
    } else if (h < P.floor_h && L.y[3] < 0.0) {
        // below the grid bottom and descending: vacuum line to r = R
        state_to_cart(L.y, x, d);
        double xd = dot3(x, d);
        double c = dot3(x, x) - P.g.R * P.g.R;
        double disc = xd * xd - c;
        if (disc >= 0.0) {
            s = c / (-xd + sqrt(disc));
            status = kGround;
        } else {
            // grazing line missing the Earth: back up to the grid bottom
            double rb = P.g.R + P.floor_h;
            double c2 = dot3(x, x) - rb * rb;
            s = -xd + sqrt(xd * xd - c2);
            graze = 1;
        }
    } else if (h >= P.exit_h) {
        status = kEscape;
    } else if (L.gp >= P.max_group || L.steps >= P.max_steps) {
        status = kMaxPath;
    }
    if (status != kNumeric && h > L.apogee) L.apogee = h;
    if (P.traj_stride > 0 && write && (L.steps % P.traj_stride == 0 || status >= 0)) put_traj(P, ray, L);

    if (status == kGround) {
#pragma unroll
        for (int i = 0; i < 3; ++i) x[i] += s * d[i];
        L.gp += s;
        L.y[6] += s;
        L.y[0] = sqrt(dot3(x, x));
        L.y[1] = atan2(sqrt(x[0] * x[0] + x[1] * x[1]), x[2]);
        L.y[2] = lon_near(x[0], x[1], P.tx_lon);
    } else if (graze) {
#pragma unroll
        for (int i = 0; i < 3; ++i) x[i] += s * d[i];
        L.gp += s;
        double ph = L.y[6] + s;
        cart_to_state(x, d, P.tx_lon, L.y);
        L.y[6] = ph;
    }
    return status;
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

// Persistent one-lane-per-ray kernel.  Each 64-lane wave loops { refill
// idle lanes from the queue; one RK4 step on every live lane } until the
// queue is drained and every lane is idle.  When the queue is drained and
// fewer than handoff_threshold rays are live, each remaining ray's state is
// written to the hand-off buffer and the lane retires (the tail kernel
// finishes it with four lanes per ray).  Every ray terminates (the group
// path grows by one step per iteration up to max_group), so every wave exits.
template <typename T, int IP>
__device__ __forceinline__ void trace_body(const TraceParams<T> *__restrict__ Pp)
{
    const TraceParams<T> &P = *Pp;
    const int lane = int(__lane_id());
    int ray = -1;            // -1 idle, -2 queue drained, >= 0 live ray
    Lane L;
    StencilCache<T, 1> sc;
    sc.clear();
    unsigned long long my_steps = 0;
    for (int iter = 0;; ++iter) {
        bool need = (ray == -1);
        if (__ballot(need)) {
            int q = wave_append(P.queue_head, need, lane);
            if (need) {
                if (q < P.n_rays) {
                    ray = P.order ? P.order[q] : q;
                    init_ray(P, ray, L, true);
                } else {
                    ray = -2;
                }
            }
        }
        if (__ballot(ray >= 0) == 0ull) break;
        if (P.handoff_threshold > 0 && (iter & 7) == 0) {
            int live = 0, head = 0;
            if (lane == 0) {
                live = __hip_atomic_load(P.live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                head = __hip_atomic_load(P.queue_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            live = __shfl(live, 0);
            head = __shfl(head, 0);
            if (head >= P.n_rays && live < P.handoff_threshold) {
                bool hand = ray >= 0;
                int slot = wave_append(P.n_handoff, hand, lane);
                if (hand) {
                    Handoff &H = P.handoff[slot];
#pragma unroll
                    for (int i = 0; i < 7; ++i) H.y[i] = L.y[i];
                    H.gp = L.gp;
                    H.apogee = L.apogee;
                    H.ray = ray;
                    H.steps = L.steps;
                    H.ntraj = L.ntraj;
                    H.pad = 0;
                    my_steps += (unsigned long long)L.steps;
                    ray = -2;
                }
                unsigned long long hm = __ballot(hand);
                if (lane == 0 && hm) atomicSub(P.live, __popcll(hm));
                break;
            }
        }
        int st = -1;
        if (ray >= 0) {
            st = advance<T, IP, 1>(P, ray, L, true, sc);
            if (st >= 0) {
                finish_ray(P, ray, L, st);
                my_steps += (unsigned long long)L.steps;
                ray = -1;
            }
        }
        unsigned long long fin = __ballot(st >= 0);
        if (lane == 0 && fin && P.handoff_threshold > 0) atomicSub(P.live, __popcll(fin));
    }
    // wave-reduce the step count, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) my_steps += __shfl_down(my_steps, off);
    if (lane == 0) atomicAdd(P.total_steps, my_steps);
}

// Tail kernel: four lanes (a quad) per handed-off ray.  The quad's lanes
// hold identical state and run identical arithmetic; only the stencil
// contraction is split (one latitude row per lane, see medium<T, 4>), so
// the results equal the one-lane kernel's bit for bit.  Lane 0 of the quad
// writes.  Launched with enough quads for the hand-off capacity; quads past
// the number of records exit at once.
template <typename T, int IP>
__device__ __forceinline__ void tail_body(const TraceParams<T> *__restrict__ Pp)
{
    const TraceParams<T> &P = *Pp;
    const int lane = int(__lane_id());
    const int slot = int(blockIdx.x) * 16 + (lane >> 2);
    const bool lead = (lane & 3) == 0;
    const int n = *P.n_handoff;
    int ray = -1;
    Lane L;
    StencilCache<T, 4> sc;
    sc.clear();
    if (slot < n) {
        const Handoff &H = P.handoff[slot];
        ray = H.ray;
        double elev_unused;
        ray_const(P, ray, L, elev_unused);
#pragma unroll
        for (int i = 0; i < 7; ++i) L.y[i] = H.y[i];
        L.gp = H.gp;
        L.apogee = H.apogee;
        L.steps = H.steps;
        L.ntraj = H.ntraj;
    }
    unsigned long long my_steps = 0;
    for (;;) {
        if (__ballot(ray >= 0) == 0ull) break;
        if (ray >= 0) {
            int st = advance<T, IP, 4>(P, ray, L, lead, sc);
            if (st >= 0) {
                if (lead) {
                    finish_ray(P, ray, L, st);
                    my_steps += (unsigned long long)(L.steps - P.handoff[slot].steps);
                }
                ray = -1;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) my_steps += __shfl_down(my_steps, off);
    if (lane == 0) atomicAdd(P.total_steps, my_steps);
}

// Launch wrappers.  The *_w2 variants ask the compiler to fit two waves per
// SIMD (at most 256 VGPRs, spilling if needed); the plain ones let it use
// the whole register file (one wave per SIMD for the FP64 path).
template <typename T, int IP>
__global__ __launch_bounds__(64) void k_trace(const TraceParams<T> *__restrict__ P) { trace_body<T, IP>(P); }
template <typename T, int IP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void k_trace_w2(const TraceParams<T> *__restrict__ P) { trace_body<T, IP>(P); }
template <typename T, int IP>
__global__ __launch_bounds__(64) void k_tail(const TraceParams<T> *__restrict__ P) { tail_body<T, IP>(P); }
template <typename T, int IP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void k_tail_w2(const TraceParams<T> *__restrict__ P) { tail_body<T, IP>(P); }

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================
struct rt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int n_cu = 0;
    // workspace (grow-only)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *stage = nullptr;      // result staging for host outputs
    size_t stage_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct rt_grid {
    rt_ctx *ctx = nullptr;
    rt_grid_geom geom{};
    double *d_f64 = nullptr;    // f_N^2 MHz^2, FP64
    float *d_f32 = nullptr;     // f_N^2 MHz^2, FP32 (mixed path)
    double B0 = 0.0;
};

namespace {

// message of the last failed rt_ctx_create on this thread
thread_local std::string g_create_error;

rt_status fail(rt_ctx *ctx, rt_status code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

#define HIP_OR_FAIL(ctx, call)                                                              \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, e_ == hipErrorOutOfMemory ? RT_E_NOMEM : RT_E_DEVICE,          \
                        std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

int popcount_modes(uint32_t m) { return int((m & 1u) != 0) + int((m & 2u) != 0); }

rt_status ensure_ws(rt_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes) return RT_OK;
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    size_t want = std::max(bytes, size_t(1) << 20);
    HIP_OR_FAIL(ctx, hipMalloc(&ctx->ws, want));
    ctx->ws_bytes = want;
    return RT_OK;
}

rt_status ensure_stage(rt_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->stage_bytes) return RT_OK;
    if (ctx->stage) (void)hipFree(ctx->stage);
    ctx->stage = nullptr;
    ctx->stage_bytes = 0;
    HIP_OR_FAIL(ctx, hipMalloc(&ctx->stage, bytes));
    ctx->stage_bytes = bytes;
    return RT_OK;
}

__global__ void k_convert(const void *src, int src_f32, double scale, size_t n, double *d64,
                          float *d32)
{
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    size_t stride = size_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) {
        double v = src_f32 ? double(static_cast<const float *>(src)[i])
                           : static_cast<const double *>(src)[i];
        v *= scale;
        d64[i] = v;
        d32[i] = float(v);
    }
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

extern "C" {

void rt_default_opts(rt_trace_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->step_km = 1.0;
    o->max_group_km = 4000.0;
    o->exit_h_km = 0.0;
    o->precision = RT_FP64;
    o->results_mem = RT_MEM_HOST;
}

rt_status rt_check_geom(const rt_grid_geom *g)
{
    if (!g) return RT_E_INVALID;
    if (g->n_lat < 4 || g->n_lon < 4 || g->n_h < 4) return RT_E_INVALID;
    if (!(g->dlat_deg > 0) || !(g->dlon_deg > 0) || !(g->dh_km > 0)) return RT_E_INVALID;
    if (!std::isfinite(g->lat0_deg) || !std::isfinite(g->lon0_deg) || !std::isfinite(g->h0_km))
        return RT_E_INVALID;
    double lat_hi = g->lat0_deg + (g->n_lat - 1) * g->dlat_deg;
    if (!(g->lat0_deg > -90.0) || !(lat_hi < 90.0)) return RT_E_INVALID;
    if (!(g->earth_radius_km > 0) || !std::isfinite(g->earth_radius_km)) return RT_E_INVALID;
    if (!(g->h0_km >= 0.0)) return RT_E_INVALID;
    if (g->dtype != RT_F64 && g->dtype != RT_F32) return RT_E_INVALID;
    if (g->quantity != RT_NE_M3 && g->quantity != RT_FN2_MHZ2) return RT_E_INVALID;
    if (g->interp != RT_INTERP_GD && g->interp != RT_INTERP_CR) return RT_E_INVALID;
    double total = double(g->n_lat) * double(g->n_lon) * double(g->n_h);
    if (total > 2.0e9) return RT_E_INVALID;
    return RT_OK;
}

rt_status rt_fan_count(const rt_fan *f, int64_t *n)
{
    if (!f || !n) return RT_E_INVALID;
    if (f->n_elev < 0 || f->n_az < 0 || f->n_freq < 0) return RT_E_INVALID;
    int nm = popcount_modes(f->modes);
    if ((f->modes & ~3u) != 0) return RT_E_INVALID;
    int64_t c = int64_t(f->n_elev) * f->n_az * f->n_freq * nm;
    if (c > INT32_MAX) return RT_E_INVALID;
    *n = c;
    return RT_OK;
}

rt_status rt_ctx_create(int32_t device, void *stream, rt_ctx **out)
{
    if (!out) return RT_E_INVALID;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device < 0 || device >= count) {
        g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e) +
                         ", count " + std::to_string(count) + ", device " + std::to_string(device);
        return RT_E_DEVICE;
    }
    rt_ctx *c = new (std::nothrow) rt_ctx();
    if (!c) return RT_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    hipDeviceProp_t prop;
    if ((e = hipSetDevice(device)) != hipSuccess ||
        (e = hipGetDeviceProperties(&prop, device)) != hipSuccess ||
        (e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        if (c->ev0) (void)hipEventDestroy(c->ev0);
        delete c;
        return RT_E_DEVICE;
    }
    c->n_cu = prop.multiProcessorCount;
    *out = c;
    return RT_OK;
}

void rt_ctx_destroy(rt_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->ws) (void)hipFree(c->ws);
    if (c->stage) (void)hipFree(c->stage);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

const char *rt_last_error(const rt_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

rt_status rt_grid_create(rt_ctx *ctx, const rt_grid_geom *geom, const void *values,
                         int32_t values_mem, rt_grid **out)
{
    if (!ctx || !out) return RT_E_INVALID;
    *out = nullptr;
    if (rt_check_geom(geom) != RT_OK) return fail(ctx, RT_E_INVALID, "invalid grid geometry");
    if (!values) return fail(ctx, RT_E_INVALID, "values is NULL");
    if (values_mem != RT_MEM_HOST && values_mem != RT_MEM_DEVICE)
        return fail(ctx, RT_E_INVALID, "values_mem must be RT_MEM_HOST or RT_MEM_DEVICE");
    size_t n = size_t(geom->n_lat) * geom->n_lon * geom->n_h;
    size_t esz = geom->dtype == RT_F32 ? 4 : 8;
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));

    // values must be finite and non-negative (checked on the host copy)
    std::vector<unsigned char> host;
    const void *hsrc = values;
    if (values_mem == RT_MEM_DEVICE) {
        host.resize(n * esz);
        HIP_OR_FAIL(ctx, hipMemcpy(host.data(), values, n * esz, hipMemcpyDeviceToHost));
        hsrc = host.data();
    }
    for (size_t i = 0; i < n; ++i) {
        double v = esz == 4 ? double(static_cast<const float *>(hsrc)[i])
                            : static_cast<const double *>(hsrc)[i];
        if (!(v >= 0.0) || !std::isfinite(v))
            return fail(ctx, RT_E_INVALID, "grid value " + std::to_string(i) +
                                               " is negative or not finite");
    }

    rt_grid *g = new (std::nothrow) rt_grid();
    if (!g) return fail(ctx, RT_E_NOMEM, "host allocation failed");
    g->ctx = ctx;
    g->geom = *geom;
    void *src = nullptr;
    hipError_t e = hipMalloc(&g->d_f64, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&g->d_f32, n * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&src, n * esz);
    if (e == hipSuccess)
        e = hipMemcpyAsync(src, hsrc, n * esz, hipMemcpyHostToDevice, ctx->stream);
    double scale = geom->quantity == RT_NE_M3 ? kKN * 1e-12 : 1.0;
    if (e == hipSuccess) {
        int blocks = int(std::min<size_t>((n + 255) / 256, 65536));
        hipLaunchKernelGGL(k_convert, dim3(blocks), dim3(256), 0, ctx->stream, src,
                           geom->dtype == RT_F32 ? 1 : 0, scale, n, g->d_f64, g->d_f32);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (src) (void)hipFree(src);
    if (e != hipSuccess) {
        if (g->d_f64) (void)hipFree(g->d_f64);
        if (g->d_f32) (void)hipFree(g->d_f32);
        delete g;
        return fail(ctx, e == hipErrorOutOfMemory ? RT_E_NOMEM : RT_E_DEVICE,
                    std::string("grid upload: ") + hipGetErrorString(e));
    }
    *out = g;
    return RT_OK;
}

void rt_grid_destroy(rt_grid *g)
{
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    if (g->d_f64) (void)hipFree(g->d_f64);
    if (g->d_f32) (void)hipFree(g->d_f32);
    delete g;
}

rt_status rt_field_set(rt_grid *g, const rt_dipole *d)
{
    if (!g) return RT_E_INVALID;
    if (!d || d->B0_tesla == 0.0) {
        g->B0 = 0.0;
        return RT_OK;
    }
    if (!std::isfinite(d->B0_tesla) || d->B0_tesla < 0.0)
        return fail(g->ctx, RT_E_INVALID, "B0 must be finite and >= 0");
    if (d->pole_lat_deg != 90.0)
        return fail(g->ctx, RT_E_UNSUPPORTED, "only the axial dipole (pole at 90N) is implemented");
    g->B0 = d->B0_tesla;
    return RT_OK;
}

}  // extern "C"

namespace {

template <typename T>
void fill_grid_dev(const rt_grid *grid, GridDev<T> &g, const T *v)
{
    const rt_grid_geom &q = grid->geom;
    g.v = v;
    g.n_lat = q.n_lat; g.n_lon = q.n_lon; g.n_h = q.n_h;
    g.lat0 = q.lat0_deg; g.lon0 = q.lon0_deg; g.h0 = q.h0_km;
    g.inv_dlat = 1.0 / q.dlat_deg; g.inv_dlon = 1.0 / q.dlon_deg; g.inv_dh = 1.0 / q.dh_km;
    g.lat_hi = q.lat0_deg + (q.n_lat - 1) * q.dlat_deg;
    g.lon_hi = q.lon0_deg + (q.n_lon - 1) * q.dlon_deg;
    g.h_hi = q.h0_km + (q.n_h - 1) * q.dh_km;
    g.R = q.earth_radius_km;
}

template <typename T>
int resident_waves(rt_ctx *ctx, const void *kernel)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess || per_cu < 1)
        per_cu = 4;
    return per_cu * ctx->n_cu;
}

// Upload the parameter block and counters, then launch the one-lane
// persistent kernel and, if hand-off is on, the four-lane tail kernel.
template <typename T>
rt_status launch_trace(rt_ctx *ctx, TraceParams<T> &P, int n_rays, char *d_params, char *d_counters,
                       int occ, int interp)
{
    struct Counters { int32_t head, trunc, live, n_handoff; unsigned long long total; } hc{};
    hc.live = n_rays;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(d_counters, &hc, sizeof(hc), hipMemcpyHostToDevice, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(d_params, &P, sizeof(P), hipMemcpyHostToDevice, ctx->stream));
    const TraceParams<T> *dp = reinterpret_cast<const TraceParams<T> *>(d_params);
    const bool cr = interp == RT_INTERP_CR;
    auto kt = occ == 2 ? (cr ? k_trace_w2<T, 1> : k_trace_w2<T, 0>) : (cr ? k_trace<T, 1> : k_trace<T, 0>);
    auto kl = occ == 2 ? (cr ? k_tail_w2<T, 1> : k_tail_w2<T, 0>) : (cr ? k_tail<T, 1> : k_tail<T, 0>);
    int max_waves = resident_waves<T>(ctx, reinterpret_cast<const void *>(kt));
    int waves = std::max(1, std::min((n_rays + 63) / 64, max_waves));
    hipLaunchKernelGGL(kt, dim3(waves), dim3(64), 0, ctx->stream, dp);
    HIP_OR_FAIL(ctx, hipGetLastError());
    if (P.handoff_threshold > 0) {
        int quads_blocks = (P.handoff_threshold + 15) / 16;
        hipLaunchKernelGGL(kl, dim3(quads_blocks), dim3(64), 0, ctx->stream, dp);
        HIP_OR_FAIL(ctx, hipGetLastError());
    }
    // hipMemcpyAsync from pageable host memory may return before the copy is
    // consumed; keep the host structs alive until the stream is synchronised
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

}  // namespace

extern "C" rt_status rt_trace(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                              const rt_trace_opts *opts, rt_results *res)
{
    if (!ctx) return RT_E_INVALID;
    if (!grid || !fan || !opts || !res) return fail(ctx, RT_E_INVALID, "NULL argument");
    if (grid->ctx != ctx) return fail(ctx, RT_E_INVALID, "grid belongs to another context");
    int64_t n64 = 0;
    if (rt_fan_count(fan, &n64) != RT_OK) return fail(ctx, RT_E_INVALID, "invalid fan");
    res->total_steps = 0;
    res->kernel_ms = 0.0;
    if (n64 == 0) return RT_OK;
    const int n_rays = int(n64);
    const rt_grid_geom &gq = grid->geom;
    if (!(opts->step_km > 0) || !std::isfinite(opts->step_km))
        return fail(ctx, RT_E_INVALID, "step_km must be > 0");
    if (!(opts->max_group_km > 0) || !std::isfinite(opts->max_group_km))
        return fail(ctx, RT_E_INVALID, "max_group_km must be > 0");
    if (opts->max_group_km / opts->step_km > 1.0e8)
        return fail(ctx, RT_E_INVALID, "max_group_km / step_km exceeds 1e8 steps");
    if (opts->precision != RT_FP64 && opts->precision != RT_MIXED)
        return fail(ctx, RT_E_INVALID, "precision must be RT_FP64 or RT_MIXED");
    if (opts->results_mem != RT_MEM_HOST && opts->results_mem != RT_MEM_DEVICE)
        return fail(ctx, RT_E_INVALID, "results_mem must be RT_MEM_HOST or RT_MEM_DEVICE");
    if (opts->tail_threshold > (1 << 24))
        return fail(ctx, RT_E_INVALID, "tail_threshold too large");
    if (opts->traj_stride < 0 || opts->traj_capacity < 0)
        return fail(ctx, RT_E_INVALID, "negative trajectory option");
    if (opts->traj_stride > 0 && (!res->traj || opts->traj_capacity < n64))
        return fail(ctx, RT_E_INVALID, "trajectory needs traj and traj_capacity >= n_rays");
    if (!(fan->tx_h_km >= 0.0) || !(fan->tx_h_km < gq.h0_km))
        return fail(ctx, RT_E_UNSUPPORTED, "transmitter must lie below the grid bottom");
    if (!std::isfinite(fan->tx_lat_deg) || std::fabs(fan->tx_lat_deg) >= 90.0 ||
        !std::isfinite(fan->tx_lon_deg))
        return fail(ctx, RT_E_INVALID, "bad transmitter position");
    for (int i = 0; i < fan->n_elev; ++i)
        if (!(fan->elev_deg[i] >= 0.0 && fan->elev_deg[i] <= 90.0))
            return fail(ctx, RT_E_INVALID, "elevation outside [0, 90]");
    for (int i = 0; i < fan->n_az; ++i)
        if (!std::isfinite(fan->az_deg[i])) return fail(ctx, RT_E_INVALID, "azimuth not finite");
    const double fH_max = kKB * 2.0 * grid->B0 / 1e6;   // MHz, at the poles on the ground
    for (int i = 0; i < fan->n_freq; ++i) {
        double f = fan->freq_mhz[i];
        if (!(f > 0.0) || !std::isfinite(f)) return fail(ctx, RT_E_INVALID, "frequency must be > 0");
        if (grid->B0 != 0.0 && f <= fH_max)
            return fail(ctx, RT_E_UNSUPPORTED, "frequency at or below the gyrofrequency (Y >= 1)");
    }
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));

    // ---- workspace layout: fan | counters | staged outputs ----
    if (opts->waves_per_simd < 0 || opts->waves_per_simd > 2)
        return fail(ctx, RT_E_INVALID, "waves_per_simd must be 0, 1 or 2");
    // register budget of the kernels: FP64 defaults to the full register
    // file (one wave per SIMD), the mixed path fits two waves anyway
    const int occ = opts->waves_per_simd == 0 ? 1 : opts->waves_per_simd;
    int tail = opts->tail_threshold;
    if (tail == 0) tail = ctx->n_cu * 64;     // library default
    if (tail < 0) tail = 0;                   // hand-off off
    tail = int(std::min<int64_t>(tail, n64));
    const size_t nf = size_t(fan->n_elev) + fan->n_az + fan->n_freq;
    const size_t off_par = align_up(nf * sizeof(double), 256);
    const size_t off_cnt = off_par + align_up(sizeof(TraceParams<double>), 256);
    const size_t off_hand = off_cnt + 256;
    const size_t ws_bytes = off_hand + size_t(tail) * sizeof(Handoff) + 256;
    rt_status st = ensure_ws(ctx, ws_bytes);
    if (st != RT_OK) return st;
    char *ws = static_cast<char *>(ctx->ws);
    double *d_fan = reinterpret_cast<double *>(ws);
    char *d_params = ws + off_par;
    char *d_counters = ws + off_cnt;
    int32_t *d_head = reinterpret_cast<int32_t *>(d_counters);
    int32_t *d_trunc = reinterpret_cast<int32_t *>(d_counters + 4);
    int32_t *d_live = reinterpret_cast<int32_t *>(d_counters + 8);
    int32_t *d_nhand = reinterpret_cast<int32_t *>(d_counters + 12);
    unsigned long long *d_total = reinterpret_cast<unsigned long long *>(d_counters + 16);
    Handoff *d_hand = reinterpret_cast<Handoff *>(ws + off_hand);

    std::vector<double> hfan(nf);
    std::copy(fan->elev_deg, fan->elev_deg + fan->n_elev, hfan.begin());
    std::copy(fan->az_deg, fan->az_deg + fan->n_az, hfan.begin() + fan->n_elev);
    std::copy(fan->freq_mhz, fan->freq_mhz + fan->n_freq, hfan.begin() + fan->n_elev + fan->n_az);
    HIP_OR_FAIL(ctx, hipMemcpyAsync(d_fan, hfan.data(), nf * sizeof(double),
                                    hipMemcpyHostToDevice, ctx->stream));

    const bool host_out = opts->results_mem == RT_MEM_HOST;
    const size_t N = size_t(n_rays);
    const int64_t per_ray = opts->traj_stride > 0 ? opts->traj_capacity / n64 : 0;
    double *dbl[7] = {res->group_km, res->phase_km, res->range_km, res->az_dev_deg,
                      res->apogee_km, res->land_lat_deg, res->land_lon_deg};
    double *dev_dbl[7];
    int32_t *dev_status = res->status, *dev_nsteps = res->n_steps, *dev_tcount = res->traj_count;
    double *dev_traj = res->traj;
    if (host_out) {
        size_t bytes = 7 * N * 8 + 3 * N * 4 + 64;
        if (per_ray > 0) bytes = align_up(bytes, 256) + size_t(per_ray) * N * 64;
        st = ensure_stage(ctx, bytes);
        if (st != RT_OK) return st;
        char *sp = static_cast<char *>(ctx->stage);
        for (int k = 0; k < 7; ++k) dev_dbl[k] = dbl[k] ? reinterpret_cast<double *>(sp + k * N * 8) : nullptr;
        char *ip = sp + 7 * N * 8;
        dev_status = res->status ? reinterpret_cast<int32_t *>(ip) : nullptr;
        dev_nsteps = res->n_steps ? reinterpret_cast<int32_t *>(ip + N * 4) : nullptr;
        dev_tcount = res->traj_count ? reinterpret_cast<int32_t *>(ip + 2 * N * 4) : nullptr;
        dev_traj = per_ray > 0 ? reinterpret_cast<double *>(sp + align_up(7 * N * 8 + 3 * N * 4 + 64, 256))
                               : nullptr;
    } else {
        for (int k = 0; k < 7; ++k) dev_dbl[k] = dbl[k];
    }

    const double la = fan->tx_lat_deg * kDeg2Rad, lo = fan->tx_lon_deg * kDeg2Rad;
    auto fill_common = [&](auto &P) {
        P.B0 = grid->B0;
        P.elev = d_fan;
        P.az = d_fan + fan->n_elev;
        P.freq = d_fan + fan->n_elev + fan->n_az;
        P.n_elev = fan->n_elev; P.n_az = fan->n_az; P.n_freq = fan->n_freq;
        P.n_mode = popcount_modes(fan->modes);
        P.mode_first = (fan->modes & RT_MODE_O) ? 1 : -1;
        P.n_rays = n_rays;
        P.tx_lon = lo;
        P.up[0] = std::cos(la) * std::cos(lo); P.up[1] = std::cos(la) * std::sin(lo); P.up[2] = std::sin(la);
        P.north[0] = -std::sin(la) * std::cos(lo); P.north[1] = -std::sin(la) * std::sin(lo);
        P.north[2] = std::cos(la);
        P.east[0] = -std::sin(lo); P.east[1] = std::cos(lo); P.east[2] = 0.0;
        P.r0 = gq.earth_radius_km + fan->tx_h_km;
        P.step = opts->step_km;
        P.max_group = opts->max_group_km;
        P.exit_h = opts->exit_h_km > 0 ? opts->exit_h_km : gq.h0_km + (gq.n_h - 1) * gq.dh_km;
        P.floor_h = gq.h0_km;
        P.max_steps = int32_t(std::ceil(opts->max_group_km / opts->step_km)) + 2;
        P.traj_stride = opts->traj_stride;
        P.traj_per_ray = per_ray;
        P.group = dev_dbl[0]; P.phase = dev_dbl[1]; P.range = dev_dbl[2]; P.azdev = dev_dbl[3];
        P.apogee = dev_dbl[4]; P.land_lat = dev_dbl[5]; P.land_lon = dev_dbl[6];
        P.status = dev_status; P.nsteps = dev_nsteps;
        P.traj = dev_traj; P.traj_count = dev_tcount;
        P.order = nullptr;
        P.queue_head = d_head;
        P.total_steps = d_total;
        P.truncated = d_trunc;
        P.live = d_live;
        P.n_handoff = d_nhand;
        P.handoff = d_hand;
        P.handoff_threshold = tail;
    };

    HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if (opts->precision == RT_MIXED) {
        TraceParams<float> P{};
        fill_grid_dev<float>(grid, P.g, grid->d_f32);
        fill_common(P);
        st = launch_trace(ctx, P, n_rays, d_params, d_counters, occ, gq.interp);
    } else {
        TraceParams<double> P{};
        fill_grid_dev<double>(grid, P.g, grid->d_f64);
        fill_common(P);
        st = launch_trace(ctx, P, n_rays, d_params, d_counters, occ, gq.interp);
    }
    if (st != RT_OK) return st;
    HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev1, ctx->stream));

    unsigned long long total = 0;
    int32_t trunc = 0;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&total, d_total, sizeof(total), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&trunc, d_trunc, sizeof(trunc), hipMemcpyDeviceToHost, ctx->stream));
    if (host_out) {
        for (int k = 0; k < 7; ++k)
            if (dbl[k])
                HIP_OR_FAIL(ctx, hipMemcpyAsync(dbl[k], dev_dbl[k], N * 8, hipMemcpyDeviceToHost, ctx->stream));
        if (res->status)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->status, dev_status, N * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (res->n_steps)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->n_steps, dev_nsteps, N * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (res->traj_count)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->traj_count, dev_tcount, N * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (per_ray > 0)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->traj, dev_traj, size_t(per_ray) * N * 64,
                                            hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    res->total_steps = int64_t(total);
    res->kernel_ms = ms;
    return trunc ? RT_W_TRAJ_TRUNCATED : RT_OK;
}
