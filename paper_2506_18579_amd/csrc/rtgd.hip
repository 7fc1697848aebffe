// rtgd.hip -- librtgd: the C-ABI host side (contexts, grids, fields,
// traces, ionograms, the request server, graph plans, the autotuner) around
// the trace kernels of rtgd_kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstddef>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <fstream>
#include <sstream>
#include <unordered_map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rtgd.h"
#include "rtgd_device.h"
#include "rtgd_kernels.h"

// ===========================================================================
// Host side
// ===========================================================================
struct rt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int n_cu = 0;
    int lds_lock = 0;           // LDS bytes per work-group that leave room for one per CU (0: none)
    int64_t wall_khz = 0;       // rate of the device's constant wall clock
    // workspace (grow-only)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *stage = nullptr;      // result staging for host outputs
    size_t stage_bytes = 0;
    void *pinned = nullptr;     // pinned host staging of fan, parameters, counters
    size_t pinned_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evm = nullptr;   // between the one-lane and the tail kernel
    // rt_trace_noalloc: the device's scratch region (address of `scratch`
    // on this context's device) and host staging of the fan, segment,
    // parameter block and counters, sized for its limits
    char *scratch = nullptr;
    alignas(256) char noalloc_host[(RT_NOALLOC_MAX_AXIS * 8 + 16384 + 255) / 256 * 256];
};

struct rt_grid {
    rt_ctx *ctx = nullptr;
    rt_grid_geom geom{};
    double *d_f64 = nullptr;    // f_N^2 MHz^2, FP64
    float *d_f32 = nullptr;     // f_N^2 MHz^2, FP32 (mixed path)
    double B0 = 0.0;
};

// Scratch region of rt_trace_noalloc: one per device (each device holds its
// own copy of a __device__ array), alive until the process ends.  Host code
// never passes the array's name to a kernel or a copy: on the host it is a
// stand-in, not a device address.  Its device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) char scratch[RT_NOALLOC_SCRATCH_BYTES];

namespace {

// message of the last failed rt_ctx_create on this thread
thread_local std::string g_create_error;

// device address of `scratch` on each device (nullptr until first looked up)
std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;

hipError_t scratch_address(int device, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the current device's copy
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<char *>(p);
    *out = static_cast<char *>(p);
    return hipSuccess;
}

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

// The trace kernels of one precision and variant (bit 0: Catmull-Rom
// interpolation, bit 1: every ray anisotropic).
struct KernelSet {
    const void *trace, *trace_w2, *trace_g, *tail, *tail_w2;
};

template <typename T, int V>
KernelSet kernel_set_of()
{
    return {(const void *)k_trace<T, V>, (const void *)k_trace_w2<T, V>, (const void *)k_trace_g<T, V>,
            (const void *)k_tail<T, V>, (const void *)k_tail_w2<T, V>};
}

template <typename T>
KernelSet kernel_set(int variant)
{
    switch (variant & 3) {
    case 0: return kernel_set_of<T, 0>();
    case 1: return kernel_set_of<T, 1>();
    case 2: return kernel_set_of<T, 2>();
    default: return kernel_set_of<T, 3>();
    }
}

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
        (e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess ||
        (e = hipEventCreate(&c->evm)) != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        if (c->ev0) (void)hipEventDestroy(c->ev0);
        if (c->ev1) (void)hipEventDestroy(c->ev1);
        if (c->evm) (void)hipEventDestroy(c->evm);
        delete c;
        return RT_E_DEVICE;
    }
    // the no-allocation scratch region of this device (only rt_trace_noalloc
    // needs it: without it that call fails, nothing else does)
    if (scratch_address(device, &c->scratch) != hipSuccess) c->scratch = nullptr;
    c->n_cu = prop.multiProcessorCount;
    // one work-group per CU for the grouped one-lane kernel: reserve more
    // than half of a CU's LDS per work-group (the kernels use none)
    {
        const size_t per_cu = prop.maxSharedMemoryPerMultiProcessor;
        const size_t lock = per_cu / 2 + 4096;
        bool ok = per_cu > 0 && lock <= prop.sharedMemPerBlock;
        for (int v = 0; ok && v < 4; ++v)
            ok = hipFuncSetAttribute(kernel_set<double>(v).trace_g, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     int(lock)) == hipSuccess &&
                 hipFuncSetAttribute(kernel_set<float>(v).trace_g, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     int(lock)) == hipSuccess;
        if (ok)
            c->lds_lock = int(lock);
    }
    int wall = 0;
    if (hipDeviceGetAttribute(&wall, hipDeviceAttributeWallClockRate, device) != hipSuccess || wall <= 0)
        wall = 100000;          // 100 MHz, the usual rate
    c->wall_khz = wall;
    *out = c;
    return RT_OK;
}

void rt_ctx_destroy(rt_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->ws) (void)hipFree(c->ws);
    if (c->stage) (void)hipFree(c->stage);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->evm) (void)hipEventDestroy(c->evm);
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
void fill_grid_dev(const rt_grid *grid, GridDev<T> &g)
{
    const rt_grid_geom &q = grid->geom;
    g.n_lat = q.n_lat; g.n_lon = q.n_lon; g.n_h = q.n_h;
    g.h0 = q.h0_km;
    // t_lat = (90 - th deg - lat0) / dlat, t_lon = (ph deg - lon0) / dlon,
    // t_h = (h - h0) / dh as affine maps of th, ph (rad) and h
    const double inv_dlat = 1.0 / q.dlat_deg, inv_dlon = 1.0 / q.dlon_deg;
    g.lat_a = -kRad2Deg * inv_dlat;
    g.lat_b = (90.0 - q.lat0_deg) * inv_dlat;
    g.lon_a = kRad2Deg * inv_dlon;
    g.lon_b = -q.lon0_deg * inv_dlon;
    g.inv_dh = 1.0 / q.dh_km;
    g.h_b = -q.h0_km * g.inv_dh;
    g.kmax_lat = double(q.n_lat - 3); g.kmax_lon = double(q.n_lon - 3); g.kmax_h = double(q.n_h - 3);
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

// One validated request of a launch: its grid, fan (host arrays) and where
// its per-ray outputs go on the device.
struct JobSeg {
    const rt_grid *grid = nullptr;
    rt_fan fan{};
    int n_rays = 0;
    double *out[7] = {};       // group, phase, range, az_dev, apogee, land_lat, land_lon
    int32_t *status = nullptr, *nsteps = nullptr;
};

// A launch: one or more requests that share the grid geometry, the
// transmitter and the options.
struct TraceJob {
    std::vector<JobSeg> segs;
    JobSeg *one = nullptr;     // set: the launch's single segment, held by the caller (no heap)
    rt_trace_opts opts{};
    int n_rays = 0;
    int tail = 0;              // launch-wide hand-off threshold actually used (0: none)
    int inwave = 0;            // in-wave switch to 16 lanes per ray
    int64_t perm = 1;          // visiting stride
    bool binned = false;       // queue sorted by wave mode
    int occ = 1;               // register budget variant
    int promote = 0;           // promotion waves (0: none)
    int promote_age = 0;       // promote rays of at least this many steps too (0: trapped and grazing rays only)
    int32_t *tcount = nullptr;
    double *traj = nullptr;
    int64_t per_ray = 0;
    size_t n_segs() const { return one ? 1 : segs.size(); }
    const JobSeg &seg(size_t k) const { return one ? *one : segs[k]; }
};

static_assert(sizeof(TraceParams<float>) <= sizeof(TraceParams<double>),
              "the workspace reserves room for the FP64 parameter block");

// Promotion waves (rt_trace_opts::promote_waves): at most, and the library
// defaults: 32 waves for launches of at least 8192 rays (smaller ones keep
// every wave for one-lane work), promoting trapped and grazing rays only.
constexpr int kMaxPromoteWaves = 64;
constexpr int kDefaultPromoteWaves = 32;
constexpr int kDefaultPromoteMinRays = 8192;
constexpr int kDefaultPromoteAge = 0;

// Counters the kernels update, read back after a launch (followed by one
// step counter per segment).
struct Counters {
    int32_t head, trunc, live, n_handoff;
    int32_t unfinished;        // rays left without a final status (k_finish)
    int32_t pad0[27];          // the promotion counters on cache lines of their own
    int32_t promo_push, promo_pop, promo_live, producers_alive, promo_err;
    int32_t pad1[27];
    // RK4 ray-steps by phase: one lane per ray, promotion rows, 16-lane rows
    // after the hand-off (or of the in-wave switch)
    unsigned long long phase_steps[3];
    unsigned long long wave_iters;   // one-lane wave iterations that stepped a ray
    int32_t pad2[8];
};
static_assert(sizeof(Counters) % 64 == 0, "counters fill whole cache lines");

// Workspace layout of a launch, the same on the device and in host staging
// (the hand-off buffer is device only): fan axes | segments | parameter
// block | counters + per-segment steps | hand-off buffer.
struct Layout {
    size_t seg, par, cnt, steps, hand, rec, ids, order, host_bytes, dev_bytes;
};

size_t fan_values(const rt_fan &f) { return size_t(f.n_elev) + f.n_az + f.n_freq; }

Layout job_layout(const TraceJob &j)
{
    size_t nf = 0;
    for (size_t k = 0; k < j.n_segs(); ++k) nf += fan_values(j.seg(k).fan);
    Layout L;
    L.seg = align_up(nf * 8, 256);
    L.par = L.seg + align_up(j.n_segs() * sizeof(Segment), 256);
    L.cnt = L.par + align_up(sizeof(TraceParams<double>), 256);
    L.steps = L.cnt + align_up(sizeof(Counters), 64);
    L.hand = L.steps + align_up(j.n_segs() * 8, 256);
    L.host_bytes = L.hand;
    L.rec = L.hand + align_up(size_t(j.tail) * sizeof(Handoff), 256);
    L.ids = L.rec + align_up(size_t(j.n_rays) * sizeof(RayRec), 256);
    L.order = L.ids + align_up(size_t(j.n_rays) * sizeof(int32_t), 256);
    L.dev_bytes = L.order + (j.binned ? size_t(j.n_rays) * sizeof(int32_t) : 0) + 256;
    return L;
}

// Check one request; on success fill seg (except the output pointers).
rt_status validate_request(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                           const rt_trace_opts *opts, JobSeg &seg)
{
    if (!grid || !fan || !opts) return fail(ctx, RT_E_INVALID, "NULL argument");
    if (grid->ctx != ctx) return fail(ctx, RT_E_INVALID, "grid belongs to another context");
    int64_t n64 = 0;
    if (rt_fan_count(fan, &n64) != RT_OK) return fail(ctx, RT_E_INVALID, "invalid fan");
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
    if (opts->tail_threshold > (1 << 24) || opts->tail_threshold < -2)
        return fail(ctx, RT_E_INVALID, "tail_threshold must be in [-2, 2^24]");
    if (opts->waves_per_simd < 0 || opts->waves_per_simd > 2)
        return fail(ctx, RT_E_INVALID, "waves_per_simd must be 0, 1 or 2");
    if (opts->ray_order < 0 || opts->ray_order > 3)
        return fail(ctx, RT_E_INVALID, "ray_order must be 0, 1, 2 or 3");
    if (opts->promote_waves < -1 || opts->promote_waves > kMaxPromoteWaves)
        return fail(ctx, RT_E_INVALID, "promote_waves must be in [-1, 64]");
    if (opts->promote_age < -1)
        return fail(ctx, RT_E_INVALID, "promote_age must be >= -1");
    if (opts->cu_layout < 0 || opts->cu_layout > 2)
        return fail(ctx, RT_E_INVALID, "cu_layout must be 0, 1 or 2");
    if (opts->traj_stride < 0 || opts->traj_capacity < 0)
        return fail(ctx, RT_E_INVALID, "negative trajectory option");
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
    seg.grid = grid;
    seg.fan = *fan;
    seg.n_rays = int(n64);
    return RT_OK;
}

// Stride of the visiting order q -> q s mod n: the first integer at or
// above 0.618 n that is coprime to n (so the map is a permutation).
int64_t visit_stride(int64_t n)
{
    if (n <= 2) return 1;
    int64_t s = int64_t(0.6180339887498949 * double(n));
    for (;; ++s) {
        int64_t a = s, b = n;
        while (b) { int64_t t = a % b; a = b; b = t; }
        if (a == 1) return s;
    }
}

// Launch-wide settings from the options and the total ray count.
void finish_job(rt_ctx *ctx, TraceJob &job, const rt_trace_opts &opts)
{
    job.opts = opts;
    int64_t n64 = 0;
    for (size_t k = 0; k < job.n_segs(); ++k) n64 += job.seg(k).n_rays;
    job.n_rays = int(n64);
    job.occ = opts.waves_per_simd == 0 ? 1 : opts.waves_per_simd;
    const int tail = opts.tail_threshold == 0 ? ctx->n_cu * 16 : opts.tail_threshold;
    job.inwave = tail == -2 ? 1 : 0;
    job.tail = tail > 0 ? int(std::min<int64_t>(tail, n64)) : 0;
    job.perm = opts.ray_order == 2 ? visit_stride(n64) : 1;
    job.binned = opts.ray_order == 3 || opts.ray_order == 0;   // the default: sorted by wave mode
    // promotion runs beside the one-lane waves; not with the in-wave switch
    const int pw = opts.promote_waves != 0 ? opts.promote_waves
                 : (n64 >= kDefaultPromoteMinRays ? kDefaultPromoteWaves : 0);
    job.promote = (pw > 0 && !job.inwave) ? pw : 0;
    job.promote_age = opts.promote_age == 0 ? kDefaultPromoteAge : std::max(0, opts.promote_age);
    job.per_ray = opts.traj_stride > 0 && n64 > 0 ? opts.traj_capacity / n64 : 0;
}

// Requests that can share one launch.
bool compatible(const JobSeg &a, const rt_trace_opts &oa, const JobSeg &b, const rt_trace_opts &ob)
{
    const rt_grid_geom &x = a.grid->geom, &y = b.grid->geom;
    return x.n_lat == y.n_lat && x.n_lon == y.n_lon && x.n_h == y.n_h && x.interp == y.interp &&
           x.lat0_deg == y.lat0_deg && x.dlat_deg == y.dlat_deg && x.lon0_deg == y.lon0_deg &&
           x.dlon_deg == y.dlon_deg && x.h0_km == y.h0_km && x.dh_km == y.dh_km &&
           x.earth_radius_km == y.earth_radius_km && a.fan.tx_lat_deg == b.fan.tx_lat_deg &&
           a.fan.tx_lon_deg == b.fan.tx_lon_deg && a.fan.tx_h_km == b.fan.tx_h_km &&
           oa.step_km == ob.step_km && oa.max_group_km == ob.max_group_km &&
           oa.exit_h_km == ob.exit_h_km && oa.precision == ob.precision &&
           oa.tail_threshold == ob.tail_threshold && oa.waves_per_simd == ob.waves_per_simd &&
           oa.ray_order == ob.ray_order && oa.promote_waves == ob.promote_waves &&
           oa.promote_age == ob.promote_age && oa.cu_layout == ob.cu_layout &&
           oa.traj_stride == 0 && ob.traj_stride == 0;
}

template <typename T>
void fill_params(const TraceJob &job, const Layout &lay, TraceParams<T> &P, char *dev, int n_producers,
                 int n_promote, int64_t wall_khz)
{
    const JobSeg &s0 = job.seg(0);
    const rt_grid_geom &gq = s0.grid->geom;
    const rt_fan *fan = &s0.fan;
    const rt_trace_opts *opts = &job.opts;
    fill_grid_dev<T>(s0.grid, P.g);
    const double la = fan->tx_lat_deg * kDeg2Rad, lo = fan->tx_lon_deg * kDeg2Rad;
    P.seg = reinterpret_cast<const Segment *>(dev + lay.seg);
    P.n_seg = int32_t(job.n_segs());
    P.n_rays = job.n_rays;
    P.tx_lon = lo;
    P.up[0] = std::cos(la) * std::cos(lo); P.up[1] = std::cos(la) * std::sin(lo); P.up[2] = std::sin(la);
    P.north[0] = -std::sin(la) * std::cos(lo); P.north[1] = -std::sin(la) * std::sin(lo);
    P.north[2] = std::cos(la);
    P.east[0] = -std::sin(lo); P.east[1] = std::cos(lo); P.east[2] = 0.0;
    P.r0 = gq.earth_radius_km + fan->tx_h_km;
    P.step = opts->step_km;
    P.step6 = opts->step_km / 6.0;
    P.short_step = series_covers_step(opts->step_km, gq.earth_radius_km) ? 1 : 0;
    P.max_group = opts->max_group_km;
    P.exit_h = opts->exit_h_km > 0 ? opts->exit_h_km : gq.h0_km + (gq.n_h - 1) * gq.dh_km;
    P.floor_h = gq.h0_km;
    P.max_steps = int32_t(std::ceil(opts->max_group_km / opts->step_km)) + 2;
    P.traj_stride = opts->traj_stride;
    P.traj_per_ray = job.per_ray;
    P.traj = job.traj;
    P.traj_count = job.tcount;
    char *cnt = dev + lay.cnt;
    P.queue_head = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, head));
    P.truncated = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, trunc));
    P.live = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, live));
    P.n_handoff = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, n_handoff));
    P.handoff = reinterpret_cast<Handoff *>(dev + lay.hand);
    P.rec = reinterpret_cast<RayRec *>(dev + lay.rec);
    P.n_producers = n_producers;
    P.promote_cap = 4 * n_promote;
    P.promote_age = job.promote_age;
    P.promo_push = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, promo_push));
    P.promo_pop = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, promo_pop));
    P.promo_live = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, promo_live));
    P.producers_alive = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, producers_alive));
    P.promo_err = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, promo_err));
    P.unfinished = reinterpret_cast<int32_t *>(cnt + offsetof(Counters, unfinished));
    P.phase_steps = reinterpret_cast<unsigned long long *>(cnt + offsetof(Counters, phase_steps));
    P.wave_iters = reinterpret_cast<unsigned long long *>(cnt + offsetof(Counters, wave_iters));
    P.promo_ids = reinterpret_cast<int32_t *>(dev + lay.ids);
    // Longest wait of an idle promotion wave while one-lane waves still run,
    // in wall-clock ticks: far above the one-lane waves' worst case (every
    // ray of a lane at max_steps, 50 us per step, a quarter of the waves
    // resident at a time), and at least 10 s.  Only a fault would reach it.
    const double lane_rays = std::ceil(double(job.n_rays) / (64.0 * std::max(1, n_producers))) + 1.0;
    double secs = std::max(10.0, 4.0 * lane_rays * double(P.max_steps) * 50e-6);
    // diagnostic override (milliseconds), for testing the timeout report
    if (const char *e = std::getenv("RTGD_PROMOTE_IDLE_MS")) {
        const double ms = std::atof(e);
        if (ms > 0.0) secs = ms * 1e-3;
    }
    P.idle_ticks = int64_t(std::min(secs * double(wall_khz) * 1e3, 9.0e18));
    P.handoff_threshold = job.tail;
    P.inwave = job.inwave;
    P.perm_stride = job.perm;
    P.order = job.binned ? reinterpret_cast<int32_t *>(dev + lay.order) : nullptr;
}

// Enqueue one launch on `stream`: stage fan axes, segment table, parameter
// block and zeroed counters in `host` (which must stay valid until the
// stream has consumed the copy), copy them to `dev` in one transfer, launch
// the one-lane persistent kernel and, with hand-off on, the sixteen-lane tail
// kernel; then copy counters and per-segment step counts back to
// `readback` (host, readback_bytes(job) bytes; NULL: into host staging,
// which a replayed upload must not see).  Events (optional) bracket the
// kernels.
rt_status enqueue_job(rt_ctx *ctx, hipStream_t stream, const TraceJob &job, char *dev, char *host,
                      hipEvent_t ev0, hipEvent_t ev1, char *readback = nullptr, hipEvent_t evm = nullptr)
{
    const Layout lay = job_layout(job);
    std::memset(host + lay.seg, 0, lay.host_bytes - lay.seg);
    double *h_fan = reinterpret_cast<double *>(host);
    Segment *h_seg = reinterpret_cast<Segment *>(host + lay.seg);
    size_t off = 0;
    int start = 0;
    // mode-sorted queue: rays of the first group (O or isotropic) of all
    // segments, then the X rays; each segment's share of a group is its rays
    // of that mode
    auto x_rays = [](const JobSeg &js) -> int {
        if (js.grid->B0 == 0.0) return 0;
        const int nm = popcount_modes(js.fan.modes);
        return nm == 2 ? js.n_rays / 2 : ((js.fan.modes & RT_MODE_O) ? 0 : js.n_rays);
    };
    int n_first = 0;
    for (size_t k = 0; k < job.n_segs(); ++k) n_first += job.seg(k).n_rays - x_rays(job.seg(k));
    int first_at = 0, x_at = n_first;
    const bool mixed = job.opts.precision == RT_MIXED;
    for (size_t k = 0; k < job.n_segs(); ++k) {
        const JobSeg &js = job.seg(k);
        const rt_fan &f = js.fan;
        double *fe = h_fan + off;
        std::copy(f.elev_deg, f.elev_deg + f.n_elev, fe);
        std::copy(f.az_deg, f.az_deg + f.n_az, fe + f.n_elev);
        std::copy(f.freq_mhz, f.freq_mhz + f.n_freq, fe + f.n_elev + f.n_az);
        const double *de = reinterpret_cast<const double *>(dev) + off;
        Segment &S = h_seg[k];
        S.elev = de;
        S.az = de + f.n_elev;
        S.freq = de + f.n_elev + f.n_az;
        S.v = mixed ? static_cast<const void *>(js.grid->d_f32) : static_cast<const void *>(js.grid->d_f64);
        S.B0 = js.grid->B0;
        for (int i = 0; i < 7; ++i) S.out[i] = js.out[i];
        S.status = js.status;
        S.nsteps = js.nsteps;
        S.steps = reinterpret_cast<unsigned long long *>(dev + lay.steps) + k;
        S.n_elev = f.n_elev;
        S.n_az = f.n_az;
        S.n_mode = popcount_modes(f.modes);
        S.mode_first = (f.modes & RT_MODE_O) ? 1 : -1;
        S.start = start;
        S.n = js.n_rays;
        S.bin_pos[0] = first_at;
        S.bin_pos[1] = x_at;
        first_at += js.n_rays - x_rays(js);
        x_at += x_rays(js);
        start += js.n_rays;
        off += fan_values(f);
    }
    // kernel variant: interpolation, and whether every ray is anisotropic
    bool aniso = true;
    for (size_t k = 0; k < job.n_segs(); ++k) aniso = aniso && job.seg(k).grid->B0 != 0.0;
    const int variant = (job.seg(0).grid->geom.interp == RT_INTERP_CR ? 1 : 0) | (aniso ? 2 : 0);
    const KernelSet ksel = mixed ? kernel_set<float>(variant) : kernel_set<double>(variant);
    const bool occ2 = job.occ == 2;
    const void *kt = occ2 ? ksel.trace_w2 : ksel.trace;
    const void *ktg = ksel.trace_g;  // the one-lane kernel grouped four waves per work-group
    const void *kl = occ2 ? ksel.tail_w2 : ksel.tail;
    const void *ks = mixed ? (const void *)k_start<float> : (const void *)k_start<double>;  // starting states
    const void *kf = mixed ? (const void *)k_finish<float> : (const void *)k_finish<double>;  // outputs
    // One-lane waves first, promotion waves after them: blocks are
    // dispatched in index order, so a promotion wave runs only once every
    // one-lane wave is resident.  All of them fit at once on an idle GPU.
    // With promotion on, a single-request launch holds at most one wave per
    // SIMD: a promotion wave runs the launch's longest rays, and beside a
    // one-lane wave on the same SIMD it would issue at half rate (the FP32
    // kernels fit two waves per SIMD).  The grouped layout goes further:
    // four-wave work-groups, one per CU, so that the promotion waves share
    // no CU (its memory pipeline and caches) with one-lane waves; it is the
    // default for every launch with promotion waves (server batches of many
    // requests included: measured as fast or faster in FP64 and 5-13 %
    // faster in mixed precision than one-wave work-groups).
    const int max_waves = resident_waves<double>(ctx, kt);
    int n_promote = job.promote > 0 && max_waves > 2 * job.promote ? job.promote : 0;
    const bool grouped = n_promote > 0 && ctx->lds_lock > 0 &&
                         job.opts.cu_layout != 1;
    int producers;
    if (grouped) {
        n_promote = (n_promote + 3) / 4 * 4;
        const int cap = 4 * ctx->n_cu;
        producers = std::max(4, std::min((job.n_rays + 63) / 64, cap - n_promote));
        producers = (producers + 3) / 4 * 4;     // whole work-groups: cap - n_promote is a multiple of 4
    } else {
        const int cap = n_promote > 0 && job.n_segs() == 1 ? std::min(max_waves, 4 * ctx->n_cu) : max_waves;
        producers = std::max(1, std::min((job.n_rays + 63) / 64, cap - n_promote));
    }
    const int waves = producers + n_promote;
    Counters hc{};
    hc.live = job.n_rays;
    hc.producers_alive = producers;
    std::memcpy(host + lay.cnt, &hc, sizeof(hc));
    // the block goes to the kernels twice: by value (kernel arguments, for
    // the trace loop) and in device memory (for the out-of-line calls)
    TraceParams<float> Pf{};
    TraceParams<double> Pd{};
    void *pargs;
    if (mixed) {
        fill_params<float>(job, lay, Pf, dev, producers, n_promote, ctx->wall_khz);
        std::memcpy(host + lay.par, &Pf, sizeof(Pf));
        pargs = &Pf;
    } else {
        fill_params<double>(job, lay, Pd, dev, producers, n_promote, ctx->wall_khz);
        std::memcpy(host + lay.par, &Pd, sizeof(Pd));
        pargs = &Pd;
    }
    HIP_OR_FAIL(ctx, hipMemcpyAsync(dev, host, lay.host_bytes, hipMemcpyHostToDevice, stream));
    void *arg = dev + lay.par;
    void *args[] = {pargs, &arg};
    const dim3 per_ray((job.n_rays + 63) / 64);
    if (ev0) HIP_OR_FAIL(ctx, hipEventRecord(ev0, stream));
    HIP_OR_FAIL(ctx, hipLaunchKernel(ks, per_ray, dim3(64), args, 0, stream));
    if (grouped)
        HIP_OR_FAIL(ctx, hipLaunchKernel(ktg, dim3(waves / 4), dim3(256), args, size_t(ctx->lds_lock), stream));
    else
        HIP_OR_FAIL(ctx, hipLaunchKernel(kt, dim3(waves), dim3(64), args, 0, stream));
    if (evm) HIP_OR_FAIL(ctx, hipEventRecord(evm, stream));
    if (job.tail > 0)
        HIP_OR_FAIL(ctx, hipLaunchKernel(kl, dim3((job.tail + 3) / 4), dim3(64), args, 0, stream));
    HIP_OR_FAIL(ctx, hipLaunchKernel(kf, per_ray, dim3(64), args, 0, stream));
    if (ev1) HIP_OR_FAIL(ctx, hipEventRecord(ev1, stream));
    HIP_OR_FAIL(ctx, hipMemcpyAsync(readback ? readback : host + lay.cnt, dev + lay.cnt, lay.hand - lay.cnt,
                                    hipMemcpyDeviceToHost, stream));
    return RT_OK;
}

// The launch error the counters report, if any: a promotion wait that
// timed out, or rays that no trace kernel finished (their outputs are NaN
// and their status -1).  Either means a fault of the launch, never a
// property of the rays.
rt_status launch_error(rt_ctx *ctx, const Counters &c)
{
    if (c.promo_err) return fail(ctx, RT_E_DEVICE, "promotion queue timed out");
    if (c.unfinished)
        return fail(ctx, RT_E_DEVICE, std::to_string(c.unfinished) + " rays were left without a final status");
    return RT_OK;
}

size_t readback_bytes(const TraceJob &job)
{
    const Layout lay = job_layout(job);
    return lay.hand - lay.cnt;
}

// Counters and per-segment step counts after the stream has finished;
// `readback` as given to enqueue_job (NULL: host staging).
void job_counters(const TraceJob &job, const char *host, Counters &c, std::vector<int64_t> &steps,
                  const char *readback = nullptr)
{
    const Layout lay = job_layout(job);
    const char *rb = readback ? readback : host + lay.cnt;
    std::memcpy(&c, rb, sizeof(c));
    steps.resize(job.n_segs());
    for (size_t k = 0; k < job.n_segs(); ++k) {
        unsigned long long v;
        std::memcpy(&v, rb + (lay.steps - lay.cnt) + 8 * k, 8);
        steps[k] = int64_t(v);
    }
}

rt_status ensure_pinned(rt_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->pinned_bytes) return RT_OK;
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    size_t want = std::max(bytes, size_t(1) << 16);
    HIP_OR_FAIL(ctx, hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_bytes = want;
    return RT_OK;
}

}  // namespace

namespace {

// Results of a finished single-request launch: device time per phase and
// the counters (ray-steps, launch errors).
rt_status trace_results(rt_ctx *ctx, const TraceJob &job, const char *host, rt_results *res,
                        int64_t &seg_steps)
{
    float ms = 0.f, ms_trace = 0.f;
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms_trace, ctx->ev0, ctx->evm));
    const Layout lay = job_layout(job);
    Counters hc;
    std::memcpy(&hc, host + lay.cnt, sizeof(hc));
    unsigned long long v;
    std::memcpy(&v, host + lay.steps, 8);
    seg_steps = int64_t(v);
    res->total_steps = seg_steps;
    res->kernel_ms = ms;
    res->trace_ms = ms_trace;
    res->tail_ms = ms - ms_trace;
    res->steps_one_lane = int64_t(hc.phase_steps[0]);
    res->steps_promoted = int64_t(hc.phase_steps[1]);
    res->steps_rows = int64_t(hc.phase_steps[2]);
    res->one_lane_wave_iters = int64_t(hc.wave_iters);
    rt_status st = launch_error(ctx, hc);
    if (st != RT_OK) return st;
    return hc.trunc ? RT_W_TRAJ_TRUNCATED : RT_OK;
}

void clear_results(rt_results *res)
{
    res->total_steps = 0;
    res->kernel_ms = res->trace_ms = res->tail_ms = 0.0;
    res->steps_one_lane = res->steps_promoted = res->steps_rows = 0;
    res->one_lane_wave_iters = 0;
}

}  // namespace

extern "C" rt_status rt_trace(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                              const rt_trace_opts *opts, rt_results *res)
{
    if (!ctx) return RT_E_INVALID;
    if (!res) return fail(ctx, RT_E_INVALID, "NULL argument");
    TraceJob job;
    job.segs.resize(1);
    rt_status st = validate_request(ctx, grid, fan, opts, job.segs[0]);
    if (st != RT_OK) return st;
    finish_job(ctx, job, *opts);
    clear_results(res);
    if (job.n_rays == 0) return RT_OK;
    const int64_t n64 = job.n_rays;
    if (opts->traj_stride > 0 && (!res->traj || opts->traj_capacity < n64))
        return fail(ctx, RT_E_INVALID, "trajectory needs traj and traj_capacity >= n_rays");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    const Layout lay = job_layout(job);
    if ((st = ensure_ws(ctx, lay.dev_bytes)) != RT_OK) return st;
    if ((st = ensure_pinned(ctx, lay.host_bytes)) != RT_OK) return st;

    const bool host_out = opts->results_mem == RT_MEM_HOST;
    const size_t N = size_t(job.n_rays);
    const int64_t per_ray = job.per_ray;
    JobSeg &js = job.segs[0];
    double *dbl[7] = {res->group_km, res->phase_km, res->range_km, res->az_dev_deg,
                      res->apogee_km, res->land_lat_deg, res->land_lon_deg};
    js.status = res->status;
    js.nsteps = res->n_steps;
    job.tcount = res->traj_count;
    job.traj = per_ray > 0 ? res->traj : nullptr;
    if (host_out) {
        size_t bytes = 7 * N * 8 + 3 * N * 4 + 64;
        if (per_ray > 0) bytes = align_up(bytes, 256) + size_t(per_ray) * N * 64;
        if ((st = ensure_stage(ctx, bytes)) != RT_OK) return st;
        char *sp = static_cast<char *>(ctx->stage);
        for (int k = 0; k < 7; ++k) js.out[k] = dbl[k] ? reinterpret_cast<double *>(sp + k * N * 8) : nullptr;
        char *ip = sp + 7 * N * 8;
        js.status = res->status ? reinterpret_cast<int32_t *>(ip) : nullptr;
        js.nsteps = res->n_steps ? reinterpret_cast<int32_t *>(ip + N * 4) : nullptr;
        job.tcount = res->traj_count ? reinterpret_cast<int32_t *>(ip + 2 * N * 4) : nullptr;
        job.traj = per_ray > 0 ? reinterpret_cast<double *>(sp + align_up(7 * N * 8 + 3 * N * 4 + 64, 256))
                               : nullptr;
    } else {
        for (int k = 0; k < 7; ++k) js.out[k] = dbl[k];
    }
    char *pinned = static_cast<char *>(ctx->pinned);
    if ((st = enqueue_job(ctx, ctx->stream, job, static_cast<char *>(ctx->ws), pinned, ctx->ev0,
                          ctx->ev1, nullptr, ctx->evm)) != RT_OK)
        return st;
    if (host_out) {
        for (int k = 0; k < 7; ++k)
            if (dbl[k])
                HIP_OR_FAIL(ctx, hipMemcpyAsync(dbl[k], js.out[k], N * 8, hipMemcpyDeviceToHost, ctx->stream));
        if (res->status)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->status, js.status, N * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (res->n_steps)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->n_steps, js.nsteps, N * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (res->traj_count)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->traj_count, job.tcount, N * 4, hipMemcpyDeviceToHost, ctx->stream));
        if (per_ray > 0)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(res->traj, job.traj, size_t(per_ray) * N * 64,
                                            hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    int64_t steps = 0;
    return trace_results(ctx, job, pinned, res, steps);
}

extern "C" rt_status rt_trace_noalloc(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                                      const rt_trace_opts *opts, rt_results *res)
{
    if (!ctx) return RT_E_INVALID;
    if (!res || !fan || !opts) return fail(ctx, RT_E_INVALID, "NULL argument");
    if (opts->results_mem != RT_MEM_DEVICE)
        return fail(ctx, RT_E_INVALID, "rt_trace_noalloc writes device results only (results_mem)");
    if (opts->traj_stride != 0) return fail(ctx, RT_E_INVALID, "rt_trace_noalloc records no trajectories");
    if (int64_t(fan->n_elev) + fan->n_az + fan->n_freq > RT_NOALLOC_MAX_AXIS)
        return fail(ctx, RT_E_INVALID, "fan axes exceed RT_NOALLOC_MAX_AXIS values");
    int64_t n64 = 0;
    if (rt_fan_count(fan, &n64) == RT_OK && n64 > RT_NOALLOC_MAX_RAYS)
        return fail(ctx, RT_E_INVALID, "fan exceeds RT_NOALLOC_MAX_RAYS rays");
    // One segment, held in place (no heap): JobSeg and the options by value.
    TraceJob job;
    JobSeg seg;
    rt_status st = validate_request(ctx, grid, fan, opts, seg);
    if (st != RT_OK) return st;
    job.one = &seg;
    finish_job(ctx, job, *opts);
    clear_results(res);
    if (job.n_rays == 0) return RT_OK;
    const Layout lay = job_layout(job);
    if (lay.dev_bytes > size_t(RT_NOALLOC_SCRATCH_BYTES) || lay.host_bytes > sizeof(ctx->noalloc_host))
        return fail(ctx, RT_E_INVALID, "launch exceeds the no-allocation scratch region");
    if (!ctx->scratch) return fail(ctx, RT_E_DEVICE, "no scratch region on this device");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    double *dbl[7] = {res->group_km, res->phase_km, res->range_km, res->az_dev_deg,
                      res->apogee_km, res->land_lat_deg, res->land_lon_deg};
    for (int k = 0; k < 7; ++k) seg.out[k] = dbl[k];
    seg.status = res->status;
    seg.nsteps = res->n_steps;
    // The staging is pageable host memory: the upload and the counter
    // read-back are ordered on the stream, and the call synchronizes before
    // it reads the counters or returns.
    if ((st = enqueue_job(ctx, ctx->stream, job, ctx->scratch, ctx->noalloc_host, ctx->ev0, ctx->ev1,
                          nullptr, ctx->evm)) != RT_OK)
        return st;
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    int64_t steps = 0;
    return trace_results(ctx, job, ctx->noalloc_host, res, steps);
}

extern "C" rt_status rt_ionogram(rt_ctx *ctx, const rt_fan *fan, const rt_results *res,
                                 double range_km, int32_t max_points, int32_t mem, double *out,
                                 int32_t *counts)
{
    if (!ctx) return RT_E_INVALID;
    if (!fan || !res || !out || !counts) return fail(ctx, RT_E_INVALID, "NULL argument");
    if (fan->n_az != 1) return fail(ctx, RT_E_INVALID, "an ionogram sweep has one azimuth");
    if (max_points < 1) return fail(ctx, RT_E_INVALID, "max_points must be >= 1");
    if (!(range_km > 0.0) || !std::isfinite(range_km))
        return fail(ctx, RT_E_INVALID, "range_km must be > 0");
    if (mem != RT_MEM_HOST && mem != RT_MEM_DEVICE)
        return fail(ctx, RT_E_INVALID, "mem must be RT_MEM_HOST or RT_MEM_DEVICE");
    if (!res->group_km || !res->phase_km || !res->range_km || !res->apogee_km || !res->status)
        return fail(ctx, RT_E_INVALID, "ionogram needs group, phase, range, apogee and status");
    int64_t n64 = 0;
    if (rt_fan_count(fan, &n64) != RT_OK) return fail(ctx, RT_E_INVALID, "invalid fan");
    for (int i = 0; i + 1 < fan->n_elev; ++i)
        if (!(fan->elev_deg[i + 1] > fan->elev_deg[i]))
            return fail(ctx, RT_E_INVALID, "elevations must be strictly increasing");
    const int n_trace = fan->n_freq * popcount_modes(fan->modes);
    if (n64 == 0 || n_trace == 0) return RT_OK;
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    const size_t N = size_t(n64);
    const size_t n_out = size_t(n_trace) * size_t(max_points) * 4;
    // device staging: elev | group phase range apogee | status | out | counts
    const size_t off_g = align_up(size_t(fan->n_elev) * 8, 256);
    const size_t off_st = off_g + (mem == RT_MEM_HOST ? align_up(4 * N * 8, 256) : 0);
    const size_t off_out = off_st + (mem == RT_MEM_HOST ? align_up(N * 4, 256) : 0);
    const size_t off_cnt = off_out + (mem == RT_MEM_HOST ? align_up(n_out * 8, 256) : 0);
    const size_t bytes = off_cnt + (mem == RT_MEM_HOST ? align_up(size_t(n_trace) * 4, 256) : 0) + 256;
    rt_status st = ensure_stage(ctx, bytes);
    if (st != RT_OK) return st;
    char *sp = static_cast<char *>(ctx->stage);
    double *d_elev = reinterpret_cast<double *>(sp);
    HIP_OR_FAIL(ctx, hipMemcpyAsync(d_elev, fan->elev_deg, size_t(fan->n_elev) * 8,
                                    hipMemcpyHostToDevice, ctx->stream));
    const double *g = res->group_km, *ph = res->phase_km, *rg = res->range_km, *ap = res->apogee_km;
    const int32_t *stt = res->status;
    double *d_out = out;
    int32_t *d_cnt = counts;
    if (mem == RT_MEM_HOST) {
        double *dg = reinterpret_cast<double *>(sp + off_g);
        const double *src[4] = {g, ph, rg, ap};
        for (int k = 0; k < 4; ++k)
            HIP_OR_FAIL(ctx, hipMemcpyAsync(dg + k * N, src[k], N * 8, hipMemcpyHostToDevice, ctx->stream));
        int32_t *ds = reinterpret_cast<int32_t *>(sp + off_st);
        HIP_OR_FAIL(ctx, hipMemcpyAsync(ds, stt, N * 4, hipMemcpyHostToDevice, ctx->stream));
        g = dg; ph = dg + N; rg = dg + 2 * N; ap = dg + 3 * N; stt = ds;
        d_out = reinterpret_cast<double *>(sp + off_out);
        d_cnt = reinterpret_cast<int32_t *>(sp + off_cnt);
    }
    hipLaunchKernelGGL(k_ionogram, dim3((n_trace + 63) / 64), dim3(64), 0, ctx->stream, d_elev,
                       fan->n_elev, n_trace, g, ph, rg, ap, stt, range_km, max_points, d_out, d_cnt);
    HIP_OR_FAIL(ctx, hipGetLastError());
    if (mem == RT_MEM_HOST) {
        HIP_OR_FAIL(ctx, hipMemcpyAsync(out, d_out, n_out * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(ctx, hipMemcpyAsync(counts, d_cnt, size_t(n_trace) * 4, hipMemcpyDeviceToHost,
                                        ctx->stream));
    }
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    return RT_OK;
}

// ===========================================================================
// Request server
// ===========================================================================
namespace {

// Per-ray outputs of one request inside the arena: 7 doubles + 2 int32.
constexpr size_t kOutBytesPerRay = 7 * 8 + 2 * 4;

struct Request {
    int64_t id = 0;
    JobSeg seg;                    // fan pointers refer to the vectors below
    rt_trace_opts opts{};
    std::vector<double> elev, az, freq;
    size_t off = 0, bytes = 0;     // arena block
    int state = 0;                 // 0 queued, 1 running, 2 done
    bool cancelled = false;
    rt_request_info info{};
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evm = nullptr;      // recorded after the trace kernel (before the tail kernel)
    bool big = false;              // the running launch has at least kStaggerRays rays
    char *dev = nullptr;
    size_t dev_bytes = 0;
    char *host = nullptr;          // pinned
    size_t host_bytes = 0;
    std::vector<int64_t> reqs;     // requests of the running launch; empty when idle
    TraceJob job;
};

// First-fit allocator over the arena (offsets, host bookkeeping only).
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(char *b, size_t n) { base = b; size = n; free_.clear(); free_[0] = n; used = 0; }
    static size_t round(size_t n) { return align_up(std::max<size_t>(n, 256), 256); }
    bool alloc(size_t n, size_t &off)
    {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                used += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct rt_server {
    rt_ctx *ctx = nullptr;
    std::vector<Slot> slots;
    Arena arena;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Request> reqs;
    std::deque<rt_request_info> done;
    int64_t next_id = 1;
    int max_batch_requests = 256;
    int64_t max_batch_rays = 1 << 20;
    std::vector<void *> retired_dev, retired_host;   // replaced slot buffers, freed when every slot is idle
    char *fetch = nullptr;     // pinned staging for rt_server_fetch to host memory
    size_t fetch_bytes = 0;
};

namespace {

// Batches of at least this many rays start staggered (see schedule).
constexpr int64_t kStaggerRays = 1 << 16;

// A slot's buffers grow while launches of the other slots may be running.
// hipFree and hipHostFree synchronize the device, so freeing the replaced
// buffers here would hold the scheduler (and every idle slot) until those
// launches end: they are retired instead, and freed once every slot is
// idle (or with the server).  A buffer grows to a quarter more than asked,
// so that growth is rare.
rt_status slot_reserve(rt_server *srv, Slot &sl, size_t dev_bytes, size_t host_bytes)
{
    rt_ctx *ctx = srv->ctx;
    if (dev_bytes > sl.dev_bytes) {
        if (sl.dev) srv->retired_dev.push_back(sl.dev);
        sl.dev = nullptr;
        sl.dev_bytes = 0;
        const size_t want = dev_bytes + dev_bytes / 4;
        HIP_OR_FAIL(ctx, hipMalloc(&sl.dev, want));
        sl.dev_bytes = want;
    }
    if (host_bytes > sl.host_bytes) {
        if (sl.host) srv->retired_host.push_back(sl.host);
        sl.host = nullptr;
        sl.host_bytes = 0;
        const size_t want = std::max<size_t>(host_bytes + host_bytes / 4, 1 << 16);
        HIP_OR_FAIL(ctx, hipHostMalloc(&sl.host, want, hipHostMallocDefault));
        sl.host_bytes = want;
    }
    return RT_OK;
}

// Free the retired slot buffers if no slot has a launch in flight.
void free_retired(rt_server *srv, bool force)
{
    if (srv->retired_dev.empty() && srv->retired_host.empty()) return;
    if (!force)
        for (const Slot &sl : srv->slots)
            if (!sl.reqs.empty()) return;
    for (void *p : srv->retired_dev) (void)hipFree(p);
    for (void *p : srv->retired_host) (void)hipHostFree(p);
    srv->retired_dev.clear();
    srv->retired_host.clear();
}

// Continuous batching: while a slot is idle, take the head of the FIFO queue
// and, in queue order, every later request that shares the head's
// geometry, transmitter and options (others are passed over and wait for a
// launch of their own), as long as their outputs fit in the arena and the
// batch limits hold; launch them together on that slot's stream.  The
// first request whose outputs do not fit stops the batch, and the head
// waits until the arena can hold its outputs.
rt_status schedule(rt_server *srv)
{
    free_retired(srv, false);
    while (!srv->queue.empty()) {
        Slot *slot = nullptr;
        for (Slot &sl : srv->slots)
            if (sl.reqs.empty()) { slot = &sl; break; }
        if (!slot) return RT_OK;
        std::vector<int64_t> ids;
        int64_t rays = 0;
        for (int64_t id : srv->queue) {
            Request &r = srv->reqs[id];
            if (!ids.empty()) {
                const Request &h = srv->reqs[ids[0]];
                if (!compatible(h.seg, h.opts, r.seg, r.opts)) continue;   // waits for its own launch
                if (int(ids.size()) >= srv->max_batch_requests || rays + r.seg.n_rays > srv->max_batch_rays)
                    break;
            }
            if (!srv->arena.alloc(r.bytes, r.off)) break;             // memory admission stays FIFO
            ids.push_back(id);
            rays += r.seg.n_rays;
        }
        if (ids.empty()) return RT_OK;                        // wait for memory
        // Staggered start: a large batch waits while another slot's large
        // launch is still in its one-lane phase.  Its persistent grid holds
        // every SIMD then, so the two would run their bulks side by side and
        // the first one's tail kernel would find no SIMD until the second's
        // one-lane waves drain; started at the first one's tail, the second
        // runs its bulk beside that launch's last rays.
        if (rays >= kStaggerRays) {
            bool wait = false;
            for (const Slot &sl : srv->slots)
                if (&sl != slot && !sl.reqs.empty() && sl.big && hipEventQuery(sl.evm) == hipErrorNotReady)
                    wait = true;
            if (wait) {
                for (int64_t id : ids) srv->arena.release(srv->reqs[id].off, srv->reqs[id].bytes);
                return RT_OK;
            }
        }
        for (int64_t id : ids)
            srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), id));
        TraceJob job;
        for (int64_t id : ids) {
            Request &r = srv->reqs[id];
            const size_t N = size_t(r.seg.n_rays);
            char *b = srv->arena.base + r.off;
            for (int k = 0; k < 7; ++k) r.seg.out[k] = reinterpret_cast<double *>(b + k * N * 8);
            r.seg.status = reinterpret_cast<int32_t *>(b + 7 * N * 8);
            r.seg.nsteps = reinterpret_cast<int32_t *>(b + 7 * N * 8 + N * 4);
            r.state = 1;
            job.segs.push_back(r.seg);
        }
        finish_job(srv->ctx, job, srv->reqs[ids[0]].opts);
        const Layout lay = job_layout(job);
        rt_status st = slot_reserve(srv, *slot, lay.dev_bytes, lay.host_bytes);
        if (st == RT_OK)
            st = enqueue_job(srv->ctx, slot->stream, job, slot->dev, slot->host, slot->ev0, slot->ev1, nullptr,
                             slot->evm);
        slot->big = rays >= kStaggerRays;
        if (st != RT_OK) {
            // leave the requests queued at the head, in order, without memory
            for (auto it = ids.rbegin(); it != ids.rend(); ++it) {
                Request &r = srv->reqs[*it];
                srv->arena.release(r.off, r.bytes);
                r.state = 0;
                srv->queue.push_front(*it);
            }
            return st;
        }
        slot->reqs = std::move(ids);
        slot->job = std::move(job);
    }
    return RT_OK;
}

}  // namespace

extern "C" rt_status rt_server_create(rt_ctx *ctx, const rt_server_opts *opts, rt_server **out)
{
    if (!ctx || !out) return RT_E_INVALID;
    *out = nullptr;
    int64_t budget = opts && opts->mem_budget_bytes > 0 ? opts->mem_budget_bytes : (int64_t(256) << 20);
    // two slots: one launch runs its bulk while the other finishes its
    // longest rays; with more, launches that each fill the GPU contend and
    // stretch one another (measured on the serving mix and on back-to-back
    // sweeps, as were the default batch limits)
    int n_slots = opts && opts->n_slots > 0 ? opts->n_slots : 2;
    if (n_slots > 64) return fail(ctx, RT_E_INVALID, "at most 64 slots");
    if (opts && (opts->max_batch_requests < 0 || opts->max_batch_rays < 0))
        return fail(ctx, RT_E_INVALID, "negative batch limit");
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    rt_server *srv = new (std::nothrow) rt_server();
    if (!srv) return fail(ctx, RT_E_NOMEM, "host allocation failed");
    srv->ctx = ctx;
    if (opts && opts->max_batch_requests > 0) srv->max_batch_requests = opts->max_batch_requests;
    if (opts && opts->max_batch_rays > 0) srv->max_batch_rays = opts->max_batch_rays;
    char *base = nullptr;
    hipError_t e = hipMalloc(&base, size_t(budget));
    if (e != hipSuccess) {
        delete srv;
        return fail(ctx, RT_E_NOMEM, "server arena allocation failed");
    }
    srv->arena.init(base, size_t(budget));
    srv->slots.resize(n_slots);
    for (auto &sl : srv->slots) {
        // non-blocking streams at the default priority
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreate(&sl.ev0)) != hipSuccess || (e = hipEventCreate(&sl.ev1)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.evm, hipEventDisableTiming)) != hipSuccess) {
            rt_server_destroy(srv);
            return fail(ctx, RT_E_DEVICE, std::string("server stream setup: ") + hipGetErrorString(e));
        }
    }
    *out = srv;
    return RT_OK;
}

extern "C" void rt_server_destroy(rt_server *srv)
{
    if (!srv) return;
    (void)hipSetDevice(srv->ctx->device);
    for (auto &sl : srv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ev0) (void)hipEventDestroy(sl.ev0);
        if (sl.ev1) (void)hipEventDestroy(sl.ev1);
        if (sl.evm) (void)hipEventDestroy(sl.evm);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    free_retired(srv, true);
    if (srv->fetch) (void)hipHostFree(srv->fetch);
    if (srv->arena.base) (void)hipFree(srv->arena.base);
    delete srv;
}

extern "C" rt_status rt_server_submit(rt_server *srv, const rt_grid *grid, const rt_fan *fan,
                                      const rt_trace_opts *opts, int64_t *id)
{
    if (!srv || !id) return RT_E_INVALID;
    rt_ctx *ctx = srv->ctx;
    if (opts && opts->traj_stride != 0)
        return fail(ctx, RT_E_UNSUPPORTED, "the server does not record trajectories");
    Request r;
    rt_status st = validate_request(ctx, grid, fan, opts, r.seg);
    if (st != RT_OK) return st;
    r.bytes = size_t(r.seg.n_rays) * kOutBytesPerRay;
    if (r.seg.n_rays > 0 && Arena::round(r.bytes) > srv->arena.size)
        return fail(ctx, RT_E_NOMEM, "request larger than the arena");
    r.id = srv->next_id++;
    r.opts = *opts;
    r.opts.results_mem = RT_MEM_DEVICE;
    r.elev.assign(fan->elev_deg, fan->elev_deg + fan->n_elev);
    r.az.assign(fan->az_deg, fan->az_deg + fan->n_az);
    r.freq.assign(fan->freq_mhz, fan->freq_mhz + fan->n_freq);
    r.info.id = r.id;
    r.info.n_rays = r.seg.n_rays;
    *id = r.id;
    const bool empty = r.seg.n_rays == 0;
    auto it = srv->reqs.emplace(r.id, std::move(r)).first;
    Request &q = it->second;
    q.seg.fan.elev_deg = q.elev.data();
    q.seg.fan.az_deg = q.az.data();
    q.seg.fan.freq_mhz = q.freq.data();
    if (empty) {                // empty fan: done at once
        q.state = 2;
        q.info.status = RT_OK;
        srv->done.push_back(q.info);
        return RT_OK;
    }
    srv->queue.push_back(q.id);
    return schedule(srv);
}

extern "C" rt_status rt_server_poll(rt_server *srv, rt_request_info *done, int32_t max, int32_t *n_done)
{
    if (!srv || !n_done || (max > 0 && !done)) return RT_E_INVALID;
    rt_ctx *ctx = srv->ctx;
    *n_done = 0;
    for (auto &sl : srv->slots) {
        if (sl.reqs.empty()) continue;
        hipError_t e = hipEventQuery(sl.ev1);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return fail(ctx, RT_E_DEVICE, std::string("request: ") + hipGetErrorString(e));
        // the counter copy follows ev1 on the stream
        HIP_OR_FAIL(ctx, hipStreamSynchronize(sl.stream));
        Counters hc;
        std::vector<int64_t> steps;
        job_counters(sl.job, sl.host, hc, steps);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, sl.ev0, sl.ev1);
        for (size_t k = 0; k < sl.reqs.size(); ++k) {
            Request &r = srv->reqs[sl.reqs[k]];
            r.info.total_steps = steps[k];
            r.info.kernel_ms = ms;
            r.info.status = launch_error(ctx, hc) != RT_OK ? RT_E_DEVICE
                          : hc.trunc ? RT_W_TRAJ_TRUNCATED : RT_OK;
            r.state = 2;
            if (r.cancelled) {
                srv->arena.release(r.off, r.bytes);
                srv->reqs.erase(r.info.id);
            } else {
                srv->done.push_back(r.info);
            }
        }
        sl.reqs.clear();
    }
    rt_status st = schedule(srv);
    if (st != RT_OK) return st;
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        done[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n_done = k;
    return RT_OK;
}

extern "C" rt_status rt_server_fetch(rt_server *srv, int64_t id, rt_results *res, int32_t mem)
{
    if (!srv || !res) return RT_E_INVALID;
    rt_ctx *ctx = srv->ctx;
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end() || it->second.state != 2)
        return fail(ctx, RT_E_INVALID, "unknown or unfinished request");
    if (mem != RT_MEM_HOST && mem != RT_MEM_DEVICE)
        return fail(ctx, RT_E_INVALID, "mem must be RT_MEM_HOST or RT_MEM_DEVICE");
    Request &r = it->second;
    const size_t N = size_t(r.seg.n_rays);
    if (N > 0) {
        double *dst[7] = {res->group_km, res->phase_km, res->range_km, res->az_dev_deg,
                          res->apogee_km, res->land_lat_deg, res->land_lon_deg};
        if (mem == RT_MEM_HOST) {
            // The request's outputs lie in one block of the arena (seven
            // FP64 arrays, then status and step count): one copy to pinned
            // staging, then host copies to the caller's arrays, rather than
            // nine copies to (pageable) caller memory.
            const size_t bytes = N * (7 * 8 + 2 * 4);
            if (bytes > srv->fetch_bytes) {
                if (srv->fetch) srv->retired_host.push_back(srv->fetch);   // freed when every slot is idle
                srv->fetch = nullptr;
                srv->fetch_bytes = 0;
                const size_t want = std::max<size_t>(bytes + bytes / 4, 1 << 20);
                HIP_OR_FAIL(ctx, hipHostMalloc(reinterpret_cast<void **>(&srv->fetch), want, hipHostMallocDefault));
                srv->fetch_bytes = want;
            }
            HIP_OR_FAIL(ctx, hipMemcpyAsync(srv->fetch, r.seg.out[0], bytes, hipMemcpyDeviceToHost, ctx->stream));
            HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
            for (int k = 0; k < 7; ++k)
                if (dst[k]) std::memcpy(dst[k], srv->fetch + size_t(k) * N * 8, N * 8);
            if (res->status) std::memcpy(res->status, srv->fetch + 7 * N * 8, N * 4);
            if (res->n_steps) std::memcpy(res->n_steps, srv->fetch + 7 * N * 8 + N * 4, N * 4);
        } else {
            for (int k = 0; k < 7; ++k)
                if (dst[k])
                    HIP_OR_FAIL(ctx, hipMemcpyAsync(dst[k], r.seg.out[k], N * 8, hipMemcpyDeviceToDevice,
                                                    ctx->stream));
            if (res->status)
                HIP_OR_FAIL(ctx, hipMemcpyAsync(res->status, r.seg.status, N * 4, hipMemcpyDeviceToDevice,
                                                ctx->stream));
            if (res->n_steps)
                HIP_OR_FAIL(ctx, hipMemcpyAsync(res->n_steps, r.seg.nsteps, N * 4, hipMemcpyDeviceToDevice,
                                                ctx->stream));
            HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
        }
        srv->arena.release(r.off, r.bytes);
    }
    res->total_steps = r.info.total_steps;
    res->kernel_ms = r.info.kernel_ms;
    srv->reqs.erase(it);
    return schedule(srv);
}

extern "C" rt_status rt_server_cancel(rt_server *srv, int64_t id)
{
    if (!srv) return RT_E_INVALID;
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) return fail(srv->ctx, RT_E_INVALID, "unknown request");
    Request &r = it->second;
    if (r.state == 0) {
        for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
            if (*q == id) { srv->queue.erase(q); break; }
        srv->reqs.erase(it);
        return schedule(srv);
    }
    if (r.state == 1) {
        r.cancelled = true;
        return RT_OK;
    }
    // finished but not fetched: release now
    for (auto d = srv->done.begin(); d != srv->done.end(); ++d)
        if (d->id == id) { srv->done.erase(d); break; }
    if (r.seg.n_rays > 0) srv->arena.release(r.off, r.bytes);
    srv->reqs.erase(it);
    return schedule(srv);
}

extern "C" rt_status rt_server_stats(const rt_server *srv, int32_t *queued, int32_t *running,
                                     int64_t *arena_used)
{
    if (!srv) return RT_E_INVALID;
    size_t run = 0;
    for (auto &sl : srv->slots) run += sl.reqs.size();
    if (queued) *queued = int32_t(srv->queue.size());
    if (running) *running = int32_t(run);
    if (arena_used) *arena_used = int64_t(srv->arena.used);
    return RT_OK;
}

// ===========================================================================
// Replayable traces (HIP graph)
// ===========================================================================
struct rt_plan {
    rt_ctx *ctx = nullptr;
    TraceJob job;
    std::vector<double> elev, az, freq;
    char *dev = nullptr;
    char *host = nullptr;          // pinned staging, read by every replay
    char *readback = nullptr;      // pinned, counters written by every replay
    hipStream_t cap = nullptr;     // private capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool launched = false;
};

extern "C" void rt_plan_destroy(rt_plan *p)
{
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    if (p->launched) (void)hipStreamSynchronize(p->ctx->stream);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->dev) (void)hipFree(p->dev);
    if (p->host) (void)hipHostFree(p->host);
    if (p->readback) (void)hipHostFree(p->readback);
    delete p;
}

extern "C" rt_status rt_plan_create(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                                    const rt_trace_opts *opts, const rt_results *res, rt_plan **out)
{
    if (!ctx) return RT_E_INVALID;
    if (!res || !out) return fail(ctx, RT_E_INVALID, "NULL argument");
    *out = nullptr;
    rt_plan *p = new (std::nothrow) rt_plan();
    if (!p) return fail(ctx, RT_E_NOMEM, "host allocation failed");
    p->ctx = ctx;
    p->job.segs.resize(1);
    JobSeg &js = p->job.segs[0];
    rt_status st = validate_request(ctx, grid, fan, opts, js);
    if (st == RT_OK && opts->traj_stride != 0) st = fail(ctx, RT_E_UNSUPPORTED, "plans do not record trajectories");
    if (st == RT_OK && opts->results_mem != RT_MEM_DEVICE)
        st = fail(ctx, RT_E_INVALID, "plans write device results (results_mem = RT_MEM_DEVICE)");
    if (st == RT_OK && js.n_rays == 0) st = fail(ctx, RT_E_INVALID, "empty fan");
    if (st != RT_OK) {
        delete p;
        return st;
    }
    p->elev.assign(fan->elev_deg, fan->elev_deg + fan->n_elev);
    p->az.assign(fan->az_deg, fan->az_deg + fan->n_az);
    p->freq.assign(fan->freq_mhz, fan->freq_mhz + fan->n_freq);
    js.fan.elev_deg = p->elev.data();
    js.fan.az_deg = p->az.data();
    js.fan.freq_mhz = p->freq.data();
    double *dbl[7] = {res->group_km, res->phase_km, res->range_km, res->az_dev_deg,
                      res->apogee_km, res->land_lat_deg, res->land_lon_deg};
    for (int k = 0; k < 7; ++k) js.out[k] = dbl[k];
    js.status = res->status;
    js.nsteps = res->n_steps;
    finish_job(ctx, p->job, *opts);
    const Layout lay = job_layout(p->job);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc(&p->dev, lay.dev_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&p->host, lay.host_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&p->readback, readback_bytes(p->job), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&p->ev0);
    if (e == hipSuccess) e = hipEventCreate(&p->ev1);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        rt_plan_destroy(p);
        return fail(ctx, e == hipErrorOutOfMemory ? RT_E_NOMEM : RT_E_DEVICE,
                    std::string("plan setup: ") + hipGetErrorString(e));
    }
    // staging is filled here and read again by every replay's upload node
    st = enqueue_job(ctx, p->cap, p->job, p->dev, p->host, nullptr, nullptr, p->readback);
    e = hipStreamEndCapture(p->cap, &p->graph);
    if (st == RT_OK && e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (st != RT_OK || e != hipSuccess) {
        rt_plan_destroy(p);
        return st != RT_OK ? st : fail(ctx, RT_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = p;
    return RT_OK;
}

extern "C" rt_status rt_plan_launch(rt_plan *p)
{
    if (!p) return RT_E_INVALID;
    rt_ctx *ctx = p->ctx;
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    HIP_OR_FAIL(ctx, hipEventRecord(p->ev0, ctx->stream));
    HIP_OR_FAIL(ctx, hipGraphLaunch(p->exec, ctx->stream));
    HIP_OR_FAIL(ctx, hipEventRecord(p->ev1, ctx->stream));
    p->launched = true;
    return RT_OK;
}

extern "C" rt_status rt_plan_wait(rt_plan *p, int64_t *total_steps, double *kernel_ms)
{
    if (!p) return RT_E_INVALID;
    rt_ctx *ctx = p->ctx;
    if (!p->launched) return fail(ctx, RT_E_INVALID, "plan not launched");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
    p->launched = false;
    Counters hc;
    std::vector<int64_t> steps;
    job_counters(p->job, p->host, hc, steps, p->readback);
    float ms = 0.f;
    HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, p->ev0, p->ev1));
    if (total_steps) *total_steps = steps[0];
    if (kernel_ms) *kernel_ms = ms;
    return launch_error(ctx, hc);
}

// ===========================================================================
// Autotuner
// ===========================================================================
namespace {

struct TuneKey {
    int32_t n_cu, n_lat, n_lon, n_h, interp, precision, field, log2_rays;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(n_cu, n_lat, n_lon, n_h, interp, precision, field, log2_rays) <
               std::tie(o.n_cu, o.n_lat, o.n_lon, o.n_h, o.interp, o.precision, o.field, o.log2_rays);
    }
};
struct TuneVal {
    int32_t tail_threshold, waves_per_simd, ray_order, promote_waves, promote_age, cu_layout;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;

int ceil_log2(int64_t n)
{
    int k = 0;
    while ((int64_t(1) << k) < n) ++k;
    return k;
}

}  // namespace

extern "C" rt_status rt_autotune(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                                 const rt_trace_opts *base, rt_trace_opts *tuned, rt_tune_info *info)
{
    if (!ctx) return RT_E_INVALID;
    if (!tuned) return fail(ctx, RT_E_INVALID, "NULL argument");
    JobSeg probe;
    rt_status st = validate_request(ctx, grid, fan, base, probe);
    if (st != RT_OK) return st;
    if (base->traj_stride != 0) return fail(ctx, RT_E_UNSUPPORTED, "tune without trajectories");
    rt_tune_info inf{};
    *tuned = *base;
    const TuneKey key{ctx->n_cu, grid->geom.n_lat, grid->geom.n_lon, grid->geom.n_h, grid->geom.interp,
                      base->precision, grid->B0 != 0.0 ? 1 : 0, ceil_log2(std::max(probe.n_rays, 1))};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            tuned->tail_threshold = it->second.tail_threshold;
            tuned->waves_per_simd = it->second.waves_per_simd;
            tuned->ray_order = it->second.ray_order;
            tuned->promote_waves = it->second.promote_waves;
            tuned->promote_age = it->second.promote_age;
            tuned->cu_layout = it->second.cu_layout;
            inf.from_cache = 1;
            if (info) *info = inf;
            return RT_OK;
        }
    }
    if (probe.n_rays == 0) {
        if (info) *info = inf;
        return RT_OK;
    }
    // scratch outputs on the device (discarded)
    const size_t N = size_t(probe.n_rays);
    char *buf = nullptr;
    HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
    HIP_OR_FAIL(ctx, hipMalloc(&buf, N * (7 * 8 + 2 * 4) + 256));
    rt_results r{};
    r.group_km = reinterpret_cast<double *>(buf);
    r.phase_km = r.group_km + N; r.range_km = r.group_km + 2 * N; r.az_dev_deg = r.group_km + 3 * N;
    r.apogee_km = r.group_km + 4 * N; r.land_lat_deg = r.group_km + 5 * N; r.land_lon_deg = r.group_km + 6 * N;
    r.status = reinterpret_cast<int32_t *>(buf + 7 * N * 8);
    r.n_steps = r.status + N;
    const int tails[4] = {-2, -1, ctx->n_cu * 8, ctx->n_cu * 16};
    const int occs[2] = {1, 2};
    const int orders[3] = {1, 2, 3};
    // one untimed run, then the median of three
    auto time_opts = [&](rt_trace_opts o, double &ms) -> rt_status {
        o.results_mem = RT_MEM_DEVICE;
        double t[3];
        for (int rep = 0; rep < 4; ++rep) {
            rt_status s2 = rt_trace(ctx, grid, fan, &o, &r);
            if (s2 != RT_OK) return s2;
            if (rep) t[rep - 1] = r.kernel_ms;
        }
        std::sort(t, t + 3);
        ms = t[1];
        return RT_OK;
    };
    double best = 1e300;
    TuneVal bv{0, 0, 0, 0, 0, 0};
    std::vector<std::pair<double, TuneVal>> tried;   // every candidate and its first-round median
    rt_trace_opts o = *base;
    o.tail_threshold = 0;
    o.waves_per_simd = 0;
    o.ray_order = 0;
    o.promote_waves = 0;
    o.promote_age = 0;
    o.cu_layout = 0;
    st = time_opts(o, inf.default_ms);
    o.promote_waves = -1;     // the first stage runs without promotion
    double best_h = 1e300;    // the best with a launch-wide hand-off or none
    TuneVal bh{0, 0, 0, 0, 0, 0};
    for (int oc : occs) {
        for (int tl : tails) {
            for (int od : orders) {
                if (st != RT_OK) break;
                o.tail_threshold = tl;
                o.waves_per_simd = oc;
                o.ray_order = od;
                double ms = 0;
                st = time_opts(o, ms);
                ++inf.n_candidates;
                if (st == RT_OK) tried.push_back({ms, TuneVal{tl, oc, od, -1, 0, 0}});
                if (st == RT_OK && ms < best) { best = ms; bv = TuneVal{tl, oc, od, -1, 0, 0}; }
                if (st == RT_OK && tl != -2 && ms < best_h) { best_h = ms; bh = TuneVal{tl, oc, od, -1, 0, 0}; }
            }
        }
    }
    // then promotion on top of the best of those without the in-wave switch
    // (promotion does not combine with it), in both work-group layouts
    const int promos[3][2] = {{16, -1}, {32, -1}, {64, -1}};
    const int layouts[2] = {2, 1};
    if (best_h < 1e300) {
        const TuneVal base_v = bh;
        for (const auto &pr : promos) {
            for (int lay : layouts) {
                if (st != RT_OK) break;
                o.tail_threshold = base_v.tail_threshold;
                o.waves_per_simd = base_v.waves_per_simd;
                o.ray_order = base_v.ray_order;
                o.promote_waves = pr[0];
                o.promote_age = pr[1];
                o.cu_layout = lay;
                double ms = 0;
                st = time_opts(o, ms);
                ++inf.n_candidates;
                const TuneVal v{base_v.tail_threshold, base_v.waves_per_simd, base_v.ray_order, pr[0], pr[1], lay};
                if (st == RT_OK) tried.push_back({ms, v});
                if (st == RT_OK && ms < best) {
                    best = ms;
                    bv = v;
                }
            }
        }
    }
    // Confirmation: single launches vary by several per cent from run to run
    // (the last rays' 16-lane steps set the launch time, and candidates are
    // often within that of each other), so the three fastest candidates and
    // the defaults are timed again, nine launches each, interleaved; the
    // candidate with the lowest median is kept only if that median is
    // clearly below the defaults'.
    if (st == RT_OK && !tried.empty()) {
        std::stable_sort(tried.begin(), tried.end(),
                         [](const std::pair<double, TuneVal> &a, const std::pair<double, TuneVal> &b) {
                             return a.first < b.first;
                         });
        const size_t nf = std::min<size_t>(3, tried.size());
        constexpr int kReps = 9;
        std::vector<rt_trace_opts> os(nf + 1, *base);
        for (size_t c = 0; c < nf; ++c) {
            const TuneVal &v = tried[c].second;
            os[c].tail_threshold = v.tail_threshold;
            os[c].waves_per_simd = v.waves_per_simd;
            os[c].ray_order = v.ray_order;
            os[c].promote_waves = v.promote_waves;
            os[c].promote_age = v.promote_age;
            os[c].cu_layout = v.cu_layout;
        }
        rt_trace_opts &od = os[nf];      // the library defaults
        od.tail_threshold = od.waves_per_simd = od.ray_order = 0;
        od.promote_waves = od.promote_age = od.cu_layout = 0;
        for (auto &oo : os) oo.results_mem = RT_MEM_DEVICE;
        std::vector<std::vector<double>> t(nf + 1);
        for (int rep = 0; rep < kReps && st == RT_OK; ++rep)
            for (size_t c = 0; c <= nf && st == RT_OK; ++c) {
                st = rt_trace(ctx, grid, fan, &os[c], &r);
                t[c].push_back(r.kernel_ms);
            }
        if (st == RT_OK) {
            for (auto &tc : t) std::sort(tc.begin(), tc.end());
            inf.default_ms = t[nf][kReps / 2];
            best = 1e300;
            for (size_t c = 0; c < nf; ++c)
                if (t[c][kReps / 2] < best) {
                    best = t[c][kReps / 2];
                    bv = tried[c].second;
                }
        }
    }
    (void)hipFree(buf);
    if (st != RT_OK) return st;
    // keep the library defaults unless a candidate is clearly faster
    if (!(best < 0.98 * inf.default_ms)) {
        best = inf.default_ms;
        bv = TuneVal{0, 0, 0, 0, 0, 0};
    }
    inf.best_ms = best;
    tuned->tail_threshold = bv.tail_threshold;
    tuned->waves_per_simd = bv.waves_per_simd;
    tuned->ray_order = bv.ray_order;
    tuned->promote_waves = bv.promote_waves;
    tuned->promote_age = bv.promote_age;
    tuned->cu_layout = bv.cu_layout;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = bv;
    }
    if (info) *info = inf;
    return RT_OK;
}

extern "C" rt_status rt_tune_cache_save(const char *path)
{
    if (!path) return RT_E_INVALID;
    std::ofstream f(path);
    if (!f) return RT_E_INVALID;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    f << "# n_cu n_lat n_lon n_h interp precision field log2_rays -> tail_threshold waves_per_simd "
         "ray_order promote_waves promote_age cu_layout\n";
    for (const auto &kv : g_tune_cache) {
        const TuneKey &k = kv.first;
        f << k.n_cu << ' ' << k.n_lat << ' ' << k.n_lon << ' ' << k.n_h << ' ' << k.interp << ' '
          << k.precision << ' ' << k.field << ' ' << k.log2_rays << ' ' << kv.second.tail_threshold << ' '
          << kv.second.waves_per_simd << ' ' << kv.second.ray_order << ' ' << kv.second.promote_waves << ' '
          << kv.second.promote_age << ' ' << kv.second.cu_layout << '\n';
    }
    return f.good() ? RT_OK : RT_E_INVALID;
}

extern "C" rt_status rt_tune_cache_load(const char *path)
{
    if (!path) return RT_E_INVALID;
    std::ifstream f(path);
    if (!f) return RT_E_INVALID;
    std::map<TuneKey, TuneVal> loaded;
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ss(line);
        TuneKey k{};
        TuneVal v{};
        if (!(ss >> k.n_cu >> k.n_lat >> k.n_lon >> k.n_h >> k.interp >> k.precision >> k.field >>
              k.log2_rays >> v.tail_threshold >> v.waves_per_simd >> v.ray_order >> v.promote_waves >>
              v.promote_age >> v.cu_layout))
            return RT_E_INVALID;
        std::string rest;
        if (ss >> rest) return RT_E_INVALID;
        if (v.waves_per_simd < 0 || v.waves_per_simd > 2 || v.tail_threshold > (1 << 24) ||
            v.tail_threshold < -2 || v.ray_order < 0 || v.ray_order > 3 || v.promote_waves < -1 ||
            v.promote_waves > kMaxPromoteWaves || v.promote_age < -1 || v.cu_layout < 0 || v.cu_layout > 2)
            return RT_E_INVALID;
        loaded[k] = v;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : loaded) g_tune_cache[kv.first] = kv.second;
    return RT_OK;
}

extern "C" void rt_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
}
