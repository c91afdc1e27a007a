// gc_lib.hip -- kernels and C ABI of the gfx950 grating-cloak ray tracer.
// The public interface is include/gcloak.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gcloak.h"
#include "gc_lane64.hpp"
#include "gc_wave.hpp"
#include "gc_adjoint.hpp"
#include "gc_corr.hpp"

using namespace gc;

// ---------------------------------------------------------------------------
// Counters: each wave folds its lanes' counts and one lane adds them.
// ---------------------------------------------------------------------------
struct DevCounters {
    unsigned long long rays, steps, rejected, events, fallbacks, failed;
};

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fold per-thread counters into the device totals (cnt may be null: nothing
// is counted).  Wave sums by shuffles, block sums in LDS, then one atomic per
// block and non-zero counter: the counters share a cache line, whose atomics
// the memory system performs one at a time, so per-wave atomics would bound a
// short kernel.  Every thread of the block calls it.
__device__ __forceinline__ void add_counters(DevCounters* c, unsigned long long rays, unsigned long long steps,
                                             unsigned long long rej, unsigned long long ev,
                                             unsigned long long fb, unsigned long long failed)
{
    if (!c) return;
    unsigned long long v[6] = {rays, steps, rej, ev, fb, failed};
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
    __shared__ unsigned long long part[4][6];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) part[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        unsigned long long sum = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += part[w][k];
        // DevCounters is six consecutive counters in the order of v
        if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(c) + k, sum);
    }
}

// ---------------------------------------------------------------------------
// FP64 kernels: one ray (trace_rays) or one pixel (render) per lane.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_trace_rays64(SceneDev s, OptsDev o, long long n, const double* org,
                                                      const double* dir, double* out_org, double* out_dir,
                                                      int* status, long long* steps, int* events,
                                                      DevCounters* cnt)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_rays = 0;
    if (i < n) {
        double r[3] = {org[3 * i], org[3 * i + 1], org[3 * i + 2]};
        double d[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
        double oo[3] = {0, 0, 0}, od[3] = {0, 0, 0};
        LaneCount lc = {0, 0, 0, 0};
        double mc = 1.0;
        int st = trace_ray64(s, o, r, d, oo, od, lc, &mc);
        if (out_org) for (int a = 0; a < 3; ++a) out_org[3 * i + a] = oo[a];
        for (int a = 0; a < 3; ++a) out_dir[3 * i + a] = od[a];
        if (status) status[i] = st;
        if (steps) steps[i] = lc.steps;
        if (events) events[i] = lc.events;
        c_rays = 1;
        c_steps = lc.steps;
        c_rej = lc.rejected;
        c_ev = lc.events;
        c_fail = st != RS_OK;
    }
    add_counters(cnt, c_rays, c_steps, c_rej, c_ev, 0, c_fail);
}

template <bool FRESNEL>
__global__ void __launch_bounds__(256) k_render64(SceneDev s, CamDev cam, OptsDev o, float* rgb,
                                                  DevCounters* cnt)
{
    long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long npx = (long long)cam.W * cam.H;
    unsigned long long c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_rays = 0;
    if (pix < npx) {
        int i = (int)(pix % cam.W), j = (int)(pix / cam.W);
        double acc[3] = {0, 0, 0};
        for (int smp = 0; smp < cam.spp; ++smp) {
            double d[3], c[3];
            camera_dir(cam, i, j, smp, d);
            LaneCount lc = {0, 0, 0, 0};
            int st;
            if (FRESNEL) {
                // every path of the sample: the primary and its reflected branches
                st = shade_ray64(s, o, cam.eye, d, lc, c);
            } else {
                double oo[3], od[3], mc = 1.0;
                st = trace_ray64(s, o, cam.eye, d, oo, od, lc, &mc);
                if (st == RS_OK) backdrop_rgb64(s, oo, od, c);
            }
            c_rays++;
            c_steps += lc.steps;
            c_rej += lc.rejected;
            c_ev += lc.events;
            if (st != RS_OK) { c_fail++; continue; }
            for (int a = 0; a < 3; ++a) acc[a] += c[a];
        }
        for (int a = 0; a < 3; ++a) rgb[3 * pix + a] = (float)(acc[a] / cam.spp);
    }
    add_counters(cnt, c_rays, c_steps, c_rej, c_ev, 0, c_fail);
}

// Reference image: flat mirror y = 0 in air.  A downward ray leaves with
// d_y negated from its reflection point; an upward one sees the backdrop
// directly.  The camera ray and the backdrop's angles or landing point are
// FP64, its tanh FP32 (backdrop_rgb_image); the same reference serves both
// precisions of the cloaked image.
__global__ void __launch_bounds__(256) k_render_flat(CamDev cam, SceneDev s, float* rgb, DevCounters* cnt)
{
    const long long npx = (long long)cam.W * cam.H;
    unsigned long long c_rays = 0, c_ev = 0;
    // grid-stride over pixels (the grid is bounded so that the counters take
    // few atomics); the loop bound is uniform over the block
    for (long long base = (long long)blockIdx.x * blockDim.x; base < npx; base += (long long)gridDim.x * blockDim.x) {
        const long long pix = base + threadIdx.x;
        if (pix >= npx) continue;
        const int i = (int)(pix % cam.W), j = (int)(pix / cam.W);
        double acc[3] = {0, 0, 0};
        for (int smp = 0; smp < cam.spp; ++smp) {
            double d[3], r[3] = {cam.eye[0], cam.eye[1], cam.eye[2]};
            camera_dir(cam, i, j, smp, d);
            if (d[1] < 0.0 && cam.eye[1] > 0.0) {
                // the reflection point on y = 0 (the backdrop plane needs it)
                const double t = -cam.eye[1] / d[1];
                r[0] += t * d[0];
                r[1] = 0.0;
                r[2] += t * d[2];
                d[1] = -d[1];
                c_ev++;
            }
            float c[3];
            backdrop_rgb_image(s, r, d, c);
            for (int a = 0; a < 3; ++a) acc[a] += (double)c[a];
        }
        c_rays += cam.spp;
        for (int a = 0; a < 3; ++a) rgb[3 * pix + a] = (float)(acc[a] / cam.spp);
    }
    add_counters(cnt, c_rays, 0, 0, c_ev, 0, 0);
}

// Blocks of k_render_flat for npx pixels: one per 256 pixels up to 8 per CU.
static unsigned flat_blocks(int n_cu, long long npx)
{
    return (unsigned)std::max<long long>(1, std::min<long long>((npx + 255) / 256, 8LL * n_cu));
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
// concurrent sub-pipelines of a batch plan (gc_tune.plan_lanes)
constexpr int kPlanMaxLanes = 3;

// Device buffers of the FP32 pipeline, grown on demand.
struct WfStore {
    long long cap_rays = 0;
    int cap_scenes = 0;
    void* rays = nullptr;       // one allocation for all per-ray arrays
    int* queues = nullptr;      // 6 x cap_rays: box (2 rounds), FP64, slow box (2 rounds), air
    void* tables = nullptr;     // scenes, cameras, offsets, image pointers
    QCtr* ctr = nullptr;
    WfTotals* tot = nullptr;
    QCtr* h_ctr = nullptr;      // pinned host copy of the counters
    int box_blocks[2] = {0, 0}; // persistent grid of k_wf_box<RK4>, <DOPRI5>
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    unsigned long long* acc = nullptr;   // Fresnel: per-sample colour sums (fixed point)
    size_t acc_bytes = 0;
    // per call
    long long fp64_steps = 0, rounds = 0, tail_rays = 0;
    double hot_ms = 0.0, event_ms = 0.0, tail_ms = 0.0, total_ms = 0.0;
};

// Device buffers of the adjoint, grown on demand.
struct AdjStore {
    double* tape = nullptr;
    size_t tape_bytes = 0;
    void* seg = nullptr;
    size_t seg_bytes = 0;
    float* srgb = nullptr;
    double* sgrad = nullptr;
    long long* ovf = nullptr;
    long long cap_samples = 0;
    float* img = nullptr;
    long long cap_pix = 0;
    AdjCC* cs = nullptr;
    unsigned long long* ctr = nullptr;   // claim (2 passes), overflow (2 passes), rays, steps, events, failed, bad
    double* red = nullptr;
    unsigned long long* h_ctr = nullptr; // pinned: ctr, then red and the correlation sums
    int blocks[2] = {0, 0};              // resident blocks of k_adj<double>, k_adj<float>
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // second pass: tapes of the long traces, their segment maps, one entry each
    double* pool = nullptr;
    double* maps = nullptr;
    AdjLong* longs = nullptr;
    long long pool_cap = 0;
    size_t longs_bytes = 0;
};

struct gc_ctx {
    int device;
    int n_cu;
    gc_tune tune;
    DevCounters* d_cnt;
    double* d_part;
    double* d_ccout;
    double* d_map_part = nullptr;   // correlation map: partial sums per (dy, row chunk, dx), grown on demand
    size_t map_part_bytes = 0;
    double* d_peak = nullptr;       // correlation map: { peak, dx, dy }
    double* d_scratch = nullptr;    // this device's copy of `scratch` (device address)
    WfStore wf;
    AdjStore adj;
};

// Scratch of gc_cross_correlate_noalloc: the block partials of the moments
// pass (kCCBlocks x 5 moments x kCCMaxCh channels), one copy per GPU for the
// life of the process.  Host code never passes this name to a kernel (on the
// host it only stands in for the symbol): it takes the device address that
// hipGetSymbolAddress returns for the current device, recorded once per
// device when the first context on it is created.
static __device__ __align__(256) double scratch[kCCBlocks * 5 * kCCMaxCh];
constexpr int kMaxDevices = 256;
static std::mutex g_scratch_mu;
static double* g_scratch_addr[kMaxDevices] = {};

static thread_local std::string g_err;

static gc_status fail(gc_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static gc_status fail(gc_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

// No C++ exception may cross the C ABI: a host allocation that throws
// becomes GC_ENOMEM.
static gc_status host_alloc_failed()
{
    try {
        g_err = "host allocation failed";
    } catch (...) {
    }
    return GC_ENOMEM;
}

#define GC_GUARD(call)                  \
    do {                                \
        try {                           \
            return (call);              \
        } catch (...) {                 \
            return host_alloc_failed(); \
        }                               \
    } while (0)

#define HIP_OK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail(GC_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));  \
    } while (0)

static double host_kepler_height(double A, double L, double x)
{
    // grating height at x: solve k x = E - e sin E, S = A cos E
    const double k = 2.0 * M_PI / L, e = A * k;
    double N = std::nearbyint(x / L);
    double M = k * (x - N * L);
    double lo = M - e, hi = M + e, E = M;
    for (int it = 0; it < 200; ++it) {
        double f = E - e * std::sin(E) - M;
        if (f > 0) hi = E; else lo = E;
        double En = E - f / (1.0 - e * std::cos(E));
        if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
        if (std::fabs(En - E) <= 1e-16 * std::fmax(1.0, std::fabs(E))) { E = En; break; }
        E = En;
    }
    return A * std::cos(E);
}

static gc_status make_scene(const gc_scene* sc, SceneDev* s)
{
    if (!sc) return fail(GC_EINVAL, "scene is null");
    if (!(std::isfinite(sc->Lambda) && sc->Lambda > 0)) return fail(GC_EINVAL, "Lambda must be finite and > 0");
    if (!std::isfinite(sc->A)) return fail(GC_EINVAL, "A must be finite");
    if (sc->A < 0) return fail(GC_EDOMAIN, "A must be >= 0");
    const double k = 2.0 * M_PI / sc->Lambda;
    if (sc->A * k >= 1.0) return fail(GC_EDOMAIN, "A k = %g >= 1: W0 is not single-valued on the cloak", sc->A * k);
    if (std::isnan(sc->half_width) || !(sc->half_width > 0)) return fail(GC_EINVAL, "half_width must be > 0");
    if (std::isnan(sc->y_top) || !(sc->y_top > sc->A)) return fail(GC_EINVAL, "y_top must exceed A");
    if (sc->cloak < GC_CLOAK_NONE || sc->cloak > GC_CLOAK_PLATE) return fail(GC_EINVAL, "cloak must be 0, 1, 2 or 3");
    if (sc->mirror != 0 && sc->mirror != 1) return fail(GC_EINVAL, "mirror must be 0 or 1");
    if (sc->mirror == 1 && (sc->cloak == GC_CLOAK_EQ1 || sc->cloak == GC_CLOAK_REFERENCED))
        return fail(GC_EUNSUPPORTED, "the flat mirror is only provided without cloak or under the plate");
    if (std::isnan(sc->sky_K) || !(sc->sky_K > 0)) return fail(GC_EINVAL, "sky_K must be > 0");
    if (sc->fresnel != 0 && sc->fresnel != 1) return fail(GC_EINVAL, "fresnel must be 0 or 1");
    if (sc->backdrop != GC_BACKDROP_SKY && sc->backdrop != GC_BACKDROP_PLANE) return fail(GC_EINVAL, "backdrop must be 0 or 1");
    if (sc->backdrop == GC_BACKDROP_PLANE &&
        !(std::isfinite(sc->backdrop_y) && std::isfinite(sc->backdrop_period) && sc->backdrop_period > 0))
        return fail(GC_EINVAL, "the backdrop plane needs a finite backdrop_y and backdrop_period > 0");
    s->L = sc->Lambda;
    s->A = sc->A;
    s->hw = sc->half_width;
    s->ytop = sc->y_top;
    s->K = sc->sky_K;
    s->k = k;
    s->e = sc->A * k;
    s->invL = 1.0 / sc->Lambda;
    s->invk = 1.0 / k;
    s->ybp = sc->A > 0 ? (1.0 + std::log(s->e)) / k : -HUGE_VAL;
    s->S_hw = (sc->mirror == 0 && std::isfinite(sc->half_width)) ? host_kepler_height(sc->A, sc->Lambda, sc->half_width) : 0.0;
    s->cloak = sc->cloak;
    s->mirror = sc->mirror;
    // Sec. 4: the referenced cloak divides every index of eq. (1) by its
    // minimum n_min = 1 / (1 + A k); the plate has index 1 / n_min
    s->nsc = sc->cloak == GC_CLOAK_REFERENCED ? 1.0 + s->e : 1.0;
    s->nsc2 = s->nsc * s->nsc;
    s->nplate = 1.0 + s->e;
    s->fresnel = sc->fresnel;
    s->backdrop = sc->backdrop;
    s->bd_y = sc->backdrop == GC_BACKDROP_PLANE ? sc->backdrop_y : 0.0;
    s->bd_P = sc->backdrop == GC_BACKDROP_PLANE ? sc->backdrop_period : 1.0;
    return GC_OK;
}

static gc_status make_camera(const gc_camera* c, CamDev* d)
{
    if (!c) return fail(GC_EINVAL, "camera is null");
    if (c->width < 1 || c->height < 1 || c->spp < 1) return fail(GC_EINVAL, "width, height and spp must be >= 1");
    if ((long long)c->width * c->height > (1ll << 31)) return fail(GC_EINVAL, "image too large");
    if (!(c->fov_y_deg > 0 && c->fov_y_deg < 180)) return fail(GC_EINVAL, "fov_y_deg must be in (0, 180)");
    double f[3];
    double n2 = 0;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(c->eye[a]) || !std::isfinite(c->target[a])) return fail(GC_EINVAL, "camera eye/target must be finite");
        f[a] = c->target[a] - c->eye[a];
        n2 += f[a] * f[a];
    }
    if (!(n2 > 0)) return fail(GC_EINVAL, "eye and target coincide");
    for (int a = 0; a < 3; ++a) f[a] /= std::sqrt(n2);
    // right = forward x up hint (+y when the hint is zero)
    double hint[3] = {c->up[0], c->up[1], c->up[2]};
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(hint[a])) return fail(GC_EINVAL, "camera up must be finite");
    if (hint[0] == 0.0 && hint[1] == 0.0 && hint[2] == 0.0) hint[1] = 1.0;
    double r[3] = {f[1] * hint[2] - f[2] * hint[1], f[2] * hint[0] - f[0] * hint[2], f[0] * hint[1] - f[1] * hint[0]};
    double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rn > 1e-12)) return fail(GC_EINVAL, "camera looks along its up vector: right vector undefined");
    for (int a = 0; a < 3; ++a) r[a] /= rn;
    if (!(c->fov_x_deg >= 0 && c->fov_x_deg < 180)) return fail(GC_EINVAL, "fov_x_deg must be in [0, 180)");
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    for (int a = 0; a < 3; ++a) {
        d->eye[a] = c->eye[a];
        d->f[a] = f[a];
        d->r[a] = r[a];
        d->u[a] = u[a];
    }
    d->t = std::tan(0.5 * c->fov_y_deg * M_PI / 180.0);
    d->aspect = c->fov_x_deg > 0 ? std::tan(0.5 * c->fov_x_deg * M_PI / 180.0) / d->t
                                 : (double)c->width / (double)c->height;
    d->W = c->width;
    d->H = c->height;
    d->spp = c->spp;
    d->jitter = c->jitter ? 1 : 0;
    d->seed = c->seed;
    d->scene_index = c->scene_index;
    return GC_OK;
}

static gc_status make_opts(const gc_opts* p, OptsDev* o)
{
    if (!p) return fail(GC_EINVAL, "opts is null");
    if (p->prec != GC_F64 && p->prec != GC_F32) return fail(GC_EINVAL, "prec must be GC_F64 or GC_F32");
    if (p->integ != GC_RK4 && p->integ != GC_DOPRI5) return fail(GC_EINVAL, "integ must be GC_RK4 or GC_DOPRI5");
    if (!(p->h > 0 && std::isfinite(p->h))) return fail(GC_EINVAL, "h must be > 0");
    if (!(p->rtol > 0 && p->atol > 0)) return fail(GC_EINVAL, "rtol and atol must be > 0");
    if (!(p->h_min > 0 && p->h_max >= p->h_min && p->h0 > 0)) return fail(GC_EINVAL, "need 0 < h_min <= h_max and h0 > 0");
    if (!(p->w_fallback >= 0)) return fail(GC_EINVAL, "w_fallback must be >= 0");
    if (p->max_events < 0 || p->max_steps < 0) return fail(GC_EINVAL, "limits must be >= 0");
    if (p->fp64_stay < 0) return fail(GC_EINVAL, "fp64_stay must be >= 0");
    o->integ = p->integ;
    o->max_events = p->max_events;
    o->max_steps = p->max_steps;
    o->h = p->h;
    o->rtol = p->rtol;
    o->atol = p->atol;
    o->h_max = p->h_max;
    o->h0 = p->h0;
    o->h_min = p->h_min;
    o->wfb2 = p->w_fallback * p->w_fallback;
    o->stay = p->fp64_stay;
    return GC_OK;
}

static gc_status read_counters(gc_ctx* ctx, gc_stats* st, hipStream_t stream)
{
    DevCounters h;
    HIP_OK(hipMemcpyAsync(&h, ctx->d_cnt, sizeof h, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    std::memset(st, 0, sizeof *st);
    st->rays = (int64_t)h.rays;
    st->accepted_steps = (int64_t)h.steps;
    st->rejected_steps = (int64_t)h.rejected;
    st->events = (int64_t)h.events;
    st->fallbacks = (int64_t)h.fallbacks;
    st->failed = (int64_t)h.failed;
    return GC_OK;
}

// ---------------------------------------------------------------------------
// Adjoint orchestration.
// ---------------------------------------------------------------------------
constexpr int kAdjCap = 256;                          // tape slots per lane, first pass
constexpr size_t kAdjTapeBudget = (size_t)8 << 30;    // bytes of tape per pass
constexpr int kAdjMaxC = 256;
// Counters of the adjoint (unsigned long long, device): claims of the two
// passes, hand-overs of the first pass (front, back of the list), overflows
// of the second, then rays, steps, events, failed, inconsistent tapes,
// steps reversed in the first pass and forward steps it took; then the
// second pass's pooled records and pooled traces.
enum { AC_CLAIM = 0, AC_OVF = 3, AC_CNT = 6, AC_POOL = 13, AC_N = 15 };
// FP32 samples handed to the FP64 second pass: paths of more steps, or
// colours more sensitive to the initial direction (per unit seed) than this
constexpr long long kAdjRerunSteps = 8000;
// hand-overs of more steps than this are queued first in the second pass
constexpr long long kAdjLongSteps = 8000;
constexpr double kAdjRerunSens = 60.0;
// Second-pass traces of at least this many tape records (C steps each, or
// events) are reversed through segment maps formed in parallel
// (k_adj_maps, k_adj_chain) after the pass, instead of one record after the
// other on their lane.  Only the longer traces pay for that: a shorter
// trace's reverse sweep on its lane (about three times its forward trace)
// ends while the longest forward traces still run; below 256 records the
// maps formed after the pass cost more than they save.  The pool holds at
// most kAdjPoolRecords records (about 1.9 GB); traces that do not fit
// reverse on their lane.
constexpr int kAdjPoolMin = 256;
constexpr long long kAdjPoolRecords = 1LL << 23;

static gc_status grow(void** p, size_t* have, size_t need, const char* what)
{
    if (need <= *have) return GC_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    if (hipMalloc(p, need) != hipSuccess) return fail(GC_ENOMEM, "%s (%zu bytes): allocation failed", what, need);
    *have = need;
    return GC_OK;
}

static gc_status adj_reserve(gc_ctx* ctx, long long n, long long npix)
{
    AdjStore& a = ctx->adj;
    if (!a.ctr) {
        if (hipMalloc((void**)&a.ctr, sizeof(unsigned long long) * AC_N) != hipSuccess ||
            hipMalloc((void**)&a.red, sizeof(double) * 2) != hipSuccess ||
            hipMalloc((void**)&a.cs, sizeof(AdjCC)) != hipSuccess ||
            hipHostMalloc((void**)&a.h_ctr, sizeof(unsigned long long) * 24) != hipSuccess)
            return fail(GC_ENOMEM, "adjoint counters: allocation failed");
        int nb = 0;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj<double>, 256, 0));
        a.blocks[0] = (nb > 0 ? nb : 1) * ctx->n_cu;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_adj<float>, 256, 0));
        a.blocks[1] = (nb > 0 ? nb : 1) * ctx->n_cu;
        for (hipEvent_t& e : a.ev) HIP_OK(hipEventCreate(&e));
    }
    if (n > a.cap_samples) {
        if (a.srgb) (void)hipFree(a.srgb);
        if (a.sgrad) (void)hipFree(a.sgrad);
        if (a.ovf) (void)hipFree(a.ovf);
        a.srgb = nullptr;
        a.sgrad = nullptr;
        a.ovf = nullptr;
        a.cap_samples = 0;
        if (hipMalloc((void**)&a.srgb, sizeof(float) * 3 * (size_t)n) != hipSuccess ||
            hipMalloc((void**)&a.sgrad, sizeof(double) * 2 * (size_t)n) != hipSuccess ||
            hipMalloc((void**)&a.ovf, sizeof(long long) * (size_t)n) != hipSuccess)
            return fail(GC_ENOMEM, "adjoint sample buffers (%lld samples): allocation failed", n);
        a.cap_samples = n;
    }
    if (npix > a.cap_pix) {
        if (a.img) (void)hipFree(a.img);
        a.img = nullptr;
        a.cap_pix = 0;
        if (hipMalloc((void**)&a.img, sizeof(float) * 3 * (size_t)npix) != hipSuccess)
            return fail(GC_ENOMEM, "adjoint image: allocation failed");
        a.cap_pix = npix;
    }
    return GC_OK;
}

// One pass of k_adj over n samples (list: indices, or null for all) with
// tapes of `cap` slots; samples it cannot finish go to out_list (null: they
// are only counted).  `rerun`: apply the FP32 hand-over criteria.
template <typename T>
static gc_status adj_pass(gc_ctx* ctx, const SceneDev& s, const CamDev& c, const OptsDev& o, int C, long long n,
                          const long long* list, long long list_front, long long* out_list, int cap, bool rerun,
                          double* sgrad, int pass, bool pooled, hipStream_t stream, long long* lanes_out = nullptr)
{
    AdjStore& a = ctx->adj;
    const int prec = sizeof(T) == 8 ? 0 : 1;
    long long lanes = (long long)a.blocks[prec] * 256;
    const long long by_budget = (long long)(kAdjTapeBudget / ((size_t)cap * kTapeFields * sizeof(double)));
    lanes = std::min(lanes, by_budget);
    lanes = std::min(lanes, (n + 255) / 256 * 256);
    lanes = std::max(256LL, lanes / 256 * 256);
    gc_status r;
    if ((r = grow((void**)&a.tape, &a.tape_bytes, (size_t)lanes * cap * kTapeFields * sizeof(double), "adjoint tape")) !=
        GC_OK)
        return r;
    if ((r = grow(&a.seg, &a.seg_bytes, (size_t)lanes * C * seg_fields<T>() * sizeof(T), "adjoint segment buffer")) != GC_OK)
        return r;
    AdjIo io;
    io.n = n;
    io.list = list;
    io.list_front = list_front;
    io.list_cap = a.cap_samples;
    io.claim = a.ctr + AC_CLAIM + pass;
    io.tape = a.tape;
    io.cap = cap;
    io.seg = a.seg;
    io.srgb = a.srgb;
    io.sgrad = sgrad;
    io.ovf = out_list;
    io.ovf_cap = a.cap_samples;
    io.n_ovf = a.ctr + AC_OVF + 2 * pass;
    io.long_steps = kAdjLongSteps;
    io.cnt = a.ctr + AC_CNT;
    io.rerun_steps = rerun ? kAdjRerunSteps : (1LL << 62);
    io.rerun_sens = rerun ? kAdjRerunSens : HUGE_VAL;
    io.pool = pooled ? a.pool : nullptr;
    io.pool_cap = a.pool_cap;
    io.pool_used = a.ctr + AC_POOL;
    io.pool_min = kAdjPoolMin;
    io.longs = a.longs;
    io.n_long = a.ctr + AC_POOL + 1;
    const T wfb2 = (T)o.wfb2;
    hipLaunchKernelGGL(k_adj<T>, dim3((unsigned)(lanes / 256)), dim3(256), 0, stream, s, c, o, wfb2, C, io);
    HIP_OK(hipGetLastError());
    if (lanes_out) *lanes_out = lanes;
    return GC_OK;
}

// Two passes: (0) all samples in precision T with tapes of kAdjCap slots;
// (1) the samples it handed over -- tapes too short, and in FP32 the long
// or sensitive traces -- in FP64 with tapes long enough for any trace the
// options allow, the longest traces first.
template <typename T>
static gc_status adj_run(gc_ctx* ctx, const SceneDev& s, const CamDev& c, const OptsDev& o, int C,
                         const float* ref, int kind, float* img, double* sgrad, double out[3], gc_stats* st,
                         hipStream_t stream)
{
    AdjStore& a = ctx->adj;
    const long long npix = (long long)c.W * c.H, n = npix * c.spp;
    gc_status r;
    HIP_OK(hipEventRecord(a.ev[0], stream));
    const long long nbm = std::min<long long>(kCCBlocks, (npix + 255) / 256);
    HIP_OK(hipMemsetAsync(a.ctr, 0, sizeof(unsigned long long) * AC_N, stream));
    if ((r = adj_pass<T>(ctx, s, c, o, C, n, nullptr, 0, a.ovf, kAdjCap, sizeof(T) == 4, sgrad, 0, false, stream)) !=
        GC_OK)
        return r;
    HIP_OK(hipEventRecord(a.ev[1], stream));
    HIP_OK(hipMemcpyAsync(a.h_ctr, a.ctr, sizeof(unsigned long long) * AC_N, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    const long long n_front = (long long)a.h_ctr[AC_OVF + 0], n_back = (long long)a.h_ctr[AC_OVF + 1];
    const long long handed = n_front + n_back;
    if (handed > 0) {
        // the second pass reads the list's front part from its start and the
        // rest from its end, where the first pass wrote them
        // every record a trace can write: one per C steps, three per event
        const long long cap2 = o.max_steps / C + 3LL * (o.max_events + 1) + 8;
        if (cap2 > (1LL << 30)) return fail(GC_EUNSUPPORTED, "max_steps / checkpoint_every too large for the tape");
        // the pool for the long traces, and one entry per handed-over sample
        if (!a.pool || !a.maps) {
            if (a.pool) (void)hipFree(a.pool);
            if (a.maps) (void)hipFree(a.maps);
            a.pool = a.maps = nullptr;
            if (hipMalloc((void**)&a.pool, sizeof(double) * kTapeFields * (size_t)kAdjPoolRecords) != hipSuccess ||
                hipMalloc((void**)&a.maps, sizeof(double) * kMapFields * (size_t)kAdjPoolRecords) != hipSuccess) {
                if (a.pool) (void)hipFree(a.pool);
                if (a.maps) (void)hipFree(a.maps);
                a.pool = a.maps = nullptr;
                a.pool_cap = 0;
                return fail(GC_ENOMEM, "adjoint tape pool: allocation failed");
            }
            a.pool_cap = kAdjPoolRecords;
        }
        if ((r = grow((void**)&a.longs, &a.longs_bytes, sizeof(AdjLong) * (size_t)handed, "adjoint pool list")) !=
            GC_OK)
            return r;
        long long lanes = 0;
        if ((r = adj_pass<double>(ctx, s, c, o, C, handed, a.ovf, n_front, nullptr, (int)cap2, false, sgrad, 1, true,
                                  stream, &lanes)) != GC_OK)
            return r;
        // the pooled traces: segment maps over all their records, then one
        // reverse sweep per trace (the per-lane segment buffers of the
        // second pass serve both)
        hipLaunchKernelGGL(k_adj_maps, dim3((unsigned)(lanes / 256)), dim3(256), 0, stream, s, o, o.wfb2, C, a.pool,
                           (const unsigned long long*)(a.ctr + AC_POOL), a.pool_cap, a.maps, (double*)a.seg);
        hipLaunchKernelGGL(k_adj_chain, dim3((unsigned)(lanes / 256)), dim3(256), 0, stream, s, o, o.wfb2, C,
                           (const double*)a.pool, (const double*)a.maps, (const AdjLong*)a.longs,
                           (const unsigned long long*)(a.ctr + AC_POOL + 1), (double*)a.seg, sgrad, a.ctr + AC_CNT);
        HIP_OK(hipGetLastError());
    }
    HIP_OK(hipEventRecord(a.ev[2], stream));
    hipLaunchKernelGGL(k_adj_image, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, stream, a.srgb, npix, c.spp,
                       img);
    hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nbm), dim3(256), 0, stream, img, ref, npix, npix, npix, 3,
                       ctx->d_part);
    hipLaunchKernelGGL(k_adj_ccstat, dim3(1), dim3(64), 0, stream, ctx->d_part, (int)nbm, npix, img, ref, a.cs);
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(1024), 0, stream, sgrad, n, c.spp, img, ref, a.cs, kind, a.red);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(a.ev[3], stream));
    HIP_OK(hipMemcpyAsync(a.h_ctr, a.ctr, sizeof(unsigned long long) * AC_N, hipMemcpyDeviceToHost, stream));
    AdjCC hc;
    HIP_OK(hipMemcpyAsync((double*)(a.h_ctr + 16), a.red, sizeof(double) * 2, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(&hc, a.cs, sizeof hc, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (a.h_ctr[AC_OVF + 2] != 0)
        return fail(GC_EDEVICE, "adjoint: %llu samples overflowed the full-length tape", a.h_ctr[AC_OVF + 2]);
    if (a.h_ctr[AC_CNT + 4] != 0)
        return fail(GC_EDEVICE, "adjoint: %llu samples with an inconsistent tape", a.h_ctr[AC_CNT + 4]);
    const double* hd = (const double*)(a.h_ctr + 16);
    if (!(hc.sff > 0)) return fail(GC_EINVAL, "reference image is constant: eq. (15) is undefined");
    if (kind == 1 && !(hc.sgg > 0)) return fail(GC_EINVAL, "rendered image is constant: NCC is undefined");
    out[0] = 1.0 - (kind == 0 ? hc.c0 : hc.ncc);
    out[1] = hd[0];          // dL/dA
    out[2] = hd[1];          // dL/dhw
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->rays = (int64_t)a.h_ctr[AC_CNT + 0];
        st->accepted_steps = (int64_t)a.h_ctr[AC_CNT + 1];
        st->events = (int64_t)a.h_ctr[AC_CNT + 2];
        st->failed = (int64_t)a.h_ctr[AC_CNT + 3];
        st->tail_rays = handed;
        st->rounds = n_front;
        st->hot_steps = (int64_t)a.h_ctr[AC_CNT + 5];
        st->first_pass_steps = (int64_t)a.h_ctr[AC_CNT + 6];
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, a.ev[0], a.ev[1]));
        st->hot_ms = ms;
        HIP_OK(hipEventElapsedTime(&ms, a.ev[1], a.ev[2]));
        st->tail_ms = ms;
        HIP_OK(hipEventElapsedTime(&ms, a.ev[0], a.ev[3]));
        st->total_ms = ms;
    }
    return GC_OK;
}

// ---------------------------------------------------------------------------
// FP32 pipeline orchestration.
// ---------------------------------------------------------------------------
static size_t wf_ray_bytes(long long n) { return (size_t)n * (8 * 8 + 10 * 4 + 14 * 4 + 3 * 4 + 4); }

static void wf_carve(void* base, long long n, WfRays& R)
{
    char* p = (char*)base;
    auto take = [&](size_t bytes) { char* r = p; p += (bytes + 255) & ~(size_t)255; return r; };
    double** d[] = {&R.rx, &R.ry, &R.rz, &R.qx, &R.qy, &R.qz, &R.z0, &R.wgt};
    for (double** q : d) *q = (double*)take(sizeof(double) * n);
    int** ip[] = {&R.cell, &R.steps, &R.rej, &R.events, &R.flags, &R.scene, &R.status, &R.fbk, &R.parent, &R.steps0};
    for (int** q : ip) *q = (int*)take(sizeof(int) * n);
    float** fp[] = {&R.fx, &R.lx, &R.y, &R.ly, &R.px, &R.lpx, &R.py, &R.lpy, &R.pz, &R.Wr, &R.Wi, &R.h, &R.tau,
                    &R.ltau};
    for (float** q : fp) *q = (float*)take(sizeof(float) * n);
    R.rgb = (float*)take(sizeof(float) * 3 * n);
}

static void wf_free(WfStore& w)
{
    void* bufs[] = {w.rays, w.queues, w.tables, w.ctr, w.tot, w.acc};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (w.h_ctr) (void)hipHostFree(w.h_ctr);
    for (hipEvent_t e : w.ev)
        if (e) (void)hipEventDestroy(e);
    w = WfStore();
}

static size_t wf_table_bytes(int ns)
{
    return (size_t)ns * (sizeof(SceneDev) + sizeof(CamDev) + sizeof(float*)) + (size_t)(ns + 1) * 2 * sizeof(long long) +
           1024;
}

static gc_status wf_reserve(gc_ctx* ctx, WfStore& w, long long n_rays, int n_scenes)
{
    if (!w.ctr) {
        if (hipMalloc(&w.ctr, sizeof(QCtr)) != hipSuccess || hipMalloc(&w.tot, sizeof(WfTotals)) != hipSuccess ||
            hipHostMalloc(&w.h_ctr, sizeof(QCtr)) != hipSuccess)
            return fail(GC_ENOMEM, "pipeline counters: allocation failed");
        int nb = 0;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_wf_box<0>, 256, 0));
        w.box_blocks[0] = (nb > 0 ? nb : 1) * ctx->n_cu;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_wf_box<1>, 256, 0));
        w.box_blocks[1] = (nb > 0 ? nb : 1) * ctx->n_cu;
        for (hipEvent_t& e : w.ev) HIP_OK(hipEventCreate(&e));
    }
    if (n_rays > w.cap_rays) {
        if (w.rays) (void)hipFree(w.rays);
        if (w.queues) (void)hipFree(w.queues);
        w.rays = nullptr;
        w.queues = nullptr;
        w.cap_rays = 0;
        long long cap = n_rays + n_rays / 8;
        if (hipMalloc(&w.rays, wf_ray_bytes(cap) + 64 * 256) != hipSuccess ||
            hipMalloc((void**)&w.queues, sizeof(int) * 6 * (size_t)cap) != hipSuccess)
            return fail(GC_ENOMEM, "pipeline ray buffers (%lld rays): allocation failed", cap);
        w.cap_rays = cap;
    }
    if (n_scenes > w.cap_scenes) {
        if (w.tables) (void)hipFree(w.tables);
        w.tables = nullptr;
        w.cap_scenes = 0;
        if (hipMalloc(&w.tables, wf_table_bytes(n_scenes)) != hipSuccess)
            return fail(GC_ENOMEM, "pipeline scene tables: allocation failed");
        w.cap_scenes = n_scenes;
    }
    return GC_OK;
}

struct WfTables {
    SceneDev* scenes;
    CamDev* cams;
    long long* ray_off;
    long long* pix_off;
    float** images;
};

static WfTables wf_tables(void* base, int ns)
{
    WfTables t;
    char* p = (char*)base;
    t.scenes = (SceneDev*)p;
    p += sizeof(SceneDev) * ns;
    t.cams = (CamDev*)p;
    p += sizeof(CamDev) * ns;
    p = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    t.ray_off = (long long*)p;
    p += sizeof(long long) * (ns + 1);
    t.pix_off = (long long*)p;
    p += sizeof(long long) * (ns + 1);
    t.images = (float**)p;
    return t;
}

// persistent grid of the in-box kernel under the context's scheduling
static unsigned wf_box_max(const gc_ctx* ctx, const WfStore& w, int integ)
{
    int box_max = w.box_blocks[integ];
    if (ctx->tune.waves_per_simd > 0) box_max = std::min(box_max, ctx->tune.waves_per_simd * ctx->n_cu);
    return (unsigned)box_max;
}

// Grid of the air kernel: its queue length is known on the device only.
static unsigned wf_air_blocks(const gc_ctx* ctx, const WfArgs& a)
{
    return (unsigned)std::max<long long>(1, std::min<long long>((a.n_rays + 255) / 256, 2ll * ctx->n_cu));
}

// Start of a launch: counters zeroed, camera (or given) rays to the box
// queues of the first round; the rays whose first leg meets the bare grating
// walk in the air kernel.  Enqueues kernels only, so that a graph can hold it.
static void wf_start(const gc_ctx* ctx, WfStore& w, const WfArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_wf_zero, dim3(1), dim3(64), 0, stream, w.ctr, w.tot, a.qbox[0], a.n_front);
    hipLaunchKernelGGL(k_wf_init, dim3((unsigned)((a.n_rays + 256 * kInitRays - 1) / (256 * kInitRays))), dim3(256), 0,
                       stream, a);
    hipLaunchKernelGGL(k_wf_air, dim3(wf_air_blocks(ctx, a)), dim3(256), 0, stream, a, 0);
}

// The parts of a round: the in-box kernel takes every ray of the round's
// queues through its visit (or to a step that needs FP64); then the FP64
// kernel takes those steps and the air kernel walks the rays that left.
// Enqueue kernels only, so that a graph can hold them; a batch plan
// captures them as separate graphs, so that events between its graph
// launches time the in-box kernel.
static void wf_round_box(const WfArgs& a, int cur, unsigned box_g, hipStream_t stream)
{
    if (a.o.integ == 0)
        hipLaunchKernelGGL(k_wf_box<0>, dim3(box_g), dim3(256), 0, stream, a, cur);
    else
        hipLaunchKernelGGL(k_wf_box<1>, dim3(box_g), dim3(256), 0, stream, a, cur);
}

static void wf_round_post(const gc_ctx* ctx, const WfArgs& a, int cur, unsigned air_g, hipStream_t stream)
{
    if (a.o.integ == 0)
        hipLaunchKernelGGL(k_wf_event<0>, dim3(air_g), dim3(256), 0, stream, a, cur);
    else
        hipLaunchKernelGGL(k_wf_event<1>, dim3(air_g), dim3(256), 0, stream, a, cur);
    hipLaunchKernelGGL(k_wf_air, dim3(wf_air_blocks(ctx, a)), dim3(256), 0, stream, a, cur ^ 1);
}

// One round: its counters' reset and both parts.  With events, ev[0] and
// ev[1] bracket the in-box kernel and ev[2] follows the other two.
static gc_status wf_round(gc_ctx* ctx, WfStore& w, const WfArgs& a, int cur, unsigned box_g, unsigned air_g,
                          const hipEvent_t* ev, hipStream_t stream)
{
    hipLaunchKernelGGL(k_wf_reset, dim3(1), dim3(64), 0, stream, w.ctr, cur);
    if (ev) HIP_OK(hipEventRecord(ev[0], stream));
    wf_round_box(a, cur, box_g, stream);
    if (ev) HIP_OK(hipEventRecord(ev[1], stream));
    wf_round_post(ctx, a, cur, air_g, stream);
    if (ev) HIP_OK(hipEventRecord(ev[2], stream));
    HIP_OK(hipGetLastError());
    return GC_OK;
}

// Run the pipeline for a filled WfArgs (tables already on the device),
// round by round, reading the queue lengths back after each.
static gc_status wf_rounds(gc_ctx* ctx, WfStore& w, WfArgs& a, unsigned len, hipStream_t stream)
{
    const unsigned box_max = wf_box_max(ctx, w, a.o.integ);
    // one round per visit of the box
    for (int round = 0; len > 0; ++round) {
        const int cur = round & 1;
        const unsigned need = (len + 255) / 256;
        const unsigned box_g = std::min<unsigned>(need, box_max);
        const unsigned air_g = std::min<unsigned>(need, (unsigned)(8 * ctx->n_cu));
        gc_status r = wf_round(ctx, w, a, cur, box_g, air_g, &w.ev[1], stream);
        if (r != GC_OK) return r;
        HIP_OK(hipMemcpyAsync(w.h_ctr, w.ctr, sizeof(QCtr), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        float t1 = 0.f, t2 = 0.f;
        HIP_OK(hipEventElapsedTime(&t1, w.ev[1], w.ev[2]));
        HIP_OK(hipEventElapsedTime(&t2, w.ev[2], w.ev[3]));
        w.hot_ms += t1;
        w.event_ms += t2;
        w.rounds += 1;
        len = w.h_ctr->box_len[cur ^ 1] + w.h_ctr->slow_len[cur ^ 1];
        if (round > 100000) return fail(GC_EDEVICE, "pipeline did not drain");
    }
    return GC_OK;
}

static gc_status wf_run(gc_ctx* ctx, WfStore& w, WfArgs& a, hipStream_t stream)
{
    w.fp64_steps = 0;
    w.rounds = 0;
    w.tail_rays = 0;
    w.hot_ms = w.event_ms = w.tail_ms = 0.0;
    HIP_OK(hipEventRecord(w.ev[0], stream));
    wf_start(ctx, w, a, stream);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(w.h_ctr, w.ctr, sizeof(QCtr), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    return wf_rounds(ctx, w, a, w.h_ctr->box_len[0] + w.h_ctr->slow_len[0], stream);
}

static WfArgs wf_args(const gc_ctx* ctx, const WfStore& w, const OptsDev& o, int ns, long long n_rays)
{
    WfArgs a;
    std::memset(&a, 0, sizeof a);
    wf_carve(w.rays, w.cap_rays, a.R);
    a.qbox[0] = w.queues;
    a.qbox[1] = w.queues + w.cap_rays;
    a.qev = w.queues + 2 * w.cap_rays;
    a.qslow[0] = w.queues + 3 * w.cap_rays;
    a.qslow[1] = w.queues + 4 * w.cap_rays;
    a.qair = w.queues + 5 * w.cap_rays;
    a.sch.slow_pxy2 = (float)(ctx->tune.slow_pxy * ctx->tune.slow_pxy);
    a.sch.slow_div = ctx->tune.slow_wave_div;
    a.sch.refill = ctx->tune.refill;
    a.ctr = w.ctr;
    WfTables t = wf_tables(w.tables, ns);
    a.scenes = t.scenes;
    a.cams = t.cams;
    a.ray_off = t.ray_off;
    a.n_scenes = ns;
    a.n_rays = n_rays;
    a.o = o;
    return a;
}

static gc_status wf_read_totals(WfStore& w, gc_stats* st, hipStream_t stream)
{
    WfTotals h;
    HIP_OK(hipEventRecord(w.ev[4], stream));
    HIP_OK(hipMemcpyAsync(&h, w.tot, sizeof h, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    float tt = 0.f;
    HIP_OK(hipEventElapsedTime(&tt, w.ev[0], w.ev[4]));
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->rays = (int64_t)h.rays;
        st->accepted_steps = (int64_t)h.steps;
        st->rejected_steps = (int64_t)h.rejected;
        st->events = (int64_t)h.events;
        st->fallbacks = (int64_t)h.fallbacks;
        st->failed = (int64_t)h.failed;
        // the in-box steps the FP32 kernel did not take: the FP64 event kernel's
        st->fp64_steps = (int64_t)h.steps - (int64_t)w.h_ctr->hot_steps;
        st->rounds = w.rounds;
        st->hot_ms = w.hot_ms;
        st->event_ms = w.event_ms;
        st->tail_ms = w.tail_ms;
        st->tail_rays = w.tail_rays;
        st->hot_steps = (int64_t)w.h_ctr->hot_steps;
        st->total_ms = tt;
    }
    return GC_OK;
}

// Render n scenes with the FP32 pipeline into the given device images.
// Reserve the store's buffers for n scenes, upload their tables and fill
// the kernel arguments (render mode).  n_pix: total pixels.
static gc_status wf_setup(gc_ctx* ctx, WfStore& w, int ns, const SceneDev* sc, const CamDev* cams, const OptsDev& o,
                          float* const* d_rgb, hipStream_t stream, WfArgs* a, long long* n_pix_out,
                          long long extra = 0)
{
    std::vector<long long> roff(ns + 1), poff(ns + 1);
    roff[0] = poff[0] = 0;
    for (int i = 0; i < ns; ++i) {
        long long npx = (long long)cams[i].W * cams[i].H;
        poff[i + 1] = poff[i] + npx;
        roff[i + 1] = roff[i] + npx * cams[i].spp;
    }
    const long long n_rays = roff[ns], n_pix = poff[ns];
    if (n_rays + extra > (1ll << 31) - 1) return fail(GC_EINVAL, "more than 2^31 - 1 samples (and branches) in one launch");
    gc_status r = wf_reserve(ctx, w, n_rays + extra, ns);
    if (r != GC_OK) return r;
    // tables: staged in host memory, copied in one go
    const size_t tb = wf_table_bytes(ns);
    std::vector<char> host(tb, 0);
    WfTables th = wf_tables(host.data(), ns);
    for (int i = 0; i < ns; ++i) {
        th.scenes[i] = sc[i];
        th.cams[i] = cams[i];
        th.images[i] = d_rgb[i];
    }
    for (int i = 0; i <= ns; ++i) { th.ray_off[i] = roff[i]; th.pix_off[i] = poff[i]; }
    HIP_OK(hipMemcpyAsync(w.tables, host.data(), tb, hipMemcpyHostToDevice, stream));
    *a = wf_args(ctx, w, o, ns, n_rays);
    *n_pix_out = n_pix;
    return GC_OK;
}

// pixel averages and counters (enqueue only)
static gc_status wf_finish(WfStore& w, const WfArgs& a, int ns, long long n_pix, hipStream_t stream)
{
    WfTables td = wf_tables(w.tables, ns);
    hipLaunchKernelGGL(k_wf_finish, dim3((unsigned)std::min((n_pix + 255) / 256, kFoldBlocks)), dim3(256), 0,
                       stream, a, (float* const*)td.images, (const long long*)td.pix_off, n_pix, w.tot);
    HIP_OK(hipGetLastError());
    return GC_OK;
}

// With Fresnel-weighted faces: the primaries' pass appends the reflected
// branches to a pool after the primaries' slots (4 per sample to start with;
// a pass that overflows it is run again with room for every branch it
// asked for); then the branches' pass (the same rounds, no further splits)
// and the weighted per-sample sums.
static gc_status wf_render_fresnel(gc_ctx* ctx, int ns, const SceneDev* sc, const CamDev* cams, const OptsDev& o,
                                   float* const* d_rgb, gc_stats* st, hipStream_t stream)
{
    WfStore& w = ctx->wf;
    long long n_rays = 0;
    for (int i = 0; i < ns; ++i) n_rays += (long long)cams[i].W * cams[i].H * cams[i].spp;
    long long cap = 4 * n_rays + 65536;
    WfArgs a;
    long long n_pix = 0;
    unsigned n_seeds = 0;
    for (int attempt = 0;; ++attempt) {
        if (n_rays + cap > (1ll << 31) - 1) cap = (1ll << 31) - 1 - n_rays;
        gc_status r = wf_setup(ctx, w, ns, sc, cams, o, d_rgb, stream, &a, &n_pix, cap);
        if (r != GC_OK) return r;
        a.seed_base = n_rays;
        a.seed_cap = (unsigned)cap;
        if ((r = wf_run(ctx, w, a, stream)) != GC_OK) return r;
        n_seeds = w.h_ctr->seed_len;
        if ((long long)n_seeds <= cap) break;
        if (attempt > 0 || n_rays + (long long)n_seeds > (1ll << 31) - 1)
            return fail(GC_ENOMEM, "%u Fresnel branches do not fit one launch", n_seeds);
        cap = n_seeds;
    }
    if (n_seeds > 0) {
        hipLaunchKernelGGL(k_wf_seed_reset, dim3(1), dim3(64), 0, stream, w.ctr);
        const unsigned g = (unsigned)std::min<long long>((n_seeds + 255) / 256, 8LL * ctx->n_cu);
        hipLaunchKernelGGL(k_wf_seed_init, dim3(g), dim3(256), 0, stream, a, n_seeds);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(w.h_ctr, w.ctr, sizeof(QCtr), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        gc_status r = wf_rounds(ctx, w, a, w.h_ctr->box_len[0] + w.h_ctr->slow_len[0], stream);
        if (r != GC_OK) return r;
    }
    gc_status r = grow((void**)&w.acc, &w.acc_bytes, sizeof(unsigned long long) * 3 * (size_t)n_rays,
                       "Fresnel colour sums");
    if (r != GC_OK) return r;
    const unsigned gf = (unsigned)std::min<long long>((n_rays + n_seeds + 255) / 256, kFoldBlocks);
    hipLaunchKernelGGL(k_fill_u64, dim3(gf), dim3(256), 0, stream, w.acc, 3 * n_rays);
    hipLaunchKernelGGL(k_wf_fresnel_fold, dim3(gf), dim3(256), 0, stream, a, n_seeds, w.acc, w.tot);
    hipLaunchKernelGGL(k_wf_fresnel_rgb, dim3(gf), dim3(256), 0, stream, a, (const unsigned long long*)w.acc);
    HIP_OK(hipGetLastError());
    w.tail_rays = n_seeds;
    if ((r = wf_finish(w, a, ns, n_pix, stream)) != GC_OK) return r;
    return wf_read_totals(w, st, stream);
}

static gc_status wf_render(gc_ctx* ctx, int ns, const SceneDev* sc, const CamDev* cams, const OptsDev& o,
                           float* const* d_rgb, gc_stats* st, hipStream_t stream)
{
    for (int i = 0; i < ns; ++i)
        if (sc[i].fresnel) return wf_render_fresnel(ctx, ns, sc, cams, o, d_rgb, st, stream);
    WfStore& w = ctx->wf;
    WfArgs a;
    long long n_pix = 0;
    gc_status r = wf_setup(ctx, w, ns, sc, cams, o, d_rgb, stream, &a, &n_pix);
    if (r != GC_OK) return r;
    if ((r = wf_run(ctx, w, a, stream)) != GC_OK) return r;
    if ((r = wf_finish(w, a, ns, n_pix, stream)) != GC_OK) return r;
    return wf_read_totals(w, st, stream);
}

static gc_status wf_trace(gc_ctx* ctx, const SceneDev& s, const OptsDev& o, long long n, const double* org,
                          const double* dir, double* out_org, double* out_dir, int* status, long long* steps,
                          int* events, hipStream_t stream)
{
    WfStore& w = ctx->wf;
    gc_status r = wf_reserve(ctx, w, n, 1);
    if (r != GC_OK) return r;
    std::vector<char> host(wf_table_bytes(1), 0);
    WfTables th = wf_tables(host.data(), 1);
    th.scenes[0] = s;
    th.ray_off[0] = 0;
    th.ray_off[1] = n;
    HIP_OK(hipMemcpyAsync(w.tables, host.data(), host.size(), hipMemcpyHostToDevice, stream));
    WfArgs a = wf_args(ctx, w, o, 1, n);
    a.in_org = org;
    a.in_dir = dir;
    r = wf_run(ctx, w, a, stream);
    if (r != GC_OK) return r;
    hipLaunchKernelGGL(k_wf_trace_out, dim3((unsigned)std::min((n + 255) / 256, kFoldBlocks)), dim3(256), 0, stream,
                       a, out_org, out_dir, status, steps, events, w.tot);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(stream));
    return GC_OK;
}

extern "C" {

const char* gc_last_error(void) { return g_err.c_str(); }

void gc_default_opts(gc_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->prec = GC_F64;
    o->integ = GC_RK4;
    o->h = 1e-3;
    o->rtol = 1e-8;
    o->atol = 1e-8;
    o->h_max = 0.02;
    o->h0 = 1e-3;
    o->h_min = 1e-12;
    o->w_fallback = 1e-2;
    o->max_events = 32;
    o->max_steps = 100000;
}

void gc_default_tune(gc_tune* t)
{
    if (!t) return;
    std::memset(t, 0, sizeof *t);
    t->slow_pxy = 0.0;
    t->slow_wave_div = 0;
    t->refill = 8;
    t->waves_per_simd = 0;
}

static gc_status set_tune_impl(gc_ctx* ctx, const gc_tune* t)
{
    if (!ctx || !t) return fail(GC_EINVAL, "ctx and tune must be non-null");
    if (!(t->slow_pxy >= 0.0 && t->slow_pxy <= 1.0)) return fail(GC_EINVAL, "slow_pxy must be in [0, 1]");
    if (t->slow_wave_div < 0) return fail(GC_EINVAL, "slow_wave_div must be >= 0");
    if (t->refill < 1 || t->refill > 64) return fail(GC_EINVAL, "refill must be in 1 .. 64");
    if (t->waves_per_simd < 0 || t->waves_per_simd > 8) return fail(GC_EINVAL, "waves_per_simd must be in 0 .. 8");
    if (t->plan_lanes < 0 || t->plan_lanes > kPlanMaxLanes) return fail(GC_EINVAL, "plan_lanes must be in 0 .. 3");
    ctx->tune = *t;
    return GC_OK;
}

gc_status gc_set_tune(gc_ctx* ctx, const gc_tune* t)
{
    GC_GUARD(set_tune_impl(ctx, t));
}

static gc_status get_tune_impl(const gc_ctx* ctx, gc_tune* t)
{
    if (!ctx || !t) return fail(GC_EINVAL, "ctx and tune must be non-null");
    *t = ctx->tune;
    return GC_OK;
}

gc_status gc_get_tune(const gc_ctx* ctx, gc_tune* t)
{
    GC_GUARD(get_tune_impl(ctx, t));
}

static gc_status create_impl(gc_ctx** out, int hip_device)
{
    if (!out) return fail(GC_EINVAL, "out is null");
    *out = nullptr;
    int n = 0;
    HIP_OK(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n) return fail(GC_EINVAL, "device %d out of range (%d devices)", hip_device, n);
    HIP_OK(hipSetDevice(hip_device));
    gc_ctx* c = new (std::nothrow) gc_ctx();
    if (!c) return fail(GC_ENOMEM, "host allocation failed");
    c->device = hip_device;
    gc_default_tune(&c->tune);
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) { delete c; return fail(GC_EDEVICE, "hipGetDeviceProperties failed"); }
        c->n_cu = prop.multiProcessorCount;
    }
    if (hip_device >= kMaxDevices) { delete c; return fail(GC_EINVAL, "device %d: at most %d devices", hip_device, kMaxDevices); }
    {
        // the device address of this GPU's `scratch`, once per device (with
        // the device current)
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_addr[hip_device]) {
            void* addr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !addr) {
                delete c;
                return fail(GC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            }
            g_scratch_addr[hip_device] = static_cast<double*>(addr);
        }
        c->d_scratch = g_scratch_addr[hip_device];
    }
    if (hipMalloc(&c->d_cnt, sizeof(DevCounters)) != hipSuccess ||
        hipMalloc(&c->d_part, sizeof(double) * kCCBlocks * 5 * kCCMaxCh) != hipSuccess ||
        hipMalloc(&c->d_ccout, sizeof(double) * kCCOut) != hipSuccess ||
        hipMalloc(&c->d_peak, sizeof(double) * 3) != hipSuccess) {
        gc_destroy(c);
        return fail(GC_ENOMEM, "device scratch allocation failed");
    }
    *out = c;
    return GC_OK;
}

gc_status gc_create(gc_ctx** out, int hip_device)
{
    GC_GUARD(create_impl(out, hip_device));
}

void gc_destroy(gc_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->d_cnt) (void)hipFree(c->d_cnt);
    if (c->d_part) (void)hipFree(c->d_part);
    if (c->d_ccout) (void)hipFree(c->d_ccout);
    if (c->d_map_part) (void)hipFree(c->d_map_part);
    if (c->d_peak) (void)hipFree(c->d_peak);
    wf_free(c->wf);
    AdjStore& a = c->adj;
    void* bufs[] = {a.tape, a.seg, a.srgb, a.sgrad, a.ovf, a.img, a.cs, a.ctr, a.red, a.pool, a.maps, a.longs};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (a.h_ctr) (void)hipHostFree(a.h_ctr);
    for (hipEvent_t e : a.ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

static gc_status trace_rays_impl(gc_ctx* ctx, const gc_scene* scene, const gc_opts* opts, int64_t n, const double* d_org,
                        const double* d_dir, double* d_out_org, double* d_out_dir, int32_t* d_status,
                        int64_t* d_steps, int32_t* d_events, hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    SceneDev s;
    OptsDev o;
    gc_status st;
    if ((st = make_scene(scene, &s)) != GC_OK) return st;
    if ((st = make_opts(opts, &o)) != GC_OK) return st;
    if (n < 0) return fail(GC_EINVAL, "n must be >= 0");
    if (n == 0) return GC_OK;
    if (!d_org || !d_dir || !d_out_dir) return fail(GC_EINVAL, "org, dir and out_dir must be non-null");
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipMemsetAsync(ctx->d_cnt, 0, sizeof(DevCounters), stream));
    long long nb = (n + 255) / 256;
    if (opts->prec == GC_F64)
        hipLaunchKernelGGL(k_trace_rays64, dim3((unsigned)nb), dim3(256), 0, stream, s, o, (long long)n, d_org,
                           d_dir, d_out_org, d_out_dir, (int*)d_status, (long long*)d_steps, (int*)d_events,
                           ctx->d_cnt);
    else
        return wf_trace(ctx, s, o, (long long)n, d_org, d_dir, d_out_org, d_out_dir, (int*)d_status,
                        (long long*)d_steps, (int*)d_events, stream);
    HIP_OK(hipGetLastError());
    return GC_OK;
}

gc_status gc_trace_rays(gc_ctx* ctx, const gc_scene* scene, const gc_opts* opts, int64_t n, const double* d_org,
                        const double* d_dir, double* d_out_org, double* d_out_dir, int32_t* d_status,
                        int64_t* d_steps, int32_t* d_events, hipStream_t stream)
{
    GC_GUARD(trace_rays_impl(ctx, scene, opts, n, d_org, d_dir, d_out_org, d_out_dir, d_status, d_steps, d_events, stream));
}

static gc_status render_impl(gc_ctx* ctx, const gc_scene* scene, const gc_camera* camera, const gc_opts* opts,
                    float* d_rgb, gc_stats* stats, hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    SceneDev s;
    CamDev c;
    OptsDev o;
    gc_status st;
    if ((st = make_scene(scene, &s)) != GC_OK) return st;
    if ((st = make_camera(camera, &c)) != GC_OK) return st;
    if ((st = make_opts(opts, &o)) != GC_OK) return st;
    if (!d_rgb) return fail(GC_EINVAL, "rgb is null");
    HIP_OK(hipSetDevice(ctx->device));
    HIP_OK(hipMemsetAsync(ctx->d_cnt, 0, sizeof(DevCounters), stream));
    long long npx = (long long)c.W * c.H;
    unsigned nb = (unsigned)((npx + 255) / 256);
    if (scene->mirror == 1 && scene->cloak == GC_CLOAK_NONE)
        hipLaunchKernelGGL(k_render_flat, dim3(flat_blocks(ctx->n_cu, npx)), dim3(256), 0, stream, c, s, d_rgb,
                           stats ? ctx->d_cnt : nullptr);
    else if (opts->prec == GC_F64 && scene->fresnel)
        hipLaunchKernelGGL(k_render64<true>, dim3(nb), dim3(256), 0, stream, s, c, o, d_rgb, ctx->d_cnt);
    else if (opts->prec == GC_F64)
        hipLaunchKernelGGL(k_render64<false>, dim3(nb), dim3(256), 0, stream, s, c, o, d_rgb, ctx->d_cnt);
    else
        return wf_render(ctx, 1, &s, &c, o, &d_rgb, stats, stream);
    HIP_OK(hipGetLastError());
    if (stats) return read_counters(ctx, stats, stream);
    return GC_OK;
}

gc_status gc_render(gc_ctx* ctx, const gc_scene* scene, const gc_camera* camera, const gc_opts* opts,
                    float* d_rgb, gc_stats* stats, hipStream_t stream)
{
    GC_GUARD(render_impl(ctx, scene, camera, opts, d_rgb, stats, stream));
}

static gc_status render_batch_impl(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                          const gc_opts* opts, float* const* d_rgb, const float* const* d_ref, double* C0,
                          gc_stats* st, hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    if (n_scenes < 1 || !scenes || !cameras || !d_rgb) return fail(GC_EINVAL, "need n_scenes >= 1 and non-null arrays");
    if (d_ref && !C0) return fail(GC_EINVAL, "C0 must be non-null when d_ref is given");
    OptsDev o;
    gc_status r;
    if ((r = make_opts(opts, &o)) != GC_OK) return r;
    if (opts->prec != GC_F32) return fail(GC_EUNSUPPORTED, "gc_render_batch runs the FP32 pipeline (prec = GC_F32)");
    std::vector<SceneDev> sd(n_scenes);
    std::vector<CamDev> cd(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        if ((r = make_scene(&scenes[i], &sd[i])) != GC_OK) return fail(r, "scene %d: %s", i, g_err.c_str());
        if (scenes[i].mirror == 1 && scenes[i].cloak == GC_CLOAK_NONE)
            return fail(GC_EUNSUPPORTED, "scene %d: flat-mirror scenes are rendered by gc_render", i);
        if ((r = make_camera(&cameras[i], &cd[i])) != GC_OK) return fail(r, "camera %d: %s", i, g_err.c_str());
        if (!d_rgb[i]) return fail(GC_EINVAL, "image pointer %d is null", i);
    }
    HIP_OK(hipSetDevice(ctx->device));
    gc_stats tmp;
    r = wf_render(ctx, n_scenes, sd.data(), cd.data(), o, d_rgb, st ? st : &tmp, stream);
    if (r != GC_OK) return r;
    if (d_ref) {
        for (int i = 0; i < n_scenes; ++i) {
            long long npix = (long long)cd[i].W * cd[i].H;
            r = gc_cross_correlate(ctx, d_rgb[i], d_ref[i], npix, 3, &C0[i], nullptr, stream);
            if (r != GC_OK) return r;
        }
    }
    return GC_OK;
}

gc_status gc_render_batch(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                          const gc_opts* opts, float* const* d_rgb, const float* const* d_ref, double* C0,
                          gc_stats* st, hipStream_t stream)
{
    GC_GUARD(render_batch_impl(ctx, n_scenes, scenes, cameras, opts, d_rgb, d_ref, C0, st, stream));
}

static gc_status render_grad_impl(gc_ctx* ctx, const gc_scene* scene, const gc_camera* camera, const gc_opts* opts,
                         const float* d_ref, int32_t loss_kind, int32_t checkpoint_every, float* d_rgb,
                         double* d_sample_dm, double* loss, double* dL_dA, double* dL_dhw, gc_stats* st,
                         hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    SceneDev s;
    CamDev c;
    OptsDev o;
    gc_status r;
    if ((r = make_scene(scene, &s)) != GC_OK) return r;
    if ((r = make_camera(camera, &c)) != GC_OK) return r;
    if ((r = make_opts(opts, &o)) != GC_OK) return r;
    if (scene->mirror == 1) return fail(GC_EUNSUPPORTED, "the flat-mirror reference does not depend on A or half_width");
    if (scene->cloak != GC_CLOAK_EQ1 || scene->fresnel || scene->backdrop != GC_BACKDROP_SKY)
        return fail(GC_EUNSUPPORTED, "the adjoint differentiates the cloak of eq. (1) with Snell faces and the sky");
    if (opts->integ != GC_RK4) return fail(GC_EUNSUPPORTED, "the adjoint differentiates the RK4 tracer (integ = GC_RK4)");
    if (!std::isfinite(scene->sky_K)) return fail(GC_EUNSUPPORTED, "sky_K = inf has no gradient");
    if (!d_ref) return fail(GC_EINVAL, "ref is null");
    if (loss_kind != GC_LOSS_C0 && loss_kind != GC_LOSS_NCC) return fail(GC_EINVAL, "unknown loss_kind %d", loss_kind);
    if (checkpoint_every < 1 || checkpoint_every > kAdjMaxC)
        return fail(GC_EINVAL, "checkpoint_every must be in [1, %d]", kAdjMaxC);
    HIP_OK(hipSetDevice(ctx->device));
    const long long npix = (long long)c.W * c.H, n = npix * c.spp;
    if ((r = adj_reserve(ctx, n, npix)) != GC_OK) return r;
    float* img = d_rgb ? d_rgb : ctx->adj.img;
    double* sgrad = d_sample_dm ? d_sample_dm : ctx->adj.sgrad;
    double out[3];
    if (opts->prec == GC_F64)
        r = adj_run<double>(ctx, s, c, o, checkpoint_every, d_ref, loss_kind, img, sgrad, out, st, stream);
    else
        r = adj_run<float>(ctx, s, c, o, checkpoint_every, d_ref, loss_kind, img, sgrad, out, st, stream);
    if (r != GC_OK) return r;
    if (loss) *loss = out[0];
    if (dL_dA) *dL_dA = out[1];
    if (dL_dhw) *dL_dhw = out[2];
    return GC_OK;
}

gc_status gc_render_grad(gc_ctx* ctx, const gc_scene* scene, const gc_camera* camera, const gc_opts* opts,
                         const float* d_ref, int32_t loss_kind, int32_t checkpoint_every, float* d_rgb,
                         double* d_sample_dm, double* loss, double* dL_dA, double* dL_dhw, gc_stats* st,
                         hipStream_t stream)
{
    GC_GUARD(render_grad_impl(ctx, scene, camera, opts, d_ref, loss_kind, checkpoint_every, d_rgb, d_sample_dm, loss, dL_dA, dL_dhw, st, stream));
}

static gc_status cross_correlate_impl(gc_ctx* ctx, const float* d_img, const float* d_ref, int64_t npix, int32_t nch,
                             double* C0, double* ncc, hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    if (!d_img || !d_ref || !C0) return fail(GC_EINVAL, "img, ref and C0 must be non-null");
    if (npix < 1 || nch < 1 || nch > kCCMaxCh) return fail(GC_EINVAL, "need npix >= 1 and 1 <= nch <= %d", kCCMaxCh);
    HIP_OK(hipSetDevice(ctx->device));
    long long nb = (npix + 255) / 256;
    if (nb > kCCBlocks) nb = kCCBlocks;
    hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nb), dim3(256), 0, stream, d_img, d_ref, (long long)npix,
                       (long long)npix, (long long)npix, nch, ctx->d_part);
    hipLaunchKernelGGL(k_cc_final, dim3(1), dim3(256), 0, stream, ctx->d_part, (int)nb, (long long)npix, nch, d_img,
                       d_ref, ctx->d_ccout);
    HIP_OK(hipGetLastError());
    double h[4];
    HIP_OK(hipMemcpyAsync(h, ctx->d_ccout, sizeof h, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (!(h[2] > 0)) return fail(GC_EINVAL, "reference image is constant: eq. (15) is undefined");
    *C0 = h[0];
    if (ncc) *ncc = h[1];
    return GC_OK;
}

gc_status gc_cross_correlate(gc_ctx* ctx, const float* d_img, const float* d_ref, int64_t npix, int32_t nch,
                             double* C0, double* ncc, hipStream_t stream)
{
    GC_GUARD(cross_correlate_impl(ctx, d_img, d_ref, npix, nch, C0, ncc, stream));
}

static gc_status cross_correlate_noalloc_impl(gc_ctx* ctx, const float* d_img, const float* d_ref, int64_t npix,
                                              int32_t nch, double* d_out, hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    if (!d_img || !d_ref || !d_out) return fail(GC_EINVAL, "img, ref and out must be non-null");
    if (npix < 1) return fail(GC_EINVAL, "need npix >= 1");
    if (nch < 1 || nch > kCCMaxCh)
        return fail(GC_EINVAL, "nch = %d: the scratch holds the moments of at most %d channels", nch, kCCMaxCh);
    if (!ctx->d_scratch) return fail(GC_EDEVICE, "scratch address not set up");
    HIP_OK(hipSetDevice(ctx->device));
    // the blocks stride over the pixels, so any npix fits the kCCBlocks
    // partials; k_cc_moments writes every partial k_cc_final reads, so
    // nothing needs clearing
    const long long nb = std::min<long long>((npix + 255) / 256, kCCBlocks);
    hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nb), dim3(256), 0, stream, d_img, d_ref, (long long)npix,
                       (long long)npix, (long long)npix, nch, ctx->d_scratch);
    hipLaunchKernelGGL(k_cc_final, dim3(1), dim3(256), 0, stream, (const double*)ctx->d_scratch, (int)nb,
                       (long long)npix, nch, d_img, d_ref, d_out);
    HIP_OK(hipGetLastError());
    return GC_OK;
}

gc_status gc_cross_correlate_noalloc(gc_ctx* ctx, const float* d_img, const float* d_ref, int64_t npix, int32_t nch,
                                     double* d_out, hipStream_t stream)
{
    GC_GUARD(cross_correlate_noalloc_impl(ctx, d_img, d_ref, npix, nch, d_out, stream));
}

static gc_status cross_correlate_map_impl(gc_ctx* ctx, const float* d_img, const float* d_ref, int32_t height,
                                         int32_t width, int64_t pitch, int32_t nch, int32_t rx, int32_t ry,
                                         double* d_map, double* peak, int32_t* peak_dx, int32_t* peak_dy,
                                         hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    if (!d_img || !d_ref || !d_map) return fail(GC_EINVAL, "img, ref and map must be non-null");
    if (height < 1 || width < 1 || pitch < width) return fail(GC_EINVAL, "need height, width >= 1 and pitch >= width");
    if (nch < 1 || nch > kCCMaxCh) return fail(GC_EINVAL, "need 1 <= nch <= %d", kCCMaxCh);
    if (rx < 0 || ry < 0 || rx >= width || ry >= height)
        return fail(GC_EINVAL, "need 0 <= rx < width and 0 <= ry < height");
    const int ndx = 2 * rx + 1, ndy = 2 * ry + 1;
    if (ndx > kCCMapMaxDx) return fail(GC_EUNSUPPORTED, "rx = %d: at most %d shifts along a row", rx, kCCMapMaxDx);
    const size_t lds = std::max<size_t>(sizeof(double) * (size_t)(2 * width + 2 * rx) * nch, sizeof(double) * 256);
    if (lds > (size_t)kCCMapLds)
        return fail(GC_EUNSUPPORTED, "(2 width + 2 rx) nch = %lld exceeds the %d doubles of LDS for two rows",
                    (long long)(2 * width + 2 * rx) * nch, kCCMapLds / 8);
    HIP_OK(hipSetDevice(ctx->device));
    // eq. (14): means and sum f'^2 of the window
    const long long npix = (long long)height * width;
    const long long nb = std::min<long long>((npix + 255) / 256, kCCBlocks);
    hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nb), dim3(256), 0, stream, d_img, d_ref, npix, (long long)width,
                       (long long)pitch, nch, ctx->d_part);
    hipLaunchKernelGGL(k_cc_final, dim3(1), dim3(256), 0, stream, ctx->d_part, (int)nb, npix, nch, d_img, d_ref,
                       ctx->d_ccout);
    // rows in chunks so that the grid holds about 4 blocks per CU
    const int n_chunks = (int)std::max<long long>(1, std::min<long long>(height, (4LL * ctx->n_cu + ndy - 1) / ndy));
    const int rpc = (height + n_chunks - 1) / n_chunks;
    const size_t need = sizeof(double) * (size_t)ndy * n_chunks * ndx;
    gc_status r;
    if ((r = grow((void**)&ctx->d_map_part, &ctx->map_part_bytes, need, "correlation map partials")) != GC_OK) return r;
    hipLaunchKernelGGL(k_cc_map_rows, dim3((unsigned)ndy, (unsigned)n_chunks), dim3(256), lds, stream, d_img, d_ref,
                       height, width, (long long)pitch, nch, rx, ry, rpc, (const double*)ctx->d_ccout,
                       ctx->d_map_part);
    hipLaunchKernelGGL(k_cc_map_final, dim3((unsigned)((ndx * ndy + 255) / 256)), dim3(256), 0, stream,
                       (const double*)ctx->d_map_part, ndx, ndy, n_chunks, (const double*)ctx->d_ccout, d_map);
    hipLaunchKernelGGL(k_cc_map_peak, dim3(1), dim3(256), 0, stream, (const double*)d_map, ndx, ndy, rx, ry,
                       ctx->d_peak);
    HIP_OK(hipGetLastError());
    double h[kCCOut];
    HIP_OK(hipMemcpyAsync(h, ctx->d_ccout, sizeof h, hipMemcpyDeviceToHost, stream));
    double pk[3];
    HIP_OK(hipMemcpyAsync(pk, ctx->d_peak, sizeof pk, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (!(h[2] > 0)) return fail(GC_EINVAL, "reference window is constant: eq. (15) is undefined");
    if (peak) *peak = pk[0];
    if (peak_dx) *peak_dx = (int32_t)pk[1];
    if (peak_dy) *peak_dy = (int32_t)pk[2];
    return GC_OK;
}

gc_status gc_cross_correlate_map(gc_ctx* ctx, const float* d_img, const float* d_ref, int32_t height, int32_t width,
                                 int64_t pitch, int32_t nch, int32_t rx, int32_t ry, double* d_map, double* peak,
                                 int32_t* peak_dx, int32_t* peak_dy, hipStream_t stream)
{
    GC_GUARD(cross_correlate_map_impl(ctx, d_img, d_ref, height, width, pitch, nch, rx, ry, d_map, peak, peak_dx,
                                      peak_dy, stream));
}

}  // extern "C"

#include "gc_autotune.hpp"
#include "gc_plan.hpp"
