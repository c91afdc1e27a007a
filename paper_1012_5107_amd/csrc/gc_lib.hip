// gc_lib.hip -- kernels and C ABI of the gfx950 grating-cloak ray tracer.
// The public interface is include/gcloak.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "gcloak.h"
#include "gc_lane64.hpp"
#include "gc_lane32.hpp"

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

__device__ __forceinline__ void add_counters(DevCounters* c, unsigned long long rays, unsigned long long steps,
                                             unsigned long long rej, unsigned long long ev,
                                             unsigned long long fb, unsigned long long failed)
{
    rays = wave_sum(rays);
    steps = wave_sum(steps);
    rej = wave_sum(rej);
    ev = wave_sum(ev);
    fb = wave_sum(fb);
    failed = wave_sum(failed);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&c->rays, rays);
        atomicAdd(&c->steps, steps);
        atomicAdd(&c->rejected, rej);
        atomicAdd(&c->events, ev);
        atomicAdd(&c->fallbacks, fb);
        atomicAdd(&c->failed, failed);
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
            double d[3], oo[3], od[3];
            camera_dir(cam, i, j, smp, d);
            LaneCount lc = {0, 0, 0, 0};
            double mc = 1.0;
            int st = trace_ray64(s, o, cam.eye, d, oo, od, lc, &mc);
            c_rays++;
            c_steps += lc.steps;
            c_rej += lc.rejected;
            c_ev += lc.events;
            if (st != RS_OK) { c_fail++; continue; }
            double c[3];
            sky_rgb<double>(s.K, od, c);
            for (int a = 0; a < 3; ++a) acc[a] += c[a];
        }
        for (int a = 0; a < 3; ++a) rgb[3 * pix + a] = (float)(acc[a] / cam.spp);
    }
    add_counters(cnt, c_rays, c_steps, c_rej, c_ev, 0, c_fail);
}

// Reference image: flat mirror y = 0 in air.  A downward ray leaves with
// d_y negated; an upward one sees the sky directly.
__global__ void __launch_bounds__(256) k_render_flat(CamDev cam, double K, float* rgb, DevCounters* cnt)
{
    long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long npx = (long long)cam.W * cam.H;
    unsigned long long c_rays = 0, c_ev = 0;
    if (pix < npx) {
        int i = (int)(pix % cam.W), j = (int)(pix / cam.W);
        double acc[3] = {0, 0, 0};
        for (int smp = 0; smp < cam.spp; ++smp) {
            double d[3], c[3];
            camera_dir(cam, i, j, smp, d);
            if (d[1] < 0.0 && cam.eye[1] > 0.0) { d[1] = -d[1]; c_ev++; }
            sky_rgb<double>(K, d, c);
            for (int a = 0; a < 3; ++a) acc[a] += c[a];
        }
        c_rays = cam.spp;
        for (int a = 0; a < 3; ++a) rgb[3 * pix + a] = (float)(acc[a] / cam.spp);
    }
    add_counters(cnt, c_rays, 0, 0, c_ev, 0, 0);
}

// ---------------------------------------------------------------------------
// FP32 kernels (one pixel per lane; the in-cloak loop runs in FP32).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_trace_rays32(SceneDev s, OptsDev o, long long n, const double* org,
                                                      const double* dir, double* out_org, double* out_dir,
                                                      int* status, long long* steps, int* events,
                                                      DevCounters* cnt)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_rays = 0, c_fb = 0;
    if (i < n) {
        double r[3] = {org[3 * i], org[3 * i + 1], org[3 * i + 2]};
        double d[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
        double oo[3] = {0, 0, 0}, od[3] = {0, 0, 0};
        LaneCount lc = {0, 0, 0, 0};
        double mc = 1.0;
        int st = trace_ray32(s, o, r, d, oo, od, lc, &mc);
        if (out_org) for (int a = 0; a < 3; ++a) out_org[3 * i + a] = oo[a];
        for (int a = 0; a < 3; ++a) out_dir[3 * i + a] = od[a];
        if (status) status[i] = st;
        if (steps) steps[i] = lc.steps;
        if (events) events[i] = lc.events;
        c_rays = 1;
        c_steps = lc.steps;
        c_rej = lc.rejected;
        c_ev = lc.events;
        c_fb = lc.fallbacks;
        c_fail = st != RS_OK;
    }
    add_counters(cnt, c_rays, c_steps, c_rej, c_ev, c_fb, c_fail);
}

__global__ void __launch_bounds__(256) k_render32(SceneDev s, CamDev cam, OptsDev o, float* rgb,
                                                  DevCounters* cnt)
{
    long long pix = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long npx = (long long)cam.W * cam.H;
    unsigned long long c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_rays = 0, c_fb = 0;
    if (pix < npx) {
        int i = (int)(pix % cam.W), j = (int)(pix / cam.W);
        float acc[3] = {0, 0, 0};
        for (int smp = 0; smp < cam.spp; ++smp) {
            double d[3], oo[3], od[3];
            camera_dir(cam, i, j, smp, d);
            LaneCount lc = {0, 0, 0, 0};
            double mc = 1.0;
            int st = trace_ray32(s, o, cam.eye, d, oo, od, lc, &mc);
            c_rays++;
            c_steps += lc.steps;
            c_rej += lc.rejected;
            c_ev += lc.events;
            c_fb += lc.fallbacks;
            if (st != RS_OK) { c_fail++; continue; }
            float df[3] = {(float)od[0], (float)od[1], (float)od[2]};
            float c[3];
            sky_rgb<float>((float)s.K, df, c);
            for (int a = 0; a < 3; ++a) acc[a] += c[a];
        }
        for (int a = 0; a < 3; ++a) rgb[3 * pix + a] = acc[a] / (float)cam.spp;
    }
    add_counters(cnt, c_rays, c_steps, c_rej, c_ev, c_fb, c_fail);
}

// ---------------------------------------------------------------------------
// Cross-correlation, eqs. (14)-(15): one pass of FP64 moments per channel
// (sum f, sum g, sum f^2, sum g^2, sum f g), then centred sums from them.
// Partials: per block, 5 x nch doubles; a single block folds them.
// ---------------------------------------------------------------------------
constexpr int kCCMaxCh = 4;
constexpr int kCCBlocks = 1024;

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_cc_moments(const float* __restrict__ g, const float* __restrict__ f,
                                                    long long npix, int nch, double* __restrict__ part)
{
    // moments of the values shifted by the first pixel's (keeps the
    // centred sums free of cancellation)
    double m[5][kCCMaxCh];
    double f0[kCCMaxCh], g0[kCCMaxCh];
#pragma unroll
    for (int c = 0; c < kCCMaxCh; ++c) {
        f0[c] = c < nch ? (double)f[c] : 0.0;
        g0[c] = c < nch ? (double)g[c] : 0.0;
#pragma unroll
        for (int q = 0; q < 5; ++q) m[q][c] = 0.0;
    }
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
#pragma unroll
        for (int c = 0; c < kCCMaxCh; ++c) {
            if (c < nch) {
                double a = (double)f[p * nch + c] - f0[c], b = (double)g[p * nch + c] - g0[c];
                m[0][c] += a;
                m[1][c] += b;
                m[2][c] += a * a;
                m[3][c] += b * b;
                m[4][c] += a * b;
            }
        }
    }
    __shared__ double red[4][5 * kCCMaxCh];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int c = 0; c < kCCMaxCh; ++c) {
            double v = wave_sum_d(m[q][c]);
            if (lane == 0) red[wave][q * kCCMaxCh + c] = v;
        }
    __syncthreads();
    if (threadIdx.x < 5 * kCCMaxCh) {
        double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        part[(long long)blockIdx.x * 5 * kCCMaxCh + threadIdx.x] = v;
    }
}

__global__ void __launch_bounds__(256) k_cc_final(const double* __restrict__ part, int nblocks, long long npix,
                                                  int nch, double* __restrict__ out)
{
    __shared__ double tot[5 * kCCMaxCh];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ double red[4][5 * kCCMaxCh];
    for (int q = 0; q < 5 * kCCMaxCh; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += part[(long long)b * 5 * kCCMaxCh + q];
        v = wave_sum_d(v);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5 * kCCMaxCh)
        tot[threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        double sfg = 0.0, sff = 0.0, sgg = 0.0;
        double N = (double)npix;
        for (int c = 0; c < nch; ++c) {
            double mf = tot[0 * kCCMaxCh + c] / N, mg = tot[1 * kCCMaxCh + c] / N;
            sff += tot[2 * kCCMaxCh + c] - N * mf * mf;
            sgg += tot[3 * kCCMaxCh + c] - N * mg * mg;
            sfg += tot[4 * kCCMaxCh + c] - N * mf * mg;
        }
        out[0] = sfg / sff;
        out[1] = sfg / sqrt(sff * sgg);
        out[2] = sff;
        out[3] = sgg;
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct gc_ctx {
    int device;
    DevCounters* d_cnt;
    double* d_part;
    double* d_ccout;
};

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
    if (sc->cloak != 0 && sc->cloak != 1) return fail(GC_EINVAL, "cloak must be 0 or 1");
    if (sc->mirror != 0 && sc->mirror != 1) return fail(GC_EINVAL, "mirror must be 0 or 1");
    if (sc->mirror == 1 && sc->cloak == 1) return fail(GC_EUNSUPPORTED, "the flat mirror is only provided without cloak");
    if (std::isnan(sc->sky_K) || !(sc->sky_K > 0)) return fail(GC_EINVAL, "sky_K must be > 0");
    s->L = sc->Lambda;
    s->A = sc->A;
    s->hw = sc->half_width;
    s->ytop = sc->y_top;
    s->K = sc->sky_K;
    s->k = k;
    s->e = sc->A * k;
    s->invL = 1.0 / sc->Lambda;
    s->ybp = sc->A > 0 ? (1.0 + std::log(s->e)) / k : -HUGE_VAL;
    s->S_hw = (sc->mirror == 0 && std::isfinite(sc->half_width)) ? host_kepler_height(sc->A, sc->Lambda, sc->half_width) : 0.0;
    s->cloak = sc->cloak;
    s->mirror = sc->mirror;
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
    double r[3] = {-f[2], 0.0, f[0]};   // f x (0, 1, 0)
    double rn = std::sqrt(r[0] * r[0] + r[2] * r[2]);
    if (!(rn > 1e-12)) return fail(GC_EINVAL, "camera looks straight along y: right vector undefined");
    r[0] /= rn;
    r[2] /= rn;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    for (int a = 0; a < 3; ++a) {
        d->eye[a] = c->eye[a];
        d->f[a] = f[a];
        d->r[a] = r[a];
        d->u[a] = u[a];
    }
    d->t = std::tan(0.5 * c->fov_y_deg * M_PI / 180.0);
    d->aspect = (double)c->width / (double)c->height;
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
    return GC_OK;
}

static gc_status read_counters(gc_ctx* ctx, gc_stats* st, hipStream_t stream)
{
    DevCounters h;
    HIP_OK(hipMemcpyAsync(&h, ctx->d_cnt, sizeof h, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    st->rays = (int64_t)h.rays;
    st->accepted_steps = (int64_t)h.steps;
    st->rejected_steps = (int64_t)h.rejected;
    st->events = (int64_t)h.events;
    st->fallbacks = (int64_t)h.fallbacks;
    st->failed = (int64_t)h.failed;
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
    o->max_steps = 10000000;
}

gc_status gc_create(gc_ctx** out, int hip_device)
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
    if (hipMalloc(&c->d_cnt, sizeof(DevCounters)) != hipSuccess ||
        hipMalloc(&c->d_part, sizeof(double) * kCCBlocks * 5 * kCCMaxCh) != hipSuccess ||
        hipMalloc(&c->d_ccout, sizeof(double) * 4) != hipSuccess) {
        gc_destroy(c);
        return fail(GC_ENOMEM, "device scratch allocation failed");
    }
    *out = c;
    return GC_OK;
}

void gc_destroy(gc_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->d_cnt) (void)hipFree(c->d_cnt);
    if (c->d_part) (void)hipFree(c->d_part);
    if (c->d_ccout) (void)hipFree(c->d_ccout);
    delete c;
}

gc_status gc_trace_rays(gc_ctx* ctx, const gc_scene* scene, const gc_opts* opts, int64_t n, const double* d_org,
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
        hipLaunchKernelGGL(k_trace_rays32, dim3((unsigned)nb), dim3(256), 0, stream, s, o, (long long)n, d_org,
                           d_dir, d_out_org, d_out_dir, (int*)d_status, (long long*)d_steps, (int*)d_events,
                           ctx->d_cnt);
    HIP_OK(hipGetLastError());
    return GC_OK;
}

gc_status gc_render(gc_ctx* ctx, const gc_scene* scene, const gc_camera* camera, const gc_opts* opts,
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
    if (scene->mirror == 1)
        hipLaunchKernelGGL(k_render_flat, dim3(nb), dim3(256), 0, stream, c, s.K, d_rgb, ctx->d_cnt);
    else if (opts->prec == GC_F64)
        hipLaunchKernelGGL(k_render64, dim3(nb), dim3(256), 0, stream, s, c, o, d_rgb, ctx->d_cnt);
    else
        hipLaunchKernelGGL(k_render32, dim3(nb), dim3(256), 0, stream, s, c, o, d_rgb, ctx->d_cnt);
    HIP_OK(hipGetLastError());
    if (stats) return read_counters(ctx, stats, stream);
    return GC_OK;
}

gc_status gc_cross_correlate(gc_ctx* ctx, const float* d_img, const float* d_ref, int64_t npix, int32_t nch,
                             double* C0, double* ncc, hipStream_t stream)
{
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    if (!d_img || !d_ref || !C0) return fail(GC_EINVAL, "img, ref and C0 must be non-null");
    if (npix < 1 || nch < 1 || nch > kCCMaxCh) return fail(GC_EINVAL, "need npix >= 1 and 1 <= nch <= %d", kCCMaxCh);
    HIP_OK(hipSetDevice(ctx->device));
    long long nb = (npix + 255) / 256;
    if (nb > kCCBlocks) nb = kCCBlocks;
    hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nb), dim3(256), 0, stream, d_img, d_ref, (long long)npix, nch,
                       ctx->d_part);
    hipLaunchKernelGGL(k_cc_final, dim3(1), dim3(256), 0, stream, ctx->d_part, (int)nb, (long long)npix, nch,
                       ctx->d_ccout);
    HIP_OK(hipGetLastError());
    double h[4];
    HIP_OK(hipMemcpyAsync(h, ctx->d_ccout, sizeof h, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (!(h[2] > 0)) return fail(GC_EINVAL, "reference image is constant: eq. (15) is undefined");
    *C0 = h[0];
    if (ncc) *ncc = h[1];
    return GC_OK;
}

}  // extern "C"
