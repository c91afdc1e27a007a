// gc_autotune.hpp -- host side of the FP32 pipeline's autotuner (included at
// the end of gc_lib.hip, after the public entry points it calls).
//
// The tuner times the whole workload for each candidate step control
// (tolerance and step cap), checks it against the FP64 path on calibration
// cameras (exit directions with an FP64 conditioning screen, and the
// zero-shift correlation of eq. (15)), keeps the fastest that passes, then
// times a fixed set of scheduling settings.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

namespace gc {

// The rays of a camera (one per pixel and sample, pixel-major), from its eye.
__global__ void __launch_bounds__(256) k_camera_rays(CamDev c, long long n, double* org, double* dir)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const long long pix = q / c.spp;
    const int smp = (int)(q - pix * c.spp);
    const int i = (int)(pix % c.W), j = (int)(pix / c.W);
    double p[3];
    camera_dir(c, i, j, smp, p);
    for (int k = 0; k < 3; ++k) {
        org[3 * q + k] = c.eye[k];
        dir[3 * q + k] = p[k];
    }
}

}  // namespace gc

namespace {

// device allocation released at scope exit
struct DevMem {
    void* p = nullptr;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem()
    {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t bytes) { return hipMalloc(&p, bytes) == hipSuccess; }
    template <class T> T* as() const { return (T*)p; }
};

gc_camera scaled_camera(const gc_camera& c, int s)
{
    gc_camera r = c;
    r.width = std::max(1, c.width / s);
    r.height = std::max(1, c.height / s);
    return r;
}

// angle between two directions, accurate for tiny angles
double angle3(const double* a, const double* b)
{
    const double na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double nb = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    double dm = 0.0, dp = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double u = a[k] / na, v = b[k] / nb;
        dm += (u - v) * (u - v);
        dp += (u + v) * (u + v);
    }
    return 2.0 * std::atan2(std::sqrt(dm), std::sqrt(dp));
}

// Host copy of a trace of the calibration rays.
struct TraceHost {
    std::vector<double> dir;
    std::vector<int32_t> status, events;
};

gc_status trace_to_host(gc_ctx* ctx, const gc_scene* sc, const gc_opts* o, long long n, const double* d_org,
                        const double* d_dir, DevMem& out_dir, DevMem& st, DevMem& ev, TraceHost& h,
                        hipStream_t stream)
{
    gc_status r = gc_trace_rays(ctx, sc, o, n, d_org, d_dir, nullptr, out_dir.as<double>(), st.as<int32_t>(),
                                nullptr, ev.as<int32_t>(), stream);
    if (r != GC_OK) return r;
    h.dir.resize(3 * n);
    h.status.resize(n);
    h.events.resize(n);
    HIP_OK(hipMemcpyAsync(h.dir.data(), out_dir.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(h.status.data(), st.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(h.events.data(), ev.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    return GC_OK;
}

// Per scene: calibration rays, the FP64 reference of the direction check and
// the FP64 correlation of the correlation check.
struct Calib {
    long long n = 0;
    DevMem org, dir;
    TraceHost ref;
    std::vector<char> well;       // compared (FP64 well-conditioned, status OK)
    gc_camera cc_cam;
    long long cc_npix = 0;
    DevMem flat;                  // flat-mirror image at the correlation size
    double c0_ref = 0.0;
};

}  // namespace

extern "C" {

void gc_default_autotune_opts(gc_autotune_opts* at)
{
    if (!at) return;
    std::memset(at, 0, sizeof *at);
    at->dir_scale = 4;
    at->cc_scale = 1;
    at->dir_tol = 1e-4;
    at->cc_tol = 1e-4;
    at->max_changed = 0.01;
    // a converged reference: the C0 of a high-amplitude scene moves by up
    // to ~1e-4 between FP64 solves at rtol 1e-8 and 1e-10 (a few dozen
    // samples trapped near the crests flip between escaping and the step
    // cap), and by ~5e-6 between 1e-10 solves at step caps 0.02 and 0.005
    at->ref_rtol = 1e-10;
    at->reps = 2;
    at->tune_sched = 1;
}

static gc_status autotune_impl(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                      const gc_opts* opts, const gc_autotune_opts* atp, gc_opts* opts_out,
                      gc_autotune_report* report, hipStream_t stream)
{
    using namespace gc;
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    if (n_scenes < 1 || !scenes || !cameras || !opts || !opts_out)
        return fail(GC_EINVAL, "need n_scenes >= 1 and non-null scenes, cameras, opts and opts_out");
    gc_autotune_opts at;
    if (atp) at = *atp; else gc_default_autotune_opts(&at);
    if (at.dir_scale < 1 || at.cc_scale < 1 || at.reps < 1 || !(at.dir_tol > 0) || !(at.cc_tol > 0) ||
        !(at.max_changed >= 0) || !(at.ref_rtol > 0))
        return fail(GC_EINVAL, "autotune options out of range");
    if (opts->prec != GC_F32) return fail(GC_EUNSUPPORTED, "the autotuner tunes the FP32 pipeline (prec = GC_F32)");
    OptsDev od;
    gc_status r = make_opts(opts, &od);
    if (r != GC_OK) return r;
    std::vector<SceneDev> sd(n_scenes);
    std::vector<CamDev> cd(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        if ((r = make_scene(&scenes[i], &sd[i])) != GC_OK) return fail(r, "scene %d: %s", i, g_err.c_str());
        if (scenes[i].mirror == 1) return fail(GC_EINVAL, "scene %d is the flat mirror: nothing to tune", i);
        if ((r = make_camera(&cameras[i], &cd[i])) != GC_OK) return fail(r, "camera %d: %s", i, g_err.c_str());
    }
    HIP_OK(hipSetDevice(ctx->device));
    gc_autotune_report rep;
    std::memset(&rep, 0, sizeof rep);
    rep.chosen = -1;
    *opts_out = *opts;

    gc_opts ref = *opts;
    ref.prec = GC_F64;
    ref.rtol = ref.atol = at.ref_rtol;

    // ---- calibration: FP64 references -----------------------------------
    std::vector<Calib> cal(n_scenes);
    long long max_cal = 0, max_ccpix = 0;
    for (int i = 0; i < n_scenes; ++i) {
        const gc_camera dc = scaled_camera(cameras[i], at.dir_scale);
        cal[i].n = (long long)dc.width * dc.height * dc.spp;
        cal[i].cc_cam = scaled_camera(cameras[i], at.cc_scale);
        cal[i].cc_npix = (long long)cal[i].cc_cam.width * cal[i].cc_cam.height;
        max_cal = std::max(max_cal, cal[i].n);
        max_ccpix = std::max(max_ccpix, cal[i].cc_npix);
    }
    DevMem pert, out_dir, st_buf, ev_buf, img64, img32;
    static_assert(GC_AUTOTUNE_MAX_CAND >= 45, "room for every candidate");
    if (!pert.alloc(sizeof(double) * 3 * max_cal) || !out_dir.alloc(sizeof(double) * 3 * max_cal) ||
        !st_buf.alloc(sizeof(int32_t) * max_cal) || !ev_buf.alloc(sizeof(int32_t) * max_cal) ||
        !img64.alloc(sizeof(float) * 3 * max_ccpix) || !img32.alloc(sizeof(float) * 3 * max_ccpix))
        return fail(GC_ENOMEM, "autotune calibration buffers: allocation failed");
    static const double kPert[2][3] = {{0.3, -0.7, 0.2}, {-0.5, 0.1, 0.8}};
    for (int i = 0; i < n_scenes; ++i) {
        Calib& c = cal[i];
        const long long n = c.n;
        if (!c.org.alloc(sizeof(double) * 3 * n) || !c.dir.alloc(sizeof(double) * 3 * n) ||
            !c.flat.alloc(sizeof(float) * 3 * c.cc_npix))
            return fail(GC_ENOMEM, "autotune calibration rays: allocation failed");
        CamDev cam;
        const gc_camera dc = scaled_camera(cameras[i], at.dir_scale);
        if ((r = make_camera(&dc, &cam)) != GC_OK) return r;
        hipLaunchKernelGGL(k_camera_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, cam, n,
                           c.org.as<double>(), c.dir.as<double>());
        HIP_OK(hipGetLastError());
        if ((r = trace_to_host(ctx, &scenes[i], &ref, n, c.org.as<double>(), c.dir.as<double>(), out_dir, st_buf,
                               ev_buf, c.ref, stream)) != GC_OK)
            return r;
        // conditioning: the FP64 exit under two perturbations of size 1e-6
        std::vector<double> d0(3 * n), dp(3 * n), kappa(n, 0.0);
        HIP_OK(hipMemcpyAsync(d0.data(), c.dir.p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        for (const auto& v : kPert) {
            const double nv = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            for (long long q = 0; q < n; ++q)
                for (int k = 0; k < 3; ++k) dp[3 * q + k] = d0[3 * q + k] + 1e-6 * v[k] / nv;
            HIP_OK(hipMemcpyAsync(pert.p, dp.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, stream));
            TraceHost tp;
            if ((r = trace_to_host(ctx, &scenes[i], &ref, n, c.org.as<double>(), pert.as<double>(), out_dir, st_buf,
                                   ev_buf, tp, stream)) != GC_OK)
                return r;
            for (long long q = 0; q < n; ++q) {
                double k = angle3(&tp.dir[3 * q], &c.ref.dir[3 * q]);
                if (tp.status[q] != c.ref.status[q] || tp.events[q] != c.ref.events[q] || !std::isfinite(k))
                    k = HUGE_VAL;
                kappa[q] = std::max(kappa[q], k);
            }
        }
        c.well.assign(n, 0);
        for (long long q = 0; q < n; ++q) {
            c.well[q] = c.ref.status[q] == GC_RAY_OK && kappa[q] <= at.dir_tol;
            rep.cal_rays++;
            rep.ill_rays += c.ref.status[q] == GC_RAY_OK && !(kappa[q] <= at.dir_tol);
        }
        // correlation reference: FP64 image and flat mirror at the correlation size
        gc_scene flat = scenes[i];
        flat.cloak = 0;
        flat.mirror = 1;
        if ((r = gc_render(ctx, &flat, &c.cc_cam, &ref, c.flat.as<float>(), nullptr, stream)) != GC_OK) return r;
        if ((r = gc_render(ctx, &scenes[i], &c.cc_cam, &ref, img64.as<float>(), nullptr, stream)) != GC_OK) return r;
        if ((r = gc_cross_correlate(ctx, img64.as<float>(), c.flat.as<float>(), c.cc_npix, 3, &c.c0_ref, nullptr,
                                    stream)) != GC_OK)
            return r;
    }

    // ---- the whole workload's images (for the timings) ---------------------
    std::vector<DevMem> imgs(n_scenes);
    std::vector<float*> d_rgb(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        if (!imgs[i].alloc(sizeof(float) * 3 * (size_t)cameras[i].width * cameras[i].height))
            return fail(GC_ENOMEM, "autotune images: allocation failed");
        d_rgb[i] = imgs[i].as<float>();
    }
    auto time_workload = [&](const gc_opts& o, double* ms, int64_t* steps) -> gc_status {
        OptsDev ox;
        gc_status e = make_opts(&o, &ox);
        if (e != GC_OK) return e;
        double best = HUGE_VAL;
        for (int k = 0; k < at.reps; ++k) {
            gc_stats st;
            e = wf_render(ctx, n_scenes, sd.data(), cd.data(), ox, d_rgb.data(), &st, stream);
            if (e != GC_OK) return e;
            best = std::min(best, st.total_ms);
            if (steps) *steps = st.accepted_steps;
        }
        *ms = best;
        return GC_OK;
    };

    // ---- step-control candidates --------------------------------------------
    // around the given tolerance, one looser: the FP32 truncation error of
    // the exit directions grows like rtol^1.5, so a factor of 3 can still
    // pass and saves steps on every ray.  The FP64 hand-over threshold is
    // the third lever: near the crests of a high-amplitude grating FP32
    // cannot resolve W (the Halley residual W - Z e^-W loses its leading
    // digits as |1 + W| shrinks), so a larger threshold hands more steps to
    // FP64.  The given threshold is tried first, then those of 0.1 and 0.3
    // that exceed it, in increasing order; the search stops after the first
    // level at which a candidate passes.
    static const double kTolFactor[] = {3.0, 1.0, 1.0 / 3.0};
    static const double kCapFactor[] = {1.0, 2.5, 5.0, 10.0, 25.0};
    const double kWfb[3] = {opts->w_fallback, 0.1, 0.3};
    const bool dp = opts->integ == GC_DOPRI5;
    const int n_tol = dp ? 3 : 1, n_cap = dp ? 5 : 1;
    double best_ms = HUGE_VAL;
    for (int wi = 0; wi < 3; ++wi) {
        if (wi > 0 && rep.chosen >= 0) break;
        if (wi > 0 && !(kWfb[wi] > opts->w_fallback)) continue;
        for (int ti = 0; ti < n_tol; ++ti)
        for (int ci = 0; ci < n_cap; ++ci) {
            gc_autotune_cand& cand = rep.cand[rep.n_cand++];
            gc_opts o = *opts;
            o.rtol = opts->rtol * kTolFactor[ti];
            o.atol = opts->atol * kTolFactor[ti];
            o.h_max = opts->h_max * kCapFactor[ci];
            o.w_fallback = kWfb[wi];
            cand.rtol = o.rtol;
            cand.h_max = o.h_max;
            cand.w_fallback = o.w_fallback;
            if ((r = time_workload(o, &cand.ms, &cand.steps)) != GC_OK) return r;
            double p99 = 0.0, mx = 0.0, chg = 0.0, cce = 0.0;
            for (int i = 0; i < n_scenes; ++i) {
                Calib& c = cal[i];
                TraceHost t;
                if ((r = trace_to_host(ctx, &scenes[i], &o, c.n, c.org.as<double>(), c.dir.as<double>(), out_dir,
                                       st_buf, ev_buf, t, stream)) != GC_OK)
                    return r;
                long long changed = 0;
                std::vector<double> err;
                err.reserve(c.n);
                for (long long q = 0; q < c.n; ++q) {
                    if (t.status[q] != c.ref.status[q] || t.events[q] != c.ref.events[q]) { ++changed; continue; }
                    if (c.well[q]) err.push_back(angle3(&t.dir[3 * q], &c.ref.dir[3 * q]));
                }
                chg = std::max(chg, (double)changed / (double)std::max(1ll, c.n));
                if (!err.empty()) {
                    const size_t k99 = (size_t)std::floor(0.99 * (double)(err.size() - 1));
                    std::nth_element(err.begin(), err.begin() + k99, err.end());
                    p99 = std::max(p99, err[k99]);
                    mx = std::max(mx, *std::max_element(err.begin(), err.end()));
                }
                // at full size the timed render's image is the one to check
                const float* img = d_rgb[i];
                if (at.cc_scale > 1) {
                    if ((r = gc_render(ctx, &scenes[i], &c.cc_cam, &o, img32.as<float>(), nullptr, stream)) != GC_OK)
                        return r;
                    img = img32.as<float>();
                }
                double c0 = 0.0;
                if ((r = gc_cross_correlate(ctx, img, c.flat.as<float>(), c.cc_npix, 3, &c0, nullptr, stream)) !=
                    GC_OK)
                    return r;
                cce = std::max(cce, std::fabs(c0 - c.c0_ref));
            }
            cand.dir_p99 = p99;
            cand.dir_max = mx;
            cand.changed = chg;
            cand.cc_err = cce;
            cand.pass = p99 <= at.dir_tol && mx <= 30.0 * at.dir_tol && chg <= at.max_changed && cce <= at.cc_tol;
            if (cand.pass && cand.ms < best_ms) {
                best_ms = cand.ms;
                rep.chosen = rep.n_cand - 1;
                *opts_out = o;
            }
        }
    }

    if (rep.chosen < 0 && rep.n_cand > 1) {
        // no candidate meets the bounds: the fastest one that is nowhere less
        // accurate than the options as given (every measured error at most
        // theirs), which keeps the reported accuracy and saves time; its pass
        // flag stays 0.  The options as given are candidate (tol 1, cap 1) of
        // the first threshold level.
        const int base = 1 * n_cap + 0;
        const gc_autotune_cand& b = rep.cand[base];
        double best = b.ms;
        for (int i = 0; i < rep.n_cand; ++i) {
            const gc_autotune_cand& c = rep.cand[i];
            if (c.ms < best && c.dir_p99 <= b.dir_p99 && c.dir_max <= b.dir_max && c.changed <= b.changed &&
                c.cc_err <= b.cc_err) {
                best = c.ms;
                rep.chosen = i;
            }
        }
        if (rep.chosen >= 0) {
            const gc_autotune_cand& c = rep.cand[rep.chosen];
            opts_out->rtol = c.rtol;
            opts_out->atol = opts->atol * (c.rtol / opts->rtol);
            opts_out->h_max = c.h_max;
            opts_out->w_fallback = c.w_fallback;
        }
    }

    // ---- scheduling ---------------------------------------------------------
    const gc_tune entry = ctx->tune;
    // the context's scheduling on entry comes back on any early exit
    struct Restore {
        gc_ctx* c;
        gc_tune t;
        bool keep;
        ~Restore()
        {
            if (!keep) c->tune = t;
        }
    } restore{ctx, entry, false};
    rep.tune = entry;
    if ((r = time_workload(*opts_out, &rep.base_tune_ms, nullptr)) != GC_OK) return r;
    rep.tune_ms = rep.base_tune_ms;
    if (at.tune_sched) {
        // (slow_pxy, slow_wave_div, refill, waves_per_simd)
        static const double kSched[][4] = {{0.0, 0, 8, 0},  {0.25, 4, 8, 0}, {0.3, 4, 8, 0}, {0.2, 8, 8, 0},
                                           {0.0, 0, 8, 2},  {0.25, 4, 8, 2}, {0.0, 0, 16, 0}, {0.3, 2, 8, 0}};
        for (const auto& s : kSched) {
            gc_tune t;
            gc_default_tune(&t);
            t.slow_pxy = s[0];
            t.slow_wave_div = (int32_t)s[1];
            t.refill = (int32_t)s[2];
            t.waves_per_simd = (int32_t)s[3];
            t.plan_lanes = entry.plan_lanes;   // batch plans only
            ctx->tune = t;
            double ms = 0.0;
            if ((r = time_workload(*opts_out, &ms, nullptr)) != GC_OK) return r;
            if (ms < rep.tune_ms) {
                rep.tune_ms = ms;
                rep.tune = t;
            }
        }
    }
    ctx->tune = rep.tune;
    restore.keep = true;
    if (report) *report = rep;
    return GC_OK;
}

gc_status gc_autotune(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                      const gc_opts* opts, const gc_autotune_opts* atp, gc_opts* opts_out,
                      gc_autotune_report* report, hipStream_t stream)
{
    GC_GUARD(autotune_impl(ctx, n_scenes, scenes, cameras, opts, atp, opts_out, report, stream));
}

}  // extern "C"
