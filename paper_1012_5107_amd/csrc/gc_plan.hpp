// gc_plan.hpp -- batched FP32 render as one HIP graph (included at the end
// of gc_lib.hip).
//
// The pipeline's rounds read their queue lengths from device memory and
// return at once when a queue is empty, so a fixed number of rounds can be
// enqueued without reading anything back.  The number of rounds a workload
// needs is a property of its rays (every ray's path is deterministic), so
// it is measured by one eager run when the plan is made; the graph then
// holds: zeroing of the counters, the camera rays' flight to the box, that
// many rounds, the pixel averages, optionally the flat-mirror references,
// and the zero-shift correlation of every scene (eq. (15)).
#pragma once

struct gc_batch_plan {
    gc_ctx* ctx = nullptr;
    WfStore w;                   // the plan's own pipeline buffers
    WfArgs a;
    int ns = 0;
    int rounds = 0;
    long long n_pix = 0;
    bool corr = false;
    double* d_cc = nullptr;      // 4 doubles per scene: C0, ncc and the two variances
    double* d_part = nullptr;    // partial moments of the correlation
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

static void plan_free(gc_batch_plan* p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_cc) (void)hipFree(p->d_cc);
    if (p->d_part) (void)hipFree(p->d_part);
    if (p->e0) (void)hipEventDestroy(p->e0);
    if (p->e1) (void)hipEventDestroy(p->e1);
    wf_free(p->w);
    delete p;
}

extern "C" {

static gc_status batch_plan_create_impl(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                               const gc_opts* opts, float* const* d_rgb, float* const* d_ref, int32_t render_refs,
                               gc_batch_plan** out)
{
    using namespace gc;
    if (!out) return fail(GC_EINVAL, "out is null");
    *out = nullptr;
    if (!ctx) return fail(GC_EINVAL, "ctx is null");
    if (n_scenes < 1 || !scenes || !cameras || !opts || !d_rgb)
        return fail(GC_EINVAL, "need n_scenes >= 1 and non-null scenes, cameras, opts and images");
    if (render_refs && !d_ref) return fail(GC_EINVAL, "render_refs needs reference images");
    OptsDev o;
    gc_status r;
    if ((r = make_opts(opts, &o)) != GC_OK) return r;
    if (opts->prec != GC_F32) return fail(GC_EUNSUPPORTED, "a batch plan runs the FP32 pipeline (prec = GC_F32)");
    std::vector<SceneDev> sd(n_scenes);
    std::vector<CamDev> cd(n_scenes);
    for (int i = 0; i < n_scenes; ++i) {
        if ((r = make_scene(&scenes[i], &sd[i])) != GC_OK) return fail(r, "scene %d: %s", i, g_err.c_str());
        if (scenes[i].mirror == 1) return fail(GC_EUNSUPPORTED, "scene %d: flat-mirror scenes are rendered by gc_render", i);
        if ((r = make_camera(&cameras[i], &cd[i])) != GC_OK) return fail(r, "camera %d: %s", i, g_err.c_str());
        if (!d_rgb[i]) return fail(GC_EINVAL, "image pointer %d is null", i);
        if (d_ref && !d_ref[i]) return fail(GC_EINVAL, "reference pointer %d is null", i);
    }
    HIP_OK(hipSetDevice(ctx->device));
    gc_batch_plan* p = new (std::nothrow) gc_batch_plan();
    if (!p) return fail(GC_ENOMEM, "host allocation failed");
    p->ctx = ctx;
    p->ns = n_scenes;
    p->corr = d_ref != nullptr;
    hipStream_t cs = nullptr;
    auto bail = [&](gc_status e) {
        if (cs) (void)hipStreamDestroy(cs);
        plan_free(p);
        return e;
    };
    if (hipStreamCreate(&cs) != hipSuccess) return bail(fail(GC_EDEVICE, "hipStreamCreate failed"));
    if (hipMalloc(&p->d_cc, sizeof(double) * 4 * n_scenes) != hipSuccess ||
        hipMalloc(&p->d_part, sizeof(double) * kCCBlocks * 5 * kCCMaxCh) != hipSuccess ||
        hipEventCreate(&p->e0) != hipSuccess || hipEventCreate(&p->e1) != hipSuccess)
        return bail(fail(GC_ENOMEM, "batch plan: allocation failed"));
    if ((r = wf_setup(ctx, p->w, n_scenes, sd.data(), cd.data(), o, d_rgb, cs, &p->a, &p->n_pix)) != GC_OK)
        return bail(r);
    // one eager run: the number of rounds this workload needs
    if ((r = wf_run(ctx, p->w, p->a, cs)) != GC_OK) return bail(r);
    if (hipStreamSynchronize(cs) != hipSuccess) return bail(fail(GC_EDEVICE, "eager run failed"));
    p->rounds = (int)p->w.rounds;

    // capture
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(fail(GC_EDEVICE, "hipStreamBeginCapture failed"));
    gc_status cr = GC_OK;
    do {
        wf_start(ctx, p->w, p->a, cs);
        const unsigned box_g = wf_box_max(ctx, p->w, o.integ);
        const unsigned air_g = (unsigned)(8 * ctx->n_cu);
        for (int round = 0; round < p->rounds && cr == GC_OK; ++round)
            cr = wf_round(ctx, p->w, p->a, round & 1, box_g, air_g, false, cs);
        if (cr != GC_OK) break;
        if ((cr = wf_finish(p->w, p->a, n_scenes, p->n_pix, cs)) != GC_OK) break;
        for (int i = 0; i < n_scenes && p->corr; ++i) {
            const long long npix = (long long)cd[i].W * cd[i].H;
            if (render_refs)
                hipLaunchKernelGGL(k_render_flat, dim3(flat_blocks(ctx->n_cu, npix)), dim3(256), 0, cs, cd[i],
                                   sd[i].K, d_ref[i], nullptr);
            long long nb = std::min<long long>((npix + 255) / 256, kCCBlocks);
            hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nb), dim3(256), 0, cs, (const float*)d_rgb[i],
                               (const float*)d_ref[i], npix, 3, p->d_part);
            hipLaunchKernelGGL(k_cc_final, dim3(1), dim3(256), 0, cs, (const double*)p->d_part, (int)nb, npix, 3,
                               p->d_cc + 4 * i);
        }
        if (hipGetLastError() != hipSuccess) cr = fail(GC_EDEVICE, "kernel launch failed during capture");
    } while (false);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    p->graph = g;
    if (cr != GC_OK) return bail(cr);
    if (ec != hipSuccess || !g) return bail(fail(GC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec)));
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(GC_EDEVICE, "hipGraphInstantiate failed"));
    (void)hipStreamDestroy(cs);
    *out = p;
    return GC_OK;
}

gc_status gc_batch_plan_create(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                               const gc_opts* opts, float* const* d_rgb, float* const* d_ref, int32_t render_refs,
                               gc_batch_plan** out)
{
    GC_GUARD(batch_plan_create_impl(ctx, n_scenes, scenes, cameras, opts, d_rgb, d_ref, render_refs, out));
}

static gc_status batch_plan_launch_impl(gc_batch_plan* p, hipStream_t stream)
{
    if (!p) return fail(GC_EINVAL, "plan is null");
    HIP_OK(hipSetDevice(p->ctx->device));
    HIP_OK(hipEventRecord(p->e0, stream));
    HIP_OK(hipGraphLaunch(p->exec, stream));
    HIP_OK(hipEventRecord(p->e1, stream));
    return GC_OK;
}

gc_status gc_batch_plan_launch(gc_batch_plan* p, hipStream_t stream)
{
    GC_GUARD(batch_plan_launch_impl(p, stream));
}

static gc_status batch_plan_results_impl(gc_batch_plan* p, double* C0, gc_stats* st, hipStream_t stream)
{
    using namespace gc;
    if (!p) return fail(GC_EINVAL, "plan is null");
    if (p->corr && !C0) return fail(GC_EINVAL, "C0 must be non-null for a plan with references");
    HIP_OK(hipSetDevice(p->ctx->device));
    WfTotals tot;
    QCtr ctr;
    std::vector<double> cc(4 * (size_t)p->ns);
    HIP_OK(hipMemcpyAsync(&tot, p->w.tot, sizeof tot, hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(&ctr, p->w.ctr, sizeof ctr, hipMemcpyDeviceToHost, stream));
    if (p->corr) HIP_OK(hipMemcpyAsync(cc.data(), p->d_cc, sizeof(double) * cc.size(), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    const int nxt = p->rounds & 1;
    if (ctr.box_len[nxt] + ctr.slow_len[nxt] != 0)
        return fail(GC_EDEVICE, "the captured %d rounds did not finish every ray", p->rounds);
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->rays = (int64_t)tot.rays;
        st->accepted_steps = (int64_t)tot.steps;
        st->rejected_steps = (int64_t)tot.rejected;
        st->events = (int64_t)tot.events;
        st->fallbacks = (int64_t)tot.fallbacks;
        st->failed = (int64_t)tot.failed;
        st->rounds = p->rounds;
        st->hot_steps = (int64_t)ctr.hot_steps;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->e0, p->e1) == hipSuccess) st->total_ms = ms;
    }
    for (int i = 0; i < p->ns && p->corr; ++i) {
        if (!(cc[4 * i + 2] > 0)) return fail(GC_EINVAL, "reference image %d is constant: eq. (15) is undefined", i);
        C0[i] = cc[4 * i];
    }
    return GC_OK;
}

gc_status gc_batch_plan_results(gc_batch_plan* p, double* C0, gc_stats* st, hipStream_t stream)
{
    GC_GUARD(batch_plan_results_impl(p, C0, st, stream));
}

void gc_batch_plan_destroy(gc_batch_plan* p)
{
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    plan_free(p);
}

}  // extern "C"
