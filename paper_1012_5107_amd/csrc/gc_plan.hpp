// gc_plan.hpp -- batched FP32 render as HIP graphs (included at the end of
// gc_lib.hip).
//
// The pipeline's rounds read their queue lengths from device memory and
// return at once when a queue is empty, so a fixed number of rounds can be
// enqueued without reading anything back.  The number of rounds a workload
// needs is a property of its rays (every ray's path is deterministic), so
// it is measured by one eager run when the plan is made; graphs launched
// back to back then hold: zeroing of the counters, the camera rays' flight
// to the box, that many rounds, the pixel averages, optionally the
// flat-mirror references, and the zero-shift correlation of every scene
// (eq. (15)).  Each round's in-box kernel is a graph of its own, so that
// events recorded between the launches time it.
//
// The same eager run records the longest first visits of the box (a visit
// cannot be split, so one that starts late ends the launch late: in a
// high-Ak scene a ray guided along z near the crests can take 1e5 steps).
// The replays' k_wf_init puts those rays at the front of round 0's queue, so
// that they are claimed when the launch starts, with raised priority.  What
// each ray computes does not depend on when it is claimed.
#pragma once

// recorded first visits: at least kRecMin steps, at most kRecCap of them;
// the kFrontMax longest go to the front of the queue
constexpr int kRecMin = 1000;
constexpr unsigned kRecCap = 65536;
constexpr int kFrontMax = 4096;

struct gc_batch_plan {
    gc_ctx* ctx = nullptr;
    WfStore w;                   // the plan's own pipeline buffers
    WfArgs a;
    int ns = 0;
    int rounds = 0;
    long long n_pix = 0;
    bool corr = false;
    double* d_cc = nullptr;      // kCCOut doubles per scene: C0, ncc, the two variances, the means
    double* d_part = nullptr;    // partial moments of the correlation
    int* d_rec = nullptr;        // (ray, steps) pairs of the eager run's long first visits
    int* d_front = nullptr;      // the front rays (ascending) and their slots
    unsigned* d_front_bits = nullptr;
    int n_front = 0;
    // the graphs, in launch order: start of the pipeline; per round, the
    // in-box kernel and the rest of the round (after the last round: pixel
    // means, references, correlations)
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    std::vector<hipEvent_t> ev_round;   // per round: before and after its in-box graph
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

static void plan_free(gc_batch_plan* p)
{
    if (!p) return;
    for (hipGraphExec_t x : p->execs) (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : p->graphs) (void)hipGraphDestroy(g);
    if (p->d_cc) (void)hipFree(p->d_cc);
    if (p->d_part) (void)hipFree(p->d_part);
    if (p->d_rec) (void)hipFree(p->d_rec);
    if (p->d_front) (void)hipFree(p->d_front);
    if (p->d_front_bits) (void)hipFree(p->d_front_bits);
    for (hipEvent_t e : p->ev_round) (void)hipEventDestroy(e);
    if (p->e0) (void)hipEventDestroy(p->e0);
    if (p->e1) (void)hipEventDestroy(p->e1);
    wf_free(p->w);
    delete p;
}

// The kFrontMax longest of the n_rec recorded first visits, in the order
// of their lengths, become the front of round 0's fast queue (p->a.front_*).
static gc_status plan_front(gc_batch_plan* p, unsigned n_rec)
{
    if (n_rec == 0) return GC_OK;
    std::vector<int> rec(2 * (size_t)n_rec);
    HIP_OK(hipMemcpy(rec.data(), p->d_rec, sizeof(int) * rec.size(), hipMemcpyDeviceToHost));
    std::vector<unsigned> order(n_rec);
    for (unsigned i = 0; i < n_rec; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](unsigned x, unsigned y) {
        return rec[2 * x + 1] != rec[2 * y + 1] ? rec[2 * x + 1] > rec[2 * y + 1] : rec[2 * x] < rec[2 * y];
    });
    const int k = (int)std::min<unsigned>(n_rec, (unsigned)kFrontMax);
    std::vector<std::pair<int, int>> fr((size_t)k);   // (ray, slot)
    for (int i = 0; i < k; ++i) fr[i] = {rec[2 * order[i]], i};
    std::sort(fr.begin(), fr.end());
    const long long n_rays = p->a.n_rays;
    std::vector<unsigned> bits((size_t)((n_rays + 31) / 32), 0u);
    std::vector<int> host(2 * (size_t)k);
    for (int i = 0; i < k; ++i) {
        const int q = fr[i].first;
        if (q < 0 || q >= n_rays || (i > 0 && q == fr[i - 1].first))
            return fail(GC_EDEVICE, "batch plan: inconsistent record of long visits");
        host[i] = q;
        host[k + i] = fr[i].second;
        bits[(size_t)q >> 5] |= 1u << (q & 31);
    }
    if (hipMalloc(&p->d_front, sizeof(int) * host.size()) != hipSuccess ||
        hipMalloc(&p->d_front_bits, sizeof(unsigned) * bits.size()) != hipSuccess)
        return fail(GC_ENOMEM, "batch plan: allocation failed");
    HIP_OK(hipMemcpy(p->d_front, host.data(), sizeof(int) * host.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(p->d_front_bits, bits.data(), sizeof(unsigned) * bits.size(), hipMemcpyHostToDevice));
    p->n_front = k;
    p->a.front_bits = p->d_front_bits;
    p->a.front_q = p->d_front;
    p->a.front_slot = p->d_front + k;
    p->a.n_front = k;
    return GC_OK;
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
        if (scenes[i].mirror == 1 && scenes[i].cloak == GC_CLOAK_NONE)
            return fail(GC_EUNSUPPORTED, "scene %d: flat-mirror scenes are rendered by gc_render", i);
        if (scenes[i].fresnel)
            return fail(GC_EUNSUPPORTED, "scene %d: Fresnel-weighted faces are rendered by the FP64 path", i);
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
    if (hipMalloc(&p->d_cc, sizeof(double) * kCCOut * n_scenes) != hipSuccess ||
        hipMalloc(&p->d_part, sizeof(double) * kCCBlocks * 5 * kCCMaxCh) != hipSuccess ||
        hipEventCreate(&p->e0) != hipSuccess || hipEventCreate(&p->e1) != hipSuccess)
        return bail(fail(GC_ENOMEM, "batch plan: allocation failed"));
    if ((r = wf_setup(ctx, p->w, n_scenes, sd.data(), cd.data(), o, d_rgb, cs, &p->a, &p->n_pix)) != GC_OK)
        return bail(r);
    // one eager run: the number of rounds this workload needs, and its long
    // first visits
    if (hipMalloc(&p->d_rec, sizeof(int) * 2 * kRecCap) != hipSuccess)
        return bail(fail(GC_ENOMEM, "batch plan: allocation failed"));
    p->a.rec = p->d_rec;
    p->a.rec_cap = kRecCap;
    p->a.rec_min = kRecMin;
    if ((r = wf_run(ctx, p->w, p->a, cs)) != GC_OK) return bail(r);
    if (hipStreamSynchronize(cs) != hipSuccess) return bail(fail(GC_EDEVICE, "eager run failed"));
    p->rounds = (int)p->w.rounds;
    p->a.rec = nullptr;
    if ((r = plan_front(p, std::min<unsigned>(p->w.h_ctr->rec_len, kRecCap))) != GC_OK) return bail(r);

    // events between the graph launches: the in-box kernel's device time
    p->ev_round.assign(2 * (size_t)p->rounds, nullptr);
    for (hipEvent_t& e : p->ev_round)
        if (hipEventCreate(&e) != hipSuccess) return bail(fail(GC_EDEVICE, "hipEventCreate failed"));

    // capture: 1 + 2 rounds graphs
    const unsigned box_g = wf_box_max(ctx, p->w, o.integ);
    const unsigned air_g = (unsigned)(8 * ctx->n_cu);
    for (int piece = 0; piece <= 2 * p->rounds; ++piece) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return bail(fail(GC_EDEVICE, "hipStreamBeginCapture failed"));
        gc_status cr = GC_OK;
        const int round = (piece - 1) / 2;   // piece 0: round 0's counters follow the start
        if (piece == 0) {
            wf_start(ctx, p->w, p->a, cs);
        } else if (piece % 2 == 1) {
            wf_round_box(p->a, round & 1, box_g, cs);
        } else {
            wf_round_post(ctx, p->a, round & 1, air_g, cs);
        }
        // the next round's counters, or the end of the render
        if (piece % 2 == 0 && round + (piece > 0) < p->rounds) {
            hipLaunchKernelGGL(k_wf_reset, dim3(1), dim3(64), 0, cs, p->w.ctr, (round + (piece > 0)) & 1);
        } else if (piece == 2 * p->rounds) {
            cr = wf_finish(p->w, p->a, n_scenes, p->n_pix, cs);
            for (int i = 0; i < n_scenes && p->corr; ++i) {
                const long long npix = (long long)cd[i].W * cd[i].H;
                if (render_refs)
                    hipLaunchKernelGGL(k_render_flat, dim3(flat_blocks(ctx->n_cu, npix)), dim3(256), 0, cs, cd[i],
                                       sd[i], d_ref[i], nullptr);
                long long nb = std::min<long long>((npix + 255) / 256, kCCBlocks);
                hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nb), dim3(256), 0, cs, (const float*)d_rgb[i],
                                   (const float*)d_ref[i], npix, npix, npix, 3, p->d_part);
                hipLaunchKernelGGL(k_cc_final, dim3(1), dim3(256), 0, cs, (const double*)p->d_part, (int)nb, npix,
                                   3, (const float*)d_rgb[i], (const float*)d_ref[i], p->d_cc + kCCOut * i);
            }
        }
        const bool launch_ok = hipGetLastError() == hipSuccess;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(cs, &g);
        if (g) p->graphs.push_back(g);
        if (cr != GC_OK) return bail(cr);
        if (!launch_ok) return bail(fail(GC_EDEVICE, "kernel launch failed during capture"));
        if (ec != hipSuccess || !g) return bail(fail(GC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec)));
        hipGraphExec_t x = nullptr;
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess || !x)
            return bail(fail(GC_EDEVICE, "hipGraphInstantiate failed"));
        p->execs.push_back(x);
    }
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
    HIP_OK(hipGraphLaunch(p->execs[0], stream));
    for (int k = 0; k < p->rounds; ++k) {
        HIP_OK(hipEventRecord(p->ev_round[2 * k], stream));
        HIP_OK(hipGraphLaunch(p->execs[1 + 2 * k], stream));
        HIP_OK(hipEventRecord(p->ev_round[2 * k + 1], stream));
        HIP_OK(hipGraphLaunch(p->execs[2 + 2 * k], stream));
    }
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
    std::vector<double> cc(kCCOut * (size_t)p->ns);
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
        st->tail_rays = p->n_front;
        st->hot_steps = (int64_t)ctr.hot_steps;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->e0, p->e1) == hipSuccess) st->total_ms = ms;
        for (int k = 0; k < p->rounds; ++k)
            if (hipEventElapsedTime(&ms, p->ev_round[2 * k], p->ev_round[2 * k + 1]) == hipSuccess) st->hot_ms += ms;
    }
    for (int i = 0; i < p->ns && p->corr; ++i) {
        if (!(cc[kCCOut * i + 2] > 0)) return fail(GC_EINVAL, "reference image %d is constant: eq. (15) is undefined", i);
        C0[i] = cc[kCCOut * i];
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
