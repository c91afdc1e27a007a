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
//
// With gc_tune.plan_lanes = G >= 2 the scenes are split into G groups of
// about equal sample counts ("lanes"), each a complete pipeline of its own
// (buffers, counters, rounds, graphs) replayed on a stream of its own: the
// groups' kernels only share the device, so while one group runs its serial
// tail (its longest visit, its FP64 hand-overs) the others' kernels fill
// the idle compute units.  Every ray computes what it computes in one
// pipeline.
#pragma once

// recorded first visits: at least kRecMin steps, at most kRecCap of them;
// the kFrontMax longest go to the front of the queue
constexpr int kRecMin = 1000;
constexpr unsigned kRecCap = 65536;
constexpr int kFrontMax = 4096;

// one sub-pipeline: its scenes (indices into the plan's), buffers, rounds
// and graphs
struct PlanLane {
    std::vector<int> scenes;
    WfStore w;
    WfArgs a;
    int rounds = 0;
    long long n_pix = 0;
    double* d_part = nullptr;    // partial moments of its correlations
    int* d_rec = nullptr;        // (ray, steps) pairs of the eager run's long first visits
    int* d_front = nullptr;      // the front rays (ascending) and their slots
    unsigned* d_front_bits = nullptr;
    int n_front = 0;
    hipStream_t stream = nullptr;   // G >= 2: the lane's own stream
    // the graphs, in launch order: start of the pipeline; per round, the
    // in-box kernel and the rest of the round (after the last round: pixel
    // means, references, correlations)
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    std::vector<hipEvent_t> ev_round;   // per round: before and after its in-box graph
    hipEvent_t e_end = nullptr;
};

struct gc_batch_plan {
    gc_ctx* ctx = nullptr;
    int ns = 0;
    bool corr = false;
    double* d_cc = nullptr;      // kCCOut doubles per scene: C0, ncc, the two variances, the means
    std::vector<PlanLane*> lanes;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

static void lane_free(PlanLane* l)
{
    if (!l) return;
    for (hipGraphExec_t x : l->execs) (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : l->graphs) (void)hipGraphDestroy(g);
    if (l->d_part) (void)hipFree(l->d_part);
    if (l->d_rec) (void)hipFree(l->d_rec);
    if (l->d_front) (void)hipFree(l->d_front);
    if (l->d_front_bits) (void)hipFree(l->d_front_bits);
    for (hipEvent_t e : l->ev_round) (void)hipEventDestroy(e);
    if (l->e_end) (void)hipEventDestroy(l->e_end);
    if (l->stream) (void)hipStreamDestroy(l->stream);
    wf_free(l->w);
    delete l;
}

static void plan_free(gc_batch_plan* p)
{
    if (!p) return;
    for (PlanLane* l : p->lanes) lane_free(l);
    if (p->d_cc) (void)hipFree(p->d_cc);
    if (p->e0) (void)hipEventDestroy(p->e0);
    if (p->e1) (void)hipEventDestroy(p->e1);
    delete p;
}

// The kFrontMax longest of the n_rec recorded first visits, in the order
// of their lengths, become the front of round 0's fast queue (l->a.front_*).
static gc_status plan_front(PlanLane* l, unsigned n_rec)
{
    if (n_rec == 0) return GC_OK;
    std::vector<int> rec(2 * (size_t)n_rec);
    HIP_OK(hipMemcpy(rec.data(), l->d_rec, sizeof(int) * rec.size(), hipMemcpyDeviceToHost));
    std::vector<unsigned> order(n_rec);
    for (unsigned i = 0; i < n_rec; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](unsigned x, unsigned y) {
        return rec[2 * x + 1] != rec[2 * y + 1] ? rec[2 * x + 1] > rec[2 * y + 1] : rec[2 * x] < rec[2 * y];
    });
    const int k = (int)std::min<unsigned>(n_rec, (unsigned)kFrontMax);
    std::vector<std::pair<int, int>> fr((size_t)k);   // (ray, slot)
    for (int i = 0; i < k; ++i) fr[i] = {rec[2 * order[i]], i};
    std::sort(fr.begin(), fr.end());
    const long long n_rays = l->a.n_rays;
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
    if (hipMalloc(&l->d_front, sizeof(int) * host.size()) != hipSuccess ||
        hipMalloc(&l->d_front_bits, sizeof(unsigned) * bits.size()) != hipSuccess)
        return fail(GC_ENOMEM, "batch plan: allocation failed");
    HIP_OK(hipMemcpy(l->d_front, host.data(), sizeof(int) * host.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(l->d_front_bits, bits.data(), sizeof(unsigned) * bits.size(), hipMemcpyHostToDevice));
    l->n_front = k;
    l->a.front_bits = l->d_front_bits;
    l->a.front_q = l->d_front;
    l->a.front_slot = l->d_front + k;
    l->a.n_front = k;
    return GC_OK;
}

// Scenes into G groups of about equal sample counts: largest first, each to
// the group with the fewest samples so far (ties: the lower group).
static std::vector<std::vector<int>> plan_groups(int ns, const std::vector<gc::CamDev>& cd, int G)
{
    std::vector<long long> rays(ns);
    for (int i = 0; i < ns; ++i) rays[i] = (long long)cd[i].W * cd[i].H * cd[i].spp;
    std::vector<int> order(ns);
    for (int i = 0; i < ns; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return rays[x] > rays[y]; });
    std::vector<std::vector<int>> g((size_t)G);
    std::vector<long long> load((size_t)G, 0);
    for (int i : order) {
        int best = 0;
        for (int j = 1; j < G; ++j)
            if (load[j] < load[best]) best = j;
        g[best].push_back(i);
        load[best] += rays[i];
    }
    for (auto& v : g) std::sort(v.begin(), v.end());
    return g;
}

// Eager run and capture of one lane (its scenes sd/cd/images, in the
// lane's order; the scenes' plan indices in l->scenes).
static gc_status lane_build(gc_ctx* ctx, PlanLane* l, const gc::OptsDev& o, const std::vector<gc::SceneDev>& sd_all,
                            const std::vector<gc::CamDev>& cd_all, float* const* d_rgb_all, float* const* d_ref_all,
                            bool render_refs, double* d_cc, hipStream_t cs)
{
    using namespace gc;
    const int n = (int)l->scenes.size();
    std::vector<SceneDev> sd(n);
    std::vector<CamDev> cd(n);
    std::vector<float*> rgb(n);
    for (int k = 0; k < n; ++k) {
        sd[k] = sd_all[l->scenes[k]];
        cd[k] = cd_all[l->scenes[k]];
        rgb[k] = d_rgb_all[l->scenes[k]];
    }
    if (hipMalloc(&l->d_part, sizeof(double) * kCCBlocks * 5 * kCCMaxCh) != hipSuccess ||
        hipMalloc(&l->d_rec, sizeof(int) * 2 * kRecCap) != hipSuccess ||
        hipEventCreate(&l->e_end) != hipSuccess)
        return fail(GC_ENOMEM, "batch plan: allocation failed");
    gc_status r;
    if ((r = wf_setup(ctx, l->w, n, sd.data(), cd.data(), o, rgb.data(), cs, &l->a, &l->n_pix)) != GC_OK) return r;
    // one eager run: the number of rounds this workload needs, and its long
    // first visits
    l->a.rec = l->d_rec;
    l->a.rec_cap = kRecCap;
    l->a.rec_min = kRecMin;
    if ((r = wf_run(ctx, l->w, l->a, cs)) != GC_OK) return r;
    if (hipStreamSynchronize(cs) != hipSuccess) return fail(GC_EDEVICE, "eager run failed");
    l->rounds = (int)l->w.rounds;
    l->a.rec = nullptr;
    if ((r = plan_front(l, std::min<unsigned>(l->w.h_ctr->rec_len, kRecCap))) != GC_OK) return r;

    // events between the graph launches: the in-box kernel's device time
    l->ev_round.assign(2 * (size_t)l->rounds, nullptr);
    for (hipEvent_t& e : l->ev_round)
        if (hipEventCreate(&e) != hipSuccess) return fail(GC_EDEVICE, "hipEventCreate failed");

    // capture: 1 + 2 rounds graphs
    const unsigned box_g = wf_box_max(ctx, l->w, o.integ);
    const unsigned air_g = (unsigned)(8 * ctx->n_cu);
    for (int piece = 0; piece <= 2 * l->rounds; ++piece) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(GC_EDEVICE, "hipStreamBeginCapture failed");
        gc_status cr = GC_OK;
        const int round = (piece - 1) / 2;   // piece 0: round 0's counters follow the start
        if (piece == 0) {
            wf_start(ctx, l->w, l->a, cs);
        } else if (piece % 2 == 1) {
            wf_round_box(l->a, round & 1, box_g, cs);
        } else {
            wf_round_post(ctx, l->a, round & 1, air_g, cs);
        }
        // the next round's counters, or the end of the render
        if (piece % 2 == 0 && round + (piece > 0) < l->rounds) {
            hipLaunchKernelGGL(k_wf_reset, dim3(1), dim3(64), 0, cs, l->w.ctr, (round + (piece > 0)) & 1);
        } else if (piece == 2 * l->rounds) {
            cr = wf_finish(l->w, l->a, n, l->n_pix, cs);
            for (int k = 0; k < n && d_ref_all; ++k) {
                const int i = l->scenes[k];
                const long long npix = (long long)cd[k].W * cd[k].H;
                if (render_refs)
                    hipLaunchKernelGGL(k_render_flat, dim3(flat_blocks(ctx->n_cu, npix)), dim3(256), 0, cs, cd[k],
                                       sd[k], d_ref_all[i], nullptr);
                long long nb = std::min<long long>((npix + 255) / 256, kCCBlocks);
                hipLaunchKernelGGL(k_cc_moments, dim3((unsigned)nb), dim3(256), 0, cs, (const float*)rgb[k],
                                   (const float*)d_ref_all[i], npix, npix, npix, 3, l->d_part);
                hipLaunchKernelGGL(k_cc_final, dim3(1), dim3(256), 0, cs, (const double*)l->d_part, (int)nb, npix,
                                   3, (const float*)rgb[k], (const float*)d_ref_all[i], d_cc + kCCOut * i);
            }
        }
        const bool launch_ok = hipGetLastError() == hipSuccess;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(cs, &g);
        if (g) l->graphs.push_back(g);
        if (cr != GC_OK) return cr;
        if (!launch_ok) return fail(GC_EDEVICE, "kernel launch failed during capture");
        if (ec != hipSuccess || !g) return fail(GC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        hipGraphExec_t x = nullptr;
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess || !x)
            return fail(GC_EDEVICE, "hipGraphInstantiate failed");
        l->execs.push_back(x);
    }
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
        hipEventCreate(&p->e0) != hipSuccess || hipEventCreate(&p->e1) != hipSuccess)
        return bail(fail(GC_ENOMEM, "batch plan: allocation failed"));
    const int G = std::max(1, std::min(std::min(ctx->tune.plan_lanes, kPlanMaxLanes), (int)n_scenes));
    for (const std::vector<int>& grp : plan_groups(n_scenes, cd, G)) {
        PlanLane* l = new (std::nothrow) PlanLane();
        if (!l) return bail(fail(GC_ENOMEM, "host allocation failed"));
        p->lanes.push_back(l);
        l->scenes = grp;
        if (G > 1 && hipStreamCreate(&l->stream) != hipSuccess)
            return bail(fail(GC_EDEVICE, "hipStreamCreate failed"));
        if ((r = lane_build(ctx, l, o, sd, cd, d_rgb, d_ref, render_refs != 0, p->d_cc, cs)) != GC_OK) return bail(r);
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
    // one lane runs on the caller's stream; several each on their own,
    // forked from it here and joined back below
    const bool fork = p->lanes.size() > 1;
    for (PlanLane* l : p->lanes)
        if (fork) HIP_OK(hipStreamWaitEvent(l->stream, p->e0, 0));
    size_t most = 0;
    for (PlanLane* l : p->lanes) most = std::max(most, l->execs.size());
    // the lanes' graphs interleaved, so that every lane starts at once
    for (size_t g = 0; g < most; ++g) {
        for (PlanLane* l : p->lanes) {
            if (g >= l->execs.size()) continue;
            hipStream_t s = fork ? l->stream : stream;
            const bool box = g % 2 == 1;   // graph 1 + 2k: round k's in-box kernel
            if (box) HIP_OK(hipEventRecord(l->ev_round[g - 1], s));
            HIP_OK(hipGraphLaunch(l->execs[g], s));
            if (box) HIP_OK(hipEventRecord(l->ev_round[g], s));
        }
    }
    for (PlanLane* l : p->lanes) {
        if (!fork) continue;
        HIP_OK(hipEventRecord(l->e_end, l->stream));
        HIP_OK(hipStreamWaitEvent(stream, l->e_end, 0));
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
    const size_t G = p->lanes.size();
    std::vector<WfTotals> tot(G);
    std::vector<QCtr> ctr(G);
    std::vector<double> cc(kCCOut * (size_t)p->ns);
    for (size_t j = 0; j < G; ++j) {
        HIP_OK(hipMemcpyAsync(&tot[j], p->lanes[j]->w.tot, sizeof(WfTotals), hipMemcpyDeviceToHost, stream));
        HIP_OK(hipMemcpyAsync(&ctr[j], p->lanes[j]->w.ctr, sizeof(QCtr), hipMemcpyDeviceToHost, stream));
    }
    if (p->corr) HIP_OK(hipMemcpyAsync(cc.data(), p->d_cc, sizeof(double) * cc.size(), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    for (size_t j = 0; j < G; ++j) {
        const int nxt = p->lanes[j]->rounds & 1;
        if (ctr[j].box_len[nxt] + ctr[j].slow_len[nxt] != 0)
            return fail(GC_EDEVICE, "the captured %d rounds did not finish every ray", p->lanes[j]->rounds);
    }
    if (st) {
        std::memset(st, 0, sizeof *st);
        // the in-box kernels' device time: the union of their launch
        // intervals (with several lanes they overlap)
        std::vector<std::pair<float, float>> iv;
        for (size_t j = 0; j < G; ++j) {
            const PlanLane* l = p->lanes[j];
            st->rays += (int64_t)tot[j].rays;
            st->accepted_steps += (int64_t)tot[j].steps;
            st->rejected_steps += (int64_t)tot[j].rejected;
            st->events += (int64_t)tot[j].events;
            st->fallbacks += (int64_t)tot[j].fallbacks;
            st->failed += (int64_t)tot[j].failed;
            st->rounds = std::max<int64_t>(st->rounds, l->rounds);
            st->tail_rays += l->n_front;
            st->hot_steps += (int64_t)ctr[j].hot_steps;
            for (int k = 0; k < l->rounds; ++k) {
                float t0 = 0.f, t1 = 0.f;
                if (hipEventElapsedTime(&t0, p->e0, l->ev_round[2 * k]) == hipSuccess &&
                    hipEventElapsedTime(&t1, p->e0, l->ev_round[2 * k + 1]) == hipSuccess)
                    iv.push_back({t0, t1});
            }
        }
        std::sort(iv.begin(), iv.end());
        float lo = 0.f, hi = -1.f;
        for (const auto& x : iv) {
            if (x.first > hi) {
                if (hi > lo) st->hot_ms += hi - lo;
                lo = x.first;
                hi = x.second;
            } else {
                hi = std::max(hi, x.second);
            }
        }
        if (hi > lo) st->hot_ms += hi - lo;
        st->fp64_steps = st->accepted_steps - st->hot_steps;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->e0, p->e1) == hipSuccess) st->total_ms = ms;
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
