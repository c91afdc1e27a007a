// gc_wave.hpp -- the FP32 render/trace pipeline as queue-driven kernels.
//
// A sample's path alternates between long stretches of integration inside
// the cloak and rare events (box faces, grating contacts, FP64 fallbacks).
// Keeping both in one kernel gives every lane the register footprint of the
// FP64 event code, so they are separate kernels that pass rays through
// queues of ray indices:
//
//   k_wf_init    one lane per sample: camera ray (or given ray), flight
//                through air (FP64) to the box, the sky, or a failure;
//   k_wf_box     persistent FP32 kernel: each wave claims rays from the box
//                queue (one atomic per wave, ballot + rank for the lanes),
//                integrates each until its next step crosses a surface or
//                needs FP64, writes the ray back and pushes it to the event
//                queue, then refills the idle lane;
//   k_wf_event   FP64: redoes the flagged step from its start with step
//                control, locates and applies the event (partial-step root
//                solve); rays still inside go to the next box queue, rays
//                that left the box to the air queue;
//   k_wf_air     FP64: flight through air to the box, the sky or a failure;
//   k_wf_finish  averages each pixel's samples and folds the counters.
//
// Rounds of (k_wf_box, k_wf_event, k_wf_air) repeat until the box queue is
// empty.
// Samples of several scenes can share one launch: every ray carries its
// scene index and the scene / camera tables live in device memory.
#pragma once
#include "gc_lane32.hpp"
#include "gc_lane64.hpp"

namespace gc {

struct QCtr {
    unsigned box_len[2];
    unsigned box_head[2];
    unsigned ev_len;
    unsigned ev_head;
    unsigned air_len;
    unsigned air_head;
    unsigned long long hot_steps;   // accepted steps taken by k_wf_box (all rounds)
};

// per-ray arrays (structure of arrays)
struct WfRays {
    double *rx, *ry, *rz, *qx, *qy, *qz;   // air state / exit point and direction
    double* z0;                             // z at the last box entry or event
    int* cell;
    float *fx, *lx, *y, *ly, *px, *lpx, *py, *lpy, *pz, *Wr, *Wi, *h, *tau, *ltau;
    int *steps, *rej, *events, *flags, *scene, *status, *fbk;
    float* rgb;   // 3 per ray
};

enum WfFlag { WF_LAST_REJ = 1 };

struct WfArgs {
    WfRays R;
    int* qbox[2];
    int* qev;
    int* qair;
    QCtr* ctr;
    const SceneDev* scenes;
    const CamDev* cams;
    const long long* ray_off;   // per scene: first ray index (n_scenes + 1 entries)
    int n_scenes;
    long long n_rays;
    OptsDev o;
    // trace_rays mode: explicit rays in, exit rays out
    const double* in_org;
    const double* in_dir;
};

__device__ __forceinline__ int scene_of(const WfArgs& a, long long q)
{
    int lo = 0, hi = a.n_scenes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.ray_off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---- storing and loading the in-box state ----------------------------------
__device__ __forceinline__ void store_box64(const WfArgs& a, long long q, const SceneDev& s, const Box64& b)
{
    const WfRays& R = a.R;
    double cellf = rint(b.u.x * s.invL);
    double off = b.u.x - cellf * s.L;
    R.cell[q] = (int)cellf;
    float hi = (float)off;
    R.fx[q] = hi;
    R.lx[q] = (float)(off - (double)hi);
    hi = (float)b.u.y;
    R.y[q] = hi;
    R.ly[q] = (float)(b.u.y - (double)hi);
    hi = (float)b.u.px;
    R.px[q] = hi;
    R.lpx[q] = (float)(b.u.px - (double)hi);
    hi = (float)b.u.py;
    R.py[q] = hi;
    R.lpy[q] = (float)(b.u.py - (double)hi);
    R.pz[q] = (float)b.pz;
    R.qz[q] = b.pz;
    R.Wr[q] = (float)b.r1.W.re;
    R.Wi[q] = (float)b.r1.W.im;
    R.h[q] = (float)b.h;
    R.tau[q] = 0.0f;
    R.ltau[q] = 0.0f;
    R.z0[q] = b.z;
    R.flags[q] = b.last_rej ? WF_LAST_REJ : 0;
}

__device__ __forceinline__ Box64 load_box64(const WfArgs& a, long long q, const SceneDev& s)
{
    const WfRays& R = a.R;
    Box64 b;
    b.u.x = (double)R.cell[q] * s.L + ((double)R.fx[q] + (double)R.lx[q]);
    b.u.y = (double)R.y[q] + (double)R.ly[q];
    b.u.px = (double)R.px[q] + (double)R.lpx[q];
    b.u.py = (double)R.py[q] + (double)R.lpy[q];
    b.pz = R.qz[q];
    b.z = R.z0[q] + b.pz * ((double)R.tau[q] + (double)R.ltau[q]);
    b.r1.W = {(double)R.Wr[q], (double)R.Wi[q]};
    if (!(isfinite(b.r1.W.re) && isfinite(b.r1.W.im))) b.r1.W = w0_cold(zarg64(s, b.u.x, b.u.y));
    rhs64(s, b.u.x, b.u.y, b.r1.W, b.r1.ax, b.r1.ay, b.r1.dW);
    b.h = (double)R.h[q];
    b.last_rej = (R.flags[q] & WF_LAST_REJ) != 0;
    return b;
}

__device__ __forceinline__ void push(int* queue, unsigned* len, int q)
{
    unsigned at = atomicAdd(len, 1u);
    queue[at] = q;
}

// terminal state: exit ray in air, or a failure (black)
__device__ __forceinline__ void finish_ray(const WfArgs& a, long long q, const SceneDev& s, int status,
                                           const double r[3], const double p[3])
{
    const WfRays& R = a.R;
    R.status[q] = status;
    R.rx[q] = r[0]; R.ry[q] = r[1]; R.rz[q] = r[2];
    R.qx[q] = p[0]; R.qy[q] = p[1]; R.qz[q] = p[2];
    float c3[3] = {0.0f, 0.0f, 0.0f};
    if (status == RS_OK) {
        double c[3];
        sky_rgb<double>(s.K, p, c);
        c3[0] = (float)c[0]; c3[1] = (float)c[1]; c3[2] = (float)c[2];
    }
    R.rgb[3 * q + 0] = c3[0];
    R.rgb[3 * q + 1] = c3[1];
    R.rgb[3 * q + 2] = c3[2];
}

// Walk through air from (r, p) and either finish the ray or set up its
// in-box state and queue it.
__device__ __forceinline__ void continue_in_air(const WfArgs& a, long long q, const SceneDev& s, double r[3],
                                                double p[3], LaneCount& cnt, int* qnext, unsigned* qnext_len)
{
    double mc = 1.0;
    int st = RS_OK;
    int ao = air_walk(s, a.o, r, p, cnt, &mc, &st);
    a.R.events[q] = cnt.events;
    if (ao == AO_FAIL) { finish_ray(a, q, s, st, r, p); return; }
    if (ao == AO_ESCAPED) { finish_ray(a, q, s, RS_OK, r, p); return; }
    Box64 b = box_enter64(s, a.o, r, p);
    store_box64(a, q, s, b);
    a.R.status[q] = RS_OK;
    push(qnext, qnext_len, (int)q);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wf_reset(QCtr* c, int cur)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->box_head[cur] = 0;
        c->box_len[cur ^ 1] = 0;
        c->box_head[cur ^ 1] = 0;
        c->ev_len = 0;
        c->ev_head = 0;
        c->air_len = 0;
        c->air_head = 0;
    }
}

__global__ void __launch_bounds__(256) k_wf_init(WfArgs a)
{
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n_rays) return;
    int si = scene_of(a, q);
    const SceneDev s = a.scenes[si];
    double r[3], p[3];
    if (a.in_org) {
        for (int i = 0; i < 3; ++i) { r[i] = a.in_org[3 * q + i]; p[i] = a.in_dir[3 * q + i]; }
        double nd = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        for (int i = 0; i < 3; ++i) p[i] /= nd;
    } else {
        const CamDev& c = a.cams[si];
        long long local = q - a.ray_off[si];
        long long pix = local / c.spp;
        int smp = (int)(local - pix * c.spp);
        int i = (int)(pix % c.W), j = (int)(pix / c.W);
        camera_dir(c, i, j, smp, p);
        for (int k = 0; k < 3; ++k) r[k] = c.eye[k];
    }
    a.R.scene[q] = si;
    a.R.fbk[q] = 0;
    a.R.steps[q] = 0;
    a.R.rej[q] = 0;
    LaneCount cnt = {0, 0, 0, 0};
    continue_in_air(a, q, s, r, p, cnt, a.qbox[0], &a.ctr->box_len[0]);
}

// The hot kernel.  INTEG: 0 RK4, 1 DOPRI5.
constexpr int kRefill = 8;

template <int INTEG>
__global__ void __launch_bounds__(256) k_wf_box(WfArgs a, int cur)
{
    const unsigned qlen = a.ctr->box_len[cur];
    const int* queue = a.qbox[cur];
    const int lane = threadIdx.x & 63;
    const float rtol = (float)a.o.rtol, atol = (float)a.o.atol;
    const float hmax = (float)a.o.h_max, hmin = (float)a.o.h_min;
    const int max_steps = a.o.max_steps > 0x7fffffffll ? 0x7fffffff : (int)a.o.max_steps;

    bool active = false;
    // a wave that finds the queue already drained does not touch the counter
    bool exhausted = *((volatile unsigned*)&a.ctr->box_head[cur]) >= qlen;
    int q = 0;
    Sc32 c;
    float ytop = 0.f, xhi = 0.f, xlo = 0.f, pz = 0.f, h = 0.f, tau = 0.f, ltau = 0.f;
    St32 u;
    Rhs32 r1;
    int steps = 0, rej = 0, mirror = 0;
    bool last_rej = false;
    double hw = 0.0, L = 1.0;
    unsigned my_steps = 0;

    for (;;) {
        if (!exhausted) {
            unsigned long long idle = __ballot(!active);
            // claim in batches: one atomic per wave for at least kRefill lanes
            // (or for all of them once the wave has run dry)
            const unsigned long long busy = __ballot(active);
            if (idle && (__popcll(idle) >= kRefill || busy == 0ull)) {
                int n = __popcll(idle);
                int leader = __ffsll((long long)idle) - 1;
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(&a.ctr->box_head[cur], (unsigned)n);
                base = __shfl(base, leader, 64);
                if (base + (unsigned)n >= qlen) exhausted = true;
                if (!active) {
                    unsigned rank = __popcll(idle & ((1ull << lane) - 1ull));
                    unsigned qi = base + rank;
                    if (qi < qlen) {
                        q = queue[qi];
                        const WfRays& R = a.R;
                        const SceneDev& s = a.scenes[R.scene[q]];
                        c = make_sc32(s, a.o.wfb2);
                        ytop = (float)s.ytop;
                        hw = s.hw;
                        L = s.L;
                        mirror = s.mirror;
                        u.cell = R.cell[q];
                        u.fx = R.fx[q]; u.lx = R.lx[q];
                        u.y = R.y[q]; u.ly = R.ly[q];
                        u.px = R.px[q]; u.lpx = R.lpx[q];
                        u.py = R.py[q]; u.lpy = R.lpy[q];
                        pz = R.pz[q];
                        h = R.h[q];
                        tau = R.tau[q];
                        ltau = R.ltau[q];
                        steps = R.steps[q];
                        rej = R.rej[q];
                        last_rej = (R.flags[q] & WF_LAST_REJ) != 0;
                        xhi = (float)(hw - (double)u.cell * L);
                        xlo = (float)(-hw - (double)u.cell * L);
                        r1.W = {R.Wr[q], R.Wi[q]};
                        refresh32(c, u.fx, u.y, r1);
                        active = true;
                    }
                }
            }
        }
        if (__ballot(active) == 0ull) break;
        if (!active) continue;

        St32 ue;
        Rhs32 re;
        bool bad = false;
        float hnext = h;
        bool flag = false;
        if (INTEG == 0) {
            rk4_step32(c, u, r1, h, ue, re, bad);
            flag = bad;
        } else {
            float err = dp5_step32(c, u, r1, h, rtol, atol, ue, re, bad);
            if (bad || !isfinite(err)) {
                flag = true;
            } else if (err > 1.0f) {
                h *= fmaxf(0.2f, 0.9f * pow_m02(err));
                last_rej = true;
                ++rej;
                if (h < hmin) {
                    // let the FP64 path take over the step control
                    h = hmin;
                    flag = true;
                } else {
                    continue;
                }
            } else {
                float fac = (err == 0.0f) ? 5.0f : 0.9f * pow_m02(err);
                fac = fminf(5.0f, fmaxf(0.2f, fac));
                if (last_rej) fac = fminf(fac, 1.0f);
                hnext = fminf(h * fac, hmax);
            }
        }
        if (!flag) {
            if (ue.cell != u.cell) {
                xhi = (float)(hw - (double)ue.cell * L);
                xlo = (float)(-hw - (double)ue.cell * L);
            }
            float xr = ue.fx + ue.lx;
            flag = !st32_finite(ue) || (ue.y + ue.ly > ytop) || (xr > xhi) || (xr < xlo) ||
                   (mirror == 0 && ue.y + re.W.re * c.invk < 0.0f);
        }
        if (flag) {
            // hand the step (from its start u, size h) to the FP64 path
            const WfRays& R = a.R;
            R.cell[q] = u.cell;
            R.fx[q] = u.fx; R.lx[q] = u.lx;
            R.y[q] = u.y; R.ly[q] = u.ly;
            R.px[q] = u.px; R.lpx[q] = u.lpx;
            R.py[q] = u.py; R.lpy[q] = u.lpy;
            R.Wr[q] = r1.W.re; R.Wi[q] = r1.W.im;
            R.h[q] = h;
            R.tau[q] = tau; R.ltau[q] = ltau;
            R.steps[q] = steps;
            R.rej[q] = rej;
            R.flags[q] = last_rej ? WF_LAST_REJ : 0;
            if (bad) R.fbk[q] += 1;
            push(a.qev, &a.ctr->ev_len, q);
            active = false;
            continue;
        }
        comp_add(tau, ltau, h);
        u = ue;
        r1 = re;
        h = hnext;
        last_rej = false;
        ++my_steps;
        if (++steps >= max_steps) {
            const WfRays& R = a.R;
            R.steps[q] = steps;
            R.rej[q] = rej;
            R.status[q] = RS_MAX_STEPS;
            R.qx[q] = 0.0; R.qy[q] = 0.0; R.qz[q] = 0.0;
            R.rgb[3 * q + 0] = 0.0f; R.rgb[3 * q + 1] = 0.0f; R.rgb[3 * q + 2] = 0.0f;
            active = false;
        }
    }
    unsigned long long total = my_steps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off, 64);
    if (lane == 0) atomicAdd(&a.ctr->hot_steps, total);
}

// One flagged step of ray q in FP64 (step control, event location and
// handling).  Returns 0 if the ray is still inside the box (state stored),
// 1 if it left the box (air state stored in rx..qz), 2 if it finished.
template <int INTEG>
__device__ __forceinline__ int event_body(const WfArgs& a, long long q, const SceneDev& s)
{
    OptsDev o = a.o;
    o.integ = INTEG;
    Box64 b = load_box64(a, q, s);
    LaneCount cnt = {a.R.steps[q], a.R.rej[q], a.R.events[q], 0};
    double r[3], p[3], mc = 1.0;
    int st = RS_OK;
    int so = box_step64(s, o, b, cnt, &mc, r, p, &st);
    if (so == SO_INSIDE && cnt.steps >= o.max_steps) { so = SO_FAIL; st = RS_MAX_STEPS; }
    a.R.steps[q] = (int)cnt.steps;
    a.R.rej[q] = (int)cnt.rejected;
    a.R.events[q] = cnt.events;
    if (so == SO_FAIL) {
        double rr[3] = {b.u.x, b.u.y, b.z}, pp[3] = {0.0, 0.0, 0.0};
        finish_ray(a, q, s, st, rr, pp);
        return 2;
    }
    if (so == SO_INSIDE) {
        store_box64(a, q, s, b);
        return 0;
    }
    a.R.rx[q] = r[0]; a.R.ry[q] = r[1]; a.R.rz[q] = r[2];
    a.R.qx[q] = p[0]; a.R.qy[q] = p[1]; a.R.qz[q] = p[2];
    return 1;
}

// Ray q in air (state in rx..qz): walk to the box (state stored, returns 0)
// or finish it (returns 2).
__device__ __forceinline__ int air_body(const WfArgs& a, long long q, const SceneDev& s)
{
    double r[3] = {a.R.rx[q], a.R.ry[q], a.R.rz[q]};
    double p[3] = {a.R.qx[q], a.R.qy[q], a.R.qz[q]};
    LaneCount cnt = {a.R.steps[q], a.R.rej[q], a.R.events[q], 0};
    double mc = 1.0;
    int st = RS_OK;
    int ao = air_walk(s, a.o, r, p, cnt, &mc, &st);
    a.R.events[q] = cnt.events;
    if (ao == AO_FAIL) { finish_ray(a, q, s, st, r, p); return 2; }
    if (ao == AO_ESCAPED) { finish_ray(a, q, s, RS_OK, r, p); return 2; }
    Box64 b = box_enter64(s, a.o, r, p);
    store_box64(a, q, s, b);
    a.R.status[q] = RS_OK;
    return 0;
}

// FP64 events (INTEG fixes the integrator so that only one is compiled in).
template <int INTEG>
__global__ void __launch_bounds__(256) k_wf_event(WfArgs a, int cur)
{
    const unsigned qlen = a.ctr->ev_len;
    int* qnext = a.qbox[cur ^ 1];
    unsigned* qnext_len = &a.ctr->box_len[cur ^ 1];
    for (unsigned qi = blockIdx.x * blockDim.x + threadIdx.x; qi < qlen; qi += gridDim.x * blockDim.x) {
        const long long q = a.qev[qi];
        const SceneDev s = a.scenes[a.R.scene[q]];
        int r = event_body<INTEG>(a, q, s);
        if (r == 0) push(qnext, qnext_len, (int)q);
        else if (r == 1) push(a.qair, &a.ctr->air_len, (int)q);
    }
}

// Rays that left the box this round: walk through air (FP64).
__global__ void __launch_bounds__(256) k_wf_air(WfArgs a, int cur)
{
    const unsigned qlen = a.ctr->air_len;
    int* qnext = a.qbox[cur ^ 1];
    unsigned* qnext_len = &a.ctr->box_len[cur ^ 1];
    for (unsigned qi = blockIdx.x * blockDim.x + threadIdx.x; qi < qlen; qi += gridDim.x * blockDim.x) {
        const long long q = a.qair[qi];
        const SceneDev s = a.scenes[a.R.scene[q]];
        if (air_body(a, q, s) == 0) push(qnext, qnext_len, (int)q);
    }
}

// FP32 in-cloak steps of one ray from its stored state until a step needs
// the FP64 path (returns 0, state of the step start stored) or the step cap
// is reached (returns 2, ray finished).
template <int INTEG>
__device__ __forceinline__ int hot_body(const WfArgs& a, long long q, const SceneDev& s)
{
    const WfRays& R = a.R;
    const Sc32 c = make_sc32(s, a.o.wfb2);
    const float rtol = (float)a.o.rtol, atol = (float)a.o.atol;
    const float hmax = (float)a.o.h_max, hmin = (float)a.o.h_min;
    const int max_steps = a.o.max_steps > 0x7fffffffll ? 0x7fffffff : (int)a.o.max_steps;
    const float ytop = (float)s.ytop;
    St32 u;
    u.cell = R.cell[q];
    u.fx = R.fx[q]; u.lx = R.lx[q];
    u.y = R.y[q]; u.ly = R.ly[q];
    u.px = R.px[q]; u.lpx = R.lpx[q];
    u.py = R.py[q]; u.lpy = R.lpy[q];
    float h = R.h[q], tau = R.tau[q], ltau = R.ltau[q];
    int steps = R.steps[q], rej = R.rej[q];
    bool last_rej = (R.flags[q] & WF_LAST_REJ) != 0;
    float xhi = (float)(s.hw - (double)u.cell * s.L), xlo = (float)(-s.hw - (double)u.cell * s.L);
    Rhs32 r1;
    r1.W = {R.Wr[q], R.Wi[q]};
    refresh32(c, u.fx, u.y, r1);
    for (;;) {
        St32 ue;
        Rhs32 re;
        bool bad = false, flag = false;
        float hnext = h;
        if (INTEG == 0) {
            rk4_step32(c, u, r1, h, ue, re, bad);
            flag = bad;
        } else {
            float err = dp5_step32(c, u, r1, h, rtol, atol, ue, re, bad);
            if (bad || !isfinite(err)) {
                flag = true;
            } else if (err > 1.0f) {
                h *= fmaxf(0.2f, 0.9f * pow_m02(err));
                last_rej = true;
                ++rej;
                if (h < hmin) { h = hmin; flag = true; } else continue;
            } else {
                float fac = (err == 0.0f) ? 5.0f : 0.9f * pow_m02(err);
                fac = fminf(5.0f, fmaxf(0.2f, fac));
                if (last_rej) fac = fminf(fac, 1.0f);
                hnext = fminf(h * fac, hmax);
            }
        }
        if (!flag) {
            if (ue.cell != u.cell) {
                xhi = (float)(s.hw - (double)ue.cell * s.L);
                xlo = (float)(-s.hw - (double)ue.cell * s.L);
            }
            float xr = ue.fx + ue.lx;
            flag = !st32_finite(ue) || (ue.y + ue.ly > ytop) || (xr > xhi) || (xr < xlo) ||
                   (s.mirror == 0 && ue.y + re.W.re * c.invk < 0.0f);
        }
        if (flag) {
            R.cell[q] = u.cell;
            R.fx[q] = u.fx; R.lx[q] = u.lx;
            R.y[q] = u.y; R.ly[q] = u.ly;
            R.px[q] = u.px; R.lpx[q] = u.lpx;
            R.py[q] = u.py; R.lpy[q] = u.lpy;
            R.Wr[q] = r1.W.re; R.Wi[q] = r1.W.im;
            R.h[q] = h;
            R.tau[q] = tau; R.ltau[q] = ltau;
            R.steps[q] = steps;
            R.rej[q] = rej;
            R.flags[q] = last_rej ? WF_LAST_REJ : 0;
            if (bad) R.fbk[q] += 1;
            return 0;
        }
        comp_add(tau, ltau, h);
        u = ue;
        r1 = re;
        h = hnext;
        last_rej = false;
        if (++steps >= max_steps) {
            R.steps[q] = steps;
            R.rej[q] = rej;
            R.status[q] = RS_MAX_STEPS;
            R.qx[q] = 0.0; R.qy[q] = 0.0; R.qz[q] = 0.0;
            R.rgb[3 * q + 0] = 0.0f; R.rgb[3 * q + 1] = 0.0f; R.rgb[3 * q + 2] = 0.0f;
            return 2;
        }
    }
}

// The last rays of a launch: few enough that round barriers would leave most
// of the GPU idle while the slowest of them sets each round's length.  Each
// is finished here in one go (FP32 steps, FP64 events, air), spread over
// `lanes` lanes per wave so that they occupy all SIMDs.
template <int INTEG>
__global__ void __launch_bounds__(64) k_wf_tail(WfArgs a, int cur, int lanes)
{
    if ((int)threadIdx.x >= lanes) return;
    const unsigned qlen = a.ctr->box_len[cur];
    const unsigned qi = blockIdx.x * (unsigned)lanes + threadIdx.x;
    if (qi >= qlen) return;
    const long long q = a.qbox[cur][qi];
    const SceneDev s = a.scenes[a.R.scene[q]];
    for (int guard = 0; guard < (1 << 20); ++guard) {
        if (hot_body<INTEG>(a, q, s) == 2) return;
        int r = event_body<INTEG>(a, q, s);
        if (r == 2) return;
        if (r == 1 && air_body(a, q, s) == 2) return;
    }
}

// Pixel averages (render mode) and counters.
struct WfTotals {
    unsigned long long rays, steps, rejected, events, failed, fallbacks;
};

__global__ void __launch_bounds__(256) k_wf_finish(WfArgs a, float* const* images, const long long* pix_off,
                                                   long long n_pix, WfTotals* tot)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c_rays = 0, c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_fb = 0;
    if (g < n_pix) {
        int lo = 0, hi = a.n_scenes - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (pix_off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const int si = lo;
        const int spp = a.cams[si].spp;
        const long long local = g - pix_off[si];
        const long long q0 = a.ray_off[si] + local * spp;
        float acc[3] = {0.f, 0.f, 0.f};
        for (int smp = 0; smp < spp; ++smp) {
            long long q = q0 + smp;
            acc[0] += a.R.rgb[3 * q + 0];
            acc[1] += a.R.rgb[3 * q + 1];
            acc[2] += a.R.rgb[3 * q + 2];
            c_rays++;
            c_steps += (unsigned)a.R.steps[q];
            c_rej += (unsigned)a.R.rej[q];
            c_ev += (unsigned)a.R.events[q];
            c_fail += a.R.status[q] != RS_OK;
            c_fb += (unsigned)a.R.fbk[q];
        }
        float inv = 1.0f / (float)spp;
        float* img = images[si];
        for (int k = 0; k < 3; ++k) img[3 * local + k] = acc[k] * inv;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c_rays += __shfl_xor(c_rays, off, 64);
        c_steps += __shfl_xor(c_steps, off, 64);
        c_rej += __shfl_xor(c_rej, off, 64);
        c_ev += __shfl_xor(c_ev, off, 64);
        c_fail += __shfl_xor(c_fail, off, 64);
        c_fb += __shfl_xor(c_fb, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&tot->fallbacks, c_fb);
        atomicAdd(&tot->rays, c_rays);
        atomicAdd(&tot->steps, c_steps);
        atomicAdd(&tot->rejected, c_rej);
        atomicAdd(&tot->events, c_ev);
        atomicAdd(&tot->failed, c_fail);
    }
}

// trace_rays mode: copy the exit rays out and fold the counters.
__global__ void __launch_bounds__(256) k_wf_trace_out(WfArgs a, double* out_org, double* out_dir, int* status,
                                                      long long* steps, int* events, WfTotals* tot)
{
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c_rays = 0, c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_fb = 0;
    if (q < a.n_rays) {
        if (out_org) { out_org[3 * q] = a.R.rx[q]; out_org[3 * q + 1] = a.R.ry[q]; out_org[3 * q + 2] = a.R.rz[q]; }
        out_dir[3 * q] = a.R.qx[q];
        out_dir[3 * q + 1] = a.R.qy[q];
        out_dir[3 * q + 2] = a.R.qz[q];
        if (status) status[q] = a.R.status[q];
        if (steps) steps[q] = a.R.steps[q];
        if (events) events[q] = a.R.events[q];
        c_rays = 1;
        c_steps = (unsigned)a.R.steps[q];
        c_rej = (unsigned)a.R.rej[q];
        c_ev = (unsigned)a.R.events[q];
        c_fail = a.R.status[q] != RS_OK;
        c_fb = (unsigned)a.R.fbk[q];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c_rays += __shfl_xor(c_rays, off, 64);
        c_steps += __shfl_xor(c_steps, off, 64);
        c_rej += __shfl_xor(c_rej, off, 64);
        c_ev += __shfl_xor(c_ev, off, 64);
        c_fail += __shfl_xor(c_fail, off, 64);
        c_fb += __shfl_xor(c_fb, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&tot->fallbacks, c_fb);
        atomicAdd(&tot->rays, c_rays);
        atomicAdd(&tot->steps, c_steps);
        atomicAdd(&tot->rejected, c_rej);
        atomicAdd(&tot->events, c_ev);
        atomicAdd(&tot->failed, c_fail);
    }
}

}  // namespace gc
