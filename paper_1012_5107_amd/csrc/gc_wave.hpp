// gc_wave.hpp -- the FP32 render/trace pipeline as queue-driven kernels.
//
// A sample's path alternates between flights through air (FP64: straight
// lines to the cloak box, contacts with the bare grating by root finding)
// and visits of the box (FP32 integration).  The two have very different
// register footprints, so they are separate kernels that pass rays through
// queues of ray indices:
//
//   k_wf_init    a few samples per lane: camera ray (or given ray), flight
//                through air to the box, the sky, or a failure; a ray whose
//                first leg meets the bare grating goes to the air queue;
//   k_wf_box     persistent FP32 kernel: each wave claims rays from the box
//                queue (one atomic per wave, ballot + rank for the lanes)
//                and integrates each through its whole visit of the box:
//                steps, the location of each event on the partial steps of
//                the same integrator, grating reflections and total
//                internal reflections; a ray that leaves the box straight
//                to the sky is finished here, any other that leaves goes to
//                the air queue, a ray whose next step needs FP64 (a stage
//                point near the branch point or a path across the branch
//                cut) goes to the FP64 queue, and the lane takes a new ray;
//   k_wf_event   FP64: that step (with step control and any event in it);
//                the ray goes on in the next round's box queue;
//   k_wf_air     FP64: the air queue's flights to the box (next box queue),
//                the bare grating, the sky or a failure;
//   k_wf_finish  averages each pixel's samples and folds the counters.
//
// Rounds of (k_wf_box, k_wf_event, k_wf_air) repeat until the box queue is
// empty; a ray needs one round per visit of the box (one or two for almost
// all), plus one per FP64 step.
// Samples of several scenes can share one launch: every ray carries its
// scene index and the scene / camera tables live in device memory.
#pragma once
#include "gc_lane32.hpp"
#include "gc_lane64.hpp"

namespace gc {

struct WfTotals {
    unsigned long long rays, steps, rejected, events, failed, fallbacks;
};
static_assert(sizeof(WfTotals) == 6 * sizeof(unsigned long long), "six consecutive counters");

struct QCtr {
    unsigned box_len[2];
    unsigned box_head[2];
    unsigned slow_len[2];           // the slow box queue of each round
    unsigned slow_head[2];
    unsigned ev_len;
    unsigned ev_head;
    unsigned air_len;               // rays whose walk through air needs the contact search
    unsigned rec_len;               // long first visits recorded (see WfArgs::rec)
    unsigned long long hot_steps;   // accepted steps taken by k_wf_box (all rounds)
    unsigned seed_len;              // Fresnel branches spawned (slots requested)
};

// per-ray arrays (structure of arrays)
struct WfRays {
    double *rx, *ry, *rz, *qx, *qy, *qz;   // air state / exit point and direction
    double* z0;                             // z at the last box entry or event
    int* cell;
    float *fx, *lx, *y, *ly, *px, *lpx, *py, *lpy, *pz, *Wr, *Wi, *h, *tau, *ltau;
    int *steps, *rej, *events, *flags, *scene, *status, *fbk;
    float* rgb;   // 3 per ray
    // Fresnel-weighted faces: the path's weight, and for a reflected branch
    // (the slots from seed_base on) its sample's primary ray and the steps
    // it inherited from it
    double* wgt;
    int *parent, *steps0;
};

// WF_FIRST_VISIT: the ray entered the box from k_wf_init (its first visit,
// in round 0's queues) and has not been handed to the FP64 kernel since
// WF_SEED_INSIDE: a Fresnel branch that starts inside the box (reflected
// at an exit face)
enum WfFlag { WF_LAST_REJ = 1, WF_FIRST_VISIT = 2, WF_SEED_INSIDE = 4 };

// Scheduling of the in-box kernel (what is computed does not depend on it).
struct WfSched {
    float slow_pxy2;   // a box entry with d_x^2 + d_y^2 below this goes to the slow queue
    int slow_div;      // every slow_div-th wave takes the slow queue first (0: none)
    int refill;        // idle lanes that make a wave claim new rays
};

struct WfArgs {
    WfRays R;
    int* qbox[2];
    int* qslow[2];     // box entries predicted to take many steps
    WfSched sch;
    int* qev;
    int* qair;         // rays in air (state in rx..qz) for the air kernel
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
    // Rays that k_wf_init puts at the front of round 0's fast box queue (so
    // that they are claimed first): a bitmap over the rays, their indices in
    // ascending order and the slot of each (n_front slots, filled with -1 by
    // k_wf_zero).  A batch plan sets them from its eager run: the visits that
    // took longest there, which would otherwise start wherever the queue
    // order puts them and end the launch late.
    const unsigned* front_bits;
    const int* front_q;
    const int* front_slot;
    int n_front;
    // Recording (null: off): k_wf_box appends (ray, steps) for every first
    // visit of at least rec_min steps, up to rec_cap pairs.
    int* rec;
    unsigned rec_cap;
    int rec_min;
    // Fresnel branches (render mode, scenes with fresnel = 1): a primary ray
    // that crosses a face appends its reflected part to the slots
    // [seed_base, seed_base + seed_cap); seed_cap = 0: no branches
    long long seed_base;
    unsigned seed_cap;
};

// A ray is a reflected branch when its slot lies in the branch pool.
__device__ __forceinline__ bool is_branch(const WfArgs& a, long long q) { return a.seed_cap > 0 && q >= a.seed_base; }

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

// The box queue a ray entering the box goes to (0 fast, 1 slow).  Its
// direction at the entry predicts the length of the visit: with a small
// in-plane part the ray crosses the box slowly in tau (p_z is conserved and
// the step is capped in tau).
__device__ __forceinline__ int box_dest(const WfArgs& a, const double p[3])
{
    const double pxy2 = p[0] * p[0] + p[1] * p[1];
    return pxy2 < (double)a.sch.slow_pxy2 * (pxy2 + p[2] * p[2]) ? 1 : 0;
}

// Append q to the next round's fast (dest 0) or slow (dest 1) box queue,
// one atomic per wave and queue.  Every active lane of the wave calls it
// together (dest < 0: nothing to append).
__device__ __forceinline__ void push_box_wave(const WfArgs& a, int nxt, int dest, int q)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long m0 = __ballot(dest == 0), m1 = __ballot(dest == 1);
    const int leader = __ffsll((long long)__ballot(1)) - 1;
    unsigned b0 = 0, b1 = 0;
    if (lane == leader) {
        if (m0) b0 = atomicAdd(&a.ctr->box_len[nxt], (unsigned)__popcll(m0));
        if (m1) b1 = atomicAdd(&a.ctr->slow_len[nxt], (unsigned)__popcll(m1));
    }
    b0 = __shfl(b0, leader, 64);
    b1 = __shfl(b1, leader, 64);
    if (dest == 0) a.qbox[nxt][b0 + (unsigned)__popcll(m0 & below)] = q;
    else if (dest == 1) a.qslow[nxt][b1 + (unsigned)__popcll(m1 & below)] = q;
}

// Append q to the air queue where `want` holds, one atomic per wave.  Every
// active lane of the wave calls it together.
__device__ __forceinline__ void push_air_wave(const WfArgs& a, bool want, int q)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long m = __ballot(want);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    unsigned b = 0;
    if (lane == leader) b = atomicAdd(&a.ctr->air_len, (unsigned)__popcll(m));
    b = __shfl(b, leader, 64);
    if (want) a.qair[b + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = q;
}

// The first leg of a walk through air from (r, p) needs no search for a
// contact with the bare grating: the metal is flat, or the ray moves up from
// above its highest point, or it enters through the top face above it.
// (Only decides which kernel walks the ray; the walk is the same.)
__device__ __forceinline__ bool air_leg_plain(const SceneDev& s, const double r[3], const double p[3])
{
    if (s.mirror == 1 || s.A == 0.0) return true;
    if (p[1] > 0.0 && r[1] >= s.A) return true;
    int face;
    air_box_entry(s, r, p, &face);
    return face == 0 && s.ytop > s.A;
}

// The walk through air from (r, p) ends at once with an escape (no face, no
// metal ahead): exactly the case in which air_walk returns AO_ESCAPED without
// an event.
__device__ __forceinline__ bool air_escapes_now(const SceneDev& s, const double r[3], const double p[3])
{
    if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]) && isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])))
        return false;
    if (!(p[1] > 0.0 && (s.mirror == 1 || s.A == 0.0 || r[1] >= s.A))) return false;
    int face;
    return !(air_box_entry(s, r, p, &face) < kInf);
}

// In-box state at an entry for the queues.  Only W (at the entry point, from
// the walk through air) is stored: the kernel that takes the ray evaluates
// the field itself, so none is evaluated here.
__device__ __forceinline__ Box64 box_entry_state(const OptsDev& o, const double r[3], const double p[3],
                                                 cx<double> W)
{
    Box64 b;
    b.u = {r[0], r[1], p[0], p[1]};
    b.z = r[2];
    b.pz = p[2];
    b.r1.W = W;
    b.r1.ax = b.r1.ay = 0.0;
    b.r1.dW = {0.0, 0.0};
    b.h = (o.integ == 0) ? o.h : o.h0;
    b.last_rej = false;
    return b;
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
        if (s.backdrop == 0) {
            // the image is FP32: so is the sky lookup
            const float pf[3] = {(float)p[0], (float)p[1], (float)p[2]};
            sky_rgb<float>((float)s.K, pf, c3);
        } else {
            // the backdrop plane: where the ray meets it, from the FP64 exit
            backdrop_rgb_image(s, r, p, c3);
        }
        if (s.fresnel && a.seed_cap > 0) {
            // the path's share of the sample's light
            const double w = R.wgt[q];
            for (int c = 0; c < 3; ++c) c3[c] = (float)(w * (double)c3[c]);
        }
    }
    R.rgb[3 * q + 0] = c3[0];
    R.rgb[3 * q + 1] = c3[1];
    R.rgb[3 * q + 2] = c3[2];
}

// Fresnel split at a face crossing of ray q at r (Sec. 3): p1 the momentum
// on the incoming side, p2 the transmitted one.  A primary ray appends the
// reflected part (weight w R, on the incoming side: `inside` for an exit)
// to the branch pool with the counts it has reached; every ray goes on with
// weight w T.  Branches never split again.
__device__ __forceinline__ void fresnel_cross(const WfArgs& a, long long q, const double r[3], const double p1[3],
                                              const double p2[3], int face, bool inside, int steps, int rej,
                                              int events)
{
    const WfRays& R = a.R;
    double refl[3];
    const double Rf = crossing_R(face, p1, p2, refl);
    const double w = R.wgt[q];
    if (a.seed_cap > 0 && !is_branch(a, q)) {
        const unsigned k = atomicAdd(&a.ctr->seed_len, 1u);
        if (k < a.seed_cap) {
            const long long b = a.seed_base + (long long)k;
            R.rx[b] = r[0]; R.ry[b] = r[1]; R.rz[b] = r[2];
            R.qx[b] = refl[0]; R.qy[b] = refl[1]; R.qz[b] = refl[2];
            R.wgt[b] = w * Rf;
            R.parent[b] = (int)q;
            R.scene[b] = R.scene[q];
            R.steps[b] = steps;
            R.steps0[b] = steps;
            R.rej[b] = rej;
            R.events[b] = events;
            R.fbk[b] = 0;
            R.flags[b] = inside ? WF_SEED_INSIDE : 0;
            R.status[b] = RS_OK;
        }
    }
    R.wgt[q] = w * (1.0 - Rf);
}

// The pipeline's walk through air from (r, p): a plate is crossed on the
// way (straight FP64 flights), and with Fresnel every face crossing splits.
// Returns as air_walk does (a plate scene never returns AO_ENTERED).
__device__ __forceinline__ int wf_air_walk(const WfArgs& a, long long q, const SceneDev& s, double r[3], double p[3],
                                           LaneCount& cnt, int* st, cx<double>* W)
{
    double mc = 1.0;
    for (;;) {
        double pa[3];
        int face = 0;
        const int ao = air_walk(s, a.o, r, p, cnt, &mc, st, W, pa, &face);
        if (ao == AO_ENTERED && s.fresnel && a.seed_cap > 0)
            fresnel_cross(a, q, r, pa, p, face, false, (int)cnt.steps, (int)cnt.rejected, cnt.events);
        if (ao != AO_ENTERED || s.cloak != CK_PLATE) return ao;
        double pin[3];
        const int ps = plate_walk64(s, a.o, r, p, cnt, &mc, pin, &face);
        if (ps != RS_OK) { *st = ps; return AO_FAIL; }
        if (s.fresnel && a.seed_cap > 0)
            fresnel_cross(a, q, r, pin, p, face, true, (int)cnt.steps, (int)cnt.rejected, cnt.events);
    }
}

// Walk through air from (r, p) (a plate is crossed on the way) and either
// finish the ray (returns -1) or set up its in-box state (returns the box
// queue it goes to).
__device__ __forceinline__ int continue_in_air(const WfArgs& a, long long q, const SceneDev& s, double r[3],
                                               double p[3], LaneCount& cnt)
{
    int st = RS_OK;
    cx<double> W;
    int ao = wf_air_walk(a, q, s, r, p, cnt, &st, &W);
    a.R.events[q] = cnt.events;
    a.R.steps[q] = (int)cnt.steps;
    a.R.rej[q] = (int)cnt.rejected;
    if (ao == AO_FAIL) { finish_ray(a, q, s, st, r, p); return -1; }
    if (ao == AO_ESCAPED) { finish_ray(a, q, s, RS_OK, r, p); return -1; }
    Box64 b = box_entry_state(a.o, r, p, W);
    store_box64(a, q, s, b);
    a.R.status[q] = RS_OK;
    return box_dest(a, p);
}

// ---------------------------------------------------------------------------
// Counters to zero at the start of a launch (a kernel, not a memset, so
// that a captured graph holds no memset node).
__global__ void __launch_bounds__(64) k_wf_zero(QCtr* c, WfTotals* t, int* qfront, int n_front)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *c = QCtr{};
        *t = WfTotals{};
        c->box_len[0] = (unsigned)n_front;   // the reserved front of round 0's fast queue
    }
    for (int i = threadIdx.x; i < n_front; i += blockDim.x) qfront[i] = -1;
}

// Slot of ray q at the front of round 0's fast queue, or -1.
__device__ __forceinline__ int front_slot_of(const WfArgs& a, long long q)
{
    if (!((a.front_bits[q >> 5] >> (q & 31)) & 1u)) return -1;
    int lo = 0, hi = a.n_front - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.front_q[mid] < q) lo = mid + 1; else hi = mid;
    }
    return a.front_q[lo] == q ? a.front_slot[lo] : -1;
}

__global__ void __launch_bounds__(256) k_wf_reset(QCtr* c, int cur)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->box_head[cur] = 0;
        c->box_len[cur ^ 1] = 0;
        c->box_head[cur ^ 1] = 0;
        c->slow_head[cur] = 0;
        c->slow_len[cur ^ 1] = 0;
        c->slow_head[cur ^ 1] = 0;
        c->ev_len = 0;
        c->ev_head = 0;
        c->air_len = 0;
    }
}

// Returns the box queue of the ray (-1: none); *deferred: the ray's first
// leg through air needs the contact search, its state is stored for the air
// kernel (so that the few such lanes do not hold up whole waves here).
__device__ __forceinline__ int init_ray(const WfArgs& a, long long q, bool* deferred)
{
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
    a.R.flags[q] = 0;
    a.R.fbk[q] = 0;
    if (a.seed_cap > 0) a.R.wgt[q] = 1.0;
    a.R.steps[q] = 0;
    a.R.rej[q] = 0;
    if (!air_leg_plain(s, r, p)) {
        a.R.events[q] = 0;
        a.R.rx[q] = r[0]; a.R.ry[q] = r[1]; a.R.rz[q] = r[2];
        a.R.qx[q] = p[0]; a.R.qy[q] = p[1]; a.R.qz[q] = p[2];
        *deferred = true;
        return -1;
    }
    LaneCount cnt = {0, 0, 0, 0};
    return continue_in_air(a, q, s, r, p, cnt);
}

// k_wf_init: camera (or given) rays and their flight to the box, kInitRays
// samples per lane.  Its appends to the three queues (fast box, slow box,
// air) take one atomic per block and queue: atomics on the queue counters
// are performed one at a time, and at one per wave they bounded the kernel.
constexpr int kInitRays = 4;

// Queue k (0 fast box, 1 slow box, 2 air) of the 3-bit code r of a lane:
// bits 0-1 the box queue + 1 (0: none), bit 2 the air queue.
__device__ __forceinline__ bool init_in_queue(unsigned codes, int r, int k)
{
    const unsigned c = (codes >> (3 * r)) & 7u;
    return k == 2 ? (c & 4u) != 0 : (c & 3u) == (unsigned)(k + 1);
}

__global__ void __launch_bounds__(256) k_wf_init(WfArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long q0 = (long long)blockIdx.x * (blockDim.x * kInitRays) + threadIdx.x;
    // the rays q0 + r * blockDim.x, r < kInitRays (coalesced for each r)
    unsigned codes = 0;
#pragma unroll 1
    for (int r = 0; r < kInitRays; ++r) {
        const long long q = q0 + (long long)r * blockDim.x;
        if (q >= a.n_rays) continue;
        bool deferred = false;
        int dest = init_ray(a, q, &deferred);
        if (dest >= 0) {
            a.R.flags[q] |= WF_FIRST_VISIT;
            const int slot = a.n_front > 0 ? front_slot_of(a, q) : -1;
            if (slot >= 0) {
                a.qbox[0][slot] = (int)q;
                dest = -1;
            }
        }
        codes |= ((unsigned)(dest + 1) | (deferred ? 4u : 0u)) << (3 * r);
    }
    // wave counts per queue, block totals in LDS, one atomic per queue
    unsigned cnt[3] = {0, 0, 0};
#pragma unroll
    for (int r = 0; r < kInitRays; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) cnt[k] += (unsigned)__popcll(__ballot(init_in_queue(codes, r, k)));
    __shared__ unsigned wcnt[4][3], base[3];
    if (lane == 0)
        for (int k = 0; k < 3; ++k) wcnt[wave][k] = cnt[k];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        unsigned tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wcnt[w][k];
        unsigned* len = k == 0 ? &a.ctr->box_len[0] : (k == 1 ? &a.ctr->slow_len[0] : &a.ctr->air_len);
        base[k] = tot ? atomicAdd(len, tot) : 0u;
    }
    __syncthreads();
    unsigned off[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        off[k] = base[k];
        for (int w = 0; w < wave; ++w) off[k] += wcnt[w][k];
    }
    int* const queue[3] = {a.qbox[0], a.qslow[0], a.qair};
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < kInitRays; ++r) {
        const int q = (int)(q0 + (long long)r * blockDim.x);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const bool in = init_in_queue(codes, r, k);
            const unsigned long long m = __ballot(in);
            if (in) queue[k][off[k] + (unsigned)__popcll(m & below)] = q;
            off[k] += (unsigned)__popcll(m);
        }
    }
}

// In-box event location in FP32: regula falsi with the Illinois
// modification on the step fraction theta, on the partial steps of the same
// integrator.  It ends at the FP32 resolution of theta or, for the grating,
// when the upper end of the bracket is on the surface to the FP32 error of W
// (a trial that lands on the surface to that error from the inside is
// followed by one just across it).
constexpr float kLocTol = 2.0e-7f;
constexpr float kLocNoiseW = 2.4e-7f;
constexpr int kLocMaxIt = 40;

// The hot kernel.  INTEG: 0 RK4, 1 DOPRI5.  Every iteration evaluates one
// step per lane: a normal step of length h, or a trial of the location of
// the event that the lane's last accepted step crossed (length theta h), so
// that lanes locating an event do not hold the others up.
//
// Rays come from two queues, the slow one holding the box entries that are
// predicted to take many steps.  A visit cannot be split, so the longest
// visits set the length of the launch unless they start early and run
// fast: every slow_div-th wave takes the slow queue first, and a wave that
// holds slow rays raises its issue priority on its SIMD.
template <int INTEG>
__global__ void __launch_bounds__(256) k_wf_box(WfArgs a, int cur)
{
    const unsigned qlen0 = a.ctr->box_len[cur], qlen1 = a.ctr->slow_len[cur];
    const int lane = threadIdx.x & 63;
    const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const unsigned kRefill = (unsigned)a.sch.refill;
    const float rtol = (float)a.o.rtol, atol = (float)a.o.atol;
    const float hmax = (float)a.o.h_max, hmin = (float)a.o.h_min;
    const int max_steps = a.o.max_steps > 0x7fffffffll ? 0x7fffffff : (int)a.o.max_steps;
    const int max_ev = a.o.max_events;

    bool active = false;
    // a wave that finds a queue already drained does not touch its counter
    bool ex0 = *((volatile unsigned*)&a.ctr->box_head[cur]) >= qlen0;
    bool ex1 = *((volatile unsigned*)&a.ctr->slow_head[cur]) >= qlen1;
    bool exhausted = ex0 && ex1;
    // the queue this wave claims from (1: slow)
    int src = (a.sch.slow_div > 0 && wave % a.sch.slow_div == 0) ? 1 : 0;
    if (src == 1 ? ex1 : ex0) src ^= 1;
    bool slow_ray = false, prio = false;
    bool rec0 = false;      // the lane's visit is the ray's first (recording)
    int q = 0;
    const SceneDev* sp = a.scenes;
    double s_hw = 0.0, s_L = 1.0;   // the lane's scene: half-width and period, kept in registers
    Sc32 c;
    float ytop = 0.f, xhi = 0.f, xlo = 0.f, pz = 0.f, h = 0.f, tau = 0.f, ltau = 0.f;
    St32 u;
    Rhs32 r1;
    int steps = 0, rej = 0, nev = 0, fbk = 0, mirror = 0;
    bool last_rej = false;
    double z0 = 0.0;
    // event location
    bool loc = false, lfin = false;
    float th = 0.f, tlo = 0.f, thi = 1.f, flo = 0.f, fhi = 0.f, hacc = 0.f, hnx = 0.f;
    int side = 0, emask = 0, lit = 0, hicode = -1;
    bool need64 = false;   // the next step from u needs FP64
    unsigned my_steps = 0;
    // a lane whose visit has ended: 0 none, 1 + the face it left through, or
    // 16 + its failure status.  The lane is idle until the wave refills, so
    // its exit is written then, together with the other lanes' (once per
    // refill instead of once per iteration in which some lane finishes).
    int pend = 0;

    for (;;) {
        if (__ballot(pend != 0)) {
            const unsigned long long idle = __ballot(!active);
            if (exhausted || (unsigned)__popcll(idle) >= kRefill || __ballot(active) == 0ull) {
                bool to_air = false;
                if (pend != 0) {
                    // the ray's exit from the box: a point and direction in air
                    const WfRays& R = a.R;
                    double r[3] = {(double)u.cell * sp->L + ((double)u.fx + (double)u.lx),
                                   (double)u.y + (double)u.ly, z0 + (double)pz * ((double)tau + (double)ltau)};
                    R.steps[q] = steps;
                    R.rej[q] = rej;
                    R.events[q] = nev;
                    R.fbk[q] = fbk;
                    if (rec0 && a.rec && steps >= a.rec_min) {
                        const unsigned k = atomicAdd(&a.ctr->rec_len, 1u);
                        if (k < a.rec_cap) { a.rec[2 * k] = q; a.rec[2 * k + 1] = steps; }
                    }
                    if (pend >= 16) {
                        const double zero[3] = {0.0, 0.0, 0.0};
                        finish_ray(a, q, *sp, pend - 16, r, zero);
                    } else {
                        // the refraction out of the face, recomputed from the
                        // same state as when the event was applied
                        double p3[3] = {(double)u.px + (double)u.lpx, (double)u.py + (double)u.lpy, (double)pz};
                        double nf[3] = {0.0, 0.0, 0.0};
                        const int face = pend - 1;
                        if (face == 0) nf[1] = 1.0; else if (face == 1) nf[0] = 1.0; else nf[0] = -1.0;
                        const double pin[3] = {p3[0], p3[1], p3[2]};
                        snell(p3, nf, 1.0);
                        if (sp->fresnel && a.seed_cap > 0) fresnel_cross(a, q, r, pin, p3, face, true, steps, rej, nev);
                        if (air_escapes_now(*sp, r, p3)) {
                            // nothing ahead: the sky, as the air kernel would
                            finish_ray(a, q, *sp, RS_OK, r, p3);
                        } else {
                            R.rx[q] = r[0]; R.ry[q] = r[1]; R.rz[q] = r[2];
                            R.qx[q] = p3[0]; R.qy[q] = p3[1]; R.qz[q] = p3[2];
                            to_air = true;
                        }
                    }
                    pend = 0;
                }
                push_air_wave(a, to_air, q);
            }
        }
        if (!exhausted) {
            unsigned long long idle = __ballot(!active);
            // claim in batches: one atomic per wave for at least kRefill lanes
            // (or for all of them once the wave has run dry)
            const unsigned long long busy = __ballot(active);
            if (idle && ((unsigned)__popcll(idle) >= kRefill || busy == 0ull)) {
                int n = __popcll(idle);
                int leader = __ffsll((long long)idle) - 1;
                const int from = src;
                const unsigned qlen = from ? qlen1 : qlen0;
                const int* queue = from ? a.qslow[cur] : a.qbox[cur];
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(from ? &a.ctr->slow_head[cur] : &a.ctr->box_head[cur], (unsigned)n);
                base = __shfl(base, leader, 64);
                if (base + (unsigned)n >= qlen) {
                    // this queue is drained: the idle lanes left over claim
                    // from the other one on the next iteration
                    if (from) ex1 = true; else ex0 = true;
                    exhausted = ex0 && ex1;
                    src ^= 1;
                }
                if (!active) {
                    unsigned rank = __popcll(idle & ((1ull << lane) - 1ull));
                    unsigned qi = base + rank;
                    // (a reserved front slot holds -1 if its ray did not come)
                    const int qn = qi < qlen ? queue[qi] : -1;
                    if (qn >= 0) {
                        q = qn;
                        // the rays at the front of round 0's fast queue run
                        // with raised priority, as the slow queue's do
                        slow_ray = from != 0 || (cur == 0 && qi < (unsigned)a.n_front);
                        const WfRays& R = a.R;
                        sp = a.scenes + R.scene[q];
                        const SceneDev& s = *sp;
                        s_hw = s.hw;
                        s_L = s.L;
                        c = make_sc32(s, a.o.wfb2);
                        ytop = (float)s.ytop;
                        mirror = s.mirror;
                        u.cell = R.cell[q];
                        u.fx = R.fx[q]; u.lx = R.lx[q];
                        u.y = R.y[q]; u.ly = R.ly[q];
                        u.px = R.px[q]; u.lpx = R.lpx[q];
                        u.py = R.py[q]; u.lpy = R.lpy[q];
                        pz = R.pz[q];
                        z0 = R.z0[q];
                        h = R.h[q];
                        tau = R.tau[q];
                        ltau = R.ltau[q];
                        steps = R.steps[q];
                        rej = R.rej[q];
                        nev = R.events[q];
                        fbk = R.fbk[q];
                        const int fl = R.flags[q];
                        last_rej = (fl & WF_LAST_REJ) != 0;
                        rec0 = (fl & WF_FIRST_VISIT) != 0;
                        xhi = (float)(s.hw - (double)u.cell * s.L);
                        xlo = (float)(-s.hw - (double)u.cell * s.L);
                        r1.W = {R.Wr[q], R.Wi[q]};
                        halley32(c, u.fx, u.y, r1.W);
                        need64 = !(accel32(c, r1) >= c.wfb2);
                        loc = false;
                        active = true;
                    }
                }
            }
        }
        if (__ballot(active) == 0ull) break;
        {
            const bool hp = __ballot(active && slow_ray) != 0ull;
            if (hp != prio) {
                prio = hp;
                if (hp) __builtin_amdgcn_s_setprio(2); else __builtin_amdgcn_s_setprio(0);
            }
        }
        if (!active) continue;

        int fin = -1;           // >= 0: the ray finishes with this status
        bool leaves = false;    // the ray left the box
        int lface = 0;          // ... through this face
        double p3[3] = {0.0, 0.0, 0.0};
        if (!loc && steps >= max_steps) {
            fin = RS_MAX_STEPS;
        } else if (!need64) {
            const float tstep = loc ? th * hacc : h;
            St32 ue;
            Rhs32 re;
            float err = 0.0f;
            bool bad = false;
            if (INTEG == 0)
                rk4_step32(c, u, r1, tstep, ue, re, bad);
            else
                err = dp5_step32(c, u, r1, tstep, rtol, atol, ue, re, bad);
            if (bad || !st32_finite(ue) || (INTEG == 1 && !loc && !isfinite(err))) {
                // this step (from u, of length h; the accepted length when
                // locating) goes to the FP64 path
                if (loc) h = hacc;
                loc = false;
                need64 = true;
                ++fbk;
            } else {
                float xh = xhi, xl = xlo;
                if (ue.cell != u.cell) {
                    xh = (float)(s_hw - (double)ue.cell * s_L);
                    xl = (float)(-s_hw - (double)ue.cell * s_L);
                }
                float e[4];
                ev_values32(c, ue, re, ytop, xh, xl, mirror, e);
                bool apply = false;
                int evc = -1;
                bool take = false;
                float hnew = 0.0f;
                if (!loc) {
                    float hnext = h;
                    bool accepted = true;
                    if (INTEG == 1) {
                        if (err > 1.0f) {
                            h *= fmaxf(0.2f, 0.9f * pow_m02(err));
                            last_rej = true;
                            ++rej;
                            accepted = false;
                            if (h < hmin) fin = RS_UNDERFLOW;
                        } else {
                            float fac = (err == 0.0f) ? 5.0f : 0.9f * pow_m02(err);
                            fac = fminf(5.0f, fmaxf(0.2f, fac));
                            if (last_rej) fac = fminf(fac, 1.0f);
                            last_rej = false;
                            hnext = fminf(h * fac, hmax);
                        }
                    }
                    if (accepted) {
                        ++steps;
                        ++my_steps;
                        emask = (e[0] < 0.0f ? 1 : 0) | (e[1] < 0.0f ? 2 : 0) | (e[2] < 0.0f ? 4 : 0) |
                                (e[3] < 0.0f ? 8 : 0);
                        if (!emask) {
                            comp_add(tau, ltau, h);
                            take = true;
                            hnew = hnext;
                        } else {
                            // the step crossed an event: locate it on the
                            // partial steps of the next iterations
                            float e0[4];
                            int c0;
                            ev_values32(c, u, r1, ytop, xhi, xlo, mirror, e0);
                            flo = fmaxf(ev_min32(e0, emask, &c0), 0.0f);
                            fhi = ev_min32(e, emask, &hicode);
                            tlo = 0.0f;
                            thi = 1.0f;
                            side = 0;
                            lit = 0;
                            lfin = false;
                            hacc = h;
                            hnx = hnext;
                            th = (flo - fhi > 0.0f) ? flo * __builtin_amdgcn_rcpf(flo - fhi) : 0.5f;
                            if (!(th > 0.0f && th < 1.0f)) th = 0.5f;
                            loc = true;
                        }
                    }
                } else {
                    // a trial of the location at theta = th
                    int code;
                    const float f = ev_min32(e, emask, &code);
                    if (lfin) {
                        apply = true;   // the recomputed upper end of the bracket
                        evc = f < 0.0f ? code : hicode;
                    } else {
                        if (f < 0.0f) {
                            thi = th;
                            fhi = f;
                            hicode = code;
                            if (side < 0) flo *= 0.5f;
                            side = -1;
                            apply = (code == 3 && f >= -kLocNoiseW);
                        } else {
                            tlo = th;
                            flo = f;
                            if (side > 0) fhi *= 0.5f;
                            side = 1;
                        }
                        ++lit;
                        if (!apply && (thi - tlo <= kLocTol || lit >= kLocMaxIt)) {
                            if (side < 0) {
                                apply = true;   // this trial is the upper end
                            } else {
                                th = thi;       // recompute the upper end next
                                lfin = true;
                            }
                        } else if (!apply) {
                            float t;
                            if (side > 0 && hicode == 3 && flo <= kLocNoiseW) {
                                const float sl = (fhi - flo) * __builtin_amdgcn_rcpf(thi - tlo);
                                t = tlo + fmaxf(2.0f * kLocNoiseW * __builtin_amdgcn_rcpf(fabsf(sl)), kLocTol);
                            } else {
                                t = (flo - fhi > 0.0f) ? (flo * thi - fhi * tlo) * __builtin_amdgcn_rcpf(flo - fhi)
                                                       : 0.5f * (tlo + thi);
                            }
                            if (lit >= 20 || !(t > tlo && t < thi)) t = 0.5f * (tlo + thi);
                            th = t;
                        }
                        evc = code;
                    }
                }
                if (apply) {
                    comp_add(tau, ltau, th * hacc);
                    take = true;
                    hnew = hnx;
                    loc = false;
                }
                if (take) {
                    // the step (or the located event's partial step) is taken
                    u = ue;
                    r1 = re;
                    h = hnew;
                    xhi = xh;
                    xlo = xl;
                }
                if (apply) {
                    // the event at the trial state ue (theta = th)
                    if (++nev > max_ev) {
                        fin = RS_MAX_EVENTS;
                    } else {
                        p3[0] = (double)u.px + (double)u.lpx;
                        p3[1] = (double)u.py + (double)u.lpy;
                        p3[2] = (double)pz;
                        if (evc == 3) {
                            // grating: the upward normal is (-Im W, 1 + Re W) on the surface
                            const double nx = -(double)re.W.im, ny = 1.0 + (double)re.W.re;
                            const double inv = 1.0 / sqrt(nx * nx + ny * ny);
                            reflect2(p3[0], p3[1], nx * inv, ny * inv);
                            split32(p3[0], u.px, u.lpx);
                            split32(p3[1], u.py, u.lpy);
                        } else {
                            double nf[3] = {0.0, 0.0, 0.0};
                            if (evc == 0) nf[1] = 1.0; else if (evc == 1) nf[0] = 1.0; else nf[0] = -1.0;
                            if (snell(p3, nf, 1.0)) {
                                leaves = true;
                                lface = evc;
                            } else {
                                split32(p3[0], u.px, u.lpx);
                                split32(p3[1], u.py, u.lpy);
                            }
                        }
                    }
                }
            }
        }
        if (need64 && fin < 0) {
            // store the state at the step start; the FP64 kernel takes it
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
            R.events[q] = nev;
            R.fbk[q] = fbk;
            R.flags[q] = last_rej ? WF_LAST_REJ : 0;
            push(a.qev, &a.ctr->ev_len, q);
            active = false;
            need64 = false;
            continue;
        }
        if (fin < 0 && !leaves) continue;
        // the visit has ended: the exit is written at the next refill
        pend = fin >= 0 ? 16 + fin : 1 + lface;
        active = false;
        loc = false;
    }
    unsigned long long total = my_steps;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off, 64);
    if (lane == 0) atomicAdd(&a.ctr->hot_steps, total);
}

// Flagged steps of ray q in FP64 (step control, event location and
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
    int so = SO_INSIDE;
    // FP64 steps while the ray stays where FP32 cannot resolve W (with a
    // margin), so that a ray lingering near the branch point does not cost
    // a round per step; from its o.stay-th hand-over on, the rest of the
    // visit (a ray that keeps coming back costs a round per return)
    double pin[3];
    int face = 0;
    const bool stay = o.stay > 0 && a.R.fbk[q] >= o.stay;
    const int nmax = stay ? 16384 : 256;
    for (int n = 0; n < nmax; ++n) {
        so = box_step64(s, o, b, cnt, &mc, r, p, &st, pin, &face);
        if (so == SO_INSIDE && cnt.steps >= o.max_steps) { so = SO_FAIL; st = RS_MAX_STEPS; }
        if (so != SO_INSIDE) break;
        const double d2 = (1.0 + b.r1.W.re) * (1.0 + b.r1.W.re) + b.r1.W.im * b.r1.W.im;
        if (!stay && d2 >= 4.0 * o.wfb2) break;
    }
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
    if (s.fresnel && a.seed_cap > 0)
        fresnel_cross(a, q, r, pin, p, face, true, (int)cnt.steps, (int)cnt.rejected, cnt.events);
    return 1;
}

// Ray q in air (state in rx..qz): walk to the box (state stored, returns 0,
// pin = the direction at the entry) or finish it (returns 2).
__device__ __forceinline__ int air_body(const WfArgs& a, long long q, const SceneDev& s, double pin[3])
{
    double r[3] = {a.R.rx[q], a.R.ry[q], a.R.rz[q]};
    double p[3] = {a.R.qx[q], a.R.qy[q], a.R.qz[q]};
    LaneCount cnt = {a.R.steps[q], a.R.rej[q], a.R.events[q], 0};
    int st = RS_OK;
    cx<double> W;
    int ao = wf_air_walk(a, q, s, r, p, cnt, &st, &W);
    a.R.events[q] = cnt.events;
    if (ao == AO_FAIL) { finish_ray(a, q, s, st, r, p); return 2; }
    if (ao == AO_ESCAPED) { finish_ray(a, q, s, RS_OK, r, p); return 2; }
    Box64 b = box_entry_state(a.o, r, p, W);
    store_box64(a, q, s, b);
    a.R.status[q] = RS_OK;
    pin[0] = p[0]; pin[1] = p[1]; pin[2] = p[2];
    return 0;
}

// FP64 events (INTEG fixes the integrator so that only one is compiled in).
template <int INTEG>
__global__ void __launch_bounds__(256) k_wf_event(WfArgs a, int cur)
{
    const unsigned qlen = a.ctr->ev_len;
    // the loop bound is uniform over the wave, so that the pushes see every lane
    for (unsigned base = blockIdx.x * blockDim.x; base < qlen; base += gridDim.x * blockDim.x) {
        const unsigned qi = base + threadIdx.x;
        int dest = -1, q = 0;
        bool air = false;
        if (qi < qlen) {
            q = a.qev[qi];
            const SceneDev s = a.scenes[a.R.scene[q]];
            int r = event_body<INTEG>(a, q, s);
            // a visit that goes on in FP32 next round: the fast queue
            if (r == 0) dest = 0;
            else if (r == 1) air = true;
        }
        push_box_wave(a, cur ^ 1, dest, q);
        push_air_wave(a, air, q);
    }
}

// The air queue (rays that left the box this round other than straight to
// the sky, or camera rays whose first leg meets the bare grating): walk
// through air in FP64; a ray that enters the box goes to box queue nxt.
__global__ void __launch_bounds__(256) k_wf_air(WfArgs a, int nxt)
{
    const unsigned len = a.ctr->air_len;
    // the loop bound is uniform over the block, so that the pushes see every lane
    for (unsigned base = blockIdx.x * blockDim.x; base < len; base += gridDim.x * blockDim.x) {
        const unsigned i = base + threadIdx.x;
        int dest = -1, q = 0;
        if (i < len) {
            q = a.qair[i];
            const SceneDev s = a.scenes[a.R.scene[q]];
            double p[3];
            if (air_body(a, q, s, p) == 0) dest = box_dest(a, p);
        }
        push_box_wave(a, nxt, dest, q);
    }
}

// Fold per-thread counters into the totals: wave sums by shuffles, block
// sums in LDS, one set of atomics per block (every thread of the block calls
// it).
__device__ __forceinline__ void add_totals(WfTotals* tot, unsigned long long c_rays, unsigned long long c_steps,
                                           unsigned long long c_rej, unsigned long long c_ev,
                                           unsigned long long c_fail, unsigned long long c_fb)
{
    unsigned long long v[6] = {c_rays, c_steps, c_rej, c_ev, c_fail, c_fb};
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    __shared__ unsigned long long part[4][6];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) part[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        unsigned long long sum = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += part[w][k];
        // WfTotals is six consecutive counters in the order of v
        if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(tot) + k, sum);
    }
}

// ---- Fresnel branches: the seed pass and the weighted sum -------------------
// Queue counters cleared for the branches' pass (the branch count and the
// in-box kernel's step total are kept).
__global__ void __launch_bounds__(64) k_wf_seed_reset(QCtr* c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int k = 0; k < 2; ++k) c->box_len[k] = c->box_head[k] = c->slow_len[k] = c->slow_head[k] = 0;
        c->ev_len = c->ev_head = c->air_len = 0;
    }
}

// Start every branch: one reflected at an exit face goes into the box at
// the face (a plate: straight on to its next face, then through air); one
// reflected at an entry walks through air.  The rays that reach the box go
// to round 0's queues.
__global__ void __launch_bounds__(256) k_wf_seed_init(WfArgs a, unsigned n_seeds)
{
    // the loop bound is uniform over the block, so that the pushes see every lane
    for (unsigned base = blockIdx.x * blockDim.x; base < n_seeds; base += gridDim.x * blockDim.x) {
        const unsigned k = base + threadIdx.x;
        int dest = -1;
        const long long q = a.seed_base + (long long)k;
        if (k < n_seeds) {
            const SceneDev s = a.scenes[a.R.scene[q]];
            double r[3] = {a.R.rx[q], a.R.ry[q], a.R.rz[q]};
            double p[3] = {a.R.qx[q], a.R.qy[q], a.R.qz[q]};
            LaneCount cnt = {a.R.steps[q], a.R.rej[q], a.R.events[q], 0};
            if (a.R.flags[q] & WF_SEED_INSIDE) {
                if (s.cloak == CK_PLATE) {
                    double mc = 1.0, pin[3];
                    int face = 0;
                    const int ps = plate_walk64(s, a.o, r, p, cnt, &mc, pin, &face);
                    a.R.events[q] = cnt.events;
                    if (ps != RS_OK) {
                        finish_ray(a, q, s, ps, r, p);
                    } else {
                        fresnel_cross(a, q, r, pin, p, face, true, (int)cnt.steps, (int)cnt.rejected, cnt.events);
                        dest = continue_in_air(a, q, s, r, p, cnt);
                    }
                } else {
                    const cx<double> W = w0_cold(zarg64(s, r[0], r[1]));
                    const Box64 b = box_entry_state(a.o, r, p, W);
                    store_box64(a, q, s, b);
                    a.R.status[q] = RS_OK;
                    dest = box_dest(a, p);
                }
            } else {
                dest = continue_in_air(a, q, s, r, p, cnt);
            }
        }
        push_box_wave(a, 0, dest, (int)q);
    }
}

// Weighted colours summed per sample in fixed point (2^-40): integer
// additions do not depend on their order, so the sum does not depend on
// which slot a branch took.  Slots [0, n_rays) are the primaries, the
// branch pool follows; a branch adds to its primary's sample.  The branches'
// own accepted steps are added to the totals.
constexpr double kFixScale = 1099511627776.0;   // 2^40

__global__ void __launch_bounds__(256) k_wf_fresnel_fold(WfArgs a, unsigned n_seeds, unsigned long long* acc,
                                                         WfTotals* tot)
{
    unsigned long long c_steps = 0;
    const long long n = a.n_rays + (long long)n_seeds;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (long long)gridDim.x * blockDim.x) {
        const long long q = g < a.n_rays ? g : a.seed_base + (g - a.n_rays);
        const long long smp = g < a.n_rays ? q : (long long)a.R.parent[q];
        if (g >= a.n_rays) c_steps += (unsigned)(a.R.steps[q] - a.R.steps0[q]);
        for (int c = 0; c < 3; ++c) {
            const float v = a.R.rgb[3 * q + c];
            if (v > 0.0f) atomicAdd(&acc[3 * smp + c], (unsigned long long)llrint((double)v * kFixScale));
        }
    }
    add_totals(tot, 0, c_steps, 0, 0, 0, 0);
}

// The sample colours from the sums (a sample whose primary path failed is
// black, as without the split).
__global__ void __launch_bounds__(256) k_wf_fresnel_rgb(WfArgs a, const unsigned long long* acc)
{
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < a.n_rays;
         q += (long long)gridDim.x * blockDim.x) {
        const bool ok = a.R.status[q] == RS_OK;
        for (int c = 0; c < 3; ++c) a.R.rgb[3 * q + c] = ok ? (float)((double)acc[3 * q + c] / kFixScale) : 0.0f;
    }
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Pixel averages (render mode) and counters (totals in WfTotals).

// Blocks of the folding kernels (k_wf_finish, k_wf_trace_out): a bounded
// grid strides over the pixels or rays, so that the counters take few atomics.
constexpr long long kFoldBlocks = 2048;

__global__ void __launch_bounds__(256) k_wf_finish(WfArgs a, float* const* images, const long long* pix_off,
                                                   long long n_pix, WfTotals* tot)
{
    unsigned long long c_rays = 0, c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_fb = 0;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < n_pix;
         g += (long long)gridDim.x * blockDim.x) {
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
    add_totals(tot, c_rays, c_steps, c_rej, c_ev, c_fail, c_fb);
}

// trace_rays mode: copy the exit rays out and fold the counters.
__global__ void __launch_bounds__(256) k_wf_trace_out(WfArgs a, double* out_org, double* out_dir, int* status,
                                                      long long* steps, int* events, WfTotals* tot)
{
    unsigned long long c_rays = 0, c_steps = 0, c_rej = 0, c_ev = 0, c_fail = 0, c_fb = 0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < a.n_rays;
         q += (long long)gridDim.x * blockDim.x) {
        if (out_org) { out_org[3 * q] = a.R.rx[q]; out_org[3 * q + 1] = a.R.ry[q]; out_org[3 * q + 2] = a.R.rz[q]; }
        out_dir[3 * q] = a.R.qx[q];
        out_dir[3 * q + 1] = a.R.qy[q];
        out_dir[3 * q + 2] = a.R.qz[q];
        if (status) status[q] = a.R.status[q];
        if (steps) steps[q] = a.R.steps[q];
        if (events) events[q] = a.R.events[q];
        c_rays++;
        c_steps += (unsigned)a.R.steps[q];
        c_rej += (unsigned)a.R.rej[q];
        c_ev += (unsigned)a.R.events[q];
        c_fail += a.R.status[q] != RS_OK;
        c_fb += (unsigned)a.R.fbk[q];
    }
    add_totals(tot, c_rays, c_steps, c_rej, c_ev, c_fail, c_fb);
}

}  // namespace gc
