// gc_lane32.hpp -- FP32 integration inside the cloak.
//
// The ray state inside the box is kept in FP32 with x split into an integer
// grating period and the offset within it (the index of eq. (1) is exactly
// Lambda-periodic in x, so the phase of Z only needs the offset), and every
// state component carries a compensation term so that the many small
// increments of a long path do not lose their low bits.
//
// FP64 is used only where the precision split requires it:
//   - Lambert W near the branch point Z = -1/e: when |1 + W| falls below
//     w_fallback (n = 1/|1 + W| is then large and FP32 loses digits), and
//     for stage points below the branch-point height, where Z can cross the
//     branch cut and a warm start could land on another branch;
//   - every event: a step flagged in FP32 as crossing a face or the grating
//     is redone from its start in FP64, and the crossing is located there
//     (root solve of the partial step), as is everything in air.
#pragma once
#include "gc_lane64.hpp"

namespace gc {

struct Sc32 {
    float L, invL, k, invk, ne, mkl2e, ybp, wfb2;
};

__device__ __forceinline__ Sc32 make_sc32(const SceneDev& s, const OptsDev& o)
{
    Sc32 c;
    c.L = (float)s.L;
    c.invL = (float)s.invL;
    c.k = (float)s.k;
    c.invk = (float)(1.0 / s.k);
    c.ne = (float)(-s.e);
    c.mkl2e = (float)(-s.k * kLog2e);
    c.ybp = (float)s.ybp;
    c.wfb2 = (float)o.wfb2;
    return c;
}

struct Rhs32 {
    float ax, ay;
    cx<float> W, dW;
};

struct St32 {
    int cell;
    float fx, y, px, py;   // leading parts (fx: offset of x inside period `cell`)
    float lx, ly, lpx, lpy;   // compensation terms
};

// One Halley step for W e^W = Z in the form W - Z e^{-W} = 0.
__device__ __forceinline__ float halley32(const Sc32& c, float fx, float y, cx<float>& W)
{
    float m = c.ne * __builtin_amdgcn_exp2f(c.mkl2e * y - W.re * 1.44269504088896341f);
    float cs, sn;
    cis_rev(fx * c.invL - W.im * 0.159154943091895336f, cs, sn);
    cx<float> q = {m * cs, m * sn};
    cx<float> f = W - q;
    cx<float> fp = {1.0f + q.re, q.im};
    cx<float> num = 2.0f * (f * fp);
    cx<float> den = 2.0f * (fp * fp) + f * q;
    float inv = __builtin_amdgcn_rcpf(norm2(den));
    cx<float> d = inv * (num * conjg(den));
    W = W - d;
    return norm2(d);
}

// RHS in FP32 at offset fx (period `cell`) and height y; W holds the
// prediction on entry.  NITER Halley steps (0 = iterate to convergence).
template <int NITER>
__device__ __forceinline__ void rhs32(const SceneDev& s, const Sc32& c, int cell, float fx, float y,
                                      Rhs32& r, int& fallbacks)
{
    if (NITER > 0) {
#pragma unroll
        for (int it = 0; it < NITER; ++it) halley32(c, fx, y, r.W);
    } else {
        for (int it = 0; it < 6; ++it) {
            float d2 = halley32(c, fx, y, r.W);
            if (!(d2 > 1e-13f * (1.0f + norm2(r.W)))) break;
        }
    }
    float d2;
    accel_from_w<float>(s, r.W, r.ax, r.ay, r.dW, d2);
    if (!(d2 >= c.wfb2) || (y < c.ybp && fabsf(fx) < 0.1f * c.L)) {
        // FP64 redo near the branch point
        double x = (double)cell * s.L + (double)fx;
        cx<double> W = {(double)r.W.re, (double)r.W.im};
        if (!(isfinite(W.re) && isfinite(W.im)) || norm2(mk(1.0 + W.re, W.im)) < 1e-6) W = w0_cold(zarg64(s, x, y));
        double ax, ay;
        cx<double> dW;
        rhs64(s, x, (double)y, W, ax, ay, dW);
        r.W = {(float)W.re, (float)W.im};
        r.dW = {(float)dW.re, (float)dW.im};
        r.ax = (float)ax;
        r.ay = (float)ay;
        fallbacks++;
    }
}

__device__ __forceinline__ void comp_add(float& hi, float& lo, float inc)
{
    float b = inc + lo;
    float t = hi + b;
    lo = b - (t - hi);
    hi = t;
}

__device__ __forceinline__ St64 promote(const SceneDev& s, const St32& u)
{
    St64 v;
    v.x = (double)u.cell * s.L + ((double)u.fx + (double)u.lx);
    v.y = (double)u.y + (double)u.ly;
    v.px = (double)u.px + (double)u.lpx;
    v.py = (double)u.py + (double)u.lpy;
    return v;
}

__device__ __forceinline__ void demote_split(double v, float& hi, float& lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

__device__ __forceinline__ St32 demote(const SceneDev& s, const St64& v)
{
    St32 u;
    double cellf = rint(v.x * s.invL);
    u.cell = (int)cellf;
    demote_split(v.x - cellf * s.L, u.fx, u.lx);
    demote_split(v.y, u.y, u.ly);
    demote_split(v.px, u.px, u.lpx);
    demote_split(v.py, u.py, u.lpy);
    return u;
}

__device__ __forceinline__ Rhs32 demote(const Rhs64& r)
{
    Rhs32 q;
    q.ax = (float)r.ax;
    q.ay = (float)r.ay;
    q.W = {(float)r.W.re, (float)r.W.im};
    q.dW = {(float)r.dW.re, (float)r.dW.im};
    return q;
}

__device__ __forceinline__ Rhs64 promote(const SceneDev& s, const St64& u, const Rhs32& r)
{
    Rhs64 q;
    q.W = {(double)r.W.re, (double)r.W.im};
    rhs64(s, u.x, u.y, q.W, q.ax, q.ay, q.dW);
    return q;
}

__device__ __forceinline__ void renorm_cell(const Sc32& c, St32& u)
{
    if (u.fx > 0.5f * c.L) { u.fx -= c.L; u.cell += 1; }
    else if (u.fx < -0.5f * c.L) { u.fx += c.L; u.cell -= 1; }
}

// Predicted W at a point displaced by (dx, dy) from the one r was taken at.
__device__ __forceinline__ void predict(Rhs32& out, const Rhs32& r, float dx, float dy)
{
    out.W = {r.W.re + r.dW.re * dx - r.dW.im * dy, r.W.im + r.dW.re * dy + r.dW.im * dx};
}

// Classical RK4 step in FP32 (one Halley step per stage from the predictor).
__device__ __forceinline__ void rk4_step32(const SceneDev& s, const Sc32& c, const St32& u, const Rhs32& r1,
                                           float h, St32& ue, Rhs32& re, int& fb)
{
    const float hh = 0.5f * h;
    Rhs32 r2, r3, r4;
    float x2 = u.fx + hh * u.px, y2 = u.y + hh * u.py;
    float p2x = u.px + hh * r1.ax, p2y = u.py + hh * r1.ay;
    predict(r2, r1, hh * u.px, hh * u.py);
    rhs32<1>(s, c, u.cell, x2, y2, r2, fb);
    float x3 = u.fx + hh * p2x, y3 = u.y + hh * p2y;
    float p3x = u.px + hh * r2.ax, p3y = u.py + hh * r2.ay;
    predict(r3, r2, x3 - x2, y3 - y2);
    rhs32<1>(s, c, u.cell, x3, y3, r3, fb);
    float x4 = u.fx + h * p3x, y4 = u.y + h * p3y;
    float p4x = u.px + h * r3.ax, p4y = u.py + h * r3.ay;
    predict(r4, r3, x4 - x3, y4 - y3);
    rhs32<1>(s, c, u.cell, x4, y4, r4, fb);
    const float h6 = h * (1.0f / 6.0f);
    ue = u;
    comp_add(ue.fx, ue.lx, h6 * (u.px + 2.0f * p2x + 2.0f * p3x + p4x));
    comp_add(ue.y, ue.ly, h6 * (u.py + 2.0f * p2y + 2.0f * p3y + p4y));
    comp_add(ue.px, ue.lpx, h6 * (r1.ax + 2.0f * r2.ax + 2.0f * r3.ax + r4.ax));
    comp_add(ue.py, ue.lpy, h6 * (r1.ay + 2.0f * r2.ay + 2.0f * r3.ay + r4.ay));
    predict(re, r4, ue.fx - x4, ue.y - y4);
    renorm_cell(c, ue);
    rhs32<1>(s, c, ue.cell, ue.fx, ue.y, re, fb);
}

// DOPRI5 step in FP32; returns the scaled RMS error (same norm as FP64).
__device__ __forceinline__ float dp5_step32(const SceneDev& s, const Sc32& c, const St32& u, const Rhs32& r1,
                                            float h, float rtol, float atol, St32& ue, Rhs32& re, int& fb)
{
    const float A[6][6] = {{(float)DP::a21, 0, 0, 0, 0, 0},
                           {(float)DP::a31, (float)DP::a32, 0, 0, 0, 0},
                           {(float)DP::a41, (float)DP::a42, (float)DP::a43, 0, 0, 0},
                           {(float)DP::a51, (float)DP::a52, (float)DP::a53, (float)DP::a54, 0, 0},
                           {(float)DP::a61, (float)DP::a62, (float)DP::a63, (float)DP::a64, (float)DP::a65, 0},
                           {(float)DP::b1, 0.0f, (float)DP::b3, (float)DP::b4, (float)DP::b5, (float)DP::b6}};
    const float E[7] = {(float)DP::e1, 0.0f, (float)DP::e3, (float)DP::e4, (float)DP::e5, (float)DP::e6,
                        (float)DP::e7};
    float kx[7], ky[7], kax[7], kay[7];
    kx[0] = u.px; ky[0] = u.py; kax[0] = r1.ax; kay[0] = r1.ay;
    Rhs32 rp = r1, rn;
    float xp = u.fx, yp = u.y;
    float x6 = 0, y6 = 0;
#pragma unroll
    for (int st = 1; st < 7; ++st) {
        float sx = 0, sy = 0, sax = 0, say = 0;
#pragma unroll
        for (int j = 0; j < st; ++j) {
            sx += A[st - 1][j] * kx[j];
            sy += A[st - 1][j] * ky[j];
            sax += A[st - 1][j] * kax[j];
            say += A[st - 1][j] * kay[j];
        }
        float x = u.fx + h * sx, y = u.y + h * sy;
        kx[st] = u.px + h * sax;
        ky[st] = u.py + h * say;
        if (st < 6) {
            predict(rn, rp, x - xp, y - yp);
            rhs32<0>(s, c, u.cell, x, y, rn, fb);
            kax[st] = rn.ax;
            kay[st] = rn.ay;
            rp = rn;
            xp = x;
            yp = y;
        } else {
            x6 = x;
            y6 = y;
            (void)sx;
        }
    }
    // 5th order end state with compensation; its RHS is the 7th stage (FSAL)
    {
        float sx = 0, sy = 0, sax = 0, say = 0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            sx += A[5][j] * kx[j];
            sy += A[5][j] * ky[j];
            sax += A[5][j] * kax[j];
            say += A[5][j] * kay[j];
        }
        ue = u;
        comp_add(ue.fx, ue.lx, h * sx);
        comp_add(ue.y, ue.ly, h * sy);
        comp_add(ue.px, ue.lpx, h * sax);
        comp_add(ue.py, ue.lpy, h * say);
    }
    predict(re, rp, x6 - xp, y6 - yp);
    float fx_end = ue.fx;
    renorm_cell(c, ue);
    rhs32<0>(s, c, ue.cell, ue.fx, ue.y, re, fb);
    (void)fx_end;
    kx[6] = ue.px;
    ky[6] = ue.py;
    kax[6] = re.ax;
    kay[6] = re.ay;
    float ex = 0, ey = 0, epx = 0, epy = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        ex += E[j] * kx[j];
        ey += E[j] * ky[j];
        epx += E[j] * kax[j];
        epy += E[j] * kay[j];
    }
    float xa0 = fabsf((float)u.cell * c.L + u.fx), xa1 = fabsf((float)ue.cell * c.L + ue.fx);
    float q0 = h * ex / (atol + rtol * fmaxf(xa0, xa1));
    float q1 = h * ey / (atol + rtol * fmaxf(fabsf(u.y), fabsf(ue.y)));
    float q2 = h * epx / (atol + rtol * fmaxf(fabsf(u.px), fabsf(ue.px)));
    float q3 = h * epy / (atol + rtol * fmaxf(fabsf(u.py), fabsf(ue.py)));
    return sqrtf(0.25f * (q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3));
}

__device__ __forceinline__ bool st32_finite(const St32& u)
{
    return isfinite(u.fx) && isfinite(u.y) && isfinite(u.px) && isfinite(u.py);
}

// FP32 counterpart of integrate_box64.
__device__ inline int integrate_box32(const SceneDev& s, const OptsDev& o, double r[3], double p[3],
                                      LaneCount& cnt, double* min_cos)
{
    const Sc32 c = make_sc32(s, o);
    const float rtol = (float)o.rtol, atol = (float)o.atol;
    double z = r[2];
    const double pz = p[2];
    St32 u;
    Rhs32 r1;
    {
        St64 u64 = {r[0], r[1], p[0], p[1]};
        Rhs64 r64;
        r64.W = w0_cold(zarg64(s, u64.x, u64.y));
        rhs64(s, u64.x, u64.y, r64.W, r64.ax, r64.ay, r64.dW);
        u = demote(s, u64);
        r1 = demote(r64);
    }
    float h = (float)((o.integ == 0) ? o.h : o.h0);
    bool last_rej = false;
    int fb = 0;
    for (;;) {
        if (cnt.steps >= o.max_steps) { cnt.fallbacks += fb; return RS_MAX_STEPS; }
        St32 ue;
        Rhs32 re;
        float hnext = h;
        if (o.integ == 0) {
            rk4_step32(s, c, u, r1, h, ue, re, fb);
        } else {
            float err = dp5_step32(s, c, u, r1, h, rtol, atol, ue, re, fb);
            if (!isfinite(err)) { cnt.fallbacks += fb; return RS_NONFINITE; }
            if (err > 1.0f) {
                h *= fmaxf(0.2f, 0.9f * __builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(err)));
                last_rej = true;
                cnt.rejected++;
                if (h < (float)o.h_min) { cnt.fallbacks += fb; return RS_UNDERFLOW; }
                continue;
            }
            float fac = (err == 0.0f) ? 5.0f : 0.9f * __builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(err));
            fac = fminf(5.0f, fmaxf(0.2f, fac));
            if (last_rej) fac = fminf(fac, 1.0f);
            last_rej = false;
            hnext = fminf(h * fac, (float)o.h_max);
        }
        cnt.steps++;
        if (!st32_finite(ue)) { cnt.fallbacks += fb; return RS_NONFINITE; }
        const double xe = (double)ue.cell * s.L + ((double)ue.fx + (double)ue.lx);
        const double ye = (double)ue.y + (double)ue.ly;
        bool ev = (ye > s.ytop) || (xe > s.hw) || (xe < -s.hw) ||
                  (s.mirror == 0 && ue.y + re.W.re * c.invk < 0.0f);
        if (!ev) {
            u = ue;
            r1 = re;
            z += pz * (double)h;
            h = hnext;
            continue;
        }
        // redo the step in FP64 and locate the crossing there
        St64 u64 = promote(s, u);
        Rhs64 r64 = promote(s, u64, r1);
        St64 ue64;
        Rhs64 re64;
        partial_step64(s, o, u64, r64, (double)h, ue64, re64);
        bool ev64 = (ue64.y > s.ytop) || (ue64.x > s.hw) || (ue64.x < -s.hw) ||
                    (s.mirror == 0 && ue64.y + re64.W.re / s.k < 0.0);
        if (!ev64) {
            u = demote(s, ue64);
            r1 = demote(re64);
            z += pz * (double)h;
            h = hnext;
            continue;
        }
        double dtau, pout[3];
        bool out = handle_events64(s, o, u64, r64, pz, (double)h, ue64, re64, &dtau, pout, min_cos);
        z += pz * dtau;
        if (++cnt.events > o.max_events) { cnt.fallbacks += fb; return RS_MAX_EVENTS; }
        if (out) {
            r[0] = u64.x; r[1] = u64.y; r[2] = z;
            p[0] = pout[0]; p[1] = pout[1]; p[2] = pout[2];
            cnt.fallbacks += fb;
            return RS_OK;
        }
        u = demote(s, u64);
        r1 = demote(r64);
        h = (o.integ == 0) ? (float)o.h : hnext;
    }
}

// Ray path with the in-cloak part in FP32 (air segments and events FP64).
__device__ inline int trace_ray32(const SceneDev& s, const OptsDev& o, const double org[3], const double dir[3],
                                  double out_org[3], double out_dir[3], LaneCount& cnt, double* min_cos)
{
    double r[3] = {org[0], org[1], org[2]};
    double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double p[3] = {dir[0] / nd, dir[1] / nd, dir[2] / nd};
    for (;;) {
        if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]) && isfinite(p[0]) && isfinite(p[1]) &&
              isfinite(p[2])))
            return RS_NONFINITE;
        int face;
        double tb = air_box_entry(s, r, p, &face);
        double xi;
        double tg = air_contact(s, r, p, &xi);
        if (!(tb < kInf) && !(tg < kInf)) {
            for (int i = 0; i < 3; ++i) { out_org[i] = r[i]; out_dir[i] = p[i]; }
            return RS_OK;
        }
        if (++cnt.events > o.max_events) return RS_MAX_EVENTS;
        if (tg <= tb) {
            for (int i = 0; i < 3; ++i) r[i] += tg * p[i];
            double nx = 0.0, ny = 1.0;
            if (!(s.mirror == 1 || s.A == 0.0)) {
                double sn, cs;
                sincos(s.k * xi, &sn, &cs);
                nx = s.e * sn;
                ny = 1.0 - s.e * cs;
                double inv = 1.0 / sqrt(nx * nx + ny * ny);
                nx *= inv;
                ny *= inv;
            }
            *min_cos = fmin(*min_cos, fabs(p[0] * nx + p[1] * ny));
            reflect2(p[0], p[1], nx, ny);
            continue;
        }
        for (int i = 0; i < 3; ++i) r[i] += tb * p[i];
        double nf[3] = {0.0, 0.0, 0.0};
        if (face == 0) { r[1] = s.ytop; nf[1] = -1.0; }
        else if (face == 1) { r[0] = s.hw; nf[0] = -1.0; }
        else { r[0] = -s.hw; nf[0] = 1.0; }
        *min_cos = fmin(*min_cos, fabs(p[0] * nf[0] + p[1] * nf[1]));
        cx<double> W = w0_cold(zarg64(s, r[0], r[1]));
        double n2 = 1.0 / sqrt(norm2(mk(1.0 + W.re, W.im)));
        if (!snell(p, nf, n2)) continue;
        int st = integrate_box32(s, o, r, p, cnt, min_cos);
        if (st != RS_OK) return st;
    }
}

}  // namespace gc
