// gc_lane32.hpp -- FP32 integration inside the cloak (the hot loop).
//
// The in-cloak ray state is FP32 with x split into an integer grating period
// and the offset within it (the index of eq. (1) is exactly Lambda-periodic
// in x, so the phase of Z only needs the offset, in revolutions), and every
// state component carries a compensation term so that the many small
// increments of a long path keep their low bits.
//
// Nothing here touches FP64.  A stage point that needs it -- |1 + W| below
// w_fallback (n = 1/|1 + W| is large near the branch point Z = -1/e and FP32
// loses digits there), or an evaluation path that crosses the branch cut
// (a crest line x = N Lambda below the branch-point height, where a warm
// start could land on another branch) -- only raises a flag; the caller then
// hands the whole step to the FP64 path.
#pragma once
#include "gc_math.hpp"

namespace gc {

// per-scene FP32 constants of the hot loop
struct Sc32 {
    float L, invL, k, invk, ne, mkl2e, ybp, wfb2;
    float kacc;   // k times the box index multiplier squared (the acceleration's scale)
};


__device__ __forceinline__ Sc32 make_sc32(const SceneDev& s, double wfb2)
{
    Sc32 c;
    c.L = (float)s.L;
    c.invL = (float)s.invL;
    c.k = (float)s.k;
    c.invk = (float)s.invk;
    c.ne = (float)(-s.e);
    c.mkl2e = (float)(-s.k * kLog2e);
    c.ybp = (float)s.ybp;
    c.wfb2 = (float)wfb2;
    c.kacc = (float)(s.k * s.nsc2);
    return c;
}

struct Rhs32 {
    float ax, ay;
    cx<float> W, dW;
};

struct St32 {
    int cell;
    float fx, y, px, py;      // leading parts (fx: offset of x inside period `cell`)
    float lx, ly, lpx, lpy;   // compensation terms
};

// One Halley step for W e^W = Z in the form W - Z e^{-W} = 0.  Returns |dW|^2.
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

// acceleration and dW/dzeta from a converged W (FP32)
__device__ __forceinline__ float accel32(const Sc32& c, Rhs32& r)
{
    cx<float> D = {1.0f + r.W.re, r.W.im};
    float d2 = norm2(D);
    float rr = __builtin_amdgcn_rcpf(d2);
    cx<float> t = conjg(r.W) * (D * D);
    float kr3 = c.kacc * rr * rr * rr;
    r.ax = -kr3 * t.im;
    r.ay = kr3 * t.re;
    cx<float> u = r.W * conjg(D);
    float kr = c.k * rr;
    r.dW = {-kr * u.im, kr * u.re};
    return d2;
}

// RHS at offset fx and height y, warm-started from the evaluation `prev`
// taken at (xp, yp) (offsets in the same period): predictor, NITER Halley
// steps (0: iterate until the update is below FP32 resolution), acceleration.
// Sets `bad` when the point needs FP64.
template <int NITER>
__device__ __forceinline__ void eval32(const Sc32& c, float fx, float y, float xp, float yp, const Rhs32& prev,
                                       Rhs32& r, bool& bad)
{
    const float dx = fx - xp, dy = y - yp;
    r.W = {prev.W.re + prev.dW.re * dx - prev.dW.im * dy, prev.W.im + prev.dW.re * dy + prev.dW.im * dx};
    if (NITER > 0) {
#pragma unroll
        for (int it = 0; it < NITER; ++it) halley32(c, fx, y, r.W);
    } else {
        // Halley converges cubically: after an update of relative size 1e-3
        // the error is far below FP32 resolution, so a second step is only
        // needed when the predictor was poor (long DOPRI5 stages near crests)
        float d2 = halley32(c, fx, y, r.W);
        for (int it = 0; it < 5 && d2 > 1e-6f * (1.0f + norm2(r.W)); ++it) d2 = halley32(c, fx, y, r.W);
    }
    const float d2 = accel32(c, r);
    // the crest line of this period is fx = 0
    bad |= !(d2 >= c.wfb2) || (fminf(y, yp) < c.ybp && fx * xp <= 0.0f);
}


__device__ __forceinline__ void comp_add(float& hi, float& lo, float inc)
{
    float b = inc + lo;
    float t = hi + b;
    lo = b - (t - hi);
    hi = t;
}

__device__ __forceinline__ bool renorm_cell(const Sc32& c, St32& u)
{
    if (u.fx > 0.5f * c.L) { u.fx -= c.L; u.cell += 1; return true; }
    if (u.fx < -0.5f * c.L) { u.fx += c.L; u.cell -= 1; return true; }
    return false;
}

// Classical RK4 step (one Halley step per stage from the predictor); re is
// the RHS at the end point, i.e. the next step's first stage.
__device__ __forceinline__ void rk4_step32(const Sc32& c, const St32& u, const Rhs32& r1, float h, St32& ue,
                                           Rhs32& re, bool& bad)
{
    const float hh = 0.5f * h;
    Rhs32 r2, r3, r4;
    float x2 = u.fx + hh * u.px, y2 = u.y + hh * u.py;
    float p2x = u.px + hh * r1.ax, p2y = u.py + hh * r1.ay;
    eval32<1>(c, x2, y2, u.fx, u.y, r1, r2, bad);
    float x3 = u.fx + hh * p2x, y3 = u.y + hh * p2y;
    float p3x = u.px + hh * r2.ax, p3y = u.py + hh * r2.ay;
    eval32<1>(c, x3, y3, x2, y2, r2, r3, bad);
    float x4 = u.fx + h * p3x, y4 = u.y + h * p3y;
    float p4x = u.px + h * r3.ax, p4y = u.py + h * r3.ay;
    eval32<1>(c, x4, y4, x3, y3, r3, r4, bad);
    const float h6 = h * (1.0f / 6.0f);
    ue = u;
    comp_add(ue.fx, ue.lx, h6 * (u.px + 2.0f * p2x + 2.0f * p3x + p4x));
    comp_add(ue.y, ue.ly, h6 * (u.py + 2.0f * p2y + 2.0f * p3y + p4y));
    comp_add(ue.px, ue.lpx, h6 * (r1.ax + 2.0f * r2.ax + 2.0f * r3.ax + r4.ax));
    comp_add(ue.py, ue.lpy, h6 * (r1.ay + 2.0f * r2.ay + 2.0f * r3.ay + r4.ay));
    // the end point's RHS (the next step's first stage), then the period shift
    eval32<1>(c, ue.fx, ue.y, x4, y4, r4, re, bad);
    renorm_cell(c, ue);
}

// DOPRI5 step in FP32; returns the scaled RMS error over (x, y, px, py).
__device__ __forceinline__ float dp5_step32(const Sc32& c, const St32& u, const Rhs32& r1, float h, float rtol,
                                            float atol, St32& ue, Rhs32& re, bool& bad)
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
#pragma unroll
    for (int st = 1; st < 6; ++st) {
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
        eval32<0>(c, x, y, xp, yp, rp, rn, bad);
        kax[st] = rn.ax;
        kay[st] = rn.ay;
        rp = rn;
        xp = x;
        yp = y;
    }
    // 5th order end state (compensated); its RHS is the 7th stage (FSAL)
    {
        float sx = 0, sy = 0, sax = 0, say = 0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (j == 1) continue;   // b2 = 0
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
    const int cell0 = u.cell;
    eval32<0>(c, ue.fx, ue.y, xp, yp, rp, re, bad);
    renorm_cell(c, ue);
    kx[6] = ue.px;
    ky[6] = ue.py;
    kax[6] = re.ax;
    kay[6] = re.ay;
    float ex = 0, ey = 0, epx = 0, epy = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        if (j == 1) continue;   // e2 = 0
        ex += E[j] * kx[j];
        ey += E[j] * ky[j];
        epx += E[j] * kax[j];
        epy += E[j] * kay[j];
    }
    float xa0 = fabsf((float)cell0 * c.L + u.fx), xa1 = fabsf((float)ue.cell * c.L + ue.fx);
    float q0 = h * ex * __builtin_amdgcn_rcpf(atol + rtol * fmaxf(xa0, xa1));
    float q1 = h * ey * __builtin_amdgcn_rcpf(atol + rtol * fmaxf(fabsf(u.y), fabsf(ue.y)));
    float q2 = h * epx * __builtin_amdgcn_rcpf(atol + rtol * fmaxf(fabsf(u.px), fabsf(ue.px)));
    float q3 = h * epy * __builtin_amdgcn_rcpf(atol + rtol * fmaxf(fabsf(u.py), fabsf(ue.py)));
    return __builtin_sqrtf(0.25f * (q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3));
}

__device__ __forceinline__ bool st32_finite(const St32& u)
{
    return isfinite(u.fx) && isfinite(u.y) && isfinite(u.px) && isfinite(u.py);
}

// Event values of an in-box state (>= 0 inside): 0 top, 1 right, 2 left,
// 3 grating (virtual coordinate y + Re W / k, zero on the trochoid).  xh /
// xl: the side faces as offsets in v's period.  Evaluated with the
// compensation terms, so that the faces are resolved to the rounding of the
// difference itself.
__device__ __forceinline__ void ev_values32(const Sc32& c, const St32& v, const Rhs32& r, float ytop, float xh,
                                            float xl, int mirror, float e[4])
{
    e[0] = (ytop - v.y) - v.ly;
    e[1] = (xh - v.fx) - v.lx;
    e[2] = (v.fx - xl) + v.lx;
    e[3] = mirror ? 1.0f : (v.y + r.W.re * c.invk) + v.ly;
}

// smallest of the event values selected by mask, and which one it is
__device__ __forceinline__ float ev_min32(const float e[4], int mask, int* code)
{
    float m = 3.0e38f;
    int k = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (((mask >> i) & 1) && e[i] < m) { m = e[i]; k = i; }
    *code = k;
    return m;
}

__device__ __forceinline__ void split32(double v, float& hi, float& lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

// err^(-1/5) through the hardware log2/exp2
__device__ __forceinline__ float pow_m02(float err)
{
    return __builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf(err));
}

}  // namespace gc
