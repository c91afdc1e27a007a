// gc_adjoint.hpp -- discrete adjoint of the RK4 ray tracer with respect to
// the scene parameters A (grating amplitude, eq. (2)) and half_width (the
// cloak box), for the cloaking-quality loss L = 1 - C0 of eq. (15).
//
// A sample's colour is Cb + m (Ca - Cb) with the sky's blend parameter m
// (see sky_rgb), so any image loss reaches the tracer through one number per
// sample: the reverse sweep is seeded with dm = 1 and returns dm/dA and
// dm/dhw; the loss-specific weights (eq. (15) at zero shift, or its Pearson
// form, whose derivatives need the finished image) are applied afterwards
// in the reduction.  Every sample is reversed through exactly the maps its
// forward trace applied:
//   sky lookup <- straight flights (their lengths fixed implicitly by the
//   surface they end on) <- grating reflections <- Snell refraction at the
//   box faces (entry: n2 = n(r; A) of eq. (1)) <- RK4 steps inside the cloak
//   <- partial steps that end on an event surface (the step length is an
//   implicit function e(Phi(u, tau)) = 0, which adds a projection).
// The in-cloak steps are not stored: the forward pass records the state
// every C steps (and at every event) on a per-lane tape; the reverse pass
// recomputes each segment of at most C steps into a per-lane buffer (with
// the Lambert values of every RK4 stage) and applies the transposed step
// Jacobians from its end to its start.
//
// Derivatives of the index field.  With D = 1 + W, W = W0(Z):
//   a_x + i a_y = i k F,  F = P conj(Q),  P = 1/D,  Q = W / D^3,
//   dW/dzeta = i k W / D,  dW/dA = W / (A D),
//   P' = -W'/D^2,  Q' = W' (1 - 2W) / D^4  (both holomorphic in zeta),
//   d/dx = d/dzeta + d/dzetabar,  d/dy = i (d/dzeta - d/dzetabar),
// so the columns of d a / d(x, y) are i k (F_z + F_zb) and -k (F_z - F_zb)
// as complex numbers, with F_z = P' conj(Q), F_zb = P conj(Q').
#pragma once
#include "gc_lane64.hpp"

namespace gc {

// ---------------------------------------------------------------------------
// Tape and segment buffer.  Both are per lane, interleaved so that the 64
// lanes of a wave touch consecutive addresses for each field.
// ---------------------------------------------------------------------------
constexpr int kTapeFields = 8;
template <typename T> constexpr int seg_fields() { return 12; }
enum AdjKind { AK_CONTACT = 0, AK_ENTRY = 1, AK_RUN = 2, AK_CKPT = 3, AK_EVENT = 4 };

// Records (fields 0..5, field 6, field 7 = tag):
//   CONTACT  air state (x, y, px, py, pz) before the flight, xi of the contact, t
//   ENTRY    air state (x, y, px, py, pz) before the flight, -, t
//   RUN      cloak state (x, y, px, py, Re W, Im W) at the start of a run, pz
//   CKPT     cloak state every C steps of a run, -
//   EVENT    cloak state before the partial step, theta (step fraction)
// tag = kind + 8 face/event + 64 transmitted + 128 steps-into-run.
struct AdjTape {
    double* base;
    long long stride, lane;
    int cap;
    __device__ __forceinline__ double* at(int slot, int f) const
    {
        return base + ((long long)slot * kTapeFields + f) * stride + lane;
    }
};

__device__ inline void tape_put(const AdjTape& t, int& n, double v0, double v1, double v2, double v3, double v4,
                                double v5, double v6, long long tag)
{
    if (n < t.cap) {
        *t.at(n, 0) = v0;
        *t.at(n, 1) = v1;
        *t.at(n, 2) = v2;
        *t.at(n, 3) = v3;
        *t.at(n, 4) = v4;
        *t.at(n, 5) = v5;
        *t.at(n, 6) = v6;
        *t.at(n, 7) = (double)tag;
    }
    ++n;
}

template <typename T>
struct AdjSeg {
    T* base;
    long long stride, lane;
    __device__ __forceinline__ T* at(int j, int f) const
    {
        return base + ((long long)j * seg_fields<T>() + f) * stride + lane;
    }
};

// Cloak state in the working precision T.  In FP32 each coordinate is an
// unevaluated sum hi + lo: the step increments are added with an error-free
// two-sum, so rounding does not accumulate along the path (stages are
// evaluated at hi).  In FP64 lo stays zero.
template <typename T>
struct AS {
    T x, y, px, py;
    cx<T> W;
    T xl, yl, pxl, pyl;
};

template <typename T>
__device__ __forceinline__ void split(double v, T& hi, T& lo)
{
    hi = (T)v;
    lo = sizeof(T) == 8 ? (T)0 : (T)(v - (double)hi);
}

template <typename T>
__device__ __forceinline__ double join(T hi, T lo) { return (double)hi + (double)lo; }

template <typename T>
__device__ inline AS<T> as_make(double x, double y, double px, double py, cx<T> W)
{
    AS<T> u;
    split(x, u.x, u.xl);
    split(y, u.y, u.yl);
    split(px, u.px, u.pxl);
    split(py, u.py, u.pyl);
    u.W = W;
    return u;
}

// hi + lo += inc (two-sum; plain addition in FP64)
template <typename T>
__device__ __forceinline__ void cadd(T& hi, T& lo, T inc)
{
    if constexpr (sizeof(T) == 8) {
        hi += inc;
    } else {
        const T b = inc + lo;
        const T s = hi + b;
        const T bb = s - hi;
        lo = (hi - (s - bb)) + (b - bb);
        hi = s;
    }
}

template <typename T> __device__ __forceinline__ cx<T> cvt(cx<double> w) { return {(T)w.re, (T)w.im}; }
// Re(conj(a) b)
template <typename T> __device__ __forceinline__ T rcm(cx<T> a, cx<T> b) { return a.re * b.re + a.im * b.im; }
// Im(conj(a) b)
template <typename T> __device__ __forceinline__ T icm(cx<T> a, cx<T> b) { return a.re * b.im - a.im * b.re; }

// ---------------------------------------------------------------------------
// Forward RK4 step in precision T.  W0 at each stage is warm-started from
// the previous stage (predictor -- second order in FP64 -- then Halley); a stage whose
// segment from the previous one crosses the branch cut, or (FP32) comes
// close to the branch point, takes W0 from scratch in FP64.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline cx<T> adj_w(const SceneDev& s, T wfb2, T x, T y, T xp, T yp, cx<T> Wp, cx<T> dWp)
{
    if (crosses_cut(s, (double)x, (double)y, (double)xp, (double)yp))
        return cvt<T>(w0_cold(zarg64(s, (double)x, (double)y)));
    cx<T> W = sizeof(T) == 8 ? predict_w<T>(s, Wp, dWp, mk<T>(x - xp, y - yp)) : Wp + dWp * mk<T>(x - xp, y - yp);
    const T fx = x - (T)s.L * rint(x * (T)s.invL);
    if constexpr (sizeof(T) == 8) {
        for (int it = 0; it < 8; ++it) {
            cx<T> w0 = W;
            halley_step<T>(s, fx, y, W);
            // cubic convergence: a relative update of 1e-7 leaves rounding
            if (!(norm2(W - w0) > (T)1e-14 * fmax((T)1e-10, norm2(W)))) break;
        }
        if (!(isfinite(W.re) && isfinite(W.im))) W = w0_cold(zarg64(s, x, y));
    } else {
        // cubic convergence: after an update below 1e-3 (relative) the
        // error left is below FP32 resolution; a second step only after a
        // poor start
        const cx<T> w0 = W;
        halley_step<T>(s, fx, y, W);
        if (norm2(W - w0) > (T)1e-6 * ((T)1 + norm2(W))) halley_step<T>(s, fx, y, W);
        T d2 = ((T)1 + W.re) * ((T)1 + W.re) + W.im * W.im;
        if (!(d2 >= wfb2) || !(isfinite(W.re) && isfinite(W.im)))
            W = cvt<T>(w0_cold(zarg64(s, (double)x, (double)y)));
    }
    return W;
}

// One RK4 step of length h from u; Wst (may be null) receives the converged
// W0 of the four stages.
template <typename T>
__device__ inline void adj_rk4(const SceneDev& s, T wfb2, const AS<T>& u, T h, AS<T>& ue, cx<T>* Wst)
{
    T a1x, a1y, a2x, a2y, a3x, a3y, a4x, a4y, d2;
    cx<T> dW1, dW2, dW3, dW4;
    accel_from_w<T>(s, u.W, a1x, a1y, dW1, d2);
    const T hh = (T)0.5 * h;
    const T x2 = u.x + hh * u.px, y2 = u.y + hh * u.py;
    const T p2x = u.px + hh * a1x, p2y = u.py + hh * a1y;
    const cx<T> W2 = adj_w<T>(s, wfb2, x2, y2, u.x, u.y, u.W, dW1);
    accel_from_w<T>(s, W2, a2x, a2y, dW2, d2);
    const T x3 = u.x + hh * p2x, y3 = u.y + hh * p2y;
    const T p3x = u.px + hh * a2x, p3y = u.py + hh * a2y;
    const cx<T> W3 = adj_w<T>(s, wfb2, x3, y3, x2, y2, W2, dW2);
    accel_from_w<T>(s, W3, a3x, a3y, dW3, d2);
    const T x4 = u.x + h * p3x, y4 = u.y + h * p3y;
    const T p4x = u.px + h * a3x, p4y = u.py + h * a3y;
    const cx<T> W4 = adj_w<T>(s, wfb2, x4, y4, x3, y3, W3, dW3);
    accel_from_w<T>(s, W4, a4x, a4y, dW4, d2);
    const T h6 = h / (T)6;
    ue = u;
    cadd(ue.x, ue.xl, h6 * (u.px + (T)2 * p2x + (T)2 * p3x + p4x));
    cadd(ue.y, ue.yl, h6 * (u.py + (T)2 * p2y + (T)2 * p3y + p4y));
    cadd(ue.px, ue.pxl, h6 * (a1x + (T)2 * a2x + (T)2 * a3x + a4x));
    cadd(ue.py, ue.pyl, h6 * (a1y + (T)2 * a2y + (T)2 * a3y + a4y));
    ue.W = adj_w<T>(s, wfb2, ue.x, ue.y, x4, y4, W4, dW4);
    if (Wst) {
        Wst[0] = u.W;
        Wst[1] = W2;
        Wst[2] = W3;
        Wst[3] = W4;
    }
}

// ---------------------------------------------------------------------------
// Field derivatives at a point from its converged W.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cx<T> dw_dA(const SceneDev& s, T x, T y, cx<T> W, cx<T> iD)
{
    if (s.A > 0.0) return (T)(1.0 / s.A) * (W * iD);
    // A = 0: W = Z to first order, dZ/dA = -k e^{-k y} cis(k x)
    const T k = (T)s.k;
    T c, sn;
    const T fx = x - (T)s.L * rint(x * (T)s.invL);
    cis_rev(fx * (T)s.invL, c, sn);
    const T m = -k * exp_e(-k * y);
    return {m * c, m * sn};
}

// d a / dx, d a / dy and d a / dA as complex numbers (a_x + i a_y)
template <typename T>
struct SJ {
    cx<T> Gx, Gy, GA;
};

template <typename T>
__device__ inline SJ<T> stage_jac(const SceneDev& s, T x, T y, cx<T> W)
{
    const T k = (T)s.k;
    const cx<T> D = {(T)1 + W.re, W.im};
    const cx<T> iD = rcp(norm2(D)) * conjg(D);
    const cx<T> iD2 = iD * iD;
    const cx<T> iD4 = iD2 * iD2;
    const cx<T> WiD = W * iD;
    const cx<T> Wp = {-k * WiD.im, k * WiD.re};
    const cx<T> WA = dw_dA<T>(s, x, y, W, iD);
    const cx<T> omw = {(T)1 - (T)2 * W.re, (T)-2 * W.im};
    const cx<T> Q = WiD * iD2;
    const cx<T> Pp = (T)-1 * (Wp * iD2), Qp = (Wp * omw) * iD4;
    const cx<T> PA = (T)-1 * (WA * iD2), QA = (WA * omw) * iD4;
    const cx<T> Fz = Pp * conjg(Q), Fzb = iD * conjg(Qp);
    const cx<T> FA = PA * conjg(Q) + iD * conjg(QA);
    const cx<T> Sm = Fz + Fzb, Df = Fz - Fzb;
    SJ<T> g;
    g.Gx = {-k * Sm.im, k * Sm.re};
    g.Gy = {-k * Df.re, -k * Df.im};
    g.GA = {-k * FA.im, k * FA.re};
    return g;
}

// index n = 1/|D| and its derivatives at a point (FP64)
__device__ inline double index_grad(const SceneDev& s, double x, double y, cx<double> W, double gn[2], double* nA)
{
    const cx<double> D = {1.0 + W.re, W.im};
    const double d2 = norm2(D);
    const cx<double> iD = (1.0 / d2) * conjg(D);
    const cx<double> WiD = W * iD;
    const cx<double> Wp = {-s.k * WiD.im, s.k * WiD.re};
    const cx<double> WA = dw_dA<double>(s, x, y, W, iD);
    const double n = 1.0 / sqrt(d2);
    const double n3 = n * n * n;
    gn[0] = -n3 * rcm(D, Wp);
    gn[1] = n3 * icm(D, Wp);
    *nA = -n3 * rcm(D, WA);
    return n;
}

// ---------------------------------------------------------------------------
// Reverse of an RK4 step.  On entry l is the adjoint of the end state
// (x, y, px, py); on return that of the start state u.  The stages are
// rebuilt from u and their W0 values.  With a non-null event gradient the
// step is the partial step ending on an event surface e = 0 (gradient ge
// in (x, y), partials eA, ehw): its length tau depends on the state and
// the parameters through e(Phi(u, tau)) = 0.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void rk4_vjp(const SceneDev& s, const AS<T>& u, const cx<T> Wst[4], T h, T l[4], double& lA,
                               const T* ge, T eA, T ehw, double& lhw)
{
    const T c[4] = {(T)0, (T)0.5 * h, (T)0.5 * h, h};
    const T w[4] = {h / (T)6, h / (T)3, h / (T)3, h / (T)6};
    T X[4], Y[4], PX[4], PY[4], AX[4], AY[4];
    SJ<T> J[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i == 0) {
            X[0] = u.x; Y[0] = u.y; PX[0] = u.px; PY[0] = u.py;
        } else {
            X[i] = u.x + c[i] * PX[i - 1];
            Y[i] = u.y + c[i] * PY[i - 1];
            PX[i] = u.px + c[i] * AX[i - 1];
            PY[i] = u.py + c[i] * AY[i - 1];
        }
        T d2;
        cx<T> dW;
        accel_from_w<T>(s, Wst[i], AX[i], AY[i], dW, d2);
        J[i] = stage_jac<T>(s, X[i], Y[i], Wst[i]);
    }
    if (ge) {
        // d Phi / d tau: forward-mode through the stages
        T Ph[4] = {(T)0, (T)0, (T)0, (T)0};
        T KD[4] = {(T)0, (T)0, (T)0, (T)0};
        const T cd[4] = {(T)0, (T)0.5, (T)0.5, (T)1};
        const T w6[4] = {(T)1 / (T)6, (T)1 / (T)3, (T)1 / (T)3, (T)1 / (T)6};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T dU[4] = {(T)0, (T)0, (T)0, (T)0};
            if (i > 0) {
                dU[0] = cd[i] * PX[i - 1] + c[i] * KD[0];
                dU[1] = cd[i] * PY[i - 1] + c[i] * KD[1];
                dU[2] = cd[i] * AX[i - 1] + c[i] * KD[2];
                dU[3] = cd[i] * AY[i - 1] + c[i] * KD[3];
            }
            const cx<T> da = dU[0] * J[i].Gx + dU[1] * J[i].Gy;
            KD[0] = dU[2];
            KD[1] = dU[3];
            KD[2] = da.re;
            KD[3] = da.im;
            Ph[0] += w6[i] * (PX[i] + h * KD[0]);
            Ph[1] += w6[i] * (PY[i] + h * KD[1]);
            Ph[2] += w6[i] * (AX[i] + h * KD[2]);
            Ph[3] += w6[i] * (AY[i] + h * KD[3]);
        }
        const T den = ge[0] * Ph[0] + ge[1] * Ph[1];
        const T cc = (Ph[0] * l[0] + Ph[1] * l[1] + Ph[2] * l[2] + Ph[3] * l[3]) / den;
        l[0] -= cc * ge[0];
        l[1] -= cc * ge[1];
        lA -= (double)(cc * eA);
        lhw -= (double)(cc * ehw);
    }
    T lu[4] = {l[0], l[1], l[2], l[3]};
    T cr[4] = {(T)0, (T)0, (T)0, (T)0};
    double la = 0.0;
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        const T kx = w[i] * l[0] + cr[0], ky = w[i] * l[1] + cr[1];
        const cx<T> La = {w[i] * l[2] + cr[2], w[i] * l[3] + cr[3]};
        const T mx = rcm(J[i].Gx, La), my = rcm(J[i].Gy, La);
        la += (double)rcm(J[i].GA, La);
        lu[0] += mx;
        lu[1] += my;
        lu[2] += kx;
        lu[3] += ky;
        cr[0] = c[i] * mx;
        cr[1] = c[i] * my;
        cr[2] = c[i] * kx;
        cr[3] = c[i] * ky;
    }
    l[0] = lu[0]; l[1] = lu[1]; l[2] = lu[2]; l[3] = lu[3];
    lA += la;
}

// The transposed map of one FP64 RK4 step applied to four adjoint vectors
// at once (the rows of L, with their dL/dA in lA): the stage values and the
// field Jacobians are formed once for all four.
__device__ inline void rk4_vjp4(const SceneDev& s, const AS<double>& u, const cx<double> Wst[4], double h,
                                double L[4][4], double lA[4])
{
    const double c[4] = {0.0, 0.5 * h, 0.5 * h, h};
    const double w[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0};
    double PX[4], PY[4], AX[4], AY[4];
    SJ<double> J[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double X, Y;
        if (i == 0) {
            X = u.x; Y = u.y; PX[0] = u.px; PY[0] = u.py;
        } else {
            X = u.x + c[i] * PX[i - 1];
            Y = u.y + c[i] * PY[i - 1];
            PX[i] = u.px + c[i] * AX[i - 1];
            PY[i] = u.py + c[i] * AY[i - 1];
        }
        double d2;
        cx<double> dW;
        accel_from_w<double>(s, Wst[i], AX[i], AY[i], dW, d2);
        J[i] = stage_jac<double>(s, X, Y, Wst[i]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double* l = L[k];
        double lu[4] = {l[0], l[1], l[2], l[3]};
        double cr[4] = {0.0, 0.0, 0.0, 0.0};
        double la = 0.0;
#pragma unroll
        for (int i = 3; i >= 0; --i) {
            const double kx = w[i] * l[0] + cr[0], ky = w[i] * l[1] + cr[1];
            const cx<double> La = {w[i] * l[2] + cr[2], w[i] * l[3] + cr[3]};
            const double mx = rcm(J[i].Gx, La), my = rcm(J[i].Gy, La);
            la += rcm(J[i].GA, La);
            lu[0] += mx;
            lu[1] += my;
            lu[2] += kx;
            lu[3] += ky;
            cr[0] = c[i] * mx;
            cr[1] = c[i] * my;
            cr[2] = c[i] * kx;
            cr[3] = c[i] * ky;
        }
        l[0] = lu[0]; l[1] = lu[1]; l[2] = lu[2]; l[3] = lu[3];
        lA[k] += la;
    }
}

// Values per tape record of a segment map (below).
constexpr int kMapFields = 20;

// The transposed map of the in-cloak steps from tape record i (a RUN or
// CKPT record) to the next record (the following checkpoint or the run's
// event): the adjoint l of the state at the segment's end becomes
// sum_k l[k] map[4k .. 4k+3] at its start, and dL/dA gains
// sum_k l[k] map[16 + k].  The segment is recomputed from its record (the
// same steps the forward pass took) and reversed once for the four unit
// seeds.  Returns false if the tape is inconsistent.  Not inlined: its
// callers (k_adj_maps, and adj_reverse for a trace the pool had no room
// for) then run the same compiled arithmetic.
__device__ __noinline__ bool adj_segment_map(const SceneDev& s_in, double wfb2, int C, double h, const AdjTape& tp_in,
                                       int i, const AdjSeg<double>& sg_in, double* map)
{
    // the scene and the buffers' descriptors in registers (read through the
    // references, they would be loaded again after every store)
    const SceneDev s = s_in;
    const AdjTape tp = tp_in;
    const AdjSeg<double> sg = sg_in;
    const long long tag = (long long)*tp.at(i, 7), tag1 = (long long)*tp.at(i + 1, 7);
    const int kind = (int)(tag & 7), kind1 = (int)(tag1 & 7);
    const long long base = kind == AK_RUN ? 0 : (tag >> 7);
    const long long nseg = (tag1 >> 7) - base;
    if ((kind != AK_RUN && kind != AK_CKPT) || (kind1 != AK_CKPT && kind1 != AK_EVENT) || nseg < 0 || nseg > C)
        return false;
    AS<double> u = as_make<double>(*tp.at(i, 0), *tp.at(i, 1), *tp.at(i, 2), *tp.at(i, 3),
                                   {*tp.at(i, 4), *tp.at(i, 5)});
    for (int q = 0; q < (int)nseg; ++q) {
        cx<double> Wst[4];
        AS<double> ue;
        adj_rk4<double>(s, wfb2, u, h, ue, Wst);
        *sg.at(q, 0) = u.x; *sg.at(q, 1) = u.y; *sg.at(q, 2) = u.px; *sg.at(q, 3) = u.py;
        *sg.at(q, 4) = u.W.re; *sg.at(q, 5) = u.W.im;
        *sg.at(q, 6) = Wst[1].re; *sg.at(q, 7) = Wst[1].im;
        *sg.at(q, 8) = Wst[2].re; *sg.at(q, 9) = Wst[2].im;
        *sg.at(q, 10) = Wst[3].re; *sg.at(q, 11) = Wst[3].im;
        u = ue;
    }
    double L[4][4] = {{1.0, 0.0, 0.0, 0.0}, {0.0, 1.0, 0.0, 0.0}, {0.0, 0.0, 1.0, 0.0}, {0.0, 0.0, 0.0, 1.0}};
    double lA[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = (int)nseg - 1; q >= 0; --q) {
        const AS<double> uq = {*sg.at(q, 0), *sg.at(q, 1), *sg.at(q, 2), *sg.at(q, 3), {*sg.at(q, 4), *sg.at(q, 5)},
                               0.0, 0.0, 0.0, 0.0};
        const cx<double> Wst[4] = {uq.W, {*sg.at(q, 6), *sg.at(q, 7)}, {*sg.at(q, 8), *sg.at(q, 9)},
                                   {*sg.at(q, 10), *sg.at(q, 11)}};
        rk4_vjp4(s, uq, Wst, h, L, lA);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) map[4 * k + r] = L[k][r];
        map[16 + k] = lA[k];
    }
    return true;
}

// ---------------------------------------------------------------------------
// Event functions inside the cloak (>= 0 inside): 0 top, 1 right, 2 left,
// 3 grating (virtual coordinate v = y + Re W / k, zero on the trochoid).
// ---------------------------------------------------------------------------
// (evaluated with the low parts of the FP32 state, so that the faces are
// exact to rounding of the difference itself)
template <typename T>
__device__ __forceinline__ T adj_event(const SceneDev& s, int ev, const AS<T>& u)
{
    switch (ev) {
    case 0: return ((T)s.ytop - u.y) - u.yl;
    case 1: return ((T)s.hw - u.x) - u.xl;
    case 2: return ((T)s.hw + u.x) + u.xl;
    default: return (u.y + u.W.re * (T)s.invk) + u.yl;
    }
}

// Rounding level of event ev: in FP64 the coordinates themselves (as large
// as y_top or half_width) set it; in FP32 the faces are differences of an
// exact constant and a compensated coordinate, and the grating carries the
// FP32 error of W.
template <typename T>
__device__ __forceinline__ T adj_event_noise(const SceneDev& s, int ev)
{
    if constexpr (sizeof(T) == 8) {
        return (T)(4.0 * 1.1102230246251565e-16 *
                   (1.0 + (isfinite(s.ytop) ? fabs(s.ytop) : 0.0) + (isfinite(s.hw) ? fabs(s.hw) : 0.0)));
    } else {
        return ev == 3 ? (T)(4.0 * 5.9604645e-8) : (T)0;
    }
}

// Smallest theta in (0, 1] at which event ev of the partial step Phi(u,
// theta h) reaches zero (f0 >= 0 at the start, f1 < 0 at the full step):
// regula falsi with the Illinois modification on the bracket.  It ends when
// the bracket is `tol` wide or when its upper end is on the surface to
// rounding (-noise <= e < 0; the event functions are differences of
// coordinates as large as y_top or half_width); a trial on the surface to
// rounding from the inside is followed by one just across it.  Returns the
// upper end of the bracket (e < 0 there) and its state in uh.
template <typename T>
__device__ __noinline__ T adj_locate(const SceneDev& s, T wfb2, int ev, const AS<T>& u, T h, T f0, T f1,
                                     const AS<T>& u_end, AS<T>& uh)
{
    const T tol = sizeof(T) == 8 ? (T)1e-14 : (T)2e-7;
    const T noise = adj_event_noise<T>(s, ev);
    T lo = (T)0, hi = (T)1, flo = f0, fhi = f1;
    uh = u_end;
    int side = 0;
    T x = (T)1;
    for (int it = 0; it < 100 && hi - lo > tol; ++it) {
        T t;
        if (side > 0 && flo <= noise && noise > (T)0) {
            // the last trial (lo) is on the surface to rounding: step across
            const T sl = (fhi - flo) / (hi - lo);
            t = lo + fmax((T)2 * noise / fabs(sl), tol);
        } else {
            t = (flo - fhi > (T)0) ? (flo * hi - fhi * lo) / (flo - fhi) : (T)0.5 * (lo + hi);
        }
        if (it >= 40 || !(t > lo && t < hi)) t = (T)0.5 * (lo + hi);
        AS<T> ut;
        adj_rk4<T>(s, wfb2, u, t * h, ut, nullptr);
        const T ft = adj_event<T>(s, ev, ut);
        if (ft < (T)0) {
            hi = t;
            fhi = ft;
            uh = ut;
            if (ft >= -noise) break;
            if (side < 0) flo *= (T)0.5;
            side = -1;
        } else {
            lo = t;
            flo = ft;
            if (side > 0) fhi *= (T)0.5;
            side = 1;
        }
        x = t;
    }
    (void)x;
    return hi;
}

// gradient of event ev at its end state ue
template <typename T>
__device__ inline void event_grad(const SceneDev& s, int ev, const AS<T>& ue, T ge[2], T* eA, T* ehw)
{
    *eA = (T)0;
    *ehw = (T)0;
    if (ev == 0) { ge[0] = (T)0; ge[1] = (T)-1; return; }
    if (ev == 1) { ge[0] = (T)-1; ge[1] = (T)0; *ehw = (T)1; return; }
    if (ev == 2) { ge[0] = (T)1; ge[1] = (T)0; *ehw = (T)1; return; }
    const T k = (T)s.k, ik = (T)s.invk;
    const cx<T> D = {(T)1 + ue.W.re, ue.W.im};
    const cx<T> iD = rcp(norm2(D)) * conjg(D);
    const cx<T> WiD = ue.W * iD;
    const cx<T> Wp = {-k * WiD.im, k * WiD.re};
    ge[0] = Wp.re * ik;
    ge[1] = (T)1 - Wp.im * ik;
    *eA = dw_dA<T>(s, ue.x, ue.y, ue.W, iD).re * ik;
}

// ---------------------------------------------------------------------------
// Reverses of the maps applied at surfaces (FP64).
// ---------------------------------------------------------------------------
// mirror reflection p' = p - 2 (p.N) N about N = m / |m| (xy only).  On
// entry lp holds the adjoint of p'; on return that of p.  lm receives the
// adjoint of m.
__device__ inline void reflect_vjp(const double p[2], const double m[2], double lp[2], double lm[2])
{
    const double r = sqrt(m[0] * m[0] + m[1] * m[1]);
    const double N[2] = {m[0] / r, m[1] / r};
    const double Nl = N[0] * lp[0] + N[1] * lp[1];
    const double pN = p[0] * N[0] + p[1] * N[1];
    const double g[2] = {-2.0 * (Nl * p[0] + pN * lp[0]), -2.0 * (Nl * p[1] + pN * lp[1])};
    const double Ng = N[0] * g[0] + N[1] * g[1];
    lm[0] = (g[0] - N[0] * Ng) / r;
    lm[1] = (g[1] - N[1] * Ng) / r;
    lp[0] -= 2.0 * Nl * N[0];
    lp[1] -= 2.0 * Nl * N[1];
}

// Snell's law at a plane with fixed unit normal nf into index n2 (as in
// snell()).  On entry lp is the adjoint of the new momentum; on return
// that of the old one; returns the adjoint of n2.
__device__ inline double snell_vjp(const double p[3], const double nf[3], double n2, double lp[3])
{
    const double pn = p[0] * nf[0] + p[1] * nf[1] + p[2] * nf[2];
    const double pt[3] = {p[0] - pn * nf[0], p[1] - pn * nf[1], p[2] - pn * nf[2]};
    const double q = n2 * n2 - (pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2]);
    const double nl = nf[0] * lp[0] + nf[1] * lp[1] + nf[2] * lp[2];
    if (q < 0.0) {
        for (int i = 0; i < 3; ++i) lp[i] -= 2.0 * nl * nf[i];
        return 0.0;
    }
    const double sg = pn >= 0.0 ? 1.0 : -1.0;
    const double r = sqrt(q);
    for (int i = 0; i < 3; ++i) lp[i] = lp[i] - nl * nf[i] - sg * nl / r * pt[i];
    return sg * nl * n2 / r;
}

// straight flight r1 = r0 + t p whose length is fixed by a surface e(r1) = 0
// (gradient ge, partials eA, ehw).  On entry lr / lp are the adjoints at
// the end (lp of the unchanged momentum); on return those at the start.
__device__ inline void flight_vjp(const double p[3], double t, const double ge[2], double eA, double ehw,
                                  double lr[2], double lp[3], double& lA, double& lhw)
{
    const double cc = (lr[0] * p[0] + lr[1] * p[1]) / (ge[0] * p[0] + ge[1] * p[1]);
    lr[0] -= cc * ge[0];
    lr[1] -= cc * ge[1];
    lp[0] += t * lr[0];
    lp[1] += t * lr[1];
    lA -= cc * eA;
    lhw -= cc * ehw;
}

// Gradient of the sky's blend parameter m (see sky_rgb) with respect to the
// direction d, times the seed lm.
__device__ inline void sky_vjp(double K, const double d[3], double lm, double lp[3])
{
    const double rho2 = d[0] * d[0] + d[2] * d[2], rho = sqrt(rho2);
    if (!(rho2 > 0.0)) {
        lp[0] = lp[1] = lp[2] = 0.0;
        return;
    }
    const double r2 = rho2 + d[1] * d[1], nrm = sqrt(r2);
    const cx<double> a = {-d[2] / rho, d[0] / rho};
    const cx<double> a2 = a * a, a4 = a2 * a2;
    const cx<double> b = {rho / nrm, d[1] / nrm};
    const cx<double> b2 = b * b, b4 = b2 * b2, b8 = b4 * b4;
    const double ta = tanh(K * a4.re), tb = tanh(K * b8.im);
    const double cphi = 0.5 * (1.0 - ta * ta) * K * (-4.0 * a4.im) * tb;
    const double cth = 0.5 * ta * (1.0 - tb * tb) * K * 8.0 * b8.re;
    const double gphi[3] = {-d[2] / rho2, 0.0, d[0] / rho2};
    const double gth[3] = {-d[1] * d[0] / (rho * r2), rho / r2, -d[1] * d[2] / (rho * r2)};
    for (int i = 0; i < 3; ++i) lp[i] = lm * (cphi * gphi[i] + cth * gth[i]);
}

// ---------------------------------------------------------------------------
// Forward trace with tape (the maps of trace_ray64, RK4 only).  With `stop`
// (a first pass, which hands such samples to the second), the trace ends
// with kAdjStopped as soon as its tape has overflowed or it has taken more
// than stop_steps steps: the second pass redoes it from the start.
// ---------------------------------------------------------------------------
constexpr int kAdjStopped = 16;   // not a ray status

template <typename T>
__device__ __forceinline__ int adj_forward_body(const SceneDev& s, const OptsDev& o, T wfb2, int C,
                                                const double org[3], const double dir[3], const AdjTape& tp,
                                                int& nrec, double out_dir[3], long long& steps, int& events,
                                                bool stop, long long stop_steps)
{
    // the scene, options and tape in registers for the step loop: read
    // through the caller's references they would be loaded again every
    // step, since the tape's stores might alias them
    const SceneDev sl = s;
    const long long max_steps = o.max_steps;
    const int max_events = o.max_events;
    const AdjTape tl = tp;
    double r[3] = {org[0], org[1], org[2]};
    const double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double p[3] = {dir[0] / nd, dir[1] / nd, dir[2] / nd};
    const T h = (T)o.h;
    nrec = 0;
    steps = 0;
    events = 0;
    for (;;) {
        // --- air ---
        for (;;) {
            if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])))
                return RS_NONFINITE;
            int face;
            const double tb = air_box_entry(s, r, p, &face);
            double xi;
            const double tg = air_contact(s, r, p, &xi);
            if (!(tb < kInf) && !(tg < kInf)) {
                out_dir[0] = p[0]; out_dir[1] = p[1]; out_dir[2] = p[2];
                return RS_OK;
            }
            if (++events > max_events) return RS_MAX_EVENTS;
            if (tg <= tb) {
                if (s.A == 0.0) xi = r[0] + tg * p[0];
                tape_put(tl, nrec, r[0], r[1], p[0], p[1], p[2], xi, tg, AK_CONTACT);
                for (int i = 0; i < 3; ++i) r[i] += tg * p[i];
                double sn, cs;
                sincos(s.k * xi, &sn, &cs);
                double nx = s.e * sn, ny = 1.0 - s.e * cs;
                const double inv = 1.0 / sqrt(nx * nx + ny * ny);
                reflect2(p[0], p[1], nx * inv, ny * inv);
                continue;
            }
            const double r0[3] = {r[0], r[1], r[2]}, p0[3] = {p[0], p[1], p[2]};
            for (int i = 0; i < 3; ++i) r[i] += tb * p[i];
            double nf[3] = {0.0, 0.0, 0.0};
            if (face == 0) { r[1] = s.ytop; nf[1] = -1.0; }
            else if (face == 1) { r[0] = s.hw; nf[0] = -1.0; }
            else { r[0] = -s.hw; nf[0] = 1.0; }
            const cx<double> W = w0_cold(zarg64(s, r[0], r[1]));
            const double n2 = 1.0 / sqrt(norm2(mk(1.0 + W.re, W.im)));
            const bool thr = snell(p, nf, n2);
            tape_put(tl, nrec, r0[0], r0[1], p0[0], p0[1], p0[2], 0.0, tb, AK_ENTRY + 8 * face + (thr ? 64 : 0));
            if (thr) break;
        }
        // --- cloak ---
        AS<T> u = as_make<T>(r[0], r[1], p[0], p[1], cvt<T>(w0_cold(zarg64(s, r[0], r[1]))));
        const double pz = p[2];
        tape_put(tl, nrec, join(u.x, u.xl), join(u.y, u.yl), join(u.px, u.pxl), join(u.py, u.pyl), u.W.re, u.W.im,
                 pz, AK_RUN);
        long long run = 0;
        for (;;) {
            if (stop && (nrec > tl.cap || steps > stop_steps)) return kAdjStopped;
            if (steps >= max_steps) return RS_MAX_STEPS;
            if (run > 0 && run % C == 0)
                tape_put(tl, nrec, join(u.x, u.xl), join(u.y, u.yl), join(u.px, u.pxl), join(u.py, u.pyl), u.W.re,
                         u.W.im, 0.0, AK_CKPT + 128 * run);
            AS<T> ue;
            adj_rk4<T>(sl, wfb2, u, h, ue, nullptr);
            ++steps;
            if (!(isfinite(ue.x) && isfinite(ue.y) && isfinite(ue.px) && isfinite(ue.py))) return RS_NONFINITE;
            T f1[4];
#pragma unroll
            for (int ev = 0; ev < 4; ++ev) f1[ev] = adj_event<T>(sl, ev, ue);
            if (!(f1[0] < (T)0 || f1[1] < (T)0 || f1[2] < (T)0 || f1[3] < (T)0)) {
                u = ue;
                ++run;
                continue;
            }
            T best = (T)2;
            int hit = -1;
            AS<T> uc = ue;
            for (int ev = 0; ev < 4; ++ev) {
                if (!(f1[ev] < (T)0)) continue;
                // copies for the call, so that the step loop's own state is
                // never addressed and stays in registers
                const AS<T> ua = u, ub = ue;
                AS<T> uh;
                const T th = adj_locate<T>(s, wfb2, ev, ua, h, fmax(adj_event<T>(sl, ev, u), (T)0), f1[ev], ub, uh);
                if (th < best) { best = th; hit = ev; uc = uh; }
            }
            if (++events > max_events) return RS_MAX_EVENTS;
            double pp[3] = {join(uc.px, uc.pxl), join(uc.py, uc.pyl), pz};
            bool thr = false;
            if (hit == 3) {
                const double nx = -(double)uc.W.im, ny = 1.0 + (double)uc.W.re;
                const double inv = 1.0 / sqrt(nx * nx + ny * ny);
                reflect2(pp[0], pp[1], nx * inv, ny * inv);
            } else {
                double nf[3] = {0.0, 0.0, 0.0};
                if (hit == 0) nf[1] = 1.0; else if (hit == 1) nf[0] = 1.0; else nf[0] = -1.0;
                thr = snell(pp, nf, 1.0);
            }
            tape_put(tl, nrec, join(u.x, u.xl), join(u.y, u.yl), join(u.px, u.pxl), join(u.py, u.pyl), u.W.re, u.W.im,
                     (double)best, AK_EVENT + 8 * hit + (thr ? 64 : 0) + 128 * run);
            if (thr) {
                r[0] = join(uc.x, uc.xl);
                r[1] = join(uc.y, uc.yl);
                p[0] = pp[0]; p[1] = pp[1]; p[2] = pp[2];
                break;
            }
            u = uc;
            split(pp[0], u.px, u.pxl);
            split(pp[1], u.py, u.pyl);
            run = 0;
            tape_put(tl, nrec, join(u.x, u.xl), join(u.y, u.yl), join(u.px, u.pxl), join(u.py, u.pyl), u.W.re, u.W.im,
                     pz, AK_RUN);
        }
    }
}

// The forward trace as one compiled function (the first and second passes
// share it); its counters live in registers and are written back at the end.
template <typename T>
__device__ __noinline__ int adj_forward(const SceneDev& s, const OptsDev& o, T wfb2, int C, const double org[3],
                                        const double dir[3], const AdjTape& tp, int& nrec, double out_dir[3],
                                        long long& steps, int& events, bool stop, long long stop_steps)
{
    int nrec_l = 0, events_l = 0;
    long long steps_l = 0;
    const int st = adj_forward_body<T>(s, o, wfb2, C, org, dir, tp, nrec_l, out_dir, steps_l, events_l, stop,
                                       stop_steps);
    nrec = nrec_l;
    steps = steps_l;
    events = events_l;
    return st;
}

// ---------------------------------------------------------------------------
// Reverse sweep over the tape.  lm: adjoint of the sample's sky parameter m.
// Accumulates dL/dA and dL/dhw of this sample.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void adj_reverse_body(const SceneDev& s_in, const OptsDev& o_in, T wfb2, int C,
                                                 const AdjTape& tp_in, int nrec, const AdjSeg<T>& sg_in,
                                                 const double out_dir[3], double lm, double& lA, double& lhw,
                                                 int& bad, double& sens, const double* maps, bool fly)
{
    // the scene, options and buffers' descriptors in registers (read through
    // the references, they would be loaded again after every store)
    const SceneDev s = s_in;
    const OptsDev o = o_in;
    const AdjTape tp = tp_in;
    const AdjSeg<T> sg = sg_in;
    const T h = (T)o.h;
    double lr[2] = {0.0, 0.0}, lp[3];
    sky_vjp(s.K, out_dir, lm, lp);
    T l[4] = {(T)0, (T)0, (T)0, (T)0};
    T lpz = (T)0;
    long long j = 0;   // box mode: l is the adjoint of the state after j steps of the current run
    for (int i = nrec - 1; i >= 0; --i) {
        const long long tag = (long long)*tp.at(i, 7);
        const int kind = (int)(tag & 7), code = (int)((tag >> 3) & 7);
        const bool thr = (tag >> 6) & 1;
        const long long run = tag >> 7;
        if (kind == AK_CONTACT) {
            const double x0 = *tp.at(i, 0), y0 = *tp.at(i, 1);
            const double p0[3] = {*tp.at(i, 2), *tp.at(i, 3), *tp.at(i, 4)};
            const double xi = *tp.at(i, 5), t = *tp.at(i, 6);
            (void)x0; (void)y0;
            // reflection about the trochoid normal m = (e sin E, 1 - e cos E), E = k xi
            double sn, cs;
            sincos(s.k * xi, &sn, &cs);
            const double m[2] = {s.e * sn, 1.0 - s.e * cs};
            double lm[2];
            reflect_vjp(p0, m, lp, lm);
            const double den = 1.0 - s.e * cs;
            const double lE = lm[0] * s.e * cs + lm[1] * s.e * sn;
            const double lde = lm[0] * sn - lm[1] * cs;
            lr[0] += lE * s.k / den;
            lA += lE * s.k * sn / den + lde * s.k;
            // flight ending on y = S(x): S' = -e sin E / den, S_A = cos E - e sin^2 E / den
            const double ge[2] = {s.e * sn / den, 1.0};
            const double eA = -(cs - s.e * sn * sn / den);
            flight_vjp(p0, t, ge, eA, 0.0, lr, lp, lA, lhw);
        } else if (kind == AK_ENTRY) {
            const double p0[3] = {*tp.at(i, 2), *tp.at(i, 3), *tp.at(i, 4)};
            const double t = *tp.at(i, 6);
            double re[2] = {*tp.at(i, 0) + t * p0[0], *tp.at(i, 1) + t * p0[1]};
            double nf[3] = {0.0, 0.0, 0.0};
            double ge[2], ehw = 0.0;
            if (code == 0) { re[1] = s.ytop; nf[1] = -1.0; ge[0] = 0.0; ge[1] = 1.0; }
            else if (code == 1) { re[0] = s.hw; nf[0] = -1.0; ge[0] = 1.0; ge[1] = 0.0; ehw = -1.0; }
            else { re[0] = -s.hw; nf[0] = 1.0; ge[0] = 1.0; ge[1] = 0.0; ehw = 1.0; }
            if (thr) {
                // leave box mode: l is the adjoint of (r_e, p_in)
                lr[0] = (double)l[0];
                lr[1] = (double)l[1];
                lp[0] = (double)l[2];
                lp[1] = (double)l[3];
                lp[2] = (double)lpz;
            }
            const cx<double> W = w0_cold(zarg64(s, re[0], re[1]));
            double gn[2], nA;
            const double n2 = index_grad(s, re[0], re[1], W, gn, &nA);
            const double ln2 = snell_vjp(p0, nf, n2, lp);
            lr[0] += ln2 * gn[0];
            lr[1] += ln2 * gn[1];
            lA += ln2 * nA;
            flight_vjp(p0, t, ge, 0.0, ehw, lr, lp, lA, lhw);
        } else if (kind == AK_EVENT) {
            // the partial step from the recorded state, and the run's pz
            const AS<T> un = as_make<T>(*tp.at(i, 0), *tp.at(i, 1), *tp.at(i, 2), *tp.at(i, 3),
                                        {(T)*tp.at(i, 4), (T)*tp.at(i, 5)});
            const T tau = (T)*tp.at(i, 6) * h;
            const int irun = i - (int)(run / C) - 1;   // the run's RUN record (one CKPT per C steps)
            if (irun < 0 || (int)(((long long)*tp.at(irun, 7)) & 7) != AK_RUN) {
                bad = 1;
                return;
            }
            const double pz = *tp.at(irun, 6);
            AS<T> ue;
            cx<T> Wst[4];
            adj_rk4<T>(s, wfb2, un, tau, ue, Wst);
            if (code == 3) {
                // grating reflection about m = (-Im W, 1 + Re W) at ue
                const double pe[2] = {join(ue.px, ue.pxl), join(ue.py, ue.pyl)};
                const double m[2] = {-(double)ue.W.im, 1.0 + (double)ue.W.re};
                double lpp[2] = {(double)l[2], (double)l[3]}, lm[2];
                reflect_vjp(pe, m, lpp, lm);
                // dm = (-Im dW, Re dW), dW = W' dzeta + W_A dA
                const cx<double> LW = {lm[1], -lm[0]};
                const cx<double> Wd = {(double)ue.W.re, (double)ue.W.im};
                const cx<double> D = {1.0 + Wd.re, Wd.im};
                const cx<double> iD = (1.0 / norm2(D)) * conjg(D);
                const cx<double> WiD = Wd * iD;
                const cx<double> Wp = {-s.k * WiD.im, s.k * WiD.re};
                const cx<double> WA = dw_dA<double>(s, (double)ue.x, (double)ue.y, Wd, iD);
                l[0] += (T)rcm(LW, Wp);
                l[1] += (T)(-icm(LW, Wp));
                lA += rcm(LW, WA);
                l[2] = (T)lpp[0];
                l[3] = (T)lpp[1];
            } else {
                double nf[3] = {0.0, 0.0, 0.0};
                if (code == 0) nf[1] = 1.0; else if (code == 1) nf[0] = 1.0; else nf[0] = -1.0;
                const double pe[3] = {join(ue.px, ue.pxl), join(ue.py, ue.pyl), pz};
                double lq[3];
                if (thr) {
                    // exit into air: adjoints come from the air side
                    lq[0] = lp[0]; lq[1] = lp[1]; lq[2] = lp[2];
                    l[0] = (T)lr[0];
                    l[1] = (T)lr[1];
                } else {
                    lq[0] = (double)l[2]; lq[1] = (double)l[3]; lq[2] = (double)lpz;
                }
                snell_vjp(pe, nf, 1.0, lq);
                l[2] = (T)lq[0];
                l[3] = (T)lq[1];
                lpz = (T)lq[2];
            }
            T ge[2], eA, ehw;
            event_grad<T>(s, code, ue, ge, &eA, &ehw);
            rk4_vjp<T>(s, un, Wst, tau, l, lA, ge, eA, ehw, lhw);
            j = run;
        } else {
            // RUN or CKPT: recompute the segment [base, j) and reverse it
            const long long base = (kind == AK_RUN) ? 0 : run;
            if (j - base < 0 || j - base > C) {
                bad = 1;
                return;
            }
            const int nseg = (int)(j - base);
            if (maps || fly) {
                // the segment's map: formed beforehand (k_adj_maps), or here
                // by the same function (a trace the pool had no room for), so
                // that both give the same result; a segment ends at the next
                // record
                if (i + 1 >= nrec) {
                    bad = 1;
                    return;
                }
                const double* m = maps ? maps + (long long)kMapFields * i : nullptr;
                double mf[kMapFields];
                if (!maps) {
                    if constexpr (sizeof(T) == 8) {
                        if (!adj_segment_map(s_in, (double)wfb2, C, o.h, tp_in, i, sg_in, mf)) mf[0] = __builtin_nan("");
                    } else {
                        mf[0] = __builtin_nan("");
                    }
                    m = mf;
                }
                if (!(m[0] == m[0])) {
                    bad = 1;
                    return;
                }
                double ln[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double lk = (double)l[k];
#pragma unroll
                    for (int r = 0; r < 4; ++r) ln[r] += lk * m[4 * k + r];
                    lA += lk * m[16 + k];
                }
                l[0] = (T)ln[0]; l[1] = (T)ln[1]; l[2] = (T)ln[2]; l[3] = (T)ln[3];
                j = base;
                continue;
            }
            AS<T> u = as_make<T>(*tp.at(i, 0), *tp.at(i, 1), *tp.at(i, 2), *tp.at(i, 3),
                                 {(T)*tp.at(i, 4), (T)*tp.at(i, 5)});
            for (int q = 0; q < nseg; ++q) {
                cx<T> Wst[4];
                AS<T> ue;
                adj_rk4<T>(s, wfb2, u, h, ue, Wst);
                *sg.at(q, 0) = u.x; *sg.at(q, 1) = u.y; *sg.at(q, 2) = u.px; *sg.at(q, 3) = u.py;
                *sg.at(q, 4) = u.W.re; *sg.at(q, 5) = u.W.im;
                *sg.at(q, 6) = Wst[1].re; *sg.at(q, 7) = Wst[1].im;
                *sg.at(q, 8) = Wst[2].re; *sg.at(q, 9) = Wst[2].im;
                *sg.at(q, 10) = Wst[3].re; *sg.at(q, 11) = Wst[3].im;
                u = ue;
            }
            for (int q = nseg - 1; q >= 0; --q) {
                // (the stages are built from hi only, so lo is not needed here)
                const AS<T> uq = {*sg.at(q, 0), *sg.at(q, 1), *sg.at(q, 2), *sg.at(q, 3), {*sg.at(q, 4), *sg.at(q, 5)},
                                  (T)0, (T)0, (T)0, (T)0};
                const cx<T> Wst[4] = {uq.W, {*sg.at(q, 6), *sg.at(q, 7)}, {*sg.at(q, 8), *sg.at(q, 9)},
                                      {*sg.at(q, 10), *sg.at(q, 11)}};
                rk4_vjp<T>(s, uq, Wst, h, l, lA, nullptr, (T)0, (T)0, lhw);
            }
            j = base;
        }
    }
    // sensitivity of the colour to the initial direction (the adjoint of
    // the camera ray's momentum): how much rounding in the trace is amplified
    sens = sqrt(lp[0] * lp[0] + lp[1] * lp[1] + lp[2] * lp[2]);
}

// The reverse sweep as one compiled function (the in-lane and pooled paths
// share it); its sums live in registers and are written back at the end.
template <typename T>
__device__ __noinline__ void adj_reverse(const SceneDev& s, const OptsDev& o, T wfb2, int C, const AdjTape& tp, int nrec,
                                         const AdjSeg<T>& sg, const double out_dir[3], double lm,
                                         double& lA, double& lhw, int& bad, double& sens, const double* maps,
                                         bool fly = false)
{
    double lA_l = lA, lhw_l = lhw, sens_l = sens;
    int bad_l = bad;
    adj_reverse_body<T>(s, o, wfb2, C, tp, nrec, sg, out_dir, lm, lA_l, lhw_l, bad_l, sens_l, maps, fly);
    lA = lA_l;
    lhw = lhw_l;
    bad = bad_l;
    sens = sens_l;
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
// correlation statistics of the finished image g against the reference f
// (eq. (14)-(15)): channel means, pooled centred sums, C0 and NCC
struct AdjCC {
    double mf[4], mg[4];
    double sff, sgg, sfg;
    double c0, ncc;
};

// A long trace of the second pass whose reverse sweep runs after its
// segment maps are formed: its tape is in the pool from record `off` on.
struct AdjLong {
    long long sidx, off;
    int nrec;
    double od[3];                 // its exit direction (the sky's argument)
};

struct AdjIo {
    long long n;                  // samples to process (list length when list is set)
    const long long* list;        // sample indices of the second pass (null: 0 .. n-1): list_front
                                  // entries from its start, the rest from its end (list_cap entries)
    long long list_front, list_cap;
    unsigned long long* claim;    // work counter (64 samples per claim)
    double* tape;
    int cap;                      // tape slots per lane
    void* seg;                    // segment buffer, C x 12 values of T per lane
    float* srgb;                  // per-sample colour (first pass)
    double* sgrad;                // per-sample dm/dA, dm/dhw
    long long* ovf;               // first pass: samples handed to the second; second pass: null
    long long ovf_cap;            // entries of ovf
    unsigned long long* n_ovf;    // first pass: hand-overs at the front / back of ovf; second: overflows
    long long long_steps;         // hand-overs of more steps go to the front
    unsigned long long* cnt;      // rays (first pass); steps, events, failed (the pass that traces the sample to
                                  // its end); inconsistent tapes; steps reversed and forward steps taken (first
                                  // pass)
    // first FP32 pass: samples whose gradient is recomputed in FP64 -- paths
    // longer than rerun_steps (their trace stops there), or whose sky
    // parameter m is more sensitive to the initial direction than rerun_sens
    // per radian (FP32 rounding would be amplified)
    long long rerun_steps;
    double rerun_sens;
    // second pass: traces of at least pool_min records copy their tape to
    // the pool (while it has room) and leave their reverse sweep to
    // k_adj_maps and k_adj_chain; null pool: every trace reverses here
    double* pool;
    long long pool_cap;           // records the pool holds
    unsigned long long* pool_used;
    int pool_min;
    AdjLong* longs;
    unsigned long long* n_long;
};

__device__ __forceinline__ unsigned long long adj_wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Persistent: each wave claims 64 consecutive samples (neighbouring pixels
// follow similar paths), traces them forward with tapes and reverses them.
template <typename T>
__device__ __forceinline__ void k_adj_body(const SceneDev& s, const CamDev& cam, const OptsDev& o, T wfb2, int C,
                                           const AdjIo& io)
{
    const long long lane = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const AdjTape tp = {io.tape, stride, lane, io.cap};
    const AdjSeg<T> sg = {(T*)io.seg, stride, lane};
    const int wl = threadIdx.x & 63;
    unsigned long long c_rays = 0, c_steps = 0, c_ev = 0, c_fail = 0, c_rev = 0, c_fwd = 0;
    for (;;) {
        unsigned long long base = 0;
        if (wl == 0) base = atomicAdd(io.claim, 64ull);
        base = __shfl(base, 0, 64);
        if (base >= (unsigned long long)io.n) break;
        const unsigned long long q = base + (unsigned long long)wl;
        if (q >= (unsigned long long)io.n) continue;
        // a second pass's entry ~sidx: a sample the first pass stopped early,
        // whose counters are taken here
        const long long qq = (long long)q;
        const long long raw = !io.list ? qq
                              : qq < io.list_front ? io.list[qq] : io.list[io.list_cap - 1 - (qq - io.list_front)];
        const bool redo = raw < 0;
        const long long sidx = redo ? ~raw : raw;
        const long long pix = sidx / cam.spp;
        const int smp = (int)(sidx - pix * cam.spp);
        const int pi = (int)(pix % cam.W), pj = (int)(pix / cam.W);
        double d[3], od[3];
        camera_dir(cam, pi, pj, smp, d);
        int nrec = 0, events = 0;
        long long steps = 0;
        const int st = adj_forward<T>(s, o, wfb2, C, cam.eye, d, tp, nrec, od, steps, events, io.ovf != nullptr,
                                      io.rerun_steps);
        const bool stopped = st == kAdjStopped;
        {
            // a later (FP64) pass overwrites the colour of the samples it redoes
            double rgb[3] = {0.0, 0.0, 0.0};
            if (st == RS_OK) sky_rgb<double>(s.K, od, rgb);
            for (int c = 0; c < 3; ++c) io.srgb[3 * sidx + c] = (float)rgb[c];
        }
        if (!io.list) {
            c_rays++;
            c_fwd += (unsigned long long)steps;
        }
        if ((!io.list && !stopped) || redo) {
            c_steps += (unsigned long long)steps;
            c_ev += (unsigned long long)events;
            c_fail += (st != RS_OK);
        }
        double gA = 0.0, ghw = 0.0;
        bool hand_over = stopped;
        if (st == RS_OK) {
            hand_over = nrec > io.cap || steps > io.rerun_steps;
            // a long trace of the second pass reverses through segment maps:
            // formed in parallel after the pass if its tape fits in the pool,
            // else here, one after the other (the same arithmetic either way)
            const bool by_maps = !hand_over && io.pool && nrec >= io.pool_min;
            if (by_maps) {
                const unsigned long long off = atomicAdd(io.pool_used, (unsigned long long)nrec);
                if (off + (unsigned long long)nrec <= (unsigned long long)io.pool_cap) {
                    double* dst = io.pool + (long long)off * kTapeFields;
                    for (int r = 0; r < nrec; ++r)
#pragma unroll
                        for (int f = 0; f < kTapeFields; ++f) dst[r * kTapeFields + f] = *tp.at(r, f);
                    const unsigned long long k = atomicAdd(io.n_long, 1ull);
                    AdjLong e;
                    e.sidx = sidx;
                    e.off = (long long)off;
                    e.nrec = nrec;
                    e.od[0] = od[0]; e.od[1] = od[1]; e.od[2] = od[2];
                    io.longs[k] = e;
                    continue;   // its dm/dA and dm/dhw come from k_adj_chain
                }
            }
            if (!hand_over) {
                int bad = 0;
                double sens = 0.0;
                adj_reverse<T>(s, o, wfb2, C, tp, nrec, sg, od, 1.0, gA, ghw, bad, sens, nullptr, by_maps);
                if (!io.list) c_rev += (unsigned long long)steps;
                if (bad) {
                    atomicAdd(&io.cnt[4], 1ull);
                    gA = ghw = 0.0;
                }
                hand_over = sens > io.rerun_sens;
            }
        }
        if (hand_over) {
            // the first pass hands the sample to the second (FP64,
            // full-length tapes): long traces from the front of the list,
            // so that they start first, the others from its back; the
            // second pass only counts a tape overflow (it cannot happen)
            if (io.ovf) {
                const long long entry = stopped ? ~sidx : sidx;
                if (steps > io.long_steps) {
                    const unsigned long long k = atomicAdd(io.n_ovf, 1ull);
                    io.ovf[k] = entry;
                } else {
                    const unsigned long long k = atomicAdd(io.n_ovf + 1, 1ull);
                    io.ovf[io.ovf_cap - 1 - (long long)k] = entry;
                }
                continue;
            }
            atomicAdd(io.n_ovf, 1ull);
            gA = ghw = 0.0;
        }
        io.sgrad[2 * sidx] = gA;
        io.sgrad[2 * sidx + 1] = ghw;
    }
    c_rays = adj_wave_sum(c_rays);
    c_steps = adj_wave_sum(c_steps);
    c_ev = adj_wave_sum(c_ev);
    c_fail = adj_wave_sum(c_fail);
    c_rev = adj_wave_sum(c_rev);
    c_fwd = adj_wave_sum(c_fwd);
    if (wl == 0) {
        atomicAdd(&io.cnt[0], c_rays);
        atomicAdd(&io.cnt[1], c_steps);
        atomicAdd(&io.cnt[2], c_ev);
        atomicAdd(&io.cnt[3], c_fail);
        atomicAdd(&io.cnt[5], c_rev);
        atomicAdd(&io.cnt[6], c_fwd);
    }
}

// The adjoint kernel: the FP64 pass (and the FP64 gradient) at one wave
// per SIMD; the FP32 first pass at two, which its registers allow with
// some of them spilled (its instruction stream, and so its results, are the
// same): the pass waits on latency, and the second wave hides part of it.
template <typename T>
__global__ void __launch_bounds__(256) k_adj(SceneDev s, CamDev cam, OptsDev o, T wfb2, int C, AdjIo io)
{
    k_adj_body<T>(s, cam, o, wfb2, C, io);
}

template <>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_adj<float>(SceneDev s, CamDev cam, OptsDev o, float wfb2, int C, AdjIo io)
{
    k_adj_body<float>(s, cam, o, wfb2, C, io);
}

// Segment maps of the pooled tapes, one RUN or CKPT record per task, all
// records of all pooled traces in parallel (grid-stride).  A record whose
// map cannot be formed gets a NaN marker, which k_adj_chain counts as an
// inconsistent tape.
__global__ void __launch_bounds__(256) k_adj_maps(SceneDev s, OptsDev o, double wfb2, int C, double* pool,
                                                  const unsigned long long* pool_used, long long pool_cap,
                                                  double* maps, double* seg)
{
    const long long lane = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const AdjSeg<double> sg = {seg, stride, lane};
    const long long taken = (long long)*pool_used;
    const long long used = taken < pool_cap ? taken : pool_cap;
    const AdjTape tp = {pool, 1, 0, (int)used};
    for (long long g = lane; g < used; g += stride) {
        const int kind = (int)((long long)pool[g * kTapeFields + 7] & 7);
        if (kind != AK_RUN && kind != AK_CKPT) continue;
        double* m = maps + g * kMapFields;
        if (g + 1 >= used || !adj_segment_map(s, wfb2, C, o.h, tp, (int)g, sg, m)) m[0] = __builtin_nan("");
    }
}

// Reverse sweeps of the pooled traces, one per lane, through their segment
// maps; writes their dm/dA and dm/dhw.
__global__ void __launch_bounds__(256) k_adj_chain(SceneDev s, OptsDev o, double wfb2, int C, const double* pool,
                                                   const double* maps, const AdjLong* longs,
                                                   const unsigned long long* n_long, double* seg, double* sgrad,
                                                   unsigned long long* cnt)
{
    const long long lane = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const AdjSeg<double> sg = {seg, stride, lane};
    const long long n = (long long)*n_long;
    for (long long k = lane; k < n; k += stride) {
        const AdjLong e = longs[k];
        const AdjTape tp = {const_cast<double*>(pool) + e.off * kTapeFields, 1, 0, e.nrec};
        double gA = 0.0, ghw = 0.0, sens = 0.0;
        int bad = 0;
        adj_reverse<double>(s, o, wfb2, C, tp, e.nrec, sg, e.od, 1.0, gA, ghw, bad, sens, maps + e.off * kMapFields);
        if (bad) {
            atomicAdd(&cnt[4], 1ull);
            gA = ghw = 0.0;
        }
        sgrad[2 * e.sidx] = gA;
        sgrad[2 * e.sidx + 1] = ghw;
    }
}

// pixel colour = mean of its samples
__global__ void __launch_bounds__(256) k_adj_image(const float* __restrict__ srgb, long long npix, int spp,
                                                   float* __restrict__ img)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    for (int c = 0; c < 3; ++c) {
        double a = 0.0;
        for (int k = 0; k < spp; ++k) a += (double)srgb[3 * (p * spp + k) + c];
        img[3 * p + c] = (float)(a / spp);
    }
}

// Correlation statistics from the block partials of k_cc_moments (5
// moments x 4 channels, shifted by the first pixel of each image).
__global__ void __launch_bounds__(64) k_adj_ccstat(const double* __restrict__ part, int nblocks, long long npix,
                                                   const float* __restrict__ img, const float* __restrict__ ref,
                                                   AdjCC* cs)
{
    __shared__ double tot[5][4];
    const int t = threadIdx.x;
    if (t < 20) {
        double v = 0.0;
        for (int b = 0; b < nblocks; ++b) v += part[(long long)b * 20 + t];
        tot[t / 4][t % 4] = v;
    }
    __syncthreads();
    if (t == 0) {
        const double N = (double)npix;
        double sff = 0.0, sgg = 0.0, sfg = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double a = tot[0][c] / N, b = tot[1][c] / N;
            cs->mf[c] = (double)ref[c] + a;
            cs->mg[c] = (double)img[c] + b;
            sff += tot[2][c] - N * a * a;
            sgg += tot[3][c] - N * b * b;
            sfg += tot[4][c] - N * a * b;
        }
        cs->mf[3] = cs->mg[3] = 0.0;
        cs->sff = sff;
        cs->sgg = sgg;
        cs->sfg = sfg;
        cs->c0 = sfg / sff;
        cs->ncc = sfg / sqrt(sff * sgg);
    }
}

// dL/dtheta = sum over samples of w_s dm_s/dtheta, w_s = sum_c dL/dg_{p,c}
// (Ca_c - Cb_c) / spp, with dL/dg = -f' / sum f'^2 for L = 1 - C0 (kind 0)
// or -(f' / sqrt(sum f'^2 sum g'^2) - NCC g' / sum g'^2) for L = 1 - NCC
// (kind 1).  One block, fixed summation order.
__global__ void __launch_bounds__(1024) k_adj_reduce(const double* __restrict__ sgrad, long long n, int spp,
                                                     const float* __restrict__ img, const float* __restrict__ ref,
                                                     const AdjCC* __restrict__ cs, int kind, double* __restrict__ out)
{
    __shared__ double red[2][1024];
    const double Ca[3] = {0.95, 0.85, 0.30}, Cb[3] = {0.10, 0.20, 0.55};
    const double af = kind == 0 ? 1.0 / cs->sff : 1.0 / sqrt(cs->sff * cs->sgg);
    const double ag = kind == 0 ? 0.0 : cs->ncc / cs->sgg;
    double a = 0.0, b = 0.0;
    for (long long q = threadIdx.x; q < n; q += blockDim.x) {
        const long long p = q / spp;
        double w = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double fp = (double)ref[3 * p + c] - cs->mf[c];
            const double gp = (double)img[3 * p + c] - cs->mg[c];
            w -= (af * fp - ag * gp) * (Ca[c] - Cb[c]);
        }
        w /= (double)spp;
        a += w * sgrad[2 * q];
        b += w * sgrad[2 * q + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            red[0][threadIdx.x] += red[0][threadIdx.x + k];
            red[1][threadIdx.x] += red[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

}  // namespace gc
