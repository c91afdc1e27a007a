// gc_lane64.hpp -- FP64 per-lane ray tracer: free flight in air, box
// entry and exit with Snell's law, integration inside the cloak, grating
// contacts, and the event machinery shared with the FP32 path.
//
// Steps of one ray (Sec. 3 and Sec. 4):
//   air:   straight line (the acceleration of eq. (11) vanishes outside the
//          cloak) to the nearest of: the cloak box (Snell refraction into
//          it), the bare grating of eq. (2) (mirror reflection), or nothing
//          (the ray escapes to the sky);
//   cloak: RK4 or DOPRI5 steps of dr/dtau = p, dp/dtau = grad(n^2)/2; a step
//          whose end leaves the box (y > y_top, |x| > half_width) or enters
//          the metal (virtual coordinate v = y + Re W / k < 0) is replaced by
//          the partial step of the same integrator that ends on that surface;
//          then the ray reflects (grating, or total internal reflection at a
//          face) or refracts out of the box.
#pragma once
#include "gc_math.hpp"

namespace gc {

constexpr double kInf = __builtin_huge_val();

struct St64 { double x, y, px, py; };

struct LaneCount {
    long long steps, rejected;
    int events;
    int fallbacks;
};

// ---------------------------------------------------------------------------
// Grating geometry, eq. (2): x = xi - A sin(k xi), y = A cos(k xi).
// ---------------------------------------------------------------------------
// Solve M = E - e sin E (e < 1) for E: safeguarded Newton in [M - e, M + e].
// It stops once the residual is at the rounding level of its terms (with
// the last Newton step applied): at that point the Newton iterate lands on
// an end of the bracket, where the safeguard would otherwise bisect on.
__device__ inline double kepler_E(double M, double e)
{
    double lo = M - e, hi = M + e;
    double E = M + e * sin(M);
    const double noise = 4.0 * 2.220446049250313e-16 * (fabs(M) + 2.0 * e + 1.0);
    for (int it = 0; it < 60; ++it) {
        double sn, c;
        sincos(E, &sn, &c);
        const double f = E - e * sn - M;
        const double dE = f / (1.0 - e * c);
        if (fabs(f) <= noise) { E -= dE; break; }
        if (f > 0.0) hi = E; else lo = E;
        double En = E - dE;
        if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
        const double step = En - E;
        E = En;
        if (fabs(step) <= 1e-15 * fmax(1.0, fabs(E))) break;
    }
    return E;
}

// trochoid parameter xi of the surface point above/below x
__device__ inline double xi_of_x(const SceneDev& s, double x)
{
    double N = rint(x * s.invL);
    double E = kepler_E(s.k * (x - N * s.L), s.e);
    return E / s.k + N * s.L;
}

// G(xi) = d_y (X(xi) - x0) - d_x (Y(xi) - y0): zero where the line through
// (x0, y0) with direction (d_x, d_y) meets the trochoid.
__device__ inline double line_G(const SceneDev& s, double xi, double x0, double y0, double dx, double dy,
                                double* dG)
{
    double sn, c;
    sincos(s.k * xi, &sn, &c);
    double X = xi - s.A * sn, Y = s.A * c;
    if (dG) *dG = dy * (1.0 - s.e * c) + dx * s.e * sn;
    return dy * (X - x0) - dx * (Y - y0);
}

// First contact of the ray r + t d (t > 0) with the bare metal surface; +inf
// if none.  Writes the trochoid parameter of the contact point to *xi_hit.
// G'(xi) = d_y - e R cos(k xi + phi) with R = |(d_x, d_y)|, so G is monotone
// between consecutive critical points k xi + phi = +-acos(d_y / (e R)) + 2 pi m.
// Above the surface sign(G) = sign(d_x); the first piece (in the direction of
// travel) over which sign(d_x) G drops from positive to non-positive holds
// the contact, found by safeguarded Newton.
__device__ __noinline__ double air_contact(const SceneDev& s, const double r[3], const double d[3], double* xi_hit)
{
    const double x0 = r[0], y0 = r[1], dx = d[0], dy = d[1];
    if (s.mirror == 1 || s.A == 0.0) {
        *xi_hit = 0.0;
        if (dy < 0.0 && y0 > 0.0) return -y0 / dy;
        if (dy < 0.0 && y0 >= 0.0) return 0.0;
        return kInf;
    }
    const double A = s.A;
    double t0 = 0.0, t1;
    if (dy < 0.0) {
        if (y0 > A) t0 = (A - y0) / dy;
        t1 = (-A - y0) / dy * (1.0 + 1e-12);
    } else if (dy > 0.0) {
        if (y0 >= A) return kInf;
        t1 = (A - y0) / dy;
    } else {
        if (y0 > A || y0 < -A || dx == 0.0) return kInf;
        t1 = s.L / fabs(dx);
    }
    const bool at_origin = (t0 == 0.0);
    if (dx == 0.0) {
        // the line stays above one surface point
        double xi = xi_of_x(s, x0);
        double S = A * cos(s.k * xi);
        *xi_hit = xi;
        double t = (S - y0) / dy;
        if (dy < 0.0 && t > 0.0) return t;
        return kInf;
    }
    const double sg = dx > 0.0 ? 1.0 : -1.0;
    const double xia = xi_of_x(s, x0 + t0 * dx);
    const double xib = xi_of_x(s, x0 + t1 * dx);
    const double R = sqrt(dx * dx + dy * dy);
    const double phi = atan2(dx, dy);
    const bool has_crit = fabs(dy) < s.e * R;
    const double alpha = has_crit ? acos(dy / (s.e * R)) : 0.0;
    double xi = xia;
    double G = sg * line_G(s, xi, x0, y0, dx, dy, nullptr);
    if (!at_origin && G <= 0.0) { *xi_hit = xia; return t0; }
    // critical phases in increasing order: c(2m) = -alpha + 2 pi m,
    // c(2m + 1) = alpha + 2 pi m; walk them by index in the travel direction
    long long j = 0;
    if (has_crit) {
        const double th = s.k * xia + phi;
        if (sg > 0.0) {
            long long m = (long long)floor((th + alpha) * kInvTwoPi);
            j = (alpha + kTwoPi * m > th) ? 2 * m + 1 : 2 * m + 2;
        } else {
            long long m = (long long)ceil((th - alpha) * kInvTwoPi) - 1;
            j = (-alpha + kTwoPi * (m + 1) < th) ? 2 * m + 2 : 2 * m + 1;
        }
    }
    for (int piece = 0; piece < 1 << 16; ++piece) {
        double xn = xib;
        if (has_crit) {
            long long m = (j >= 0) ? j / 2 : -((-j + 1) / 2);
            double tn = ((j - 2 * m) == 1 ? alpha : -alpha) + kTwoPi * (double)m;
            double xc = (tn - phi) / s.k;
            xn = (sg > 0.0) ? fmin(xc, xib) : fmax(xc, xib);
            j += (sg > 0.0) ? 1 : -1;
        }
        double Gn = sg * line_G(s, xn, x0, y0, dx, dy, nullptr);
        if (G > 0.0 && Gn <= 0.0) {
            // monotone bracket [xi, xn]: safeguarded Newton on G
            double lo = xi, hi = xn;   // sg*G(lo) > 0 >= sg*G(hi)
            double z = 0.5 * (lo + hi);
            for (int it = 0; it < 100; ++it) {
                double dG;
                double g = sg * line_G(s, z, x0, y0, dx, dy, &dG);
                dG *= sg;
                // residual at the rounding level of G's terms: converged
                // (see kepler_E); the last Newton step stays in the bracket
                const double noise = 4.0 * 2.220446049250313e-16 *
                                     (fabs(dy) * (fabs(z) + A + fabs(x0)) + fabs(dx) * (A + fabs(y0)));
                if (fabs(g) <= noise) {
                    const double zn = z - g / dG;
                    if ((zn - lo) * (zn - hi) <= 0.0 && isfinite(zn)) z = zn;
                    break;
                }
                if (g > 0.0) lo = z; else hi = z;
                double zn = z - g / dG;
                bool inside = (zn - lo) * (zn - hi) < 0.0;
                if (!inside || !isfinite(zn)) zn = 0.5 * (lo + hi);
                double step = fabs(zn - z);
                z = zn;
                if (step <= 1e-15 * fmax(1.0, fabs(z)) || fabs(hi - lo) <= 1e-15 * fmax(1.0, fabs(z))) break;
            }
            *xi_hit = z;
            double sn, c;
            sincos(s.k * z, &sn, &c);
            double X = z - A * sn, Y = A * c;
            double t = fabs(dx) >= fabs(dy) ? (X - x0) / dx : (Y - y0) / dy;
            return t;
        }
        if (xn == xib) return kInf;
        xi = xn;
        G = Gn;
    }
    return kInf;
}

// Entry of the straight ray into the cloak box from air (face code: 0 top,
// 1 right x = +hw, 2 left x = -hw; -1 none).
__device__ inline double air_box_entry(const SceneDev& s, const double r[3], const double d[3], int* face)
{
    double best = kInf;
    *face = -1;
    if (!s.cloak) return best;
    if (d[1] < 0.0 && r[1] > s.ytop) {
        double t = (s.ytop - r[1]) / d[1];
        double xe = r[0] + t * d[0];
        if (fabs(xe) <= s.hw && t < best) { best = t; *face = 0; }
    }
    if (d[0] < 0.0 && r[0] > s.hw) {
        double t = (s.hw - r[0]) / d[0];
        double ye = r[1] + t * d[1];
        if (ye <= s.ytop && ye >= s.S_hw && t < best) { best = t; *face = 1; }
    }
    if (d[0] > 0.0 && r[0] < -s.hw) {
        double t = (-s.hw - r[0]) / d[0];
        double ye = r[1] + t * d[1];
        if (ye <= s.ytop && ye >= s.S_hw && t < best) { best = t; *face = 2; }
    }
    return best;
}

// Snell's law at a plane with unit normal nf (from medium 1 into 2): keep the
// tangential part, choose the normal part for |p'| = n2; total internal
// reflection when n2^2 < |p_t|^2.  Returns true if transmitted.
__device__ inline bool snell(double p[3], const double nf[3], double n2)
{
    double pn = p[0] * nf[0] + p[1] * nf[1] + p[2] * nf[2];
    double pt[3] = {p[0] - pn * nf[0], p[1] - pn * nf[1], p[2] - pn * nf[2]};
    double q = n2 * n2 - (pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2]);
    if (q < 0.0) {
        for (int i = 0; i < 3; ++i) p[i] -= 2.0 * pn * nf[i];
        return false;
    }
    double pnn = (pn >= 0.0 ? 1.0 : -1.0) * sqrt(q);
    for (int i = 0; i < 3; ++i) p[i] = pt[i] + pnn * nf[i];
    return true;
}

__device__ inline void reflect2(double& px, double& py, double nx, double ny)
{
    double pn = px * nx + py * ny;
    px -= 2.0 * pn * nx;
    py -= 2.0 * pn * ny;
}

// ---------------------------------------------------------------------------
// One FP64 integrator step inside the cloak.  k1 = (p, a1) at u with the
// converged W1 and dW1 = dW/dzeta there.  Returns the end state and the
// W, a, dW at the end point (the next step's first stage).
// ---------------------------------------------------------------------------
struct Rhs64 {
    double ax, ay;
    cx<double> W, dW;
};

__device__ inline void rhs_at(const SceneDev& s, double x, double y, double xp, double yp, const Rhs64& prev,
                              Rhs64& out)
{
    out.W = predict_w<double>(s, prev.W, prev.dW, mk(x - xp, y - yp));
    rhs64(s, x, y, out.W, out.ax, out.ay, out.dW, crosses_cut(s, x, y, xp, yp));
}

__device__ inline void rk4_step64(const SceneDev& s, const St64& u, const Rhs64& r1, double h, St64& ue,
                                  Rhs64& re)
{
    const double hh = 0.5 * h;
    Rhs64 r2, r3, r4;
    double x2 = u.x + hh * u.px, y2 = u.y + hh * u.py;
    double p2x = u.px + hh * r1.ax, p2y = u.py + hh * r1.ay;
    rhs_at(s, x2, y2, u.x, u.y, r1, r2);
    double x3 = u.x + hh * p2x, y3 = u.y + hh * p2y;
    double p3x = u.px + hh * r2.ax, p3y = u.py + hh * r2.ay;
    rhs_at(s, x3, y3, x2, y2, r2, r3);
    double x4 = u.x + h * p3x, y4 = u.y + h * p3y;
    double p4x = u.px + h * r3.ax, p4y = u.py + h * r3.ay;
    rhs_at(s, x4, y4, x3, y3, r3, r4);
    const double h6 = h / 6.0;
    ue.x = u.x + h6 * (u.px + 2.0 * p2x + 2.0 * p3x + p4x);
    ue.y = u.y + h6 * (u.py + 2.0 * p2y + 2.0 * p3y + p4y);
    ue.px = u.px + h6 * (r1.ax + 2.0 * r2.ax + 2.0 * r3.ax + r4.ax);
    ue.py = u.py + h6 * (r1.ay + 2.0 * r2.ay + 2.0 * r3.ay + r4.ay);
    rhs_at(s, ue.x, ue.y, x4, y4, r4, re);
}

// One DOPRI5 step; returns the scaled RMS error over (x, y, px, py) and the
// 5th order end state with its RHS (FSAL).
template <typename T>
__device__ __forceinline__ T dp_comb6(T k1, T k2, T k3, T k4, T k5, T k6, T c1, T c2, T c3, T c4, T c5, T c6)
{
    return c1 * k1 + c2 * k2 + c3 * k3 + c4 * k4 + c5 * k5 + c6 * k6;
}

__device__ inline double dp5_step64(const SceneDev& s, const St64& u, const Rhs64& r1, double h, double rtol,
                                    double atol, St64& ue, Rhs64& re)
{
    double kx[7], ky[7], kax[7], kay[7];
    Rhs64 rp = r1, rn;
    double xp = u.x, yp = u.y;
    kx[0] = u.px; ky[0] = u.py; kax[0] = r1.ax; kay[0] = r1.ay;
    const double A[6][6] = {{DP::a21, 0, 0, 0, 0, 0},
                            {DP::a31, DP::a32, 0, 0, 0, 0},
                            {DP::a41, DP::a42, DP::a43, 0, 0, 0},
                            {DP::a51, DP::a52, DP::a53, DP::a54, 0, 0},
                            {DP::a61, DP::a62, DP::a63, DP::a64, DP::a65, 0},
                            {DP::b1, 0.0, DP::b3, DP::b4, DP::b5, DP::b6}};
#pragma unroll
    for (int st = 1; st < 7; ++st) {
        double sx = 0, sy = 0, sax = 0, say = 0;
#pragma unroll
        for (int j = 0; j < st; ++j) {
            sx += A[st - 1][j] * kx[j];
            sy += A[st - 1][j] * ky[j];
            sax += A[st - 1][j] * kax[j];
            say += A[st - 1][j] * kay[j];
        }
        double x = u.x + h * sx, y = u.y + h * sy;
        kx[st] = u.px + h * sax;
        ky[st] = u.py + h * say;
        rhs_at(s, x, y, xp, yp, rp, rn);
        kax[st] = rn.ax;
        kay[st] = rn.ay;
        rp = rn;
        xp = x;
        yp = y;
        if (st == 6) { ue.x = x; ue.y = y; ue.px = kx[6]; ue.py = ky[6]; }
    }
    re = rp;
    const double E[7] = {DP::e1, 0.0, DP::e3, DP::e4, DP::e5, DP::e6, DP::e7};
    double ex = 0, ey = 0, epx = 0, epy = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        ex += E[j] * kx[j];
        ey += E[j] * ky[j];
        epx += E[j] * kax[j];
        epy += E[j] * kay[j];
    }
    double q0 = h * ex / (atol + rtol * fmax(fabs(u.x), fabs(ue.x)));
    double q1 = h * ey / (atol + rtol * fmax(fabs(u.y), fabs(ue.y)));
    double q2 = h * epx / (atol + rtol * fmax(fabs(u.px), fabs(ue.px)));
    double q3 = h * epy / (atol + rtol * fmax(fabs(u.py), fabs(ue.py)));
    return sqrt(0.25 * (q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3));
}

__device__ inline void partial_step64(const SceneDev& s, const OptsDev& o, const St64& u, const Rhs64& r1,
                                      double h, St64& ue, Rhs64& re)
{
    if (o.integ == 0) rk4_step64(s, u, r1, h, ue, re);
    else (void)dp5_step64(s, u, r1, h, o.rtol, o.atol, ue, re);
}

// event functions, >= 0 inside the box: 0 top, 1 right, 2 left, 3 grating
__device__ inline double event_fn(const SceneDev& s, int ev, const St64& u, const Rhs64& r)
{
    switch (ev) {
    case 0: return s.ytop - u.y;
    case 1: return s.hw - u.x;
    case 2: return s.hw + u.x;
    default: return u.y + r.W.re / s.k;
    }
}

// d/dtau of event function `ev` at state u with RHS r
__device__ inline double event_rate(const SceneDev& s, int ev, const St64& u, const Rhs64& r)
{
    switch (ev) {
    case 0: return -u.py;
    case 1: return -u.px;
    case 2: return u.px;
    default: return u.py + (u.px * r.dW.re - u.py * r.dW.im) / s.k;   // v = y + Re W / k
    }
}

// Root in (0, 1) of the cubic Hermite interpolant of an event function with
// values f0 >= 0 > f1 and slopes m0, m1 (per unit theta): the first sign
// change on an 8-point grid, refined by bisection + Newton on the cubic.
__device__ inline double hermite_root(double f0, double f1, double m0, double m1, double* slope)
{
    auto P = [&](double t, double* dp) {
        double t2 = t * t, t3 = t2 * t;
        if (dp) *dp = (6 * t2 - 6 * t) * f0 + (3 * t2 - 4 * t + 1) * m0 + (-6 * t2 + 6 * t) * f1 + (3 * t2 - 2 * t) * m1;
        return (2 * t3 - 3 * t2 + 1) * f0 + (t3 - 2 * t2 + t) * m0 + (-2 * t3 + 3 * t2) * f1 + (t3 - t2) * m1;
    };
    double lo = 0.0, hi = 1.0;
    for (int i = 1; i <= 8; ++i) {
        double t = i * 0.125;
        if (P(t, nullptr) < 0.0) { hi = t; lo = t - 0.125; break; }
    }
    double t = 0.5 * (lo + hi);
    for (int it = 0; it < 40; ++it) {
        double dp;
        double p = P(t, &dp);
        if (p < 0.0) hi = t; else lo = t;
        double tn = (dp != 0.0) ? t - p / dp : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - t) < 1e-15 || hi - lo < 1e-15) { t = tn; break; }
        t = tn;
    }
    P(t, slope);
    return t;
}

// Rounding level of the event functions: they are differences of
// coordinates as large as y_top or half_width, so values within a few ulps
// of those are zero to working precision.
__device__ inline double event_noise64(const SceneDev& s)
{
    const double scale = 1.0 + (isfinite(s.ytop) ? fabs(s.ytop) : 0.0) + (isfinite(s.hw) ? fabs(s.hw) : 0.0);
    return 4.0 * 1.1102230246251565e-16 * scale;
}

// Smallest theta in (0, 1] at which event `ev` of the partial step Phi(theta h)
// crosses zero.  f0 / f1: event values at the step start / full-step end
// (f1 < 0), rates d0 / d1 their tau-derivatives.  The first trial is the
// root of the cubic Hermite interpolant; then Newton / secant steps
// safeguarded by the bracket [lo, hi] (e >= 0 at lo, e < 0 at hi).  It ends
// when the bracket is 1e-14 wide or when the upper end is on the surface to
// rounding (-noise <= e < 0); a trial that lands on the surface to rounding
// from the inside is followed by one placed just across it.  Returns hi.
__device__ inline double locate_event(const SceneDev& s, const OptsDev& o, int ev, const St64& u,
                                      const Rhs64& r1, double h, double f0, double f1, double d0, double d1,
                                      const St64& u_end, const Rhs64& r_end, St64& u_hi, Rhs64& r_hi)
{
    u_hi = u_end;
    r_hi = r_end;
    const double fnoise = event_noise64(s);
    double lo = 0.0, hi = 1.0;
    double slope = 0.0;
    double x = hermite_root(fmax(f0, 0.0), f1, h * d0, h * d1, &slope);
    double xprev = -1.0, fprev = 0.0;
    for (int it = 0; it < 60; ++it) {
        St64 ue;
        Rhs64 re;
        partial_step64(s, o, u, r1, x * h, ue, re);
        const double fx = event_fn(s, ev, ue, re);
        if (fx < 0.0) {
            hi = x;
            u_hi = ue;
            r_hi = re;
            if (fx >= -fnoise) break;
        } else {
            lo = x;
        }
        if (hi - lo <= 1e-14) break;
        double sl = slope;
        if (xprev >= 0.0 && x != xprev && fx != fprev) sl = (fx - fprev) / (x - xprev);
        double t;
        if (fx >= 0.0 && fx <= fnoise && sl != 0.0)
            t = x + fmax(2.0 * fnoise / fabs(sl), 1e-14);
        else
            t = (sl != 0.0) ? x - fx / sl : 0.5 * (lo + hi);
        if (it >= 20 || !(t > lo && t < hi)) t = 0.5 * (lo + hi);
        xprev = x;
        fprev = fx;
        x = t;
    }
    return hi;
}

// Handle the end of a step that crossed at least one event (FP64).
// u, r1: state and RHS at the step start; ue, re: full-step end.  On return
// u / r1 hold the post-event state (momentum updated) and the return value
// tells whether the ray left the box (out_p then holds the momentum in air,
// out_z advanced accordingly).  *dtau receives the tau advanced.
__device__ inline bool handle_events64(const SceneDev& s, const OptsDev& o, St64& u, Rhs64& r1, double pz,
                                       double h, const St64& ue, const Rhs64& re, double* dtau,
                                       double out_p[3], double* min_cos, double* pin_out = nullptr,
                                       int* face_out = nullptr)
{
    double best = 2.0;
    int hit = -1;
    St64 uc = ue;
    Rhs64 rc = re;
    for (int ev = 0; ev < 4; ++ev) {
        if (ev == 3 && s.mirror == 1) continue;
        double f1 = event_fn(s, ev, ue, re);
        if (!(f1 < 0.0)) continue;
        double f0 = event_fn(s, ev, u, r1);
        St64 uh;
        Rhs64 rh;
        double th = locate_event(s, o, ev, u, r1, h, f0, f1, event_rate(s, ev, u, r1), event_rate(s, ev, ue, re),
                                 ue, re, uh, rh);
        if (th < best) { best = th; hit = ev; uc = uh; rc = rh; }
    }
    *dtau = best * h;
    u = uc;
    r1 = rc;
    if (hit == 3) {
        // grating contact: on the surface W = -A k e^{i k xi}, so the upward
        // normal (A k sin k xi, 1 - A k cos k xi) is (-Im W, 1 + Re W)
        double nx = -rc.W.im, ny = 1.0 + rc.W.re;
        double inv = 1.0 / sqrt(nx * nx + ny * ny);
        nx *= inv;
        ny *= inv;
        double pa = sqrt(u.px * u.px + u.py * u.py + pz * pz);
        *min_cos = fmin(*min_cos, fabs(u.px * nx + u.py * ny) / pa);
        reflect2(u.px, u.py, nx, ny);
        return false;
    }
    double nf[3] = {0.0, 0.0, 0.0};
    if (hit == 0) nf[1] = 1.0; else if (hit == 1) nf[0] = 1.0; else nf[0] = -1.0;
    double p[3] = {u.px, u.py, pz};
    double pa = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    *min_cos = fmin(*min_cos, fabs(p[0] * nf[0] + p[1] * nf[1]) / pa);
    const double pin[3] = {p[0], p[1], p[2]};
    bool through = snell(p, nf, 1.0);
    u.px = p[0];
    u.py = p[1];
    if (!through) return false;
    out_p[0] = p[0];
    out_p[1] = p[1];
    out_p[2] = p[2];
    if (pin_out) { pin_out[0] = pin[0]; pin_out[1] = pin[1]; pin_out[2] = pin[2]; }
    if (face_out) *face_out = hit;
    return true;
}

// Outcome of one step inside the box.
enum StepOutcome { SO_INSIDE = 0, SO_EXITED = 1, SO_FAIL = 2 };

// In-box stepper state carried between steps.
struct Box64 {
    St64 u;
    Rhs64 r1;
    double z, pz, h;
    bool last_rej;
};

// One accepted integrator step from b (FP64), with DOPRI5 step control, event
// detection, location and handling.  On SO_EXITED r_out / p_out hold the
// point where the ray left the box and its momentum in air.  On SO_FAIL
// *status holds the reason.
__device__ inline int box_step64(const SceneDev& s, const OptsDev& o, Box64& b, LaneCount& cnt,
                                 double* min_cos, double r_out[3], double p_out[3], int* status,
                                 double* pin_out = nullptr, int* face_out = nullptr)
{
    St64 ue;
    Rhs64 re;
    double h = b.h, hnext = b.h;
    for (;;) {
        if (o.integ == 0) {
            rk4_step64(s, b.u, b.r1, h, ue, re);
            break;
        }
        double err = dp5_step64(s, b.u, b.r1, h, o.rtol, o.atol, ue, re);
        if (!isfinite(err)) { *status = RS_NONFINITE; return SO_FAIL; }
        if (err > 1.0) {
            h *= fmax(0.2, 0.9 * pow(err, -0.2));
            b.last_rej = true;
            cnt.rejected++;
            if (h < o.h_min) { *status = RS_UNDERFLOW; return SO_FAIL; }
            continue;
        }
        double fac = (err == 0.0) ? 5.0 : 0.9 * pow(err, -0.2);
        fac = fmin(5.0, fmax(0.2, fac));
        if (b.last_rej) fac = fmin(fac, 1.0);
        b.last_rej = false;
        hnext = fmin(h * fac, o.h_max);
        break;
    }
    cnt.steps++;
    if (!(isfinite(ue.x) && isfinite(ue.y) && isfinite(ue.px) && isfinite(ue.py))) {
        *status = RS_NONFINITE;
        return SO_FAIL;
    }
    bool ev = (ue.y > s.ytop) || (ue.x > s.hw) || (ue.x < -s.hw) ||
              (s.mirror == 0 && ue.y + re.W.re / s.k < 0.0);
    if (!ev) {
        b.u = ue;
        b.r1 = re;
        b.z += b.pz * h;
        b.h = hnext;
        return SO_INSIDE;
    }
    double dtau, pout[3];
    bool out = handle_events64(s, o, b.u, b.r1, b.pz, h, ue, re, &dtau, pout, min_cos, pin_out, face_out);
    b.z += b.pz * dtau;
    b.h = (o.integ == 0) ? o.h : hnext;
    if (++cnt.events > o.max_events) { *status = RS_MAX_EVENTS; return SO_FAIL; }
    if (!out) return SO_INSIDE;
    r_out[0] = b.u.x; r_out[1] = b.u.y; r_out[2] = b.z;
    p_out[0] = pout[0]; p_out[1] = pout[1]; p_out[2] = pout[2];
    return SO_EXITED;
}

// Stepper state on entry into the box at (r, p) (p already refracted).
// In-box state just inside a face at r; W is W0 at r (the value the walk
// through air used for the index at the face).
__device__ inline Box64 box_enter64(const SceneDev& s, const OptsDev& o, const double r[3], const double p[3],
                                    cx<double> W)
{
    Box64 b;
    b.u = {r[0], r[1], p[0], p[1]};
    b.z = r[2];
    b.pz = p[2];
    b.r1.W = W;
    rhs64(s, b.u.x, b.u.y, b.r1.W, b.r1.ax, b.r1.ay, b.r1.dW);
    b.h = (o.integ == 0) ? o.h : o.h0;
    b.last_rej = false;
    return b;
}

// Integrate inside the box from (r, p) just inside a face.  On RS_OK r, p
// hold the exit point and the momentum in air (pin_out, face_out: the
// momentum just inside the exit face and the face, 0 top, 1 right, 2 left).
__device__ inline int integrate_box64(const SceneDev& s, const OptsDev& o, double r[3], double p[3],
                                      cx<double> W, LaneCount& cnt, double* min_cos, double* pin_out = nullptr,
                                      int* face_out = nullptr)
{
    Box64 b = box_enter64(s, o, r, p, W);
    for (;;) {
        if (cnt.steps >= o.max_steps) return RS_MAX_STEPS;
        int st = RS_OK;
        int so = box_step64(s, o, b, cnt, min_cos, r, p, &st, pin_out, face_out);
        if (so == SO_FAIL) return st;
        if (so == SO_EXITED) return RS_OK;
    }
}

// Outcome of a walk through air.
enum AirOutcome { AO_ESCAPED = 0, AO_ENTERED = 1, AO_FAIL = 2 };

// Straight flight from (r, p) through air, reflecting off the bare grating,
// until the ray escapes (p = unit exit direction) or enters the box (r on the
// face, p refracted inside, *w_in = W0 at r).  The acceleration of eq. (11)
// vanishes outside the cloak.
__device__ inline int air_walk(const SceneDev& s, const OptsDev& o, double r[3], double p[3], LaneCount& cnt,
                               double* min_cos, int* status, cx<double>* w_in, double* pair_out = nullptr,
                               int* face_out = nullptr)
{
    // highest point of the metal: a ray that enters through the top face
    // above it has met no metal on the way
    const double s_top = (s.mirror == 1 || s.A == 0.0) ? 0.0 : s.A;
    for (;;) {
        if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]) && isfinite(p[0]) && isfinite(p[1]) &&
              isfinite(p[2]))) {
            *status = RS_NONFINITE;
            return AO_FAIL;
        }
        int face;
        double tb = air_box_entry(s, r, p, &face);
        double xi = 0.0;
        const double tg = (face == 0 && s.ytop > s_top) ? kInf : air_contact(s, r, p, &xi);
        if (!(tb < kInf) && !(tg < kInf)) return AO_ESCAPED;
        if (++cnt.events > o.max_events) { *status = RS_MAX_EVENTS; return AO_FAIL; }
        if (tg <= tb) {
            for (int i = 0; i < 3; ++i) r[i] += tg * p[i];
            double nx = 0.0, ny = 1.0;
            if (!(s.mirror == 1 || s.A == 0.0)) {
                double sn, c;
                sincos(s.k * xi, &sn, &c);
                nx = s.e * sn;
                ny = 1.0 - s.e * c;
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
        // the box index at the entry point: eq. (1) (times 1 / n_min for the
        // referenced cloak) or the plate's
        cx<double> W = {0.0, 0.0};
        double n2 = s.nplate;
        if (s.cloak != CK_PLATE) {
            W = w0_cold(zarg64(s, r[0], r[1]));
            n2 = s.nsc / sqrt(norm2(mk(1.0 + W.re, W.im)));
        }
        const double pa[3] = {p[0], p[1], p[2]};
        if (!snell(p, nf, n2)) continue;
        *w_in = W;
        if (pair_out) { pair_out[0] = pa[0]; pair_out[1] = pa[1]; pair_out[2] = pa[2]; }
        if (face_out) *face_out = face;
        return AO_ENTERED;
    }
}

// Straight flight inside the homogeneous plate (CK_PLATE: the index is
// constant, so the acceleration of eq. (11) vanishes) from (r, p) just
// inside a face, |p| = nplate: to the top or a side face ahead, or to the
// mirror (reflection, as in air).  A face refracts into air by Snell's law or
// reflects totally.  On RS_OK r, p hold the exit point and the momentum in
// air (pin_out, face_out as for integrate_box64).
__device__ inline int plate_walk64(const SceneDev& s, const OptsDev& o, double r[3], double p[3], LaneCount& cnt,
                                   double* min_cos, double* pin_out = nullptr, int* face_out = nullptr)
{
    for (;;) {
        if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]) && isfinite(p[0]) && isfinite(p[1]) &&
              isfinite(p[2])))
            return RS_NONFINITE;
        const double pa = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        const double d[3] = {p[0] / pa, p[1] / pa, p[2] / pa};
        double tf = kInf;
        int face = -1;
        if (d[1] > 0.0) { const double t = (s.ytop - r[1]) / d[1]; if (t < tf) { tf = t; face = 0; } }
        if (d[0] > 0.0 && isfinite(s.hw)) { const double t = (s.hw - r[0]) / d[0]; if (t < tf) { tf = t; face = 1; } }
        if (d[0] < 0.0 && isfinite(s.hw)) { const double t = (-s.hw - r[0]) / d[0]; if (t < tf) { tf = t; face = 2; } }
        double xi = 0.0;
        const double tg = air_contact(s, r, d, &xi);
        if (++cnt.events > o.max_events) return RS_MAX_EVENTS;
        if (tg <= tf) {
            for (int i = 0; i < 3; ++i) r[i] += tg * d[i];
            double nx = 0.0, ny = 1.0;
            if (!(s.mirror == 1 || s.A == 0.0)) {
                double sn, c;
                sincos(s.k * xi, &sn, &c);
                nx = s.e * sn;
                ny = 1.0 - s.e * c;
                const double inv = 1.0 / sqrt(nx * nx + ny * ny);
                nx *= inv;
                ny *= inv;
            }
            *min_cos = fmin(*min_cos, fabs(d[0] * nx + d[1] * ny));
            reflect2(p[0], p[1], nx, ny);
            continue;
        }
        if (!(tf < kInf)) return RS_NONFINITE;
        for (int i = 0; i < 3; ++i) r[i] += tf * d[i];
        double nf[3] = {0.0, 0.0, 0.0};
        if (face == 0) { r[1] = s.ytop; nf[1] = 1.0; }
        else if (face == 1) { r[0] = s.hw; nf[0] = 1.0; }
        else { r[0] = -s.hw; nf[0] = -1.0; }
        *min_cos = fmin(*min_cos, fabs(d[0] * nf[0] + d[1] * nf[1]));
        const double pin[3] = {p[0], p[1], p[2]};
        if (!snell(p, nf, 1.0)) continue;   // total internal reflection
        if (pin_out) { pin_out[0] = pin[0]; pin_out[1] = pin[1]; pin_out[2] = pin[2]; }
        if (face_out) *face_out = face;
        return RS_OK;
    }
}

// Complete path of one ray in FP64.  Returns the status; the exit point and
// the unit exit direction go to out_org / out_dir.
__device__ inline int trace_ray64(const SceneDev& s, const OptsDev& o, const double org[3], const double dir[3],
                                  double out_org[3], double out_dir[3], LaneCount& cnt, double* min_cos)
{
    double r[3] = {org[0], org[1], org[2]};
    double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double p[3] = {dir[0] / nd, dir[1] / nd, dir[2] / nd};
    for (;;) {
        int st = RS_OK;
        cx<double> W;
        int ao = air_walk(s, o, r, p, cnt, min_cos, &st, &W);
        if (ao == AO_FAIL) return st;
        if (ao == AO_ESCAPED) {
            for (int i = 0; i < 3; ++i) { out_org[i] = r[i]; out_dir[i] = p[i]; }
            return RS_OK;
        }
        st = (s.cloak == CK_PLATE) ? plate_walk64(s, o, r, p, cnt, min_cos) : integrate_box64(s, o, r, p, W, cnt, min_cos);
        if (st != RS_OK) return st;
    }
}

// Fresnel reflectance of unpolarised light at a face (Sec. 3: the Fresnel
// equations), from the normal components of the momentum on the two sides:
// pn = |p . N| in the medium of index n1 (= n1 cos of incidence), qn = |q . N|
// of the transmitted momentum in index n2 (= n2 cos of transmission).
__device__ inline double fresnel_R(double pn, double qn, double n1, double n2)
{
    const double rs = (pn - qn) / (pn + qn);
    const double a = n2 * n2 * pn, b = n1 * n1 * qn;
    const double rp = (a - b) / (a + b);
    return 0.5 * (rs * rs + rp * rp);
}

// R at a crossing of the face with outward normal of index `face` (0 top,
// 1 right, 2 left): p1 the momentum on the incoming side, p2 the
// transmitted one; and p1 reflected about the face into refl.
__device__ inline double crossing_R(int face, const double p1[3], const double p2[3], double refl[3])
{
    double nf[3] = {0.0, 0.0, 0.0};
    if (face == 0) nf[1] = 1.0; else if (face == 1) nf[0] = 1.0; else nf[0] = -1.0;
    const double n1 = sqrt(p1[0] * p1[0] + p1[1] * p1[1] + p1[2] * p1[2]);
    const double n2 = sqrt(p2[0] * p2[0] + p2[1] * p2[1] + p2[2] * p2[2]);
    const double d1 = p1[0] * nf[0] + p1[1] * nf[1] + p1[2] * nf[2];
    const double d2 = p2[0] * nf[0] + p2[1] * nf[1] + p2[2] * nf[2];
    for (int i = 0; i < 3; ++i) refl[i] = p1[i] - 2.0 * d1 * nf[i];
    return fresnel_R(fabs(d1), fabs(d2), n1, n2);
}

// Colour of one camera sample in FP64 (the plain path): the backdrop seen
// along the primary path, weighted by the Fresnel transmissions of its face
// crossings, plus, with Fresnel, the path reflected at each of those
// crossings (weight the primary's times R), traced to its end without
// further splits -- rays reflected more than once are neglected (Sec. 3).
// A branch continues the light path up to its crossing, so its caps count
// from the primary's counts there; it runs when it is created, the primary
// waiting in `held`.  Returns the primary's status (a failed sample is
// black); a branch that fails adds nothing.  cnt receives the work of all
// paths.
__device__ inline int shade_ray64(const SceneDev& s, const OptsDev& o, const double org[3], const double dir[3],
                                  LaneCount& cnt, double rgb[3])
{
    struct Leg {
        double r[3], p[3];
        cx<double> W;      // W0 at r for a leg that starts inside (eq. (1) scenes)
        double w;
        bool inside;
        LaneCount pc;      // the path's own counts (its caps)
    };
    const double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    Leg cur = {{org[0], org[1], org[2]}, {dir[0] / nd, dir[1] / nd, dir[2] / nd}, {0.0, 0.0}, 1.0, false,
               {0, 0, 0, 0}};
    Leg held;
    bool branch = false;   // cur is a reflected branch (the primary is held)
    rgb[0] = rgb[1] = rgb[2] = 0.0;
    long long work_steps = 0, work_rej = 0;
    int work_ev = 0;
    for (;;) {
        double mc = 1.0;
        int st = RS_OK;
        bool ended = false, crossed = false;
        double p1[3], p2[3];
        int face = 0;
        const LaneCount before = cur.pc;
        if (!cur.inside) {
            const int ao = air_walk(s, o, cur.r, cur.p, cur.pc, &mc, &st, &cur.W, p1, &face);
            if (ao == AO_FAIL) {
                ended = true;
            } else if (ao == AO_ESCAPED) {
                double c[3];
                backdrop_rgb64(s, cur.r, cur.p, c);
                for (int k = 0; k < 3; ++k) rgb[k] += cur.w * c[k];
                ended = true;
            } else {
                for (int i = 0; i < 3; ++i) p2[i] = cur.p[i];
                cur.inside = true;
                crossed = true;
            }
        } else {
            st = (s.cloak == CK_PLATE) ? plate_walk64(s, o, cur.r, cur.p, cur.pc, &mc, p1, &face)
                                       : integrate_box64(s, o, cur.r, cur.p, cur.W, cur.pc, &mc, p1, &face);
            if (st != RS_OK) {
                ended = true;
            } else {
                for (int i = 0; i < 3; ++i) p2[i] = cur.p[i];
                cur.inside = false;
                crossed = true;
            }
        }
        work_steps += cur.pc.steps - before.steps;
        work_rej += cur.pc.rejected - before.rejected;
        work_ev += cur.pc.events - before.events;
        if (ended) {
            if (!branch) {
                if (st != RS_OK) rgb[0] = rgb[1] = rgb[2] = 0.0;
                cnt.steps += work_steps;
                cnt.rejected += work_rej;
                cnt.events += work_ev;
                return st;
            }
            cur = held;        // the branch is done: back to the primary
            branch = false;
            continue;
        }
        if (crossed && s.fresnel) {
            double refl[3];
            const double R = crossing_R(face, p1, p2, refl);
            if (!branch) {
                held = cur;
                held.w = cur.w * (1.0 - R);
                // the reflected path stays on the incoming side of the face
                Leg b = cur;
                b.w = cur.w * R;
                b.inside = !cur.inside;
                for (int i = 0; i < 3; ++i) b.p[i] = refl[i];
                if (b.inside && s.cloak != CK_PLATE) b.W = w0_cold(zarg64(s, b.r[0], b.r[1]));
                cur = b;
                branch = true;
            } else {
                cur.w *= 1.0 - R;
            }
        }
    }
}

}  // namespace gc
