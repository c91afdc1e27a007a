/*
 * gco.c -- plain, slow FP64 CPU oracle for Newtonian ray tracing of the
 * grating cloak (Halimeh, Schmied, Wegener, Opt. Express 2010).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: every quantity
 * here is written out again from the paper's equations.
 *
 * What is computed, in the paper's order:
 *   - the index profile, eq. (1), with the principal Lambert function W0 of
 *     eq. (13) evaluated by Halley iteration from a cold start;
 *   - its gradient, eq. (12), and the ray acceleration used for integration,
 *     grad(n^2)/2 = n grad n (Sec. 3);
 *   - the trochoid grating of eq. (2) (height S(x) by solving the Kepler-type
 *     equation x = xi - A sin(k xi)), and its normal;
 *   - straight rays in air, Snell refraction at the cloak/air interface, and
 *     mirror reflection at the metal grating (Sec. 3 and Sec. 4);
 *   - Newton-type ray equation inside the cloak (Sec. 3, eq. (11)), written in
 *     the equivalent parameter tau with dr/dtau = p, dp/dtau = grad(n^2)/2 and
 *     |p| = n (dt = n^2 dtau turns it into eq. (11));
 *   - pinhole camera, procedural sky, image averaging;
 *   - mean subtraction and zero-shift cross-correlation, eqs. (14), (15).
 *
 * Readings where the paper is silent (integrator, event rules, camera, sky,
 * colour handling) follow the project's design notes; each is restated at the
 * function that implements it.
 *
 * Parameter blocks are flat arrays so that this file needs no header shared
 * with anything else:
 *   scene[11] = { Lambda, A, half_width, y_top, cloak, mirror, sky_K, fresnel,
 *                 backdrop, backdrop_y, backdrop_period }
 *               cloak: 0 -> n = 1 everywhere, 1 -> eq. (1) inside the box,
 *                      2 -> referenced cloak: eq. (1) / n_min inside the box,
 *                           n_min = 1 / (1 + A k) (Sec. 4, Figs. 5-7),
 *                      3 -> homogeneous dielectric plate of index
 *                           1 / n_min = 1 + A k filling the box (Sec. 4)
 *               mirror: 0 -> trochoid eq. (2), 1 -> flat mirror y = 0
 *               fresnel: 0 -> Snell + total internal reflection, weight 1;
 *                        1 -> Fresnel-weighted faces with one reflected
 *                             branch per crossing of the primary ray (Sec. 3)
 *               backdrop: 0 -> sky at infinity; 1 -> patterned plane
 *                         y = backdrop_y (the photograph, Sec. 4)
 *   opts[10]  = { integrator (0 RK4, 1 DOPRI5), h, rtol, atol, h_max,
 *                 max_events, max_steps, h0, h_min, diagnostics }
 *   camera[16]= { eye xyz, target xyz, fov_y_deg, width, height, spp,
 *                 jitter, scene_index, up xyz, fov_x_deg }  (seed passed
 *                 separately; up = 0 -> +y; fov_x_deg = 0 -> square pixels)
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846

enum { RAY_OK = 0, RAY_MAX_STEPS = 1, RAY_MAX_EVENTS = 2, RAY_NONFINITE = 3,
       RAY_STEP_UNDERFLOW = 4 };

typedef struct {
    double L, A, hw, ytop, K;
    int cloak, mirror, fresnel, backdrop;
    double bd_y, bd_P;   /* backdrop plane height and pattern period */
    double k, e;         /* k = 2 pi / Lambda, e = A k */
    double nscale;       /* index multiplier inside the box: 1 / n_min = 1 + A k for cloak 2, else 1 */
} oscene;

enum { CLOAK_NONE = 0, CLOAK_EQ1 = 1, CLOAK_REF = 2, CLOAK_PLATE = 3 };

void gco_sky(double K, const double d[3], double rgb[3]);

typedef struct {
    int integ;
    double h, rtol, atol, hmax, h0, hmin;
    long max_events;
    long max_steps;
    int diag;      /* 1: record the drift of |p|^2 - n^2 at every accepted step */
} oopts;

static void load_scene(const double* s, oscene* o)
{
    o->L = s[0]; o->A = s[1]; o->hw = s[2]; o->ytop = s[3];
    o->cloak = (int)s[4]; o->mirror = (int)s[5]; o->K = s[6];
    o->fresnel = (int)s[7]; o->backdrop = (int)s[8]; o->bd_y = s[9]; o->bd_P = s[10];
    o->k = 2.0 * ORC_PI / o->L;
    o->e = o->A * o->k;
    /* Sec. 4: referencing divides every index of the cloak by its minimum,
       n_min = 1 / (1 + A k) (the trough of the grating, on the surface) */
    o->nscale = (o->cloak == CLOAK_REF) ? 1.0 + o->e : 1.0;
}

static void load_opts(const double* p, oopts* o)
{
    o->integ = (int)p[0]; o->h = p[1]; o->rtol = p[2]; o->atol = p[3];
    o->hmax = p[4]; o->max_events = (long)p[5]; o->max_steps = (long)p[6];
    o->h0 = p[7]; o->hmin = p[8]; o->diag = (int)p[9];
}

/* ------------------------------------------------------------------------ */
/* Lambert W, principal branch (eq. (13) names it; Sec. 2).                  */
/* Halley's iteration for w e^w = z (Corless, Gonnet, Hare, Jeffrey, Knuth,  */
/* Adv. Comput. Math. 5 (1996)), tried from these starts in turn:            */
/*   |z| < 1/4           : Taylor series  z - z^2 + 3 z^3 / 2                */
/*   |z + 1/e| < 0.3     : branch-point series -1 + p - p^2/3 + 11 p^3 / 72, */
/*                         p = sqrt(2 (e z + 1)), principal square root     */
/*   always              : log(1 + z), then the asymptotic form              */
/*                         L1 - L2 + L2 / L1 with L1 = log z, L2 = log L1    */
/* The cut is z in (-inf, -1/e]; on it the value continuous from above is    */
/* taken (complex.h's log/sqrt follow the sign of a zero imaginary part).    */
/* Returns 0 when converged with |w e^w - z| <= 1e-14 max(|z|, 1e-300) and w */
/* inside the image of the principal branch, 1 otherwise.                    */
/* ------------------------------------------------------------------------ */
static int w0_in_principal_range(cplx w)
{
    double a = creal(w), b = cimag(w);
    if (fabs(b) >= ORC_PI) return 0;
    if (b == 0.0) return a >= -1.0 - 1e-12;
    /* boundary of the principal range: a = -b cot b */
    return a > -b * cos(b) / sin(b) - 1e-10;
}

static int w0_halley(cplx z, cplx w, cplx* out)
{
    for (int it = 0; it < 64; ++it) {
        cplx ew = cexp(w);
        cplx f = w * ew - z;
        cplx wp1 = w + 1.0;
        if (wp1 == 0.0) break;   /* exactly at the branch point */
        cplx d = f / (ew * wp1 - (w + 2.0) * f / (2.0 * wp1));
        w -= d;
        if (!(cabs(d) > 4.0 * DBL_EPSILON * fmax(1.0, cabs(w)))) break;
    }
    *out = w;
    double res = cabs(w * cexp(w) - z);
    int ok = isfinite(creal(w)) && isfinite(cimag(w)) &&
             res <= 1e-14 * fmax(cabs(z), 1e-300) && w0_in_principal_range(w);
    return ok ? 0 : 1;
}

static int orc_w0(cplx z, cplx* out)
{
    const double E = 2.71828182845904523536;
    /* e split into a double plus a small correction so that e z + 1 keeps
       its low bits near the branch point */
    const double E_LO = 1.4456468917292502e-16;
    double az = cabs(z);
    if (az == 0.0) { *out = 0.0; return 0; }
    cplx ezp1 = (E * z + 1.0) + E_LO * z;
    cplx p = csqrt(2.0 * ezp1);
    cplx L1 = clog(z), L2 = clog(L1);
    cplx guess[4];
    int ng = 0;
    if (az < 0.25) guess[ng++] = z - z * z + 1.5 * z * z * z;
    if (cabs(z + 1.0 / E) < 0.3) guess[ng++] = -1.0 + p - p * p / 3.0 + 11.0 / 72.0 * p * p * p;
    guess[ng++] = clog(1.0 + z);
    guess[ng++] = L1 - L2 + L2 / L1;
    /* the first start whose Halley limit passes the residual and the
       principal-range checks wins; otherwise the first limit is returned */
    cplx first = 0.0;
    for (int g = 0; g < ng; ++g) {
        cplx w;
        if (w0_halley(z, guess[g], &w) == 0) { *out = w; return 0; }
        if (g == 0) first = w;
    }
    *out = first;
    return 1;
}

/* Argument of W0 in eq. (1): i c k e^{ik(x+iy)} with c = iA, i.e.
   Z = -A k e^{-k y} (cos kx + i sin kx).  x is reduced modulo Lambda first
   (the profile is Lambda-periodic in x). */
static cplx orc_Z(const oscene* s, double x, double y)
{
    double xr = x - s->L * floor(x / s->L + 0.5);
    double ph = s->k * xr;
    double m = -s->e * exp(-s->k * y);
    return m * cos(ph) + I * (m * sin(ph));
}

/* eq. (1): n = 1 / |1 + W0(Z)| (untruncated profile). */
static double orc_index_raw(const oscene* s, double x, double y, int* bad)
{
    cplx w;
    int r = orc_w0(orc_Z(s, x, y), &w);
    if (bad) *bad |= r;
    return 1.0 / cabs(1.0 + w);
}

/* Ray acceleration grad(n^2)/2 = n grad n for eq. (1).  With W = W0(Z):
   a_x + i a_y = i k conj(W) (1 + W)^2 / |1 + W|^6.  (eq. (12) times n; the
   test-suite checks the two against each other and against differences.) */
static void orc_accel(const oscene* s, double x, double y, double* ax, double* ay, int* bad)
{
    cplx w;
    int r = orc_w0(orc_Z(s, x, y), &w);
    if (bad) *bad |= r;
    cplx d = 1.0 + w;
    double d2 = creal(d) * creal(d) + cimag(d) * cimag(d);
    cplx a = I * s->k * conj(w) * d * d / (d2 * d2 * d2);
    *ax = creal(a);
    *ay = cimag(a);
}

/* Index inside the box: eq. (1) (cloak 1), eq. (1) / n_min (cloak 2, the
   referenced cloak of Sec. 4) or the plate's 1 / n_min = 1 + A k (cloak 3). */
static double box_index(const oscene* s, double x, double y, int* bad)
{
    if (s->cloak == CLOAK_PLATE) return 1.0 + s->e;
    return s->nscale * orc_index_raw(s, x, y, bad);
}

/* eq. (12), literally: grad n in terms of W0. */
static void orc_grad_n_eq12(const oscene* s, double x, double y, double* gx, double* gy)
{
    cplx w;
    orc_w0(orc_Z(s, x, y), &w);
    double re1 = 1.0 + creal(w), im = cimag(w);
    double m2 = re1 * re1 + im * im;
    double m3 = m2 * sqrt(m2);
    *gx = (2.0 * re1 * im / m2 - im) * s->k / m3;
    *gy = ((im * im - re1 * re1) / m2 + re1) * s->k / m3;
}

/* ------------------------------------------------------------------------ */
/* Trochoid grating, eq. (2): x = xi - A sin(k xi), y = A cos(k xi).         */
/* For given x, xi solves Kepler's equation M = E - e sin E with M = k x,    */
/* E = k xi, eccentricity e = A k < 1 (unique root in [M - e, M + e]).       */
/* Safeguarded Newton (bisection when Newton leaves the bracket).            */
/* Returns the height S(x) = A cos(k xi); *Eout = k xi reduced to [-pi,pi).  */
/* ------------------------------------------------------------------------ */
static double orc_surface(const oscene* s, double x, double* Eout)
{
    if (s->mirror == 1) { if (Eout) *Eout = 0.0; return 0.0; }
    double N = floor(x / s->L + 0.5);
    double M = s->k * (x - N * s->L);
    double e = s->e;
    double lo = M - e, hi = M + e;
    double E = M + e * sin(M);
    if (E < lo || E > hi) E = M;
    for (int it = 0; it < 200; ++it) {
        double f = E - e * sin(E) - M;
        if (f > 0) hi = E; else lo = E;
        double fp = 1.0 - e * cos(E);
        double En = E - f / fp;
        if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
        double dE = En - E;
        E = En;
        if (fabs(dE) <= 1e-15 * fmax(1.0, fabs(E)) || hi - lo <= 1e-15) break;
    }
    if (Eout) *Eout = E;
    return s->A * cos(E);
}

/* Upward unit normal of the grating at parameter E = k xi (points out of the
   metal, +y side).  From eq. (2): tangent (1 - e cos E, -e sin E). */
static void orc_grating_normal(const oscene* s, double E, double* nx, double* ny)
{
    if (s->mirror == 1) { *nx = 0.0; *ny = 1.0; return; }
    double a = s->e * sin(E), b = 1.0 - s->e * cos(E);
    double r = sqrt(a * a + b * b);
    *nx = a / r;
    *ny = b / r;
}

/* ------------------------------------------------------------------------ */
/* Ray state and integrators.                                                */
/* Only (x, y, px, py) evolve non-trivially: n does not depend on z, so p_z  */
/* is constant and z advances by p_z per unit tau.                           */
/* ------------------------------------------------------------------------ */
typedef struct { double v[4]; } st4;   /* x, y, px, py */

/* dr/dtau = p, dp/dtau = grad(n^2)/2 with n the box index: for the
   referenced cloak n = s n1 (s = 1 / n_min) and grad(n^2)/2 = s^2 n1 grad n1. */
static void rhs(const oscene* s, const st4* u, st4* du, int* bad)
{
    double ax, ay;
    orc_accel(s, u->v[0], u->v[1], &ax, &ay, bad);
    const double s2 = s->nscale * s->nscale;
    du->v[0] = u->v[2];
    du->v[1] = u->v[3];
    du->v[2] = s2 * ax;
    du->v[3] = s2 * ay;
}

static void axpy(st4* out, const st4* u, double h, const st4* k)
{
    for (int i = 0; i < 4; ++i) out->v[i] = u->v[i] + h * k->v[i];
}

/* Classical 4-stage Runge-Kutta step of size h. */
static void rk4_step(const oscene* s, const st4* u, double h, st4* out, int* bad)
{
    st4 k1, k2, k3, k4, t;
    rhs(s, u, &k1, bad);
    axpy(&t, u, 0.5 * h, &k1); rhs(s, &t, &k2, bad);
    axpy(&t, u, 0.5 * h, &k2); rhs(s, &t, &k3, bad);
    axpy(&t, u, h, &k3);       rhs(s, &t, &k4, bad);
    for (int i = 0; i < 4; ++i)
        out->v[i] = u->v[i] + (h / 6.0) * (k1.v[i] + 2.0 * k2.v[i] + 2.0 * k3.v[i] + k4.v[i]);
}

/* Dormand-Prince 5(4) tableau (Dormand & Prince, J. Comput. Appl. Math. 6
   (1980) 19-26): 5th-order solution propagated, 4th-order embedded for the
   error estimate, first-same-as-last. */
static const double DP_A[7][6] = {
    { 0 },
    { 1.0 / 5 },
    { 3.0 / 40, 9.0 / 40 },
    { 44.0 / 45, -56.0 / 15, 32.0 / 9 },
    { 19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729 },
    { 9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656 },
    { 35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84 },
};
static const double DP_B5[7] = { 35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0.0 };
static const double DP_B4[7] = { 5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640,
                                 -92097.0 / 339200, 187.0 / 2100, 1.0 / 40 };

/* The tableau as used above (test access): A[7][6] row-major, then b5[7],
   then b4[7]. */
void gco_dp5_tableau(double* out)
{
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 6; ++j) out[6 * i + j] = DP_A[i][j];
    for (int i = 0; i < 7; ++i) { out[42 + i] = DP_B5[i]; out[49 + i] = DP_B4[i]; }
}

/* One DOPRI5 step of size h from u with k1 = f(u) given.  Writes the 5th
   order result, the 4th order result and k7 = f(result). */
static void dp5_step(const oscene* s, const st4* u, const st4* k1, double h,
                     st4* y5, st4* y4, st4* k7, int* bad)
{
    st4 K[7];
    K[0] = *k1;
    for (int st = 1; st < 7; ++st) {
        st4 t = *u;
        for (int j = 0; j < st; ++j)
            for (int i = 0; i < 4; ++i) t.v[i] += h * DP_A[st][j] * K[j].v[i];
        if (st == 6) *y5 = t;
        rhs(s, &t, &K[st], bad);
    }
    for (int i = 0; i < 4; ++i) {
        double a5 = 0.0, a4 = 0.0;
        for (int j = 0; j < 7; ++j) { a5 += DP_B5[j] * K[j].v[i]; a4 += DP_B4[j] * K[j].v[i]; }
        y5->v[i] = u->v[i] + h * a5;
        y4->v[i] = u->v[i] + h * a4;
    }
    *k7 = K[6];
}

/* ------------------------------------------------------------------------ */
/* Box B = { |x| <= hw, y <= y_top, y above the grating } (cloak = 1).       */
/* Event functions, all >= 0 inside B.                                       */
/* ------------------------------------------------------------------------ */
enum { EV_NONE = -1, EV_TOP = 0, EV_RIGHT = 1, EV_LEFT = 2, EV_GRATING = 3 };

static double event_value(const oscene* s, int ev, const st4* u)
{
    switch (ev) {
    case EV_TOP:   return s->ytop - u->v[1];
    case EV_RIGHT: return s->hw - u->v[0];
    case EV_LEFT:  return s->hw + u->v[0];
    default:       return u->v[1] - orc_surface(s, u->v[0], NULL);
    }
}

/* Snell's law at a planar face with unit normal nf (pointing from medium 1
   into medium 2): the tangential part of p is kept and the normal part is
   chosen so that |p'| = n2.  Total internal reflection when n2^2 < |p_t|^2:
   mirror reflection about the face.  Returns 1 if transmitted. */
static int snell(double p[3], const double nf[3], double n2)
{
    double pn = p[0] * nf[0] + p[1] * nf[1] + p[2] * nf[2];
    double pt[3] = { p[0] - pn * nf[0], p[1] - pn * nf[1], p[2] - pn * nf[2] };
    double pt2 = pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2];
    double q = n2 * n2 - pt2;
    if (q < 0.0) {
        for (int i = 0; i < 3; ++i) p[i] -= 2.0 * pn * nf[i];
        return 0;
    }
    double pnn = (pn >= 0.0 ? 1.0 : -1.0) * sqrt(q);
    for (int i = 0; i < 3; ++i) p[i] = pt[i] + pnn * nf[i];
    return 1;
}

static void reflect(double p[3], double nx, double ny)
{
    double pn = p[0] * nx + p[1] * ny;
    p[0] -= 2.0 * pn * nx;
    p[1] -= 2.0 * pn * ny;
}

/* First contact of the straight line r + t d (t > 0, d in the xy-plane
   projection) with the metal surface.  Returns +inf if none.
   g(t) = y(t) - S(x(t)) >= 0 above the metal.  |S'(x)| <= e / sqrt(1 - e^2)
   (maximum slope of the trochoid), so |g'| <= L with
   L = |d_y| + |d_x| e / sqrt(1 - e^2): marching with steps g/L never steps
   over a crossing.  A minimum step of 1e-9 guarantees progress near
   tangency.  The bracket is then refined by bisection to 1e-15. */
static double air_contact(const oscene* s, const double r[3], const double d[3])
{
    double x0 = r[0], y0 = r[1], dx = d[0], dy = d[1];
    if (s->mirror == 1 || s->A == 0.0) {
        if (dy < 0.0 && y0 > 0.0) return -y0 / dy;
        if (dy < 0.0 && y0 >= 0.0) return 0.0;
        return INFINITY;
    }
    double A = s->A;
    double t0 = 0.0, t1;
    if (dy < 0.0) {
        if (y0 > A) t0 = (A - y0) / dy;
        t1 = (-A - y0) / dy * (1.0 + 1e-12);   /* just below the troughs */
    } else if (dy > 0.0) {
        if (y0 >= A) return INFINITY;
        t1 = (A - y0) / dy;
    } else {
        if (y0 > A || y0 < -A || dx == 0.0) return INFINITY;
        t1 = s->L / fabs(dx);
    }
    if (dx == 0.0) {
        /* a vertical line x = x0 meets the trochoid of eq. (2) only at
           (x0, S(x0)): a contact when it moves down onto that point */
        double S = orc_surface(s, x0, NULL);
        if (dy < 0.0 && y0 > S) return (S - y0) / dy;
        return INFINITY;
    }
    double L = fabs(dy) + fabs(dx) * s->e / sqrt(1.0 - s->e * s->e);
    double t = t0, tprev = t0;
    /* a ray that starts on the surface (just reflected) is not in contact */
    int at_origin = (t0 == 0.0);
    for (long it = 0; it < 100000000L; ++it) {
        double g = y0 + t * dy - orc_surface(s, x0 + t * dx, NULL);
        /* a rising ray leaves the band at y = A >= S(x): there g >= 0
           exactly, so a g <= 0 at that end is rounding, not a crossing */
        if (g <= 0.0 && !(at_origin && t == t0) && !(dy > 0.0 && t >= t1)) {
            if (t == t0) return t0;   /* touches the surface where it enters the band */
            double lo = tprev, hi = t;
            for (int b = 0; b < 200 && hi - lo > 1e-15 * fmax(1.0, fabs(hi)); ++b) {
                double mid = 0.5 * (lo + hi);
                double gm = y0 + mid * dy - orc_surface(s, x0 + mid * dx, NULL);
                if (gm <= 0.0) hi = mid; else lo = mid;
            }
            return hi;
        }
        if (t >= t1) return INFINITY;
        tprev = t;
        double step = (g > 0.0 ? g : 0.0) / L;
        if (step < 1e-9) step = 1e-9;
        t += step;
        if (t > t1) t = t1;
    }
    return INFINITY;
}

/* Entry of the straight line into the cloak box from air.  Faces: top
   (y = y_top, |x| <= hw), right (x = hw) and left (x = -hw), the side faces
   spanning from the grating height at that x up to y_top. */
static double air_box_entry(const oscene* s, const double r[3], const double d[3], int* face)
{
    double best = INFINITY;
    *face = EV_NONE;
    if (!s->cloak) return best;
    if (d[1] < 0.0 && r[1] > s->ytop) {
        double t = (s->ytop - r[1]) / d[1];
        double xe = r[0] + t * d[0];
        if (fabs(xe) <= s->hw && t < best) { best = t; *face = EV_TOP; }
    }
    if (d[0] < 0.0 && r[0] > s->hw) {
        double t = (s->hw - r[0]) / d[0];
        double ye = r[1] + t * d[1];
        if (ye <= s->ytop && ye >= orc_surface(s, s->hw, NULL) && t < best) { best = t; *face = EV_RIGHT; }
    }
    if (d[0] > 0.0 && r[0] < -s->hw) {
        double t = (-s->hw - r[0]) / d[0];
        double ye = r[1] + t * d[1];
        if (ye <= s->ytop && ye >= orc_surface(s, -s->hw, NULL) && t < best) { best = t; *face = EV_LEFT; }
    }
    return best;
}

static void face_normal(int face, double nf[3])
{
    nf[0] = nf[1] = nf[2] = 0.0;
    if (face == EV_TOP) nf[1] = 1.0;
    else if (face == EV_RIGHT) nf[0] = 1.0;
    else nf[0] = -1.0;
}

typedef struct {
    long steps;       /* accepted integrator steps inside the box */
    long rejected;    /* rejected DOPRI5 attempts */
    long events;      /* box entries, exits, internal reflections, grating contacts */
    long contacts;    /* grating reflections */
    double min_cos;   /* smallest |p_hat . N| over all contacts and face crossings */
    long bad_w;       /* Lambert-W evaluations that failed their check */
    double max_H;     /* diagnostics: max | |p|^2 - n^2 | / n^2 at step ends */
    long bsteps, brejected;  /* steps / rejections taken in Fresnel-reflected branches */
    long branch_events;  /* events of Fresnel-reflected branches */
    long branch_failed;  /* Fresnel-reflected branches that failed (they add nothing) */
} trace_info;

static int all_finite(const double* a, int n)
{
    for (int i = 0; i < n; ++i) if (!isfinite(a[i])) return 0;
    return 1;
}

/* Integration inside the box from (r, p) on entry until the ray leaves B
   through a face into air.  Grating contacts and total internal reflections
   at faces are handled inside.  Returns a ray status; on RAY_OK, r and p hold
   the exit point and the refracted momentum (|p| = 1), p_in the momentum
   just inside the face and n_face the face's outward normal. */
static int integrate_box(const oscene* s, const oopts* o, double r[3], double p[3],
                         trace_info* ti, double p_in[3], double n_face[3])
{
    st4 u = { { r[0], r[1], p[0], p[1] } };
    double z = r[2], pz = p[2];
    double h = (o->integ == 0) ? o->h : o->h0;
    int last_rej = 0;
    int bad = 0;
    st4 k1;
    int have_k1 = 0;
    for (;;) {
        if (ti->steps >= o->max_steps) return RAY_MAX_STEPS;
        st4 y5, y4, k7;
        double hs = h, hnext = h;
        if (o->integ == 0) {
            rk4_step(s, &u, h, &y5, &bad);
        } else {
            if (!have_k1) { rhs(s, &u, &k1, &bad); have_k1 = 1; }
            dp5_step(s, &u, &k1, h, &y5, &y4, &k7, &bad);
            double acc = 0.0;
            for (int i = 0; i < 4; ++i) {
                double sc = o->atol + o->rtol * fmax(fabs(u.v[i]), fabs(y5.v[i]));
                double q = (y5.v[i] - y4.v[i]) / sc;
                acc += q * q;
            }
            double err = sqrt(acc / 4.0);
            if (!isfinite(err)) return RAY_NONFINITE;
            if (err > 1.0) {
                double fac = 0.9 * pow(err, -0.2);
                if (fac < 0.2) fac = 0.2;
                h *= fac;
                last_rej = 1;
                ti->rejected++;
                if (h < o->hmin) return RAY_STEP_UNDERFLOW;
                continue;
            }
            double fac = (err == 0.0) ? 5.0 : 0.9 * pow(err, -0.2);
            if (fac > 5.0) fac = 5.0;
            if (fac < 0.2) fac = 0.2;
            if (last_rej && fac > 1.0) fac = 1.0;
            last_rej = 0;
            hnext = h * fac;
            if (hnext > o->hmax) hnext = o->hmax;
        }
        ti->steps++;
        if (!all_finite(y5.v, 4)) return RAY_NONFINITE;
        /* events at the end of the step */
        int hit = EV_NONE;
        double theta = 2.0;
        for (int ev = 0; ev < 4; ++ev) {
            if (event_value(s, ev, &y5) >= 0.0) continue;
            /* smallest theta in (0, 1] with the event function of the partial
               step crossing zero: bisection over the partial step size. */
            double lo = 0.0, hi = 1.0;
            while (hi - lo > 1e-14) {
                double mid = 0.5 * (lo + hi);
                st4 ym, y4m, k7m;
                if (o->integ == 0) rk4_step(s, &u, mid * hs, &ym, &bad);
                else dp5_step(s, &u, &k1, mid * hs, &ym, &y4m, &k7m, &bad);
                if (event_value(s, ev, &ym) < 0.0) hi = mid; else lo = mid;
            }
            if (hi < theta) { theta = hi; hit = ev; }
        }
        if (o->diag) {
            double n = box_index(s, y5.v[0], y5.v[1], NULL);
            double H = fabs(y5.v[2] * y5.v[2] + y5.v[3] * y5.v[3] + pz * pz - n * n) / (n * n);
            if (H > ti->max_H) ti->max_H = H;
        }
        if (hit == EV_NONE) {
            u = y5;
            z += pz * hs;
            if (o->integ == 1) { k1 = k7; h = hnext; }
            continue;
        }
        /* advance to the event with the partial step */
        {
            st4 ye, y4e, k7e;
            if (o->integ == 0) rk4_step(s, &u, theta * hs, &ye, &bad);
            else dp5_step(s, &u, &k1, theta * hs, &ye, &y4e, &k7e, &bad);
            u = ye;
            z += pz * theta * hs;
        }
        h = (o->integ == 0) ? o->h : hnext;
        have_k1 = 0;
        if (++ti->events > o->max_events) return RAY_MAX_EVENTS;
        double pp[3] = { u.v[2], u.v[3], pz };
        double pabs = sqrt(pp[0] * pp[0] + pp[1] * pp[1] + pp[2] * pp[2]);
        if (hit == EV_GRATING) {
            double E, nx, ny;
            orc_surface(s, u.v[0], &E);
            orc_grating_normal(s, E, &nx, &ny);
            double c = fabs(pp[0] * nx + pp[1] * ny) / pabs;
            if (c < ti->min_cos) ti->min_cos = c;
            reflect(pp, nx, ny);
            ti->contacts++;
            u.v[2] = pp[0]; u.v[3] = pp[1];
            continue;
        }
        /* face crossing from inside: n1 = eq. (1) at the crossing, n2 = 1 */
        double nf[3];
        face_normal(hit, nf);
        {
            double c = fabs(pp[0] * nf[0] + pp[1] * nf[1]) / pabs;
            if (c < ti->min_cos) ti->min_cos = c;
        }
        double pin[3] = { pp[0], pp[1], pp[2] };
        int through = snell(pp, nf, 1.0);
        u.v[2] = pp[0]; u.v[3] = pp[1];
        if (!through) continue;   /* total internal reflection: stay inside */
        r[0] = u.v[0]; r[1] = u.v[1]; r[2] = z;
        p[0] = pp[0]; p[1] = pp[1]; p[2] = pp[2];
        for (int i = 0; i < 3; ++i) { p_in[i] = pin[i]; n_face[i] = nf[i]; }
        if (bad) ti->bad_w++;
        return RAY_OK;
    }
}

/* Inside the homogeneous plate (cloak 3) rays are straight (the index is
   constant, so the acceleration of eq. (11) vanishes): from (r, p) just
   inside a face, |p| = n_plate, to the nearest of the top face, a side face
   or the mirror (reflection, as in air).  Faces refract into air by Snell's
   law or reflect totally.  Same outputs as integrate_box. */
static int plate_walk(const oscene* s, const oopts* o, double r[3], double p[3], trace_info* ti,
                      double p_in[3], double n_face[3])
{
    for (;;) {
        if (!all_finite(r, 3) || !all_finite(p, 3)) return RAY_NONFINITE;
        double pa = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        double d[3] = { p[0] / pa, p[1] / pa, p[2] / pa };
        /* faces ahead, from inside: distances along the unit direction */
        double tf = INFINITY;
        int face = EV_NONE;
        if (d[1] > 0.0) { double t = (s->ytop - r[1]) / d[1]; if (t < tf) { tf = t; face = EV_TOP; } }
        if (d[0] > 0.0 && isfinite(s->hw)) { double t = (s->hw - r[0]) / d[0]; if (t < tf) { tf = t; face = EV_RIGHT; } }
        if (d[0] < 0.0 && isfinite(s->hw)) { double t = (-s->hw - r[0]) / d[0]; if (t < tf) { tf = t; face = EV_LEFT; } }
        double tg = air_contact(s, r, d);
        if (++ti->events > o->max_events) return RAY_MAX_EVENTS;
        if (tg <= tf) {
            for (int i = 0; i < 3; ++i) r[i] += tg * d[i];
            double E, nx, ny;
            orc_surface(s, r[0], &E);
            orc_grating_normal(s, E, &nx, &ny);
            double c = fabs(d[0] * nx + d[1] * ny);
            if (c < ti->min_cos) ti->min_cos = c;
            reflect(p, nx, ny);
            ti->contacts++;
            continue;
        }
        if (!isfinite(tf)) return RAY_NONFINITE;   /* no face ahead: cannot happen in a finite box */
        for (int i = 0; i < 3; ++i) r[i] += tf * d[i];
        if (face == EV_TOP) r[1] = s->ytop;
        else if (face == EV_RIGHT) r[0] = s->hw;
        else r[0] = -s->hw;
        double nf[3];
        face_normal(face, nf);
        {
            double c = fabs(d[0] * nf[0] + d[1] * nf[1]);
            if (c < ti->min_cos) ti->min_cos = c;
        }
        double pin[3] = { p[0], p[1], p[2] };
        if (!snell(p, nf, 1.0)) continue;   /* total internal reflection */
        for (int i = 0; i < 3; ++i) { p_in[i] = pin[i]; n_face[i] = nf[i]; }
        return RAY_OK;
    }
}

/* Fresnel reflectance of unpolarised light at a face (Sec. 3: the Fresnel
   equations), from the normal components of the momentum on the two sides:
   pn = |p . N| in the medium of index n1 (= n1 cos of incidence) and
   qn = |q . N| of the transmitted momentum in index n2 (= n2 cos of
   transmission).  r_s = (pn - qn) / (pn + qn),
   r_p = (n2^2 pn - n1^2 qn) / (n2^2 pn + n1^2 qn), R = (r_s^2 + r_p^2) / 2. */
static double fresnel_R(double pn, double qn, double n1, double n2)
{
    double rs = (pn - qn) / (pn + qn);
    double a = n2 * n2 * pn, b = n1 * n1 * qn;
    double rp = (a - b) / (a + b);
    return 0.5 * (rs * rs + rp * rp);
}

/* Backdrop colour for a ray leaving the scene from r along the unit
   direction d.  backdrop 0: the sky at infinity (gco_sky).  backdrop 1: the
   plane y = bd_y (the photograph in front of which the camera sits, Sec. 4)
   patterned with m = 1/2 + 1/2 tanh(K cos(2 pi x / P)) tanh(K cos(2 pi z / P))
   at the point the ray meets it; a ray that does not rise to the plane sees
   m = 0.  rgb = Cb + m (Ca - Cb) with the sky's two colours. */
static void backdrop_rgb(const oscene* s, const double r[3], const double d[3], double rgb[3])
{
    if (s->backdrop == 0) { gco_sky(s->K, d, rgb); return; }
    const double Ca[3] = { 0.95, 0.85, 0.30 }, Cb[3] = { 0.10, 0.20, 0.55 };
    double m = 0.0;
    if (d[1] > 0.0 && r[1] < s->bd_y) {
        double t = (s->bd_y - r[1]) / d[1];
        double X = r[0] + t * d[0], Zc = r[2] + t * d[2];
        double a = cos(2.0 * ORC_PI * X / s->bd_P), b = cos(2.0 * ORC_PI * Zc / s->bd_P);
        double ta = isinf(s->K) ? (a > 0 ? 1.0 : (a < 0 ? -1.0 : 0.0)) : tanh(s->K * a);
        double tb = isinf(s->K) ? (b > 0 ? 1.0 : (b < 0 ? -1.0 : 0.0)) : tanh(s->K * b);
        m = 0.5 + 0.5 * ta * tb;
    }
    for (int c = 0; c < 3; ++c) rgb[c] = Cb[c] + m * (Ca[c] - Cb[c]);
}

static int trace_path(const oscene* s, const oopts* o, const double r0[3], const double p0[3], int inside,
                      double w, int split, double rgb[3], double out_org[3], double out_dir[3],
                      trace_info* ti);

/* A Fresnel-reflected branch from r with momentum q: traced as a path of
   its own, never split again.  It continues the light path up to the
   split, so its caps (max_steps, max_events) count from the primary path's
   counts there; the work it does is added to the branch counters, the
   primary path's own counts are left as they were. */
static void run_branch(const oscene* s, const oopts* o, const double r[3], const double q[3], int inside, double w,
                       double rgb[3], trace_info* ti)
{
    trace_info tb = *ti;
    double so[3], sd[3];
    int st = trace_path(s, o, r, q, inside, w, 0, rgb, so, sd, &tb);
    ti->bsteps += tb.steps - ti->steps;
    ti->brejected += tb.rejected - ti->rejected;
    ti->branch_events += tb.events - ti->events;
    if (st != RAY_OK) ti->branch_failed++;
}

/* One path from (r, p) until it escapes: in air (inside = 0, |p| = 1) or
   just inside a face of the box (inside = 1, |p| = the box index there).
   w is the path's weight.  At every face crossing that transmits, Fresnel
   (fresnel = 1) splits the ray: the path goes on with weight w T, and when
   `split` is set the reflected part (weight w R) is traced as a path of its
   own that is never split again -- rays reflected more than once are
   neglected (Sec. 3); without `split` the reflected part is dropped.  Total
   internal reflection keeps the whole weight.  On escape w times the
   backdrop colour is added to rgb (may be NULL); out_org / out_dir receive
   where and in which direction this path left.  Failures of a reflected
   branch contribute nothing and do not change the returned status. */
static int trace_path(const oscene* s, const oopts* o, const double r0[3], const double p0[3], int inside,
                      double w, int split, double rgb[3], double out_org[3], double out_dir[3],
                      trace_info* ti)
{
    double r[3] = { r0[0], r0[1], r0[2] };
    double p[3] = { p0[0], p0[1], p0[2] };
    for (;;) {
        if (!all_finite(r, 3) || !all_finite(p, 3)) return RAY_NONFINITE;
        if (inside) {
            double pin[3], nf[3];
            int st = (s->cloak == CLOAK_PLATE) ? plate_walk(s, o, r, p, ti, pin, nf)
                                               : integrate_box(s, o, r, p, ti, pin, nf);
            if (st != RAY_OK) return st;
            if (s->fresnel) {
                double n1 = sqrt(pin[0] * pin[0] + pin[1] * pin[1] + pin[2] * pin[2]);
                double pn = fabs(pin[0] * nf[0] + pin[1] * nf[1] + pin[2] * nf[2]);
                double qn = fabs(p[0] * nf[0] + p[1] * nf[1] + p[2] * nf[2]);
                double R = fresnel_R(pn, qn, n1, 1.0);
                if (split) {
                    double q[3];
                    double pd = pin[0] * nf[0] + pin[1] * nf[1] + pin[2] * nf[2];
                    for (int i = 0; i < 3; ++i) q[i] = pin[i] - 2.0 * pd * nf[i];
                    run_branch(s, o, r, q, 1, w * R, rgb, ti);
                }
                w *= 1.0 - R;
            }
            inside = 0;
            continue;
        }
        /* in air: straight line (the acceleration of eq. (11) vanishes) */
        int face;
        double tb = air_box_entry(s, r, p, &face);
        double tg = air_contact(s, r, p);
        if (!isfinite(tb) && !isfinite(tg)) {
            for (int i = 0; i < 3; ++i) { out_org[i] = r[i]; out_dir[i] = p[i]; }
            if (rgb) {
                double c[3];
                backdrop_rgb(s, r, p, c);
                for (int k = 0; k < 3; ++k) rgb[k] += w * c[k];
            }
            return RAY_OK;
        }
        if (++ti->events > o->max_events) return RAY_MAX_EVENTS;
        if (tg <= tb) {
            for (int i = 0; i < 3; ++i) r[i] += tg * p[i];
            double E, nx, ny;
            orc_surface(s, r[0], &E);
            orc_grating_normal(s, E, &nx, &ny);
            double c = fabs(p[0] * nx + p[1] * ny);
            if (c < ti->min_cos) ti->min_cos = c;
            reflect(p, nx, ny);
            ti->contacts++;
            continue;
        }
        for (int i = 0; i < 3; ++i) r[i] += tb * p[i];
        if (face == EV_TOP) r[1] = s->ytop;
        else if (face == EV_RIGHT) r[0] = s->hw;
        else r[0] = -s->hw;
        double nf[3];
        face_normal(face, nf);
        for (int i = 0; i < 3; ++i) nf[i] = -nf[i];   /* from air into the box */
        {
            double c = fabs(p[0] * nf[0] + p[1] * nf[1]);
            if (c < ti->min_cos) ti->min_cos = c;
        }
        int bad = 0;
        double n2 = box_index(s, r[0], r[1], &bad);
        if (bad) ti->bad_w++;
        double pa[3] = { p[0], p[1], p[2] };
        if (!snell(p, nf, n2)) continue;   /* reflected back into air */
        if (s->fresnel) {
            double pn = fabs(pa[0] * nf[0] + pa[1] * nf[1] + pa[2] * nf[2]);
            double qn = fabs(p[0] * nf[0] + p[1] * nf[1] + p[2] * nf[2]);
            double R = fresnel_R(pn, qn, 1.0, n2);
            if (split) {
                double q[3];
                double pd = pa[0] * nf[0] + pa[1] * nf[1] + pa[2] * nf[2];
                for (int i = 0; i < 3; ++i) q[i] = pa[i] - 2.0 * pd * nf[i];
                run_branch(s, o, r, q, 0, w * R, rgb, ti);
            }
            w *= 1.0 - R;
        }
        inside = 1;
    }
}

/* Full path of one ray from (org, dir) until it escapes (the primary path:
   Fresnel-reflected parts are not followed).  Returns the ray status; exit
   position and unit direction in out_*. */
static int trace_one(const oscene* s, const oopts* o, const double org[3], const double dir[3],
                     double out_org[3], double out_dir[3], trace_info* ti)
{
    double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double p[3] = { dir[0] / nd, dir[1] / nd, dir[2] / nd };
    memset(ti, 0, sizeof(*ti));
    ti->min_cos = 1.0;
    return trace_path(s, o, org, p, 0, 1.0, 0, NULL, out_org, out_dir, ti);
}

/* Colour of one camera sample: every path of the sample (the primary one
   and, with Fresnel, its once-reflected branches) adds its weight times the
   backdrop.  Returns the primary path's status; a failed sample is black. */
static int shade_one(const oscene* s, const oopts* o, const double org[3], const double dir[3], double rgb[3],
                     trace_info* ti)
{
    double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double p[3] = { dir[0] / nd, dir[1] / nd, dir[2] / nd };
    double oo[3], od[3];
    memset(ti, 0, sizeof(*ti));
    ti->min_cos = 1.0;
    rgb[0] = rgb[1] = rgb[2] = 0.0;
    int st = trace_path(s, o, org, p, 0, 1.0, s->fresnel, rgb, oo, od, ti);
    if (st != RAY_OK) rgb[0] = rgb[1] = rgb[2] = 0.0;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Camera and jitter.                                                        */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the n-th output of the      */
/* generator seeded with `seed` is mix(seed + (n + 1) * 0x9E3779B97F4A7C15). */
/* Uniform in [0,1): top 53 bits times 2^-53.                                */
/* ------------------------------------------------------------------------ */
uint64_t gco_splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double u01(uint64_t seed, uint64_t n)
{
    return (double)(gco_splitmix64(seed, n) >> 11) * (1.0 / 9007199254740992.0);
}

static void normalize3(double v[3])
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= r; v[1] /= r; v[2] /= r;
}

/* Pinhole camera (Sec. 4: a point camera).  Forward f = target - eye, right
   r = f x up (up = the camera's up hint, +y when it is zero), image up
   u = r x f; row 0 at the top.  The vertical opening angle is fov_y; the
   horizontal one is fov_x, or follows from square pixels when fov_x = 0
   (the paper's camera: 50 deg horizontally, 42 vertically).  Sample s of
   pixel (i, j) goes through (i + u, j + v) with u, v the jitter values (1/2
   without jitter). */
void gco_camera_ray(const double* cam, uint64_t seed, int i, int j, int s,
                    double org[3], double dir[3])
{
    double f[3] = { cam[3] - cam[0], cam[4] - cam[1], cam[5] - cam[2] };
    normalize3(f);
    double hint[3] = { cam[12], cam[13], cam[14] };
    if (hint[0] == 0.0 && hint[1] == 0.0 && hint[2] == 0.0) hint[1] = 1.0;
    double r[3] = { f[1] * hint[2] - f[2] * hint[1], f[2] * hint[0] - f[0] * hint[2], f[0] * hint[1] - f[1] * hint[0] };
    normalize3(r);
    double up[3] = { r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0] };
    int W = (int)cam[7], H = (int)cam[8], spp = (int)cam[9], jitter = (int)cam[10];
    long scene = (long)cam[11];
    double t = tan(0.5 * cam[6] * ORC_PI / 180.0);
    double aspect = cam[15] > 0.0 ? tan(0.5 * cam[15] * ORC_PI / 180.0) / t : (double)W / (double)H;
    double du = 0.5, dv = 0.5;
    if (jitter) {
        uint64_t c = ((((uint64_t)scene * (uint64_t)H + (uint64_t)j) * (uint64_t)W + (uint64_t)i) *
                      (uint64_t)spp + (uint64_t)s) * 2ULL;
        du = u01(seed, c);
        dv = u01(seed, c + 1);
    }
    double sx = (2.0 * (i + du) / W - 1.0) * t * aspect;
    double sy = (1.0 - 2.0 * (j + dv) / H) * t;
    for (int k = 0; k < 3; ++k) {
        org[k] = cam[k];
        dir[k] = f[k] + sx * r[k] + sy * up[k];
    }
    normalize3(dir);
}

/* Procedural backdrop at infinity: an 8 x 8 latitude-longitude checkerboard
   smoothed with tanh of sharpness K (K = inf gives hard squares).
   phi = atan2(d_x, -d_z), theta = atan2(d_y, hypot(d_x, d_z)),
   m = 1/2 + 1/2 tanh(K cos 4 phi) tanh(K sin 8 theta),
   rgb = Cb + m (Ca - Cb), Ca = (0.95, 0.85, 0.30), Cb = (0.10, 0.20, 0.55). */
void gco_sky(double K, const double d[3], double rgb[3])
{
    const double Ca[3] = { 0.95, 0.85, 0.30 }, Cb[3] = { 0.10, 0.20, 0.55 };
    double phi = atan2(d[0], -d[2]);
    double th = atan2(d[1], hypot(d[0], d[2]));
    double a = cos(4.0 * phi), b = sin(8.0 * th);
    double ta = isinf(K) ? (a > 0 ? 1.0 : (a < 0 ? -1.0 : 0.0)) : tanh(K * a);
    double tb = isinf(K) ? (b > 0 ? 1.0 : (b < 0 ? -1.0 : 0.0)) : tanh(K * b);
    double m = 0.5 + 0.5 * ta * tb;
    for (int c = 0; c < 3; ++c) rgb[c] = Cb[c] + m * (Ca[c] - Cb[c]);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (called through ctypes by the test-suite).         */
/* ------------------------------------------------------------------------ */
int gco_lambertw(double zr, double zi, double* wr, double* wi)
{
    cplx w;
    int r = orc_w0(zr + I * zi, &w);
    *wr = creal(w);
    *wi = cimag(w);
    return r;
}

double gco_index(const double* scene, double x, double y)
{
    oscene s;
    load_scene(scene, &s);
    return orc_index_raw(&s, x, y, NULL);
}

void gco_accel(const double* scene, double x, double y, double out[2])
{
    oscene s;
    load_scene(scene, &s);
    orc_accel(&s, x, y, &out[0], &out[1], NULL);
}

void gco_grad_n_eq12(const double* scene, double x, double y, double out[2])
{
    oscene s;
    load_scene(scene, &s);
    orc_grad_n_eq12(&s, x, y, &out[0], &out[1]);
}

double gco_surface(const double* scene, double x, double* xi)
{
    oscene s;
    load_scene(scene, &s);
    double E;
    double S = orc_surface(&s, x, &E);
    if (xi) {
        double N = floor(x / s.L + 0.5);
        *xi = E / s.k + N * s.L;
    }
    return S;
}

/* Trace n rays.  info (may be NULL) gets 7 values per ray:
   steps, rejected, events, contacts, min_cos, bad_w, max_H. */
void gco_trace_rays(const double* scene, const double* opts, long n,
                    const double* org, const double* dir, double* out_org, double* out_dir,
                    int* status, double* info, int nthreads)
{
    oscene s;
    oopts o;
    load_scene(scene, &s);
    load_opts(opts, &o);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (long i = 0; i < n; ++i) {
        trace_info ti;
        double oo[3] = { 0, 0, 0 }, od[3] = { 0, 0, 0 };
        int st = trace_one(&s, &o, org + 3 * i, dir + 3 * i, oo, od, &ti);
        for (int k = 0; k < 3; ++k) { out_org[3 * i + k] = oo[k]; out_dir[3 * i + k] = od[k]; }
        status[i] = st;
        if (info) {
            info[7 * i + 0] = (double)ti.steps;
            info[7 * i + 1] = (double)ti.rejected;
            info[7 * i + 2] = (double)ti.events;
            info[7 * i + 3] = (double)ti.contacts;
            info[7 * i + 4] = ti.min_cos;
            info[7 * i + 5] = (double)ti.bad_w;
            info[7 * i + 6] = ti.max_H;
        }
    }
}

/* Render selected pixels (or all when npix < 0) of a scene.
   rgb: 3 floats per listed pixel (or H x W x 3).  Each pixel is the mean of
   its spp sample colours (shade_one: the backdrop seen along every path of
   the sample, weighted); a failed sample contributes black.
   counters[4] (may be NULL): rays, accepted steps, rejected steps, failed. */
void gco_render_pixels(const double* scene, const double* cam, uint64_t seed, const double* opts,
                       long npix, const long* pix, double* rgb, double* counters, int nthreads)
{
    oscene s;
    oopts o;
    load_scene(scene, &s);
    load_opts(opts, &o);
    int W = (int)cam[7], H = (int)cam[8], spp = (int)cam[9];
    long total = npix < 0 ? (long)W * H : npix;
    double c_rays = 0, c_steps = 0, c_rej = 0, c_fail = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : c_rays, c_steps, c_rej, c_fail)
#endif
    for (long q = 0; q < total; ++q) {
        long pidx = npix < 0 ? q : pix[q];
        int i = (int)(pidx % W), j = (int)(pidx / W);
        double acc[3] = { 0, 0, 0 };
        for (int smp = 0; smp < spp; ++smp) {
            double org[3], dir[3], c[3];
            trace_info ti;
            gco_camera_ray(cam, seed, i, j, smp, org, dir);
            int st = shade_one(&s, &o, org, dir, c, &ti);
            c_rays += 1;
            c_steps += (double)(ti.steps + ti.bsteps);
            c_rej += (double)(ti.rejected + ti.brejected);
            if (st != RAY_OK) { c_fail += 1; continue; }
            for (int k = 0; k < 3; ++k) acc[k] += c[k];
        }
        for (int k = 0; k < 3; ++k) rgb[3 * q + k] = acc[k] / spp;
    }
    if (counters) {
        counters[0] = c_rays; counters[1] = c_steps; counters[2] = c_rej; counters[3] = c_fail;
    }
}

/* eqs. (14), (15) at zero shift.  Images are npix x nch (channel fastest).
   Each channel's spatial mean is subtracted (eq. (14)); the sums are then
   pooled over channels: C = sum f' g' / sum f'^2 (eq. (15) at (0, 0)), and
   the Pearson form sum f' g' / sqrt(sum f'^2 sum g'^2) is reported beside
   it.  Accumulation in long double, two passes. */
void gco_cross_correlate(const float* f, const float* g, long npix, int nch, double out[2])
{
    long double sfg = 0, sff = 0, sgg = 0;
    for (int c = 0; c < nch; ++c) {
        long double mf = 0, mg = 0;
        for (long i = 0; i < npix; ++i) { mf += f[i * nch + c]; mg += g[i * nch + c]; }
        mf /= npix;
        mg /= npix;
        for (long i = 0; i < npix; ++i) {
            long double a = f[i * nch + c] - mf, b = g[i * nch + c] - mg;
            sfg += a * b;
            sff += a * a;
            sgg += b * b;
        }
    }
    out[0] = (double)(sfg / sff);
    out[1] = (double)(sfg / sqrtl(sff * sgg));
}

/* Same on double images (oracle renders). */
void gco_cross_correlate_f64(const double* f, const double* g, long npix, int nch, double out[2])
{
    long double sfg = 0, sff = 0, sgg = 0;
    for (int c = 0; c < nch; ++c) {
        long double mf = 0, mg = 0;
        for (long i = 0; i < npix; ++i) { mf += f[i * nch + c]; mg += g[i * nch + c]; }
        mf /= npix;
        mg /= npix;
        for (long i = 0; i < npix; ++i) {
            long double a = f[i * nch + c] - mf, b = g[i * nch + c] - mg;
            sfg += a * b;
            sff += a * a;
            sgg += b * b;
        }
    }
    out[0] = (double)(sfg / sff);
    out[1] = (double)(sfg / sqrtl(sff * sgg));
}

/* eq. (15) at every shift (Sec. 5): the correlation map C(dx, dy) of the
   image g against the reference f, both H x W pixels of nch channels
   (channel fastest) stored with a row pitch of `pitch` pixels, so that a
   window of a larger image can be passed.  dx is the shift along a row
   (columns, to the right), dy along a column (rows, downwards: row 0 is the
   top of the image), in pixels, |dx| <= rx, |dy| <= ry.
   Eq. (14): each channel's mean over the whole window is subtracted.  The
   numerator of eq. (15) is the sum over the pixels (j, i) for which both
   (j, i) and (j + dy, i + dx) lie in the window -- the finite photograph
   holds nothing outside -- pooled over channels; the denominator is the
   sum of f'^2 over the whole window.  So C(0, 0) is the zero-shift
   coefficient, and an image that is f shifted within the frame gives a
   maximum below 1 at that shift (equal to 1 only for an infinite
   photograph, as Sec. 5 notes).
   map: (2 ry + 1) x (2 rx + 1) doubles, row-major, C(dx, dy) at
   (dy + ry) (2 rx + 1) + (dx + rx).  peak: { maximum of the map, its dx,
   its dy }, the first maximum in that row-major order on ties.  Direct
   sums in long double. */
void gco_cross_correlate_map(const float* f, const float* g, long H, long W, long pitch, int nch,
                             int rx, int ry, double* map, double peak[3])
{
    long double mf[8], mg[8];
    long double sff = 0;
    for (int c = 0; c < nch; ++c) {
        long double a = 0, b = 0;
        for (long j = 0; j < H; ++j)
            for (long i = 0; i < W; ++i) {
                a += f[(j * pitch + i) * nch + c];
                b += g[(j * pitch + i) * nch + c];
            }
        mf[c] = a / (long double)(H * W);
        mg[c] = b / (long double)(H * W);
        for (long j = 0; j < H; ++j)
            for (long i = 0; i < W; ++i) {
                long double d = f[(j * pitch + i) * nch + c] - mf[c];
                sff += d * d;
            }
    }
    long nx = 2L * rx + 1;
    double best = -INFINITY;
    int bdx = 0, bdy = 0;
    for (int dy = -ry; dy <= ry; ++dy)
        for (int dx = -rx; dx <= rx; ++dx) {
            long double s = 0;
            for (long j = 0; j < H; ++j) {
                long jj = j + dy;
                if (jj < 0 || jj >= H) continue;
                for (long i = 0; i < W; ++i) {
                    long ii = i + dx;
                    if (ii < 0 || ii >= W) continue;
                    for (int c = 0; c < nch; ++c)
                        s += (f[(j * pitch + i) * nch + c] - mf[c]) * (g[(jj * pitch + ii) * nch + c] - mg[c]);
                }
            }
            double v = (double)(s / sff);
            map[(long)(dy + ry) * nx + (dx + rx)] = v;
            if (v > best) { best = v; bdx = dx; bdy = dy; }
        }
    peak[0] = best;
    peak[1] = bdx;
    peak[2] = bdy;
}

/* ------------------------------------------------------------------------ */
/* Forward-mode derivatives with respect to the parameters (A, half_width)  */
/* of the discrete RK4 tracer above.  Every map the tracer applies -- RK4   */
/* steps, partial steps ending on an event (with the event time implicit    */
/* in e(Phi(tau*)) = 0), reflections, Snell refraction, straight flight,    */
/* the sky lookup -- is differentiated exactly, so the result is the        */
/* derivative of the computed image, not of the continuous problem.         */
/* ------------------------------------------------------------------------ */

/* acceleration, its Jacobian d a / d(x, y) and d a / dA.  With D = 1 + W:
   a_x + i a_y = i k F,  F = P conj(Q),  P = 1/D,  Q = W / D^3 (both
   holomorphic in zeta = x + i y), dW/dzeta = i k W / D, dW/dA = W / (A D);
   d/dx = d/dzeta + d/dzetabar, d/dy = i (d/dzeta - d/dzetabar). */
static void orc_accel_jac(const oscene* s, double x, double y, double a[2], double J[2][2], double aA[2])
{
    cplx W;
    orc_w0(orc_Z(s, x, y), &W);
    cplx D = 1.0 + W;
    cplx Wp = I * s->k * W / D;
    cplx WA = (s->A > 0.0) ? W / (s->A * D) : -s->k * cexp(I * s->k * (x + I * y));
    cplx P = 1.0 / D, Q = W / (D * D * D);
    cplx Pp = -Wp / (D * D), Qp = Wp * (1.0 - 2.0 * W) / (D * D * D * D);
    cplx PA = -WA / (D * D), QA = WA * (1.0 - 2.0 * W) / (D * D * D * D);
    cplx F = P * conj(Q);
    cplx Fz = Pp * conj(Q), Fzb = P * conj(Qp);
    cplx FA = PA * conj(Q) + P * conj(QA);
    cplx ax = I * s->k * F;
    cplx dx = I * s->k * (Fz + Fzb);
    cplx dy = -s->k * (Fz - Fzb);
    cplx dA = I * s->k * FA;
    a[0] = creal(ax); a[1] = cimag(ax);
    J[0][0] = creal(dx); J[1][0] = cimag(dx);
    J[0][1] = creal(dy); J[1][1] = cimag(dy);
    aA[0] = creal(dA); aA[1] = cimag(dA);
}

/* index and its derivatives d n / d(x, y), d n / dA */
static double orc_index_jac(const oscene* s, double x, double y, double dn[2], double* nA)
{
    cplx W;
    orc_w0(orc_Z(s, x, y), &W);
    cplx D = 1.0 + W;
    cplx Wp = I * s->k * W / D;
    cplx WA = (s->A > 0.0) ? W / (s->A * D) : -s->k * cexp(I * s->k * (x + I * y));
    double n = 1.0 / cabs(D);
    double n3 = n * n * n;
    dn[0] = -n3 * creal(conj(D) * Wp);
    dn[1] = n3 * cimag(conj(D) * Wp);
    *nA = -n3 * creal(conj(D) * WA);
    return n;
}

/* grating geometry at x: E = k xi, height S, slope S' = dS/dx, S_A = dS/dA
   at fixed x, and E_x = dE/dx, E_A = dE/dA at fixed x */
static void orc_surface_jac(const oscene* s, double x, double* E, double* S, double* Sx, double* SA,
                            double* Ex, double* EA)
{
    *S = orc_surface(s, x, E);
    double e = s->e, sn = sin(*E), cs = cos(*E);
    double den = 1.0 - e * cs;
    *Ex = s->k / den;
    *EA = s->k * sn / den;
    *Sx = -e * sn / den;
    *SA = cs - e * sn * sn / den;
}

/* unit upward normal at x and its tangent for dx (position) and dA */
static void orc_normal_tan(const oscene* s, double x, double dx, double dA, double N[2], double dN[2])
{
    double E, S, Sx, SA, Ex, EA;
    orc_surface_jac(s, x, &E, &S, &Sx, &SA, &Ex, &EA);
    double e = s->e, sn = sin(E), cs = cos(E);
    double dE = Ex * dx + EA * dA;
    double de = s->k * dA;
    double m[2] = { e * sn, 1.0 - e * cs };
    double dm[2] = { de * sn + e * cs * dE, -de * cs + e * sn * dE };
    double r = sqrt(m[0] * m[0] + m[1] * m[1]);
    N[0] = m[0] / r; N[1] = m[1] / r;
    double ndm = N[0] * dm[0] + N[1] * dm[1];
    dN[0] = (dm[0] - N[0] * ndm) / r;
    dN[1] = (dm[1] - N[1] * ndm) / r;
}

/* p' = p - 2 (p.N) N in 3D with N = (N0, N1, 0), and its tangent */
static void reflect_tan(double p[3], double dp[3], const double N[2], const double dN[2])
{
    double pn = p[0] * N[0] + p[1] * N[1];
    double dpn = dp[0] * N[0] + dp[1] * N[1] + p[0] * dN[0] + p[1] * dN[1];
    for (int i = 0; i < 2; ++i) {
        dp[i] -= 2.0 * (dpn * N[i] + pn * dN[i]);
        p[i] -= 2.0 * pn * N[i];
    }
}

/* Snell at a plane face with fixed unit normal nf, n2 with tangent dn2 */
static int snell_tan(double p[3], double dp[3], const double nf[3], double n2, double dn2)
{
    double pn = p[0] * nf[0] + p[1] * nf[1] + p[2] * nf[2];
    double dpn = dp[0] * nf[0] + dp[1] * nf[1] + dp[2] * nf[2];
    double pt[3], dpt[3];
    for (int i = 0; i < 3; ++i) { pt[i] = p[i] - pn * nf[i]; dpt[i] = dp[i] - dpn * nf[i]; }
    double q = n2 * n2 - (pt[0] * pt[0] + pt[1] * pt[1] + pt[2] * pt[2]);
    if (q < 0.0) {
        for (int i = 0; i < 3; ++i) { p[i] -= 2.0 * pn * nf[i]; dp[i] -= 2.0 * dpn * nf[i]; }
        return 0;
    }
    double dq = 2.0 * n2 * dn2 - 2.0 * (pt[0] * dpt[0] + pt[1] * dpt[1] + pt[2] * dpt[2]);
    double sg = pn >= 0.0 ? 1.0 : -1.0;
    double r = sqrt(q);
    for (int i = 0; i < 3; ++i) {
        p[i] = pt[i] + sg * r * nf[i];
        dp[i] = dpt[i] + sg * dq / (2.0 * r) * nf[i];
    }
    return 1;
}

/* RK4 step of size tau from u with parameter tangents du[j] (j = 0: A,
   j = 1: half_width); also returns d out / d tau */
static void rk4_step_tan(const oscene* s, const st4* u, const double du[2][4], double tau, st4* out,
                         double dout[2][4], double dtau[4])
{
    static const double c[4] = { 0.0, 0.5, 0.5, 1.0 }, w[4] = { 1.0, 2.0, 2.0, 1.0 };
    double K[4][4], dK[4][2][4], tK[4][4];
    for (int i = 0; i < 4; ++i) {
        double U[4], dU[2][4], tU[4];
        for (int q = 0; q < 4; ++q) {
            U[q] = u->v[q] + (i ? c[i] * tau * K[i - 1][q] : 0.0);
            tU[q] = i ? c[i] * K[i - 1][q] + c[i] * tau * tK[i - 1][q] : 0.0;
            for (int j = 0; j < 2; ++j) dU[j][q] = du[j][q] + (i ? c[i] * tau * dK[i - 1][j][q] : 0.0);
        }
        double a[2], J[2][2], aA[2];
        orc_accel_jac(s, U[0], U[1], a, J, aA);
        K[i][0] = U[2]; K[i][1] = U[3]; K[i][2] = a[0]; K[i][3] = a[1];
        tK[i][0] = tU[2]; tK[i][1] = tU[3];
        tK[i][2] = J[0][0] * tU[0] + J[0][1] * tU[1];
        tK[i][3] = J[1][0] * tU[0] + J[1][1] * tU[1];
        for (int j = 0; j < 2; ++j) {
            dK[i][j][0] = dU[j][2];
            dK[i][j][1] = dU[j][3];
            dK[i][j][2] = J[0][0] * dU[j][0] + J[0][1] * dU[j][1] + (j == 0 ? aA[0] : 0.0);
            dK[i][j][3] = J[1][0] * dU[j][0] + J[1][1] * dU[j][1] + (j == 0 ? aA[1] : 0.0);
        }
    }
    for (int q = 0; q < 4; ++q) {
        double sum = 0.0, tsum = 0.0;
        for (int i = 0; i < 4; ++i) { sum += w[i] * K[i][q]; tsum += w[i] * tK[i][q]; }
        out->v[q] = u->v[q] + (tau / 6.0) * (K[0][q] + 2.0 * K[1][q] + 2.0 * K[2][q] + K[3][q]);
        dtau[q] = sum / 6.0 + (tau / 6.0) * tsum;
        for (int j = 0; j < 2; ++j) {
            double ds = 0.0;
            for (int i = 0; i < 4; ++i) ds += w[i] * dK[i][j][q];
            dout[j][q] = du[j][q] + (tau / 6.0) * ds;
        }
    }
}

/* FNV-1a over the event codes and the number of integrator steps between
   events: equal signatures mean equal event sequences on the same step
   grid.  The discrete map is smooth between signature changes; where the
   event moves from the end of one step to the start of the next, the map
   has a kink because the derivative of an RK4 step with respect to its
   length differs from the right-hand side at its end by the local error. */
static uint64_t sig_add(uint64_t h, uint64_t code)
{
    h ^= code + 1;
    return h * 0x100000001B3ULL;
}

/* trace with tangents (RK4 only).  dir_out: unit exit direction; ddir[j]:
   its derivative wrt A (j = 0) and half_width (j = 1). */
static int trace_one_tan(const oscene* s, const oopts* o, const double org[3], const double dir[3],
                         double dir_out[3], double ddir[2][3], uint64_t* sig, trace_info* ti)
{
    double r[3] = { org[0], org[1], org[2] };
    double nd = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double p[3] = { dir[0] / nd, dir[1] / nd, dir[2] / nd };
    double dr[2][3] = { { 0 } }, dp[2][3] = { { 0 } };
    uint64_t h = 0xcbf29ce484222325ULL;
    memset(ti, 0, sizeof(*ti));
    ti->min_cos = 1.0;
    for (;;) {
        int face;
        double tb = air_box_entry(s, r, p, &face);
        double tg = air_contact(s, r, p);
        if (!isfinite(tb) && !isfinite(tg)) {
            for (int i = 0; i < 3; ++i) { dir_out[i] = p[i]; ddir[0][i] = dp[0][i]; ddir[1][i] = dp[1][i]; }
            *sig = h;
            return RAY_OK;
        }
        if (++ti->events > o->max_events) { *sig = h; return RAY_MAX_EVENTS; }
        if (tg <= tb) {
            /* contact with the bare grating: g(t) = y0 + t py - S(x0 + t px) = 0 */
            double t = tg;
            double xc = r[0] + t * p[0];
            double E, S, Sx, SA, Ex, EA;
            orc_surface_jac(s, xc, &E, &S, &Sx, &SA, &Ex, &EA);
            double gt = p[1] - Sx * p[0];
            for (int j = 0; j < 2; ++j) {
                double dt = -(dr[j][1] + t * dp[j][1] - Sx * (dr[j][0] + t * dp[j][0]) - (j == 0 ? SA : 0.0)) / gt;
                for (int i = 0; i < 3; ++i) dr[j][i] += dt * p[i] + t * dp[j][i];
            }
            for (int i = 0; i < 3; ++i) r[i] += t * p[i];
            double p0[3] = { p[0], p[1], p[2] };
            for (int j = 0; j < 2; ++j) {
                double N[2], dN[2], pp[3] = { p0[0], p0[1], p0[2] };
                orc_normal_tan(s, r[0], dr[j][0], j == 0 ? 1.0 : 0.0, N, dN);
                reflect_tan(pp, dp[j], N, dN);
                if (j == 1) for (int i = 0; i < 3; ++i) p[i] = pp[i];
            }
            ti->contacts++;
            h = sig_add(h, 1);
            continue;
        }
        /* entry into the box */
        double t = tb;
        for (int j = 0; j < 2; ++j) {
            double dt;
            if (face == EV_TOP) dt = -(dr[j][1] + t * dp[j][1]) / p[1];
            else if (face == EV_RIGHT) dt = ((j == 1 ? 1.0 : 0.0) - dr[j][0] - t * dp[j][0]) / p[0];
            else dt = (-(j == 1 ? 1.0 : 0.0) - dr[j][0] - t * dp[j][0]) / p[0];
            for (int i = 0; i < 3; ++i) dr[j][i] += dt * p[i] + t * dp[j][i];
        }
        for (int i = 0; i < 3; ++i) r[i] += t * p[i];
        if (face == EV_TOP) r[1] = s->ytop; else if (face == EV_RIGHT) r[0] = s->hw; else r[0] = -s->hw;
        double nf[3];
        face_normal(face, nf);
        for (int i = 0; i < 3; ++i) nf[i] = -nf[i];
        double dn[2], nA;
        double n2 = orc_index_jac(s, r[0], r[1], dn, &nA);
        int through = 1;
        {
            double p0[3] = { p[0], p[1], p[2] };
            for (int j = 0; j < 2; ++j) {
                double pp[3] = { p0[0], p0[1], p0[2] };
                double dn2 = dn[0] * dr[j][0] + dn[1] * dr[j][1] + (j == 0 ? nA : 0.0);
                through = snell_tan(pp, dp[j], nf, n2, dn2);
                if (j == 1) for (int i = 0; i < 3; ++i) p[i] = pp[i];
            }
        }
        h = sig_add(h, 10 + face + (through ? 0 : 4));
        if (!through) continue;
        /* integrate inside the box (RK4) */
        st4 u = { { r[0], r[1], p[0], p[1] } };
        double du[2][4];
        for (int j = 0; j < 2; ++j) { du[j][0] = dr[j][0]; du[j][1] = dr[j][1]; du[j][2] = dp[j][0]; du[j][3] = dp[j][1]; }
        double pz = p[2], dpz[2] = { dp[0][2], dp[1][2] };
        int bad = 0;
        long run = 0;   /* steps since the last event: part of the signature */
        for (;;) {
            if (ti->steps >= o->max_steps) { *sig = h; return RAY_MAX_STEPS; }
            st4 y5;
            double dy5[2][4], dtau[4];
            rk4_step_tan(s, &u, du, o->h, &y5, dy5, dtau);
            ti->steps++;
            run++;
            int hit = EV_NONE;
            double theta = 2.0;
            for (int ev = 0; ev < 4; ++ev) {
                if (event_value(s, ev, &y5) >= 0.0) continue;
                double lo = 0.0, hi = 1.0;
                while (hi - lo > 1e-14) {
                    double mid = 0.5 * (lo + hi);
                    st4 ym;
                    rk4_step(s, &u, mid * o->h, &ym, &bad);
                    if (event_value(s, ev, &ym) < 0.0) hi = mid; else lo = mid;
                }
                if (hi < theta) { theta = hi; hit = ev; }
            }
            if (hit == EV_NONE) {
                u = y5;
                memcpy(du, dy5, sizeof du);
                continue;
            }
            /* partial step to the event; tau* implicit in e(Phi(tau*)) = 0 */
            st4 ye;
            double dye[2][4], dte[4];
            double taus = theta * o->h;
            rk4_step_tan(s, &u, du, taus, &ye, dye, dte);
            double ge[4] = { 0, 0, 0, 0 }, eA = 0.0, ehw = 0.0;
            if (hit == EV_TOP) ge[1] = -1.0;
            else if (hit == EV_RIGHT) { ge[0] = -1.0; ehw = 1.0; }
            else if (hit == EV_LEFT) { ge[0] = 1.0; ehw = 1.0; }
            else {
                double E, S, Sx, SA, Ex, EA;
                orc_surface_jac(s, ye.v[0], &E, &S, &Sx, &SA, &Ex, &EA);
                ge[0] = -Sx; ge[1] = 1.0; eA = -SA;
            }
            double gt = ge[0] * dte[0] + ge[1] * dte[1];
            for (int j = 0; j < 2; ++j) {
                double num = ge[0] * dye[j][0] + ge[1] * dye[j][1] + (j == 0 ? eA : ehw);
                double dts = -num / gt;
                for (int q = 0; q < 4; ++q) du[j][q] = dye[j][q] + dte[q] * dts;
            }
            u = ye;
            h = sig_add(h, (uint64_t)run);
            run = 0;
            if (++ti->events > o->max_events) { *sig = h; return RAY_MAX_EVENTS; }
            double pp3[3] = { u.v[2], u.v[3], pz };
            double dpp[2][3] = { { du[0][2], du[0][3], dpz[0] }, { du[1][2], du[1][3], dpz[1] } };
            if (hit == EV_GRATING) {
                double p0[3] = { pp3[0], pp3[1], pp3[2] };
                for (int j = 0; j < 2; ++j) {
                    double N[2], dN[2], q3[3] = { p0[0], p0[1], p0[2] };
                    orc_normal_tan(s, u.v[0], du[j][0], j == 0 ? 1.0 : 0.0, N, dN);
                    reflect_tan(q3, dpp[j], N, dN);
                    if (j == 1) for (int i = 0; i < 3; ++i) pp3[i] = q3[i];
                }
                ti->contacts++;
                h = sig_add(h, 20);
            } else {
                double nfb[3];
                face_normal(hit, nfb);
                double p0[3] = { pp3[0], pp3[1], pp3[2] };
                int thr = 1;
                for (int j = 0; j < 2; ++j) {
                    double q3[3] = { p0[0], p0[1], p0[2] };
                    thr = snell_tan(q3, dpp[j], nfb, 1.0, 0.0);
                    if (j == 1) for (int i = 0; i < 3; ++i) pp3[i] = q3[i];
                }
                h = sig_add(h, 30 + hit + (thr ? 0 : 4));
                if (thr) {
                    r[0] = u.v[0]; r[1] = u.v[1];
                    for (int i = 0; i < 3; ++i) p[i] = pp3[i];
                    for (int j = 0; j < 2; ++j) {
                        dr[j][0] = du[j][0]; dr[j][1] = du[j][1]; dr[j][2] = 0.0;
                        for (int i = 0; i < 3; ++i) dp[j][i] = dpp[j][i];
                    }
                    break;
                }
            }
            u.v[2] = pp3[0]; u.v[3] = pp3[1];
            for (int j = 0; j < 2; ++j) { du[j][2] = dpp[j][0]; du[j][3] = dpp[j][1]; dpz[j] = dpp[j][2]; }
        }
    }
}

/* sky colour and its gradient with respect to the (unnormalised) direction */
static void sky_grad(double K, const double d[3], double rgb[3], double g[3][3])
{
    const double Ca[3] = { 0.95, 0.85, 0.30 }, Cb[3] = { 0.10, 0.20, 0.55 };
    double rho2 = d[0] * d[0] + d[2] * d[2], rho = sqrt(rho2);
    double r2 = rho2 + d[1] * d[1];
    double phi = atan2(d[0], -d[2]);
    double th = atan2(d[1], rho);
    double A4 = cos(4.0 * phi), B8 = sin(8.0 * th);
    double ta = tanh(K * A4), tb = tanh(K * B8);
    double m = 0.5 + 0.5 * ta * tb;
    double dphi[3] = { -d[2] / rho2, 0.0, d[0] / rho2 };
    double dth[3] = { -d[1] * d[0] / (rho * r2), rho / r2, -d[1] * d[2] / (rho * r2) };
    double dm[3];
    for (int i = 0; i < 3; ++i)
        dm[i] = 0.5 * ((1.0 - ta * ta) * K * (-4.0 * sin(4.0 * phi)) * dphi[i] * tb +
                       ta * (1.0 - tb * tb) * K * 8.0 * cos(8.0 * th) * dth[i]);
    for (int c = 0; c < 3; ++c) {
        rgb[c] = Cb[c] + m * (Ca[c] - Cb[c]);
        for (int i = 0; i < 3; ++i) g[c][i] = dm[i] * (Ca[c] - Cb[c]);
    }
}

/* Per-sample render with derivatives (RK4 only).  For each listed pixel
   (or all when npix < 0) and sample: rgb (3), d rgb / dA (3),
   d rgb / d half_width (3), event signature, status.  Outputs are indexed
   (pixel, sample). */
int gco_render_samples_tan(const double* scene, const double* cam, uint64_t seed, const double* opts,
                           long npix, const long* pix, double* rgb, double* drgb_A, double* drgb_hw,
                           uint64_t* sig, int* status, int nthreads)
{
    oscene s;
    oopts o;
    load_scene(scene, &s);
    load_opts(opts, &o);
    if (o.integ != 0 || s.mirror == 1 || !isfinite(s.K) || s.cloak > CLOAK_EQ1 || s.fresnel || s.backdrop) return -1;
    int W = (int)cam[7], H = (int)cam[8], spp = (int)cam[9];
    long total = npix < 0 ? (long)W * H : npix;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (long q = 0; q < total; ++q) {
        long pidx = npix < 0 ? q : pix[q];
        int i = (int)(pidx % W), j = (int)(pidx / W);
        for (int smp = 0; smp < spp; ++smp) {
            long k = q * spp + smp;
            double org[3], dir[3], od[3], dd[2][3], c[3], g[3][3];
            trace_info ti;
            gco_camera_ray(cam, seed, i, j, smp, org, dir);
            int st = trace_one_tan(&s, &o, org, dir, od, dd, &sig[k], &ti);
            status[k] = st;
            if (st != RAY_OK) {
                for (int a = 0; a < 3; ++a) { rgb[3 * k + a] = 0.0; drgb_A[3 * k + a] = 0.0; drgb_hw[3 * k + a] = 0.0; }
                continue;
            }
            sky_grad(s.K, od, c, g);
            for (int a = 0; a < 3; ++a) {
                rgb[3 * k + a] = c[a];
                drgb_A[3 * k + a] = g[a][0] * dd[0][0] + g[a][1] * dd[0][1] + g[a][2] * dd[0][2];
                drgb_hw[3 * k + a] = g[a][0] * dd[1][0] + g[a][1] * dd[1][1] + g[a][2] * dd[1][2];
            }
        }
    }
    return 0;
}

/* exported pointwise derivative helpers (for the test-suite) */
void gco_accel_jac(const double* scene, double x, double y, double out[8])
{
    oscene s;
    load_scene(scene, &s);
    double a[2], J[2][2], aA[2];
    orc_accel_jac(&s, x, y, a, J, aA);
    out[0] = a[0]; out[1] = a[1];
    out[2] = J[0][0]; out[3] = J[0][1]; out[4] = J[1][0]; out[5] = J[1][1];
    out[6] = aA[0]; out[7] = aA[1];
}

int gco_trace_rays_tan(const double* scene, const double* opts, long n, const double* org, const double* dir,
                       double* out_dir, double* ddir, int* status, uint64_t* sig, int nthreads)
{
    oscene s;
    oopts o;
    load_scene(scene, &s);
    load_opts(opts, &o);
    if (o.integ != 0 || s.mirror == 1 || s.cloak > CLOAK_EQ1 || s.fresnel || s.backdrop) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (long i = 0; i < n; ++i) {
        trace_info ti;
        double od[3], dd[2][3];
        status[i] = trace_one_tan(&s, &o, org + 3 * i, dir + 3 * i, od, dd, &sig[i], &ti);
        for (int k = 0; k < 3; ++k) {
            out_dir[3 * i + k] = od[k];
            ddir[6 * i + k] = dd[0][k];
            ddir[6 * i + 3 + k] = dd[1][k];
        }
    }
    return 0;
}
