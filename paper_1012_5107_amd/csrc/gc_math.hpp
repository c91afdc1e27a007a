// gc_math.hpp -- device math for the gfx950 grating-cloak ray tracer.
//
// Index profile of the grating cloak (Sec. 2, eq. (1)):
//     n = 1 / |1 + W|,  W = W0(Z),  Z = i c k e^{ik(x+iy)} = -A k e^{-ky} e^{ikx}
// (c = iA).  Rays follow dr/dtau = p, dp/dtau = grad(n^2)/2 = a with
//     a_x + i a_y = i k conj(W) (1 + W)^2 / |1 + W|^6,
// which is eq. (12) multiplied by n and is eq. (11) after dt = n^2 dtau.
//
// The Lambert function is never started cold inside the integration loop.
// With Q = Z e^{-W} = -A k exp(-k y - Re W) cis(k x - Im W) the equation
// W e^W = Z reads f(W) = W - Q = 0, f' = 1 + Q, f'' = -Q, and one Halley
// step W <- W - 2 f f' / (2 f'^2 + f Q) costs a single complex exponential.
// The start is a first-order predictor from the previous evaluation,
// W + (dW/dzeta) dzeta with dW/dzeta = i k W / (1 + W).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gc {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kInvTwoPi = 0.15915494309189533577;
constexpr double kLog2e = 1.44269504088896340736;
constexpr double kInvE = 0.36787944117144232160;

// ---------------------------------------------------------------------------
// Launch-time parameter blocks (kernel arguments live in constant memory).
// ---------------------------------------------------------------------------
// cloak kinds: none; eq. (1); eq. (1) / n_min with n_min = 1 / (1 + A k) (the
// referenced cloak of Sec. 4); a homogeneous plate of index 1 / n_min
enum CloakKind { CK_NONE = 0, CK_EQ1 = 1, CK_REF = 2, CK_PLATE = 3 };

struct SceneDev {
    double L, A, hw, ytop, K;
    double k, e, invL;
    double invk;       // 1 / k
    double ybp;        // branch-point height (1 + ln(A k)) / k: Z crosses the cut only below it
    double S_hw;       // grating height at x = +-half_width
    double nsc;        // index multiplier inside the box: 1 + A k for the referenced cloak, else 1
    double nsc2;       // nsc^2 (the acceleration grad(n^2)/2 scales by it)
    double nplate;     // the plate's index 1 + A k (cloak CK_PLATE)
    double bd_y, bd_P; // backdrop plane y = bd_y and its pattern period (backdrop 1)
    int cloak, mirror;
    int fresnel;       // 1: Fresnel-weighted faces with one reflected branch per crossing
    int backdrop;      // 0: sky at infinity, 1: patterned plane
};

struct CamDev {
    double eye[3], f[3], r[3], u[3];
    double t, aspect;
    int W, H, spp, jitter;
    uint64_t seed;
    long long scene_index;
};

struct OptsDev {
    int integ;         // 0 RK4, 1 DOPRI5
    int max_events;
    long long max_steps;
    double h, rtol, atol, h_max, h0, h_min;
    double wfb2;       // |1 + W|^2 below which FP32 hands the step to FP64
    int stay;          // hand-overs after which the FP64 kernel keeps the visit (0: never)
};

enum RayStatus { RS_OK = 0, RS_MAX_STEPS = 1, RS_MAX_EVENTS = 2, RS_NONFINITE = 3, RS_UNDERFLOW = 4 };

// ---------------------------------------------------------------------------
// Minimal complex arithmetic.
// ---------------------------------------------------------------------------
template <typename T> struct cx { T re, im; };

template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }

// ---------------------------------------------------------------------------
// Elementary functions: FP32 maps onto the hardware transcendental unit
// (v_exp_f32 is 2^x, v_sin/v_cos take revolutions), FP64 uses the device
// math library.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float exp_e(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ __forceinline__ double exp_e(double x) { return exp(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
// cis(2 pi r) for |r| <= 1
__device__ __forceinline__ void cis_rev(float r, float& c, float& s)
{
    c = __builtin_amdgcn_cosf(r);
    s = __builtin_amdgcn_sinf(r);
}
__device__ __forceinline__ void cis_rev(double r, double& c, double& s) { sincospi(2.0 * r, &s, &c); }

// ---------------------------------------------------------------------------
// Lambert W0 from scratch (FP64): entry points, evaluation paths that cross
// the branch cut, and recovery.  Halley iteration on f = W - z e^{-W}
// from the textbook starts (Corless et al., Adv. Comput. Math. 5 (1996)):
// Taylor series near 0, the branch-point series near -1/e, log(1 + z) and
// the asymptotic log z - log log z.  The first start whose limit has a small
// residual and lies in the principal range is kept.
// ---------------------------------------------------------------------------
__device__ inline cx<double> cexp_d(cx<double> w)
{
    double s, c;
    sincos(w.im, &s, &c);
    double m = exp(w.re);
    return {m * c, m * s};
}
__device__ inline cx<double> clog_d(cx<double> z) { return {log(hypot(z.re, z.im)), atan2(z.im, z.re)}; }
__device__ inline cx<double> csqrt_d(cx<double> z)
{
    double r = hypot(z.re, z.im);
    double a = sqrt(0.5 * (r + fabs(z.re)));
    if (a == 0.0) return {0.0, 0.0};
    double b = 0.5 * z.im / a;
    if (z.re >= 0.0) return {a, b};
    return {fabs(b), copysign(a, z.im)};
}
__device__ inline cx<double> cdiv_d(cx<double> a, cx<double> b)
{
    double inv = 1.0 / norm2(b);
    return inv * (a * conjg(b));
}

__device__ inline bool w0_principal(cx<double> w)
{
    if (!(fabs(w.im) < kPi)) return false;
    if (w.im == 0.0) return w.re >= -1.0 - 1e-12;
    double s, c;
    sincos(w.im, &s, &c);
    return w.re > -w.im * c / s - 1e-10;
}

__device__ inline bool w0_refine(cx<double> z, cx<double>& w)
{
    for (int it = 0; it < 40; ++it) {
        cx<double> q = z * cexp_d(mk(-w.re, -w.im));
        cx<double> f = w - q;
        cx<double> fp = mk(1.0 + q.re, q.im);
        cx<double> den = 2.0 * (fp * fp) + f * q;
        if (den.re == 0.0 && den.im == 0.0) break;
        cx<double> d = cdiv_d(2.0 * (f * fp), den);
        w = w - d;
        if (!(norm2(d) > 1e-32 * fmax(1.0, norm2(w)))) break;
    }
    cx<double> res = w * cexp_d(w) - z;
    return isfinite(w.re) && isfinite(w.im) &&
           norm2(res) <= 1e-28 * fmax(norm2(z), 1e-300) && w0_principal(w);
}

__device__ __noinline__ cx<double> w0_cold(cx<double> z)
{
    double az2 = norm2(z);
    if (az2 == 0.0) return z;
    if (az2 < 1e-6) {
        // |z| < 1e-3 (every entry through the top face): the Taylor series of
        // W0 at 0, sum (-n)^(n-1) z^n / n!, through z^6 leaves a relative
        // error below 2.4e-17
        const double c[6] = {1.0, -1.0, 1.5, -8.0 / 3.0, 125.0 / 24.0, -10.8};
        cx<double> t = mk(c[5], 0.0);
        for (int n = 4; n >= 0; --n) t = mk(c[n], 0.0) + t * z;
        return t * z;
    }
    // the starts in order; each is formed only if the ones before it failed
    cx<double> first = z;
    bool have = false;
    auto attempt = [&](cx<double> w, cx<double>& out) {
        bool ok = w0_refine(z, w);
        if (ok) { out = w; return true; }
        if (!have) { first = w; have = true; }
        return false;
    };
    cx<double> w;
    if (az2 < 0.0625 && attempt(z - z * z + 1.5 * (z * z * z), w)) return w;
    cx<double> zb = mk(z.re + kInvE, z.im);
    if (norm2(zb) < 0.09) {
        // p = sqrt(2 (e z + 1)) with e z + 1 = e (z + 1/e)
        cx<double> p = csqrt_d(mk(2.0 * 2.71828182845904523536, 0.0) * zb);
        if (attempt(mk(-1.0, 0.0) + p - (1.0 / 3.0) * (p * p) + (11.0 / 72.0) * (p * p * p), w)) return w;
    }
    if (attempt(clog_d(mk(1.0 + z.re, z.im)), w)) return w;
    {
        cx<double> l1 = clog_d(z), l2 = clog_d(l1);
        if (attempt(l1 - l2 + cdiv_d(l2, l1), w)) return w;
    }
    return first;
}

// Z at (x, y) in FP64 with x reduced to the central period.
__device__ inline cx<double> zarg64(const SceneDev& s, double x, double y)
{
    double xr = x - s.L * rint(x * s.invL);
    double c, sn;
    cis_rev(xr * s.invL, c, sn);
    double m = -s.e * exp(-s.k * y);
    return {m * c, m * sn};
}

// ---------------------------------------------------------------------------
// Right-hand side: W0 update, acceleration and dW/dzeta at (x, y).
// `fx` is x inside its period (|fx| <= L/2 up to a small overshoot): the
// phase of Z only needs fx / L in revolutions.
// On entry W holds the predicted value; on exit the converged one.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void halley_step(const SceneDev& s, T fx, T y, cx<T>& W)
{
    const T k = (T)s.k, e = (T)s.e, invL = (T)s.invL;
    T m = -e * exp_e(-k * y - W.re);
    T c, sn;
    cis_rev(fx * invL - W.im * (T)kInvTwoPi, c, sn);
    cx<T> q = {m * c, m * sn};
    cx<T> f = W - q;
    cx<T> fp = {(T)1 + q.re, q.im};
    cx<T> num = (T)2 * (f * fp);
    cx<T> den = (T)2 * (fp * fp) + f * q;
    T inv = rcp(norm2(den));
    cx<T> d = inv * (num * conjg(den));
    W = W - d;
}

// acceleration and derivative of W from a converged W
template <typename T>
__device__ __forceinline__ void accel_from_w(const SceneDev& s, cx<T> W, T& ax, T& ay, cx<T>& dW, T& d2)
{
    const T k = (T)s.k;
    cx<T> D = {(T)1 + W.re, W.im};
    d2 = norm2(D);
    T r = rcp(d2);
    cx<T> D2 = D * D;
    cx<T> t = conjg(W) * D2;
    T r3 = r * r * r;
    // i k t r^3
    ax = -k * t.im * r3;
    ay = k * t.re * r3;
    // dW/dzeta = i k W conj(D) / |D|^2
    cx<T> u = W * conjg(D);
    dW = {-k * u.im * r, k * u.re * r};
}

// Warm start for W0 at zeta + dz from the converged W and W' = dW/dzeta at
// zeta (W is analytic in zeta = x + i y, since Z = -A k e^{i k zeta}), to
// second order: W'' = i k W' / (1 + W)^2.  Near the branch point the series
// converges on a short segment only; there the quadratic term is dropped
// unless it is well below the linear one.
template <typename T>
__device__ __forceinline__ cx<T> predict_w(const SceneDev& s, cx<T> W, cx<T> dW, cx<T> dz)
{
    const cx<T> lin = dW * dz;
    const cx<T> cD = {(T)1 + W.re, -W.im};            // conj(1 + W)
    const T id2 = rcp(norm2(cD));
    const cx<T> iD2 = (id2 * id2) * (cD * cD);         // 1 / (1 + W)^2
    const cx<T> ikdW = {-(T)s.k * dW.im, (T)s.k * dW.re};
    const cx<T> quad = (T)0.5 * ((ikdW * iD2) * (dz * dz));
    return norm2(quad) < (T)0.25 * norm2(lin) ? (W + lin) + quad : W + lin;
}

// FP64 right-hand side with warm start: iterate Halley to convergence.
// FP64 right-hand side with a warm start: W holds the prediction on entry;
// Halley steps until the update is at rounding level.  `cold` asks for W0
// from scratch instead (the evaluation path crossed the branch cut).
__device__ inline void rhs64(const SceneDev& s, double x, double y, cx<double>& W,
                             double& ax, double& ay, cx<double>& dW, bool cold = false)
{
    if (cold) {
        W = w0_cold(zarg64(s, x, y));
    } else {
        double fx = x - s.L * rint(x * s.invL);
        // Halley converges cubically: after an update of relative size
        // 1e-7 the error left is about C 1e-21, with C ~ 1 / |1 + W|^2
        // (below 1e4 where this path runs), i.e. at rounding level
        for (int it = 0; it < 8; ++it) {
            cx<double> w0 = W;
            halley_step<double>(s, fx, y, W);
            double d2 = norm2(W - w0);
            if (!(d2 > 1e-14 * fmax(1e-10, norm2(W)))) break;
        }
        if (!(isfinite(W.re) && isfinite(W.im))) W = w0_cold(zarg64(s, x, y));
    }
    double d2;
    accel_from_w<double>(s, W, ax, ay, dW, d2);
    // grad(n^2)/2 of the box index: the referenced cloak's is nsc^2 times eq. (1)'s
    ax *= s.nsc2;
    ay *= s.nsc2;
}

// Z = -A k e^{-ky} e^{ikx} lies on the branch cut (-inf, -1/e] exactly on the
// crest lines x = N Lambda below the branch-point height y_bp = (1 + ln A k)/k.
// A warm start carried from (xp, yp) to (x, y) can only change branch if the
// segment between them crosses such a line below y_bp.
__device__ __forceinline__ bool crosses_cut(const SceneDev& s, double x, double y, double xp, double yp)
{
    return fmin(y, yp) < s.ybp && floor(x * s.invL) != floor(xp * s.invL);
}

// Dormand-Prince 5(4) tableau (Dormand & Prince, J. Comput. Appl. Math. 6
// (1980) 19-26): 5th-order weights b, and e = b - b* (5th minus 4th order).
struct DP {
    static constexpr double a21 = 1.0 / 5;
    static constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
    static constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
    static constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561, a54 = -212.0 / 729;
    static constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                            a65 = -5103.0 / 18656;
    static constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784,
                            b6 = 11.0 / 84;
    static constexpr double e1 = 35.0 / 384 - 5179.0 / 57600, e3 = 500.0 / 1113 - 7571.0 / 16695,
                            e4 = 125.0 / 192 - 393.0 / 640, e5 = -2187.0 / 6784 + 92097.0 / 339200,
                            e6 = 11.0 / 84 - 187.0 / 2100, e7 = -1.0 / 40;
};

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output number n of the
// generator seeded with `seed`.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double uniform53(uint64_t seed, uint64_t n)
{
    return (double)(splitmix64(seed, n) >> 11) * 1.1102230246251565404e-16;
}

// Camera sample direction (unit) for pixel (i, j), sample s.
__device__ inline void camera_dir(const CamDev& c, int i, int j, int smp, double d[3])
{
    double du = 0.5, dv = 0.5;
    if (c.jitter) {
        uint64_t ctr = ((((uint64_t)c.scene_index * (uint64_t)c.H + (uint64_t)j) * (uint64_t)c.W +
                         (uint64_t)i) * (uint64_t)c.spp + (uint64_t)smp) * 2ull;
        du = uniform53(c.seed, ctr);
        dv = uniform53(c.seed, ctr + 1ull);
    }
    double sx = (2.0 * (i + du) / c.W - 1.0) * c.t * c.aspect;
    double sy = (1.0 - 2.0 * (j + dv) / c.H) * c.t;
    double n2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        d[a] = c.f[a] + sx * c.r[a] + sy * c.u[a];
        n2 += d[a] * d[a];
    }
    double inv = 1.0 / sqrt(n2);
    for (int a = 0; a < 3; ++a) d[a] *= inv;
}

// Sky colour for a unit direction: with azimuth phi = atan2(d_x, -d_z) and
// elevation theta = atan2(d_y, hypot(d_x, d_z)), cos 4 phi and sin 8 theta
// are taken as the real / imaginary parts of powers of the unit complex
// numbers (-d_z + i d_x)/rho and (rho + i d_y)/|d|, rho = hypot(d_x, d_z).
template <typename T>
__device__ inline void sky_rgb(T K, const T d[3], T rgb[3])
{
    T rho = sqrt(d[0] * d[0] + d[2] * d[2]);
    T nrm = sqrt(rho * rho + d[1] * d[1]);
    cx<T> a = {rho > (T)0 ? -d[2] / rho : (T)1, rho > (T)0 ? d[0] / rho : (T)0};
    cx<T> a2 = a * a;
    cx<T> a4 = a2 * a2;
    cx<T> b = {rho / nrm, d[1] / nrm};
    cx<T> b2 = b * b, b4 = b2 * b2, b8 = b4 * b4;
    T c4 = a4.re, s8 = b8.im;
    T ta, tb;
    if (isinf(K)) {
        ta = c4 > 0 ? (T)1 : (c4 < 0 ? (T)-1 : (T)0);
        tb = s8 > 0 ? (T)1 : (s8 < 0 ? (T)-1 : (T)0);
    } else {
        ta = tanh(K * c4);
        tb = tanh(K * s8);
    }
    T m = (T)0.5 + (T)0.5 * ta * tb;
    const T Ca[3] = {(T)0.95, (T)0.85, (T)0.30};
    const T Cb[3] = {(T)0.10, (T)0.20, (T)0.55};
    for (int c = 0; c < 3; ++c) rgb[c] = Cb[c] + m * (Ca[c] - Cb[c]);
}

// The sky of an FP32 image from an FP64 direction: the unit complex numbers
// and their powers in FP64 (the tanh arguments are K = 16 times them), tanh
// in FP32 on the FP64-formed argument.  Rounding the argument moves tanh by at
// most 6e-8 |x| sech^2 x < 3e-8, below the FP32 resolution of the image.
__device__ inline void sky_rgb_image(double K, const double d[3], float rgb[3])
{
    const double rho = sqrt(d[0] * d[0] + d[2] * d[2]);
    const double nrm = sqrt(rho * rho + d[1] * d[1]);
    const double ir = rho > 0.0 ? 1.0 / rho : 0.0, in = 1.0 / nrm;
    cx<double> a = {rho > 0.0 ? -d[2] * ir : 1.0, d[0] * ir};
    cx<double> a2 = a * a;
    cx<double> a4 = a2 * a2;
    cx<double> b = {rho * in, d[1] * in};
    cx<double> b2 = b * b, b4 = b2 * b2, b8 = b4 * b4;
    const double c4 = a4.re, s8 = b8.im;
    float ta, tb;
    if (isinf(K)) {
        ta = c4 > 0 ? 1.0f : (c4 < 0 ? -1.0f : 0.0f);
        tb = s8 > 0 ? 1.0f : (s8 < 0 ? -1.0f : 0.0f);
    } else {
        ta = tanhf((float)(K * c4));
        tb = tanhf((float)(K * s8));
    }
    const float m = 0.5f + 0.5f * ta * tb;
    const float Ca[3] = {0.95f, 0.85f, 0.30f};
    const float Cb[3] = {0.10f, 0.20f, 0.55f};
    for (int c = 0; c < 3; ++c) rgb[c] = Cb[c] + m * (Ca[c] - Cb[c]);
}

// Backdrop plane (backdrop 1): the ray from r along d meets y = bd_y at
// (X, Z) (FP64), where the pattern is m = 1/2 + 1/2 tanh(K cos(2 pi X / P))
// tanh(K cos(2 pi Z / P)); a ray that does not rise to the plane sees
// m = 0.  Returns m.
__device__ inline double plane_m64(const SceneDev& s, const double r[3], const double d[3], double* ca,
                                   double* cb)
{
    *ca = 0.0;
    *cb = 0.0;
    if (!(d[1] > 0.0 && r[1] < s.bd_y)) return -1.0;
    const double t = (s.bd_y - r[1]) / d[1];
    const double X = r[0] + t * d[0], Z = r[2] + t * d[2];
    const double iP = 1.0 / s.bd_P;
    // cos(2 pi u) with u reduced to [-1/2, 1/2]
    double sa, sb;
    sincospi(2.0 * (X * iP - rint(X * iP)), &sa, ca);
    sincospi(2.0 * (Z * iP - rint(Z * iP)), &sb, cb);
    return 0.0;
}

// Colour of the backdrop seen by a ray leaving from r along the unit d:
// the sky at infinity (backdrop 0) or the plane (backdrop 1), FP64.
__device__ inline void backdrop_rgb64(const SceneDev& s, const double r[3], const double d[3], double rgb[3])
{
    if (s.backdrop == 0) { sky_rgb<double>(s.K, d, rgb); return; }
    double ca, cb, m = 0.0;
    if (plane_m64(s, r, d, &ca, &cb) == 0.0) {
        double ta, tb;
        if (isinf(s.K)) {
            ta = ca > 0 ? 1.0 : (ca < 0 ? -1.0 : 0.0);
            tb = cb > 0 ? 1.0 : (cb < 0 ? -1.0 : 0.0);
        } else {
            ta = tanh(s.K * ca);
            tb = tanh(s.K * cb);
        }
        m = 0.5 + 0.5 * ta * tb;
    }
    const double Ca[3] = {0.95, 0.85, 0.30};
    const double Cb[3] = {0.10, 0.20, 0.55};
    for (int c = 0; c < 3; ++c) rgb[c] = Cb[c] + m * (Ca[c] - Cb[c]);
}

// The same for an FP32 image: the landing point and the cosines in FP64,
// tanh in FP32 on the FP64-formed argument (as sky_rgb_image does for the
// sky); the sky at infinity in FP32 from the FP64 direction.
__device__ inline void backdrop_rgb_image(const SceneDev& s, const double r[3], const double d[3], float rgb[3])
{
    if (s.backdrop == 0) {
        sky_rgb_image(s.K, d, rgb);
        return;
    }
    double ca, cb;
    float m = 0.0f;
    if (plane_m64(s, r, d, &ca, &cb) == 0.0) {
        float ta, tb;
        if (isinf(s.K)) {
            ta = ca > 0 ? 1.0f : (ca < 0 ? -1.0f : 0.0f);
            tb = cb > 0 ? 1.0f : (cb < 0 ? -1.0f : 0.0f);
        } else {
            ta = tanhf((float)(s.K * ca));
            tb = tanhf((float)(s.K * cb));
        }
        m = 0.5f + 0.5f * ta * tb;
    }
    const float Ca[3] = {0.95f, 0.85f, 0.30f};
    const float Cb[3] = {0.10f, 0.20f, 0.55f};
    for (int c = 0; c < 3; ++c) rgb[c] = Cb[c] + m * (Ca[c] - Cb[c]);
}

}  // namespace gc
