"""ctypes wrapper of the FP64 CPU oracle (``oracle/gco.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library never
loads this module or its shared object, and this module imports nothing from
the GPU package.

Inputs are the plain dictionaries built by the workload recipes (scene,
camera, step options); they are flattened here into the oracle's own
parameter arrays.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgco.so")
SRC_PATH = os.path.join(_HERE, "gco.c")

RAY_OK, RAY_MAX_STEPS, RAY_MAX_EVENTS, RAY_NONFINITE, RAY_STEP_UNDERFLOW = range(5)

_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    import subprocess
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB_PATH, SRC_PATH, "-lm"]
    if force or not os.path.exists(LIB_PATH):
        subprocess.check_call(cmd)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.gco_lambertw.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        L.gco_lambertw.restype = ctypes.c_int
        L.gco_index.argtypes = [dp, ctypes.c_double, ctypes.c_double]
        L.gco_index.restype = ctypes.c_double
        L.gco_accel.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.gco_grad_n_eq12.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.gco_surface.argtypes = [dp, ctypes.c_double, dp]
        L.gco_surface.restype = ctypes.c_double
        L.gco_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.gco_splitmix64.restype = ctypes.c_uint64
        L.gco_camera_ray.argtypes = [dp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        L.gco_sky.argtypes = [ctypes.c_double, dp, dp]
        L.gco_trace_rays.argtypes = [dp, dp, ctypes.c_long, dp, dp, dp, dp,
                                     ctypes.POINTER(ctypes.c_int), dp, ctypes.c_int]
        L.gco_render_pixels.argtypes = [dp, dp, ctypes.c_uint64, dp, ctypes.c_long,
                                        ctypes.POINTER(ctypes.c_long), dp, dp, ctypes.c_int]
        L.gco_cross_correlate.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                          ctypes.c_long, ctypes.c_int, dp]
        L.gco_cross_correlate_f64.argtypes = [dp, dp, ctypes.c_long, ctypes.c_int, dp]
        L.gco_cross_correlate_map.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                              ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, dp, dp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.gco_accel_jac.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.gco_dp5_tableau.argtypes = [dp]
        L.gco_trace_rays_tan.argtypes = [dp, dp, ctypes.c_long, dp, dp, dp, dp,
                                         ctypes.POINTER(ctypes.c_int), u64p, ctypes.c_int]
        L.gco_trace_rays_tan.restype = ctypes.c_int
        L.gco_render_samples_tan.argtypes = [dp, dp, ctypes.c_uint64, dp, ctypes.c_long,
                                             ctypes.POINTER(ctypes.c_long), dp, dp, dp, u64p,
                                             ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.gco_render_samples_tan.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def scene_array(sc):
    return np.array([sc["Lambda"], sc["A"], sc["half_width"], sc["y_top"],
                     sc["cloak"], sc["mirror"], sc["sky_K"], sc.get("fresnel", 0),
                     sc.get("backdrop", 0), sc.get("backdrop_y", 0.0), sc.get("backdrop_period", 1.0)],
                    dtype=np.float64)


def opts_array(o):
    integ = {"rk4": 0, "dopri5": 1}[o["integrator"]]
    return np.array([integ, o["h"], o["rtol"], o["atol"], o["h_max"], o["max_events"],
                     o["max_steps"], o["h0"], o["h_min"], float(o.get("diagnostics", 0))],
                    dtype=np.float64)


def camera_array(c):
    return np.array(list(c["eye"]) + list(c["target"]) +
                    [c["fov_y_deg"], c["width"], c["height"], c["spp"], c["jitter"],
                     c["scene_index"]] + list(c.get("up", (0.0, 0.0, 0.0))) + [c.get("fov_x_deg", 0.0)],
                    dtype=np.float64)


# --- pointwise functions -----------------------------------------------------

def lambertw(z):
    """Principal branch W0(z); returns (w, ok)."""
    wr, wi = ctypes.c_double(), ctypes.c_double()
    r = lib().gco_lambertw(float(np.real(z)), float(np.imag(z)), ctypes.byref(wr), ctypes.byref(wi))
    return complex(wr.value, wi.value), r == 0


def index(sc, x, y):
    s = scene_array(sc)
    return lib().gco_index(_dp(s), float(x), float(y))


def accel(sc, x, y):
    s = scene_array(sc)
    out = np.zeros(2)
    lib().gco_accel(_dp(s), float(x), float(y), _dp(out))
    return out


def grad_n_eq12(sc, x, y):
    s = scene_array(sc)
    out = np.zeros(2)
    lib().gco_grad_n_eq12(_dp(s), float(x), float(y), _dp(out))
    return out


def surface(sc, x):
    """Grating height S(x) and the trochoid parameter xi of eq. (2)."""
    s = scene_array(sc)
    xi = ctypes.c_double()
    S = lib().gco_surface(_dp(s), float(x), ctypes.byref(xi))
    return S, xi.value


def splitmix64(seed, n):
    return int(lib().gco_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(n)))


def camera_ray(cam, i, j, s=0):
    c = camera_array(cam)
    org, d = np.zeros(3), np.zeros(3)
    lib().gco_camera_ray(_dp(c), ctypes.c_uint64(cam["seed"]), int(i), int(j), int(s), _dp(org), _dp(d))
    return org, d


def camera_rays(cam):
    """All sample rays of a camera, ordered (row j, column i, sample s)."""
    W, H, spp = cam["width"], cam["height"], cam["spp"]
    org = np.zeros((H * W * spp, 3))
    d = np.zeros((H * W * spp, 3))
    q = 0
    for j in range(H):
        for i in range(W):
            for s in range(spp):
                org[q], d[q] = camera_ray(cam, i, j, s)
                q += 1
    return org, d


def dp5_tableau():
    """The oracle's Dormand-Prince tableau: (A 7 x 6, b5, b4)."""
    out = np.zeros(56)
    lib().gco_dp5_tableau(_dp(out))
    return out[:42].reshape(7, 6), out[42:49], out[49:56]


def sky(K, d):
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(3)
    lib().gco_sky(float(K), _dp(d), _dp(out))
    return out


# --- ray tracing and rendering ------------------------------------------------

def trace_rays(sc, o, org, d, nthreads=0):
    """Trace rays; returns dict with exit origin/direction, status and
    per-ray info (steps, rejected, events, contacts, min_cos, bad_w, max_H)."""
    org = np.ascontiguousarray(org, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    n = org.shape[0]
    s, p = scene_array(sc), opts_array(o)
    oo, od = np.zeros((n, 3)), np.zeros((n, 3))
    st = np.zeros(n, dtype=np.int32)
    info = np.zeros((n, 7))
    lib().gco_trace_rays(_dp(s), _dp(p), n, _dp(org), _dp(d), _dp(oo), _dp(od),
                         st.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(info), int(nthreads))
    return dict(org=oo, dir=od, status=st, steps=info[:, 0].astype(np.int64),
                rejected=info[:, 1].astype(np.int64), events=info[:, 2].astype(np.int64),
                contacts=info[:, 3].astype(np.int64), min_cos=info[:, 4],
                bad_w=info[:, 5].astype(np.int64), max_H=info[:, 6])


def render(sc, cam, o, pixels=None, nthreads=0):
    """Render all pixels (H x W x 3) or the listed linear pixel indices
    (len x 3).  Returns (rgb, counters) with counters = dict(rays, steps,
    rejected, failed)."""
    s, c, p = scene_array(sc), camera_array(cam), opts_array(o)
    W, H = cam["width"], cam["height"]
    cnt = np.zeros(4)
    if pixels is None:
        rgb = np.zeros((H, W, 3))
        lib().gco_render_pixels(_dp(s), _dp(c), ctypes.c_uint64(cam["seed"]), _dp(p), -1, None,
                                _dp(rgb), _dp(cnt), int(nthreads))
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        rgb = np.zeros((pix.size, 3))
        lib().gco_render_pixels(_dp(s), _dp(c), ctypes.c_uint64(cam["seed"]), _dp(p), pix.size,
                                pix.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                _dp(rgb), _dp(cnt), int(nthreads))
    return rgb, dict(rays=int(cnt[0]), steps=int(cnt[1]), rejected=int(cnt[2]), failed=int(cnt[3]))


def cross_correlate(f, g):
    """eq. (15) at zero shift (C0) and the Pearson form (NCC)."""
    f = np.asarray(f)
    g = np.asarray(g)
    nch = f.shape[-1] if f.ndim == 3 else 1
    npix = f.size // nch
    out = np.zeros(2)
    if f.dtype == np.float32 and g.dtype == np.float32:
        ff, gg = np.ascontiguousarray(f), np.ascontiguousarray(g)
        fp = ff.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        gp = gg.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        lib().gco_cross_correlate(fp, gp, npix, nch, _dp(out))
    else:
        ff = np.ascontiguousarray(f, dtype=np.float64)
        gg = np.ascontiguousarray(g, dtype=np.float64)
        lib().gco_cross_correlate_f64(_dp(ff), _dp(gg), npix, nch, _dp(out))
    return float(out[0]), float(out[1])


def cross_correlate_map(f, g, rx, ry, cols=None):
    """eq. (15) at every shift |dx| <= rx, |dy| <= ry of the image g against
    the reference f (H x W x C float32, or H x W): returns (map, peak, dx,
    dy) with map[dy + ry, dx + rx] = C(dx, dy) (dx along a row, dy down the
    rows) and the first maximum in row-major order.  cols = (c0, c1) takes
    the column window [c0, c1) of both images (passed with their row pitch,
    not copied)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    g = np.ascontiguousarray(g, dtype=np.float32)
    if f.ndim == 2:
        f, g = f[:, :, None], g[:, :, None]
    H, Wfull, nch = f.shape
    c0, c1 = (0, Wfull) if cols is None else cols
    out = np.zeros((2 * ry + 1, 2 * rx + 1))
    pk = np.zeros(3)
    off = c0 * nch
    fp = ctypes.cast(f.ctypes.data + 4 * off, ctypes.POINTER(ctypes.c_float))
    gp = ctypes.cast(g.ctypes.data + 4 * off, ctypes.POINTER(ctypes.c_float))
    lib().gco_cross_correlate_map(fp, gp, H, c1 - c0, Wfull, nch, int(rx), int(ry), _dp(out), _dp(pk))
    return out, float(pk[0]), int(pk[1]), int(pk[2])


# --- derivatives with respect to the scene parameters (A, half_width) --------

def accel_jac(sc, x, y):
    """Acceleration a(x, y), its Jacobian d a / d(x, y) (2 x 2, rows a_x,
    a_y) and d a / dA."""
    s = scene_array(sc)
    out = np.zeros(8)
    lib().gco_accel_jac(_dp(s), float(x), float(y), _dp(out))
    return out[0:2].copy(), out[2:6].reshape(2, 2).copy(), out[6:8].copy()


def trace_rays_tan(sc, o, org, d, nthreads=0):
    """RK4 tracer with forward-mode tangents.  Returns dict with the unit exit
    direction, its derivatives d_A and d_hw (n x 3 each), status and the
    event-sequence signature of every ray."""
    if o["integrator"] != "rk4" or sc["mirror"]:
        raise ValueError("tangents are provided for RK4 and cloak / grating scenes only")
    org = np.ascontiguousarray(org, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    n = org.shape[0]
    s, p = scene_array(sc), opts_array(o)
    od = np.zeros((n, 3))
    dd = np.zeros((n, 2, 3))
    st = np.zeros(n, dtype=np.int32)
    sig = np.zeros(n, dtype=np.uint64)
    r = lib().gco_trace_rays_tan(_dp(s), _dp(p), n, _dp(org), _dp(d), _dp(od), _dp(dd),
                                 st.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                 sig.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), int(nthreads))
    if r != 0:
        raise ValueError("unsupported tangent configuration")
    return dict(dir=od, d_A=dd[:, 0], d_hw=dd[:, 1], status=st, sig=sig)


def render_samples_tan(sc, cam, o, pixels=None, nthreads=0):
    """Per-sample colours and their derivatives with respect to A and
    half_width.  Arrays are (npix, spp, 3) (colours, d_A, d_hw) and (npix,
    spp) (signature, status); pixels are all pixels in row-major order or
    the listed linear indices."""
    if o["integrator"] != "rk4" or sc["mirror"] or not np.isfinite(sc["sky_K"]):
        raise ValueError("tangents are provided for RK4, cloak / grating scenes and finite sky_K only")
    s, c, p = scene_array(sc), camera_array(cam), opts_array(o)
    W, H, spp = cam["width"], cam["height"], cam["spp"]
    if pixels is None:
        npix, pix, pp = W * H, None, -1
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        npix, pp = pix.size, pix.size
    rgb = np.zeros((npix, spp, 3))
    dA = np.zeros((npix, spp, 3))
    dhw = np.zeros((npix, spp, 3))
    sig = np.zeros((npix, spp), dtype=np.uint64)
    st = np.zeros((npix, spp), dtype=np.int32)
    r = lib().gco_render_samples_tan(
        _dp(s), _dp(c), ctypes.c_uint64(cam["seed"]), _dp(p), pp,
        None if pix is None else pix.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
        _dp(rgb), _dp(dA), _dp(dhw), sig.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        st.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(nthreads))
    if r != 0:
        raise ValueError("unsupported tangent configuration")
    return dict(rgb=rgb, d_A=dA, d_hw=dhw, sig=sig, status=st)


def loss_weights(ref, img, loss="ncc"):
    """dL/dg for the image g = img against the reference f = ref (both
    H x W x 3), with f' and g' the deviations from the channel means
    (eq. (14)), pooled over channels:
      L = 1 - C0,  C0 = sum f' g' / sum f'^2 (eq. (15) at zero shift):
          dL/dg = -f' / sum f'^2  (sum f' = 0 per channel, so the mean of
          g drops out);
      L = 1 - NCC, NCC = sum f' g' / sqrt(sum f'^2 sum g'^2):
          dL/dg = -(f' / sqrt(sum f'^2 sum g'^2) - NCC g' / sum g'^2).
    Returns (L, dL/dg)."""
    f = np.asarray(ref, dtype=np.float64)
    g = np.asarray(img, dtype=np.float64)
    fp = f - f.reshape(-1, 3).mean(axis=0)
    gp = g - g.reshape(-1, 3).mean(axis=0)
    sff, sgg, sfg = float((fp * fp).sum()), float((gp * gp).sum()), float((fp * gp).sum())
    if loss == "c0":
        return 1.0 - sfg / sff, -fp / sff
    ncc = sfg / np.sqrt(sff * sgg)
    return 1.0 - ncc, -(fp / np.sqrt(sff * sgg) - ncc * gp / sgg)


def render_grad(sc, cam, o, ref, loss="ncc", nthreads=0):
    """Loss L (1 - NCC or 1 - C0, see loss_weights) of the rendered image
    against the reference image `ref` (H x W x 3) and its derivatives dL/dA,
    dL/dhw, by forward-mode tangents: dL/dtheta = sum dL/dg dg/dtheta.
    Returns dict(loss, dA, dhw, image, tan)."""
    t = render_samples_tan(sc, cam, o, nthreads=nthreads)
    H, W = cam["height"], cam["width"]
    g = t["rgb"].mean(axis=1).reshape(H, W, 3)
    gA = t["d_A"].mean(axis=1).reshape(H, W, 3)
    ghw = t["d_hw"].mean(axis=1).reshape(H, W, 3)
    L, wgt = loss_weights(np.asarray(ref).reshape(H, W, 3), g, loss)
    return dict(loss=L, dA=float((wgt * gA).sum()), dhw=float((wgt * ghw).sum()), image=g, tan=t)
