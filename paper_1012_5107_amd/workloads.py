"""Seeded synthetic workloads: scenes, cameras and step-control settings.

This module holds only input recipes (plain numbers and a seeded sampler for
the multi-scene batch).  It contains none of the method's arithmetic and is
shared by the GPU tests, the CPU oracle tests and the benchmark.

Scene fields follow the paper's notation (Sec. 2): grating period ``Lambda``,
half peak-to-peak amplitude ``A`` (eq. (2)); the cloak of eq. (1) fills the
box |x| <= half_width, grating < y <= y_top.  There is no public dataset for
this method: the backdrop of the paper's renderings is a photograph that is
not available, so the workloads use a procedural sky, or, for the paper's
own scene, a procedural pattern on the plane of the photograph.
"""
import math

import numpy as np

SQRT45 = math.sqrt(45.0)


# cloak kinds: none, eq. (1), eq. (1) divided by its minimum n_min = 1 / (1 + A k)
# (the referenced cloak of Sec. 4), homogeneous dielectric plate of index 1 / n_min
CLOAK_NONE, CLOAK_EQ1, CLOAK_REFERENCED, CLOAK_PLATE = 0, 1, 2, 3
# backdrops: the sky at infinity, or a patterned plane (the photograph)
BACKDROP_SKY, BACKDROP_PLANE = 0, 1


def scene(A=0.1, half_width=2.0, y_top=1.5, Lambda=1.0, cloak=1, mirror=0, sky_K=16.0, fresnel=0,
          backdrop=BACKDROP_SKY, backdrop_y=0.0, backdrop_period=1.0):
    return dict(Lambda=float(Lambda), A=float(A), half_width=float(half_width),
                y_top=float(y_top), cloak=int(cloak), mirror=int(mirror), sky_K=float(sky_K),
                fresnel=int(fresnel), backdrop=int(backdrop), backdrop_y=float(backdrop_y),
                backdrop_period=float(backdrop_period))


def reference_scene(sc):
    """Flat mirror at y = 0 in air (no grating, no cloak)."""
    r = dict(sc)
    r.update(cloak=0, mirror=1)
    return r


def plate_reference_scene(sc):
    """Flat mirror at y = 0 under a homogeneous dielectric plate of index
    1 / n_min = 1 + A k filling the cloak's box (Sec. 4, Figs. 5-7 (a))."""
    r = dict(sc)
    r.update(cloak=CLOAK_PLATE, mirror=1)
    return r


def uncloaked_scene(sc):
    """The bare trochoid grating without the index profile."""
    r = dict(sc)
    r.update(cloak=0, mirror=0)
    return r


def camera(width, height, spp=1, jitter=False, seed=0, eye=(0.0, 3.0, 6.0),
           target=(0.0, 0.0, 0.0), fov_y_deg=40.0, scene_index=0, up=(0.0, 0.0, 0.0), fov_x_deg=0.0):
    """Pinhole camera; up = (0, 0, 0) means +y; fov_x_deg = 0 means square
    pixels (the horizontal opening from the vertical one and the aspect)."""
    return dict(eye=tuple(float(v) for v in eye), target=tuple(float(v) for v in target),
                fov_y_deg=float(fov_y_deg), width=int(width), height=int(height),
                spp=int(spp), jitter=int(bool(jitter)), seed=int(seed),
                scene_index=int(scene_index), up=tuple(float(v) for v in up), fov_x_deg=float(fov_x_deg))


def orbit_eye(az_deg, el_deg, R):
    az, el = math.radians(az_deg), math.radians(el_deg)
    return (R * math.sin(az) * math.cos(el), R * math.sin(el), R * math.cos(az) * math.cos(el))


def opts(integrator="rk4", h=1e-3, rtol=1e-8, atol=None, h_max=0.02, max_events=32,
         max_steps=100_000, h0=1e-3, h_min=1e-12, w_fallback=1e-2, fp64_stay=0):
    return dict(integrator=integrator, h=float(h), rtol=float(rtol),
                atol=float(rtol if atol is None else atol), h_max=float(h_max),
                max_events=int(max_events), max_steps=int(max_steps), h0=float(h0),
                h_min=float(h_min), w_fallback=float(w_fallback), fp64_stay=int(fp64_stay))


# --- the five workloads -------------------------------------------------------

def plain_64():
    """64 x 64, one ray through each pixel centre, A = 0.1, box |x| <= 2,
    RK4 with h = 1e-3."""
    return scene(A=0.1, half_width=2.0), camera(64, 64), opts("rk4", h=1e-3)


def plain_vs_fp32_512():
    """512 x 512, 4 jittered samples (seed 0), A = 0.1, box |x| <= 4,
    DOPRI5 with rtol 1e-8 (FP64) and 1e-5 (FP32)."""
    sc = scene(A=0.1, half_width=4.0)
    cam = camera(512, 512, spp=4, jitter=True, seed=0)
    return sc, cam, opts("dopri5", rtol=1e-8), opts("dopri5", rtol=1e-5)


def branch_stress_1024():
    """1024 x 1024, 8 spp (seed 2), A = 0.15 (A k = 0.942), grazing camera at
    elevation 10 deg, distance 12, box |x| <= 4."""
    sc = scene(A=0.15, half_width=4.0)
    cam = camera(1024, 1024, spp=8, jitter=True, seed=2, eye=orbit_eye(0.0, 10.0, 12.0))
    return sc, cam, opts("dopri5", rtol=1e-5)


def grad_256():
    """256 x 256, 4 spp (seed 3), A = 0.08, half-width 3, RK4 h = 1e-3."""
    sc = scene(A=0.08, half_width=3.0)
    cam = camera(256, 256, spp=4, jitter=True, seed=3)
    return sc, cam, opts("rk4", h=1e-3)


def batch_64(seed=1012, n_scenes=64, jitter_seed=1, resolutions=(256, 512, 1024)):
    """64 scenes from one seed: A ~ U[0.02, 0.15], half-width ~ U[2, 8],
    resolution uniform over {256, 512, 1024}, camera azimuth ~ U[-60, 60] deg
    and elevation ~ U[15, 60] deg at distance sqrt(45) aimed at the origin,
    4 jittered spp (jitter seed 1); y_top = 1.5."""
    rng = np.random.default_rng(seed)
    scenes, cams = [], []
    for s in range(n_scenes):
        A = rng.uniform(0.02, 0.15)
        hw = rng.uniform(2.0, 8.0)
        res = int(rng.choice(resolutions))
        az = rng.uniform(-60.0, 60.0)
        el = rng.uniform(15.0, 60.0)
        scenes.append(scene(A=A, half_width=hw))
        cams.append(camera(res, res, spp=4, jitter=True, seed=jitter_seed,
                           eye=orbit_eye(az, el, SQRT45), scene_index=s))
    return scenes, cams


# --- the paper's scene (Sec. 4, Figs. 2-7; Sec. 5, Table 1) -----------------
# The observer stands d = 2.64 units above the mirror and looks down at it
# with a 50 x 42 degree field of view; the grating (Lambda = 1,
# A = 3 / (16 pi)) runs along the image's vertical (tan(21 deg) = Lambda / d:
# three maxima in view).  The photograph she stands in front of is replaced
# by a patterned plane at her height; the cloak covers the whole mirror.
PAPER_A = 3.0 / (16.0 * math.pi)
PAPER_D = 2.64
PAPER_HEIGHTS = (1.1, 0.55, 0.41)
PAPER_FOVS = (0.0, 10.0, 25.0, 50.0)


def paper_scene(kind, height=1.1, fresnel=1, period=0.5, sky_K=16.0):
    """kind: 'flat' (Fig. 3 (a)), 'grating' (3 (b)), 'cloak' (3 (c), eq. (1)),
    'plate' (5-7 (a): plate of index 1 / n_min on the flat mirror),
    'plate_grating' (5-7 (b)), 'referenced' (5-7 (c))."""
    cloak, mirror = {"flat": (CLOAK_NONE, 1), "grating": (CLOAK_NONE, 0), "cloak": (CLOAK_EQ1, 0),
                     "plate": (CLOAK_PLATE, 1), "plate_grating": (CLOAK_PLATE, 0),
                     "referenced": (CLOAK_REFERENCED, 0)}[kind]
    return scene(A=PAPER_A, half_width=math.inf, y_top=height, cloak=cloak, mirror=mirror, sky_K=sky_K,
                 fresnel=fresnel if cloak != CLOAK_NONE else 0, backdrop=BACKDROP_PLANE, backdrop_y=PAPER_D,
                 backdrop_period=period)


def paper_camera(width=301, height=251, spp=4, seed=4):
    """The observer's point camera: at (0, d, 0) looking down, the image's up
    along +x (across the grooves), 50 deg horizontally and 42 vertically;
    an odd width puts a column on the vertical centre line (FOV 0)."""
    return camera(width, height, spp=spp, jitter=spp > 1, seed=seed, eye=(0.0, PAPER_D, 0.0),
                  target=(0.0, 0.0, 0.0), up=(1.0, 0.0, 0.0), fov_y_deg=42.0, fov_x_deg=50.0)


def fov_columns(cam, fov_deg):
    """Columns [c0, c1) whose centres lie within the horizontal field of view
    fov_deg about the vertical centre line (0: the centre column)."""
    W = cam["width"]
    tx = math.tan(math.radians(0.5 * cam["fov_x_deg"]))
    lim = math.tan(math.radians(0.5 * fov_deg))
    cols = [i for i in range(W) if abs((2.0 * (i + 0.5) / W - 1.0) * tx) <= lim + 1e-12]
    if not cols:
        cols = [W // 2]
    return cols[0], cols[-1] + 1


# The step control the benchmark times: the autotuner's choices on these
# workloads (bench.py --autotune on reruns the search; its pick can change
# from run to run with the timings, so the tests and the benchmark use the
# recorded one).
def batch_timed_opts():
    return opts("dopri5", rtol=1e-7, h_max=0.05, w_fallback=0.3, fp64_stay=4)


def single_timed_opts():
    """512 x 512 x 4: FP32 step control and the in-box kernel's scheduling
    (slow_pxy, slow_wave_div, refill, waves_per_simd)."""
    return opts("dopri5", rtol=3e-7, h_max=0.5), dict(slow_pxy=0.25, slow_wave_div=4, refill=8, waves_per_simd=2)


# Bound on the zero-shift correlation error of every batch scene against the
# converged FP64 solve (rtol 1e-10): the workload's stated accuracy.  A
# scene's C0 rests partly on a few dozen samples trapped near the crests of a
# high-amplitude grating, which end at the step cap or escape depending on
# any change of the integration (FP64 solves at rtol 1e-8 and 1e-10 differ by
# 7e-5 on the worst scene): the reference has to be the converged one.
BATCH_C0_BOUND = 1e-4


def sample_pixels(width, height, count, seed):
    """Seeded, sorted subset of linear pixel indices (row-major)."""
    rng = np.random.default_rng(seed)
    n = width * height
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)
