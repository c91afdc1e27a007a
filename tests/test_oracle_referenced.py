"""Pins of the oracle's referenced cloak, dielectric plate, Fresnel faces,
backdrop plane and general camera (Sec. 3 and Sec. 4).

Each test ties the tracer to something fixed independently of it: refraction
through a homogeneous slab on a flat mirror in closed form (Snell's law and
the slab's lateral displacement), the Fresnel equations in their textbook
angular form, the paper's statement that the referenced cloak's ideal image
is that of the flat mirror under a plate of index 1 / n_min (exact in 2D,
where the cloak is), the geometry of where a reflected ray meets the
backdrop plane, the camera's opening angles, and time reversal.  No GPU.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1012_5107_amd import workloads as W

K2PI = 2.0 * math.pi


def _unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _angle(a, b):
    a, b = _unit(a), _unit(b)
    return 2 * np.arctan2(np.linalg.norm(a - b, axis=-1), np.linalg.norm(a + b, axis=-1))


def _slab_exit(org, d, h, n):
    """Closed form for a ray from org along unit d (d_y < 0) through a plate
    0 <= y <= h of index n on the flat mirror y = 0: entry point on y = h,
    lateral displacement 2 h tan(theta') inside (Snell: sin theta' =
    sin theta / n), exit on y = h with the mirror direction."""
    t1 = (h - org[:, 1]) / d[:, 1]
    P1 = org + t1[:, None] * d
    s = np.hypot(d[:, 0], d[:, 2])
    sp = s / n
    tp = sp / np.sqrt(1.0 - sp * sp)
    hor = np.stack([d[:, 0], np.zeros_like(s), d[:, 2]], axis=1) / np.where(s > 0, s, 1.0)[:, None]
    exit_pt = P1 + (2.0 * h * tp)[:, None] * hor
    return exit_pt, d * [1, -1, 1]


def _fresnel_R_angular(cos_i, n1, n2):
    """Unpolarised reflectance from the Fresnel equations (angles)."""
    sin_i = np.sqrt(1.0 - cos_i ** 2)
    sin_t = n1 / n2 * sin_i
    cos_t = np.sqrt(1.0 - sin_t ** 2)
    rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t)
    rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t)
    return 0.5 * (rs ** 2 + rp ** 2)


def _camera_rays(cam):
    org, d = O.camera_rays(cam)
    return org, d


# --------------------------------------------------------------------------
# the plate of index 1 / n_min on the flat mirror (Figs. 5-7 (a))
# --------------------------------------------------------------------------

@pytest.mark.parametrize("A,h", [(3.0 / (16 * math.pi), 1.1), (0.1, 0.41)])
def test_plate_on_flat_mirror_closed_form(A, h):
    sc = W.plate_reference_scene(W.scene(A=A, half_width=1e9, y_top=h))
    n = 1.0 + A * K2PI
    cam = W.camera(9, 7, eye=(0.3, 2.64, 0.5), fov_y_deg=42.0)
    org, d = _camera_rays(cam)
    r = O.trace_rays(sc, W.opts(), org, d)
    assert np.all(r["status"] == 0)
    P, dref = _slab_exit(org, d, h, n)
    assert np.max(_angle(r["dir"], dref)) < 1e-15
    assert np.max(np.abs(r["org"] - P)) < 1e-12
    # events: entry, mirror, exit
    assert np.all(r["events"] == 3) and np.all(r["contacts"] == 1)


def test_plate_total_internal_reflection_at_the_side_faces():
    # Inside a plate entered through its top face the momentum keeps its
    # tangential part (d_x, d_z) and |p| = n; at a side face (normal x) the
    # tangential part has |p_t|^2 = n^2 - d_x^2 >= n^2 - 1 > 1 for n > sqrt(2):
    # total internal reflection, which folds x back into |x| <= hw.
    # Unfolded, the ray crosses the plate down and up once: x moves by
    # 2 h d_x / |p_y| with |p_y| = sqrt(n^2 - d_x^2 - d_z^2); folding that
    # into the box gives the exit point and the sign of d_x.
    A, hw, h = 0.1, 0.5, 1.0
    n = 1.0 + A * K2PI
    assert n > math.sqrt(2.0)
    sc = W.plate_reference_scene(W.scene(A=A, half_width=hw, y_top=h))
    d = _unit([[0.9, -0.3, 0.3162], [-0.6, -0.7, 0.2], [0.2, -0.95, -0.1], [0.1, -0.95, 0.05]])
    xe = np.array([0.3, -0.1, 0.45, 0.0])
    org = np.stack([xe - 3.0 * d[:, 0], h - 3.0 * d[:, 1], -3.0 * d[:, 2]], axis=1)
    r = O.trace_rays(sc, W.opts(), org, d)
    assert np.all(r["status"] == 0)
    py = np.sqrt(n * n - d[:, 0] ** 2 - d[:, 2] ** 2)
    u = xe + 2.0 * h * d[:, 0] / py
    v = np.mod(u + hw, 4.0 * hw)
    x_exit = np.where(v <= 2.0 * hw, v - hw, 3.0 * hw - v)
    sign = np.where(v <= 2.0 * hw, 1.0, -1.0)
    n_side = np.abs(np.floor((u + hw) / (2.0 * hw)))
    assert np.max(np.abs(r["org"][:, 0] - x_exit)) < 1e-13
    assert np.max(np.abs(r["org"][:, 2] - (org[:, 2] + 3.0 * d[:, 2] + 2.0 * h * d[:, 2] / py))) < 1e-13
    want = np.stack([sign * d[:, 0], -d[:, 1], d[:, 2]], axis=1)
    assert np.max(_angle(r["dir"], want)) < 1e-15
    # entry, mirror, exit and one event per side-face reflection
    assert np.array_equal(r["events"], 3 + n_side.astype(int))
    assert sorted(set(n_side.astype(int))) == [0, 1, 2]


# --------------------------------------------------------------------------
# Fresnel faces (Sec. 3): one reflected branch per crossing of the primary
# --------------------------------------------------------------------------

@pytest.mark.parametrize("K", [16.0, math.inf])
def test_fresnel_plate_colour_closed_form(K):
    # A plate on the flat mirror (no side faces in view) with the sky at
    # infinity: every path leaves with the mirror direction d', so a pixel
    # is w sky(d') with w = R (top-face reflection) + T^2 (the primary path)
    # + T R T (reflected once inside, transmitted on its second arrival);
    # the path reflected twice inside is neglected.  R at the top face is
    # the same from air and from inside (the angles are Snell partners).
    A, h = 0.1, 0.55
    n = 1.0 + A * K2PI
    sc = W.plate_reference_scene(W.scene(A=A, half_width=1e9, y_top=h, fresnel=1, sky_K=K))
    cam = W.camera(7, 5, eye=(0.0, 3.0, 6.0), fov_y_deg=40.0)
    rgb, cnt = O.render(sc, cam, W.opts())
    org, d = _camera_rays(cam)
    R = _fresnel_R_angular(-d[:, 1], 1.0, n)
    T = 1.0 - R
    w = R + T * T + T * R * T
    want = np.array([w[q] * O.sky(K, d[q] * [1, -1, 1]) for q in range(len(d))]).reshape(5, 7, 3)
    assert np.max(np.abs(rgb - want)) < 1e-14
    assert cnt["failed"] == 0
    # the reflectance at normal incidence is ((n - 1) / (n + 1))^2
    assert abs(_fresnel_R_angular(np.array([1.0]), 1.0, n)[0] - ((n - 1) / (n + 1)) ** 2) < 1e-16


def test_fresnel_brewster_and_grazing():
    # the angular form used above: r_p vanishes at Brewster's angle
    # tan(theta_B) = n2 / n1, and R -> 1 at grazing incidence
    n = 1.6
    tb = math.atan(n)
    R = _fresnel_R_angular(np.array([math.cos(tb)]), 1.0, n)[0]
    ci, ct = math.cos(tb), math.sqrt(1 - (math.sin(tb) / n) ** 2)
    rs = (ci - n * ct) / (ci + n * ct)
    assert abs(R - 0.5 * rs * rs) < 1e-16
    assert _fresnel_R_angular(np.array([1e-9]), 1.0, n)[0] > 1 - 1e-8


def test_fresnel_dims_the_cloaked_image():
    # Sec. 4: the Fresnel transmissions make the primary image slightly
    # dimmer; with the reflected branches the total weight stays below 1
    sc = W.scene(A=0.1, half_width=2.0, cloak=W.CLOAK_REFERENCED)
    cam = W.camera(8, 8)
    op = W.opts("dopri5", rtol=1e-9)
    g0, _ = O.render(sc, cam, op)
    g1, _ = O.render(dict(sc, fresnel=1), cam, op)
    assert 0 < np.mean(g0) - np.mean(g1) < 0.05


# --------------------------------------------------------------------------
# the referenced cloak (Sec. 4, Figs. 5-7 (c))
# --------------------------------------------------------------------------

def _in_plane_rays(angles_deg, x0s, y0=7.0):
    org, d = [], []
    for a in angles_deg:
        for x0 in x0s:
            org.append([x0, y0, 0.0])
            d.append([math.sin(math.radians(a)), -math.cos(math.radians(a)), 0.0])
    return np.array(org), np.array(d)


def test_referenced_cloak_is_the_plate_in_two_dimensions():
    # Dividing the cloak's indices by n_min maps the virtual half-space above
    # the flat mirror onto a homogeneous medium of index 1 / n_min: in-plane
    # rays through the untruncated referenced cloak (|n - 1/n_min| < 1e-16
    # above y = 6) leave like rays through a plate of that index and height
    # on the flat mirror, in direction and exit point.
    A, ytop = 0.1, 6.0
    n = 1.0 + A * K2PI
    sc = W.scene(A=A, half_width=1e9, y_top=ytop, cloak=W.CLOAK_REFERENCED)
    org, d = _in_plane_rays([20.0, 45.0, -35.0], [0.0, 0.37])
    P, dref = _slab_exit(org, d, ytop, n)
    r = O.trace_rays(sc, W.opts("dopri5", rtol=1e-12, h_max=0.005), org, d)
    assert np.all(r["status"] == 0)
    assert np.max(_angle(r["dir"], dref)) < 1e-10
    assert np.max(np.abs(r["org"][:, 0] - P[:, 0])) < 1e-10
    # RK4 converges to it at fourth order (a ray that meets the grating near
    # a crest, where the referenced index reaches (1 + Ak) / (1 - Ak) = 4.4,
    # needs the smallest steps)
    errs = []
    for h in (1e-3, 5e-4):
        r = O.trace_rays(sc, W.opts("rk4", h=h), org, d)
        assert np.all(r["status"] == 0)
        errs.append(max(np.max(_angle(r["dir"], dref)), np.max(np.abs(r["org"][:, 0] - P[:, 0]))))
    assert errs[-1] < 5e-5
    assert errs[0] / errs[1] > 10
    # the unreferenced cloak gives the flat mirror's exit point instead
    r1 = O.trace_rays(dict(sc, cloak=W.CLOAK_EQ1), W.opts("rk4", h=1e-3), org, d)
    P, _ = _slab_exit(org, d, ytop, n)
    assert np.min(np.abs(r1["org"][:, 0] - P[:, 0])) > 1e-2


def test_referenced_index_scales_by_one_over_nmin():
    # inside the box the referenced cloak's acceleration is (1 / n_min)^2
    # times eq. (1)'s: the same path in space, traversed 1 / n_min times
    # faster in tau; an in-plane ray through the truncated referenced cloak
    # with the faces refracting like the plate still conserves p_z and is
    # time reversible
    sc = W.scene(A=0.1, half_width=2.0, cloak=W.CLOAK_REFERENCED)
    cam = W.camera(16, 16)
    op = W.opts("dopri5", rtol=1e-12, h_max=0.01)
    pix = [(3, 6), (8, 8), (12, 10)]
    org = np.array([O.camera_ray(cam, i, j)[0] for i, j in pix])
    d = np.array([O.camera_ray(cam, i, j)[1] for i, j in pix])
    r = O.trace_rays(sc, op, org, d)
    assert np.all(r["status"] == 0) and np.all(r["steps"] > 50)
    assert np.array_equal(r["dir"][:, 2], d[:, 2] / np.linalg.norm(d, axis=1))
    b = O.trace_rays(sc, op, r["org"] + 5.0 * r["dir"], -r["dir"])
    assert np.all(b["status"] == 0)
    assert np.max(_angle(b["dir"], -d)) < 1e-9
    dist = np.linalg.norm(np.cross(org - b["org"], b["dir"]), axis=1)
    assert np.max(dist) < 1e-8


def test_plate_on_grating_time_reversal():
    # Figs. 5-7 (b): the plate on the bare grating -- straight flights,
    # Snell at the faces, mirror reflections at the trochoid
    sc = W.scene(A=0.1, half_width=2.0, y_top=0.55, cloak=W.CLOAK_PLATE)
    cam = W.camera(16, 16, eye=(0.2, 2.64, 1.0))
    pix = [(2, 3), (8, 8), (13, 12), (5, 14)]
    org = np.array([O.camera_ray(cam, i, j)[0] for i, j in pix])
    d = np.array([O.camera_ray(cam, i, j)[1] for i, j in pix])
    r = O.trace_rays(sc, W.opts(), org, d)
    assert np.all(r["status"] == 0) and np.all(r["contacts"] >= 1)
    b = O.trace_rays(sc, W.opts(), r["org"] + 3.0 * r["dir"], -r["dir"])
    assert np.all(b["status"] == 0)
    assert np.max(_angle(b["dir"], -d)) < 1e-12
    dist = np.linalg.norm(np.cross(org - b["org"], b["dir"]), axis=1)
    assert np.max(dist) < 1e-11


# --------------------------------------------------------------------------
# the backdrop plane and the camera (Sec. 4)
# --------------------------------------------------------------------------

def test_backdrop_plane_landing_points():
    # the photograph is the plane y = 2.64 holding the camera; over the flat
    # mirror a ray returns to it at eye + (t1 + t2) d_xz with t1 = t2 =
    # 2.64 / |d_y|; hard squares (K = inf) make the colour Ca where
    # cos(2 pi X / P) cos(2 pi Z / P) > 0 and Cb where it is < 0
    P = 0.37
    sc = W.scene(A=0.1, cloak=0, mirror=1, sky_K=math.inf, backdrop=W.BACKDROP_PLANE, backdrop_y=2.64,
                 backdrop_period=P)
    cam = W.camera(11, 9, eye=(0.05, 2.64, -0.02), target=(0.05, 0.0, -0.02), up=(1.0, 0.0, 0.0),
                   fov_y_deg=42.0, fov_x_deg=50.0)
    rgb, cnt = O.render(sc, cam, W.opts())
    org, d = _camera_rays(cam)
    t = 2.0 * 2.64 / -d[:, 1]
    X = org[:, 0] + t * d[:, 0]
    Z = org[:, 2] + t * d[:, 2]
    s = np.cos(K2PI * X / P) * np.cos(K2PI * Z / P)
    Ca, Cb = np.array([0.95, 0.85, 0.30]), np.array([0.10, 0.20, 0.55])
    want = np.where(s[:, None] > 0, Ca, Cb).reshape(9, 11, 3)
    assert np.min(np.abs(s)) > 1e-6
    assert np.max(np.abs(rgb - want)) < 1e-15
    # both colours occur
    assert 0 < np.sum(s > 0) < s.size


def test_plate_moves_the_backdrop_landing_point():
    # with the plate the ray reaches the plane displaced by the slab's
    # 2 h (tan theta - tan theta') towards the camera: the plate narrows the
    # field of view (Sec. 4)
    A, h, P = 3.0 / (16 * math.pi), 1.1, 0.53
    n = 1.0 + A * K2PI
    sc = W.plate_reference_scene(W.scene(A=A, half_width=1e9, y_top=h, sky_K=math.inf,
                                         backdrop=W.BACKDROP_PLANE, backdrop_y=2.64, backdrop_period=P))
    cam = W.camera(11, 9, eye=(0.0, 2.64, 0.0), target=(0.0, 0.0, 0.0), up=(1.0, 0.0, 0.0),
                   fov_y_deg=42.0, fov_x_deg=50.0)
    org, d = _camera_rays(cam)
    r = O.trace_rays(sc, W.opts(), org, d)
    Pt, dref = _slab_exit(org, d, h, n)
    t = (2.64 - h) / dref[:, 1]
    X = Pt[:, 0] + t * dref[:, 0]
    Z = Pt[:, 2] + t * dref[:, 2]
    s = np.cos(K2PI * X / P) * np.cos(K2PI * Z / P)
    Ca, Cb = np.array([0.95, 0.85, 0.30]), np.array([0.10, 0.20, 0.55])
    rgb, _ = O.render(sc, cam, W.opts())
    want = np.where(s[:, None] > 0, Ca, Cb).reshape(9, 11, 3)
    assert np.min(np.abs(s)) > 1e-6
    assert np.max(np.abs(rgb - want)) < 1e-15
    # every landing point is closer to the camera's axis than without the plate
    t0 = 2.0 * 2.64 / -d[:, 1]
    R0 = np.hypot(t0 * d[:, 0], t0 * d[:, 2])
    R1 = np.hypot(X, Z)
    off = R0 > 1e-9
    assert np.all(R1[off] < R0[off])


def test_camera_up_hint_and_horizontal_opening():
    # looking straight down with the image's up along +x: the centre pixel
    # looks along -y, the middle of the top row along +x by 2/3 of
    # tan(fov_y / 2), the middle of the right column along +z by 2/3 of
    # tan(fov_x / 2) (right = forward x up)
    cam = W.camera(3, 3, eye=(0.0, 2.64, 0.0), target=(0.0, 0.0, 0.0), up=(1.0, 0.0, 0.0),
                   fov_y_deg=42.0, fov_x_deg=50.0)
    ty, tx = math.tan(math.radians(21.0)), math.tan(math.radians(25.0))
    _, d = O.camera_ray(cam, 1, 1)
    assert np.max(np.abs(d - [0, -1, 0])) < 1e-16
    _, d = O.camera_ray(cam, 1, 0)
    assert np.max(np.abs(d - _unit([2 / 3 * ty, -1, 0]))) < 1e-15
    _, d = O.camera_ray(cam, 2, 1)
    assert np.max(np.abs(d - _unit([0, -1, 2 / 3 * tx]))) < 1e-15
    # with up = 0 the old convention (world up +y) holds
    c2 = W.camera(3, 3)
    c3 = dict(c2, up=(0.0, 1.0, 0.0))
    assert np.array_equal(O.camera_ray(c2, 0, 2)[1], O.camera_ray(c3, 0, 2)[1])
