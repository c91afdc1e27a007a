"""Python binding of ``libgcloak.so`` (C ABI in ``include/gcloak.h``).

Argument marshalling only: torch provides device memory and the current
stream; every step of the computation runs in the library's HIP kernels.
Importing this module loads the library and fails loudly when it has not been
built (``python -m paper_1012_5107_amd.build``) -- there is no fallback.
"""
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgcloak.so")

GC_OK, GC_EINVAL, GC_EDOMAIN, GC_ENOMEM, GC_EDEVICE, GC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GC_F64, GC_F32 = 0, 1
GC_LOSS_C0, GC_LOSS_NCC = 0, 1
SKY_CA = (0.95, 0.85, 0.30)   # sky colours: colour = CB + m (CA - CB)
SKY_CB = (0.10, 0.20, 0.55)
GC_RK4, GC_DOPRI5 = 0, 1
RAY_OK, RAY_MAX_STEPS, RAY_MAX_EVENTS, RAY_NONFINITE, RAY_STEP_UNDERFLOW = range(5)


class GcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gcloak error {status}: {msg}")
        self.status = status


class Scene(ctypes.Structure):
    _fields_ = [("Lambda", ctypes.c_double), ("A", ctypes.c_double), ("half_width", ctypes.c_double),
                ("y_top", ctypes.c_double), ("cloak", ctypes.c_int32), ("mirror", ctypes.c_int32),
                ("sky_K", ctypes.c_double), ("fresnel", ctypes.c_int32), ("backdrop", ctypes.c_int32),
                ("backdrop_y", ctypes.c_double), ("backdrop_period", ctypes.c_double)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("target", ctypes.c_double * 3), ("fov_y_deg", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("spp", ctypes.c_int32),
                ("jitter", ctypes.c_int32), ("seed", ctypes.c_uint64), ("scene_index", ctypes.c_int64),
                ("up", ctypes.c_double * 3), ("fov_x_deg", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("integ", ctypes.c_int32), ("h", ctypes.c_double),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double), ("h_max", ctypes.c_double),
                ("h0", ctypes.c_double), ("h_min", ctypes.c_double), ("w_fallback", ctypes.c_double),
                ("max_events", ctypes.c_int32), ("fp64_stay", ctypes.c_int32), ("max_steps", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("rays", ctypes.c_int64), ("accepted_steps", ctypes.c_int64), ("rejected_steps", ctypes.c_int64),
                ("events", ctypes.c_int64), ("fallbacks", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("fp64_steps", ctypes.c_int64), ("rounds", ctypes.c_int64), ("tail_rays", ctypes.c_int64), ("hot_steps", ctypes.c_int64),
                ("hot_ms", ctypes.c_double), ("event_ms", ctypes.c_double), ("tail_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("first_pass_steps", ctypes.c_int64)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is ctypes.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class Tune(ctypes.Structure):
    _fields_ = [("slow_pxy", ctypes.c_double), ("slow_wave_div", ctypes.c_int32), ("refill", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32), ("plan_lanes", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class AutotuneOpts(ctypes.Structure):
    _fields_ = [("dir_scale", ctypes.c_int32), ("cc_scale", ctypes.c_int32), ("dir_tol", ctypes.c_double),
                ("cc_tol", ctypes.c_double), ("max_changed", ctypes.c_double), ("ref_rtol", ctypes.c_double),
                ("reps", ctypes.c_int32), ("tune_sched", ctypes.c_int32)]


AUTOTUNE_MAX_CAND = 48


class AutotuneCand(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("h_max", ctypes.c_double), ("w_fallback", ctypes.c_double),
                ("ms", ctypes.c_double), ("steps", ctypes.c_int64),
                ("dir_p99", ctypes.c_double), ("dir_max", ctypes.c_double), ("changed", ctypes.c_double),
                ("cc_err", ctypes.c_double), ("pass_", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class AutotuneReport(ctypes.Structure):
    _fields_ = [("n_cand", ctypes.c_int32), ("chosen", ctypes.c_int32), ("cand", AutotuneCand * AUTOTUNE_MAX_CAND),
                ("tune", Tune), ("tune_ms", ctypes.c_double), ("base_tune_ms", ctypes.c_double),
                ("cal_rays", ctypes.c_int64), ("ill_rays", ctypes.c_int64)]

    def as_dict(self):
        cands = []
        for i in range(self.n_cand):
            c = self.cand[i]
            cands.append(dict(rtol=c.rtol, h_max=c.h_max, w_fallback=c.w_fallback, ms=c.ms, steps=int(c.steps), dir_p99=c.dir_p99, dir_max=c.dir_max,
                              changed=c.changed, cc_err=c.cc_err, passed=bool(c.pass_)))
        return dict(candidates=cands, chosen=int(self.chosen), tune=self.tune.as_dict(), tune_ms=self.tune_ms,
                    base_tune_ms=self.base_tune_ms, cal_rays=int(self.cal_rays), ill_rays=int(self.ill_rays))


# every symbol the header declares
EXPORTS = ["gc_create", "gc_destroy", "gc_last_error", "gc_default_opts", "gc_trace_rays", "gc_render",
           "gc_render_batch", "gc_render_grad", "gc_cross_correlate", "gc_default_tune", "gc_set_tune",
           "gc_get_tune", "gc_default_autotune_opts", "gc_autotune", "gc_batch_plan_create", "gc_batch_plan_launch",
           "gc_batch_plan_results", "gc_batch_plan_destroy", "gc_cross_correlate_map",
           "gc_cross_correlate_noalloc"]

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1012_5107_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.gc_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    L.gc_create.restype = ctypes.c_int
    L.gc_destroy.argtypes = [vp]
    L.gc_destroy.restype = None
    L.gc_last_error.argtypes = []
    L.gc_last_error.restype = ctypes.c_char_p
    L.gc_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.gc_default_opts.restype = None
    L.gc_trace_rays.argtypes = [vp, ctypes.POINTER(Scene), ctypes.POINTER(Opts), i64, vp, vp, vp, vp, vp, vp, vp,
                                vp]
    L.gc_trace_rays.restype = ctypes.c_int
    L.gc_render.argtypes = [vp, ctypes.POINTER(Scene), ctypes.POINTER(Camera), ctypes.POINTER(Opts), vp,
                            ctypes.POINTER(Stats), vp]
    L.gc_render.restype = ctypes.c_int
    L.gc_render_batch.argtypes = [vp, i32, ctypes.POINTER(Scene), ctypes.POINTER(Camera), ctypes.POINTER(Opts),
                                  ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(Stats), vp]
    L.gc_render_batch.restype = ctypes.c_int
    dptr = ctypes.POINTER(ctypes.c_double)
    L.gc_render_grad.argtypes = [vp, ctypes.POINTER(Scene), ctypes.POINTER(Camera), ctypes.POINTER(Opts), vp, i32,
                                 i32, vp, vp, dptr, dptr, dptr, ctypes.POINTER(Stats), vp]
    L.gc_render_grad.restype = ctypes.c_int
    L.gc_cross_correlate.argtypes = [vp, vp, vp, i64, i32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), vp]
    L.gc_cross_correlate.restype = ctypes.c_int
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.gc_cross_correlate_map.argtypes = [vp, vp, vp, i32, i32, i64, i32, i32, i32, vp, ctypes.POINTER(ctypes.c_double),
                                         i32p, i32p, vp]
    L.gc_cross_correlate_map.restype = ctypes.c_int
    L.gc_cross_correlate_noalloc.argtypes = [vp, vp, vp, i64, i32, vp, vp]
    L.gc_cross_correlate_noalloc.restype = ctypes.c_int
    L.gc_default_tune.argtypes = [ctypes.POINTER(Tune)]
    L.gc_default_tune.restype = None
    L.gc_set_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    L.gc_set_tune.restype = ctypes.c_int
    L.gc_get_tune.argtypes = [vp, ctypes.POINTER(Tune)]
    L.gc_get_tune.restype = ctypes.c_int
    L.gc_default_autotune_opts.argtypes = [ctypes.POINTER(AutotuneOpts)]
    L.gc_default_autotune_opts.restype = None
    L.gc_autotune.argtypes = [vp, i32, ctypes.POINTER(Scene), ctypes.POINTER(Camera), ctypes.POINTER(Opts),
                              ctypes.POINTER(AutotuneOpts), ctypes.POINTER(Opts), ctypes.POINTER(AutotuneReport), vp]
    L.gc_autotune.restype = ctypes.c_int
    L.gc_batch_plan_create.argtypes = [vp, i32, ctypes.POINTER(Scene), ctypes.POINTER(Camera), ctypes.POINTER(Opts),
                                       ctypes.POINTER(vp), ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    L.gc_batch_plan_create.restype = ctypes.c_int
    L.gc_batch_plan_launch.argtypes = [vp, vp]
    L.gc_batch_plan_launch.restype = ctypes.c_int
    L.gc_batch_plan_results.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(Stats), vp]
    L.gc_batch_plan_results.restype = ctypes.c_int
    L.gc_batch_plan_destroy.argtypes = [vp]
    L.gc_batch_plan_destroy.restype = None
    _lib = L
    return L


def _check(st):
    if st != GC_OK:
        raise GcError(st, load().gc_last_error().decode())


# --- struct marshalling ------------------------------------------------------

def make_scene(sc):
    return Scene(sc["Lambda"], sc["A"], sc["half_width"], sc["y_top"], int(sc["cloak"]), int(sc["mirror"]),
                 sc["sky_K"], int(sc.get("fresnel", 0)), int(sc.get("backdrop", 0)), float(sc.get("backdrop_y", 0.0)),
                 float(sc.get("backdrop_period", 1.0)))


def make_camera(c):
    cam = Camera()
    cam.eye[:] = list(c["eye"])
    cam.target[:] = list(c["target"])
    cam.fov_y_deg = c["fov_y_deg"]
    cam.width, cam.height, cam.spp = c["width"], c["height"], c["spp"]
    cam.jitter = int(c["jitter"])
    cam.seed = c["seed"]
    cam.scene_index = c.get("scene_index", 0)
    cam.up[:] = list(c.get("up", (0.0, 0.0, 0.0)))
    cam.fov_x_deg = c.get("fov_x_deg", 0.0)
    return cam


def make_opts(o, prec="f64"):
    p = Opts()
    load().gc_default_opts(ctypes.byref(p))
    p.prec = {"f64": GC_F64, "f32": GC_F32}[prec]
    p.integ = {"rk4": GC_RK4, "dopri5": GC_DOPRI5}[o["integrator"]]
    p.h, p.rtol, p.atol = o["h"], o["rtol"], o["atol"]
    p.h_max, p.h0, p.h_min = o["h_max"], o["h0"], o["h_min"]
    p.w_fallback = o.get("w_fallback", 1e-2)
    p.max_events = o["max_events"]
    p.fp64_stay = o.get("fp64_stay", 0)
    p.max_steps = o["max_steps"]
    return p


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Owns one library context on a device."""

    def __init__(self, device=0):
        L = load()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = ctypes.c_void_p()
        _check(L.gc_create(ctypes.byref(h), self.device.index or 0))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().gc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ------------------------------------------------------------
    def trace_rays(self, scene, opts, org, dirs, prec="f64", stream=None):
        """Trace rays from device tensors org, dirs (n x 3 float64).  Returns
        (exit_org, exit_dir, status, steps, events) device tensors."""
        org = org.to(self.device, torch.float64).contiguous()
        dirs = dirs.to(self.device, torch.float64).contiguous()
        n = org.shape[0]
        oo = torch.empty_like(org)
        od = torch.empty_like(dirs)
        st = torch.empty(n, dtype=torch.int32, device=self.device)
        steps = torch.empty(n, dtype=torch.int64, device=self.device)
        ev = torch.empty(n, dtype=torch.int32, device=self.device)
        sc, op = make_scene(scene), make_opts(opts, prec)
        _check(load().gc_trace_rays(self._h, ctypes.byref(sc), ctypes.byref(op), n, org.data_ptr(),
                                    dirs.data_ptr(), oo.data_ptr(), od.data_ptr(), st.data_ptr(), steps.data_ptr(),
                                    ev.data_ptr(), _stream_handle(stream)))
        return oo, od, st, steps, ev

    def tune(self, **kw):
        """Read the context's scheduling of the FP32 pipeline (gc_tune as a
        dict); keyword arguments set those fields first."""
        L = load()
        t = Tune()
        _check(L.gc_get_tune(self._h, ctypes.byref(t)))
        if kw:
            for k, v in kw.items():
                if k not in t.as_dict():
                    raise KeyError(k)
                setattr(t, k, v)
            _check(L.gc_set_tune(self._h, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, scenes, cameras, opts, stream=None, **at_kw):
        """Autotune the FP32 pipeline for a workload (one scene/camera dict or
        lists of them): returns (tuned opts dict, report dict).  The chosen
        scheduling is installed in this context.  Keyword arguments set
        gc_autotune_opts fields (dir_scale, cc_scale, dir_tol, cc_tol,
        max_changed, ref_rtol, reps, tune_sched)."""
        L = load()
        if isinstance(scenes, dict):
            scenes, cameras = [scenes], [cameras]
        n = len(scenes)
        sc_arr = (Scene * n)(*[make_scene(s) for s in scenes])
        cam_arr = (Camera * n)(*[make_camera(c) for c in cameras])
        op = make_opts(opts, "f32")
        at = AutotuneOpts()
        L.gc_default_autotune_opts(ctypes.byref(at))
        for k, v in at_kw.items():
            if k not in dict(AutotuneOpts._fields_):
                raise KeyError(k)
            setattr(at, k, v)
        out = Opts()
        rep = AutotuneReport()
        _check(L.gc_autotune(self._h, n, sc_arr, cam_arr, ctypes.byref(op), ctypes.byref(at), ctypes.byref(out),
                             ctypes.byref(rep), _stream_handle(stream)))
        tuned = dict(opts, h_max=out.h_max, rtol=out.rtol, atol=out.atol, w_fallback=out.w_fallback)
        return tuned, rep.as_dict()

    def render(self, scene, camera, opts, prec="f64", out=None, stats=True, stream=None):
        """Render an H x W x 3 float32 image on the device.  Returns
        (image, stats dict or None)."""
        H, W = camera["height"], camera["width"]
        img = out if out is not None else torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
        sc, cam, op = make_scene(scene), make_camera(camera), make_opts(opts, prec)
        st = Stats()
        _check(load().gc_render(self._h, ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(op), img.data_ptr(),
                                ctypes.byref(st) if stats else None, _stream_handle(stream)))
        return img, (st.as_dict() if stats else None)

    def render_batch(self, scenes, cameras, opts, refs=None, outs=None, stream=None):
        """Render several scenes in one FP32 pipeline launch.  Returns (list of
        H x W x 3 images, list of C0 or None, stats dict)."""
        n = len(scenes)
        imgs = outs if outs is not None else [
            torch.empty((c["height"], c["width"], 3), dtype=torch.float32, device=self.device) for c in cameras]
        sc = (Scene * n)(*[make_scene(x) for x in scenes])
        cam = (Camera * n)(*[make_camera(x) for x in cameras])
        op = make_opts(opts, "f32")
        ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in imgs])
        rp = None
        c0 = None
        if refs is not None:
            refs = [r.to(self.device, torch.float32).contiguous() for r in refs]
            rp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in refs])
            c0 = (ctypes.c_double * n)()
        st = Stats()
        _check(load().gc_render_batch(self._h, n, sc, cam, ctypes.byref(op), ptrs, rp, c0, ctypes.byref(st),
                                      _stream_handle(stream)))
        return imgs, (list(c0) if c0 is not None else None), st.as_dict()

    def batch_plan(self, scenes, cameras, opts, outs, refs=None, render_refs=True):
        """Capture a batched FP32 render (and, with refs, the flat-mirror
        references and C0 per scene) as one HIP graph: see BatchPlan."""
        return BatchPlan(self, scenes, cameras, opts, outs, refs, render_refs)

    def render_grad(self, scene, camera, opts, ref, prec="f64", loss="ncc", checkpoint_every=64, out=None,
                    sample_dm=False, stream=None):
        """Loss 1 - NCC (loss="ncc") or 1 - C0 of eq. (15) (loss="c0")
        against the device reference image `ref` (H x W x 3) and its
        derivatives with respect to A and half_width (discrete adjoint of the
        RK4 tracer).  Returns dict(loss, dA, dhw, image, sample_dm (n x 2
        float64 tensor of dm/dA, dm/dhw per sample, or None), stats)."""
        H, W, spp = camera["height"], camera["width"], camera["spp"]
        ref = ref.to(self.device, torch.float32).contiguous()
        img = out if out is not None else torch.empty((H, W, 3), dtype=torch.float32, device=self.device)
        sg = torch.empty((H * W * spp, 2), dtype=torch.float64, device=self.device) if sample_dm else None
        sc, cam, op = make_scene(scene), make_camera(camera), make_opts(opts, prec)
        kind = {"c0": GC_LOSS_C0, "ncc": GC_LOSS_NCC}[loss]
        lv, dA, dhw = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = Stats()
        _check(load().gc_render_grad(self._h, ctypes.byref(sc), ctypes.byref(cam), ctypes.byref(op), ref.data_ptr(),
                                     kind, int(checkpoint_every), img.data_ptr(),
                                     sg.data_ptr() if sg is not None else None, ctypes.byref(lv), ctypes.byref(dA),
                                     ctypes.byref(dhw), ctypes.byref(st), _stream_handle(stream)))
        return dict(loss=lv.value, dA=dA.value, dhw=dhw.value, image=img, sample_dm=sg, stats=st.as_dict())

    def cross_correlate(self, img, ref, stream=None):
        """eq. (15) at zero shift and the Pearson form, from device images."""
        img = img.to(self.device, torch.float32).contiguous()
        ref = ref.to(self.device, torch.float32).contiguous()
        nch = img.shape[-1] if img.dim() == 3 else 1
        npix = img.numel() // nch
        c0, ncc = ctypes.c_double(), ctypes.c_double()
        _check(load().gc_cross_correlate(self._h, img.data_ptr(), ref.data_ptr(), npix, nch, ctypes.byref(c0),
                                         ctypes.byref(ncc), _stream_handle(stream)))
        return c0.value, ncc.value

    def cross_correlate_noalloc(self, img, ref, out, stream=None):
        """gc_cross_correlate_noalloc: the zero-shift correlation into the
        device tensor out (12 float64: C0, ncc, sum f'^2, sum g'^2, 4 means
        of f, 4 of g), asynchronously, with no allocation in the library.
        img and ref must be contiguous float32 device tensors."""
        nch = img.shape[-1] if img.dim() == 3 else 1
        npix = img.numel() // nch
        _check(load().gc_cross_correlate_noalloc(self._h, img.data_ptr(), ref.data_ptr(), npix, nch, out.data_ptr(),
                                                 _stream_handle(stream)))
        return out

    def cross_correlate_map(self, img, ref, rx, ry, cols=None, stream=None):
        """eq. (15) at every shift |dx| <= rx, |dy| <= ry of the device image
        img (g, H x W x C float32) against ref (f).  cols = (c0, c1) takes the
        column window [c0, c1) of both (passed with the row pitch, not
        copied).  Returns (map (2 ry + 1) x (2 rx + 1) float64 device tensor,
        map[dy + ry, dx + rx] = C(dx, dy), peak value, peak dx, peak dy)."""
        img = img.to(self.device, torch.float32).contiguous()
        ref = ref.to(self.device, torch.float32).contiguous()
        if img.dim() == 2:
            img, ref = img[:, :, None], ref[:, :, None]
        H, Wfull, nch = img.shape
        c0, c1 = (0, Wfull) if cols is None else cols
        m = torch.empty((2 * ry + 1, 2 * rx + 1), dtype=torch.float64, device=self.device)
        pk, dx, dy = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int32()
        off = c0 * nch * 4
        _check(load().gc_cross_correlate_map(self._h, img.data_ptr() + off, ref.data_ptr() + off, H, c1 - c0, Wfull,
                                             nch, int(rx), int(ry), m.data_ptr(), ctypes.byref(pk), ctypes.byref(dx),
                                             ctypes.byref(dy), _stream_handle(stream)))
        return m, pk.value, dx.value, dy.value


_default = {}


class BatchPlan:
    """A batched FP32 render captured as one HIP graph (gc_batch_plan): the
    images (and flat-mirror references, when refs are given with
    render_refs) are device tensors the plan writes on every launch."""

    def __init__(self, ctx, scenes, cameras, opts, outs, refs=None, render_refs=True):
        L = load()
        n = len(scenes)
        self.n = n
        self.outs, self.refs = list(outs), (list(refs) if refs is not None else None)
        sc_arr = (Scene * n)(*[make_scene(s) for s in scenes])
        cam_arr = (Camera * n)(*[make_camera(c) for c in cameras])
        op = make_opts(opts, "f32")
        rgb = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.outs])
        ref = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.refs]) if self.refs is not None else None
        h = ctypes.c_void_p()
        _check(L.gc_batch_plan_create(ctx._h, n, sc_arr, cam_arr, ctypes.byref(op), rgb, ref,
                                      int(bool(render_refs and refs is not None)), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(load().gc_batch_plan_launch(self._h, _stream_handle(stream)))

    def results(self, stream=None):
        """(C0 list or None, stats dict); synchronises the stream."""
        c0 = (ctypes.c_double * self.n)()
        st = Stats()
        _check(load().gc_batch_plan_results(self._h, c0 if self.refs is not None else None, ctypes.byref(st),
                                            _stream_handle(stream)))
        return (list(c0) if self.refs is not None else None), st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load().gc_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_tune():
    """gc_tune defaults as a dict."""
    t = Tune()
    load().gc_default_tune(ctypes.byref(t))
    return t.as_dict()


def context(device=0):
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def render(scene, camera, opts, prec="f64", device=0):
    return context(device).render(scene, camera, opts, prec)


def trace_rays(scene, opts, org, dirs, prec="f64", device=0):
    return context(device).trace_rays(scene, opts, org, dirs, prec)


def render_batch(scenes, cameras, opts, refs=None, device=0):
    return context(device).render_batch(scenes, cameras, opts, refs)


def cross_correlate(img, ref, device=0):
    return context(device).cross_correlate(img, ref)


def cross_correlate_map(img, ref, rx, ry, cols=None, device=0):
    return context(device).cross_correlate_map(img, ref, rx, ry, cols)


def render_grad(scene, camera, opts, ref, prec="f64", loss="ncc", checkpoint_every=64, device=0):
    return context(device).render_grad(scene, camera, opts, ref, prec, loss, checkpoint_every)


class CloakLoss(torch.autograd.Function):
    """L(A, half_width) = 1 - NCC (or 1 - C0 of eq. (15)) between the image
    of the cloak and a reference image, as a differentiable function of a
    float64 tensor params = [A, half_width].  The forward call runs the
    library's adjoint once; backward scales its two derivatives by the
    incoming gradient."""

    @staticmethod
    def forward(fctx, params, scene, camera, opts, ref, prec="f64", loss="ncc", checkpoint_every=64, device=0):
        p = params.detach().to("cpu", torch.float64)
        sc = dict(scene, A=float(p[0]), half_width=float(p[1]))
        r = context(device).render_grad(sc, camera, opts, ref, prec, loss, checkpoint_every)
        fctx.save_for_backward(torch.tensor([r["dA"], r["dhw"]], dtype=torch.float64))
        fctx.params_device = params.device
        return torch.tensor(r["loss"], dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        grad = (grad_out.detach().to("cpu", torch.float64) * g).to(fctx.params_device)
        return grad, None, None, None, None, None, None, None, None


def cloak_loss(params, scene, camera, opts, ref, prec="f64", loss="ncc", checkpoint_every=64, device=0):
    """Differentiable cloaking-quality loss (see CloakLoss)."""
    return CloakLoss.apply(params, scene, camera, opts, ref, prec, loss, checkpoint_every, device)
