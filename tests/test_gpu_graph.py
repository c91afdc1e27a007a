"""The batched FP32 render captured as HIP graphs (gc_batch_plan): every
replay must reproduce the eager batch render bit for bit (images, flat
references, C0 and counters), also with other work and synchronisations
between the replays."""
import pytest

torch = pytest.importorskip("torch")

from paper_1012_5107_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1012_5107_amd import binding
    return binding


def _workload():
    scenes = [W.scene(A=0.1, half_width=3.0), W.scene(A=0.05, half_width=2.2), W.scene(A=0.13, half_width=5.0)]
    cams = [W.camera(64, 48, spp=2, jitter=True, seed=1), W.camera(40, 40, spp=1, jitter=False, seed=2),
            W.camera(72, 56, spp=2, jitter=True, seed=3, eye=W.orbit_eye(20.0, 35.0, 7.0))]
    return scenes, cams, W.opts("dopri5", rtol=1e-6)


def test_plan_replays_match_eager_batch(B):
    scenes, cams, op = _workload()
    ctx = B.Context(0)
    try:
        refs_e = [ctx.render(W.reference_scene(s), c, op, prec="f32")[0] for s, c in zip(scenes, cams)]
        imgs_e, c0_e, st_e = ctx.render_batch(scenes, cams, op, refs=refs_e)
        outs = [torch.full_like(i, float("nan")) for i in imgs_e]
        refs = [torch.full_like(r, float("nan")) for r in refs_e]
        plan = ctx.batch_plan(scenes, cams, op, outs, refs=refs, render_refs=True)
        try:
            for rep in range(3):
                for t in outs + refs:
                    t.fill_(float("nan"))
                torch.cuda.synchronize()
                plan.launch()
                c0, st = plan.results()
                for a, b in zip(outs, imgs_e):
                    assert torch.equal(a, b), rep
                for a, b in zip(refs, refs_e):
                    assert torch.equal(a, b), rep
                assert c0 == c0_e, rep
                for k in ("rays", "accepted_steps", "rejected_steps", "events", "failed", "fallbacks"):
                    assert st[k] == st_e[k], (rep, k)
                assert st["rounds"] == st_e["rounds"] and st["total_ms"] > 0
                # unrelated eager work between replays
                ctx.render(scenes[1], cams[1], op, prec="f32")
                torch.cuda.synchronize()
        finally:
            plan.close()
        # without references: images only
        plan = ctx.batch_plan(scenes[:2], cams[:2], op, outs[:2])
        try:
            plan.launch()
            c0, st = plan.results()
            assert c0 is None
            assert torch.equal(outs[0], imgs_e[0]) and torch.equal(outs[1], imgs_e[1])
        finally:
            plan.close()
        with pytest.raises(B.GcError):   # flat-mirror scenes are not batched
            ctx.batch_plan([W.reference_scene(scenes[0])], cams[:1], op, outs[:1])
    finally:
        ctx.close()


@pytest.mark.parametrize("tune", [dict(slow_pxy=0.0, slow_wave_div=0), dict(slow_pxy=0.3, slow_wave_div=4)])
def test_plan_front_of_queue_replays_match_eager(B, tune):
    """The plan's eager run records the longest first visits of the box and
    its graph claims those rays first (the front of the first round's
    queue); every replay still reproduces the eager render bit for bit."""
    sc, cam, _, op = W.plain_vs_fp32_512()
    cam = dict(cam, width=192, height=192, spp=2)
    ctx = B.Context(0)
    try:
        ctx.tune(**tune)
        ref_e = ctx.render(W.reference_scene(sc), cam, op, prec="f32")[0]
        imgs_e, c0_e, st_e = ctx.render_batch([sc], [cam], op, refs=[ref_e])
        out = torch.full_like(imgs_e[0], float("nan"))
        ref = torch.full_like(ref_e, float("nan"))
        plan = ctx.batch_plan([sc], [cam], op, [out], refs=[ref], render_refs=True)
        try:
            for rep in range(3):
                out.fill_(float("nan"))
                ref.fill_(float("nan"))
                torch.cuda.synchronize()
                plan.launch()
                c0, st = plan.results()
                assert st["tail_rays"] > 0, "no long first visit was put at the front"
                assert torch.equal(out, imgs_e[0]), rep
                assert torch.equal(ref, ref_e), rep
                assert c0 == c0_e, rep
                for k in ("rays", "accepted_steps", "rejected_steps", "events", "failed", "fallbacks"):
                    assert st[k] == st_e[k], (rep, k)
                ctx.render(sc, dict(cam, width=32, height=32, spp=1), op, prec="f32")
                torch.cuda.synchronize()
        finally:
            plan.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("lanes", [2, 3])
def test_plan_lanes_replays_match_eager_batch(B, lanes):
    """A plan split into concurrent sub-pipelines (gc_tune.plan_lanes): each
    group of scenes runs on a stream of its own; every replay reproduces the
    eager batch bit for bit, and the counters add up to the eager run's."""
    scenes, cams, op = _workload()
    ctx = B.Context(0)
    try:
        refs_e = [ctx.render(W.reference_scene(s), c, op, prec="f32")[0] for s, c in zip(scenes, cams)]
        imgs_e, c0_e, st_e = ctx.render_batch(scenes, cams, op, refs=refs_e)
        ctx.tune(plan_lanes=lanes)
        outs = [torch.full_like(i, float("nan")) for i in imgs_e]
        refs = [torch.full_like(r, float("nan")) for r in refs_e]
        plan = ctx.batch_plan(scenes, cams, op, outs, refs=refs, render_refs=True)
        try:
            for rep in range(3):
                for t in outs + refs:
                    t.fill_(float("nan"))
                torch.cuda.synchronize()
                plan.launch()
                c0, st = plan.results()
                for a, b in zip(outs, imgs_e):
                    assert torch.equal(a, b), rep
                for a, b in zip(refs, refs_e):
                    assert torch.equal(a, b), rep
                assert c0 == c0_e, rep
                for k in ("rays", "accepted_steps", "rejected_steps", "events", "failed", "fallbacks"):
                    assert st[k] == st_e[k], (rep, k)
                assert 0 < st["hot_ms"] <= st["total_ms"]
                ctx.render(scenes[1], cams[1], op, prec="f32")
                torch.cuda.synchronize()
        finally:
            plan.close()
        with pytest.raises(B.GcError):
            ctx.tune(plan_lanes=4)
    finally:
        ctx.close()
