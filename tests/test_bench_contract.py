"""bench.py's command-line contract on the CPU: it measures one GPU and says
so, and exits before touching a GPU, for any other GPU count."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    if env:
        e.update(env)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                          env=e, timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run(["--gpus", "2"])
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""   # no result line


def test_distributed_launch_exits_with_a_message():
    r = _run(["--gpus", "1"], env={"WORLD_SIZE": "4"})
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = _run(["--help"])
    assert r.returncode == 0
    for w in ("single", "batch", "stress", "grad"):
        assert w in r.stdout


def test_traffic_tables_resolve_the_options_the_benchmark_uses(monkeypatch):
    """The measured HBM bytes per launch are found for the options the
    autotuner forms by products (3 x 1e-7, 1e-7 / 3), for every workload
    whose roofline reports them, while the in-box kernel's sources are the
    ones they were measured with; an unmeasured setting, or any change of
    those sources, gives None."""
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "MEASURED_SHA", bench._kernel_sha())
    # the batch's recorded options, formed as the autotuner forms them
    assert bench._measured(bench.TRAFFIC_K_WF_BOX_BATCH, (3 * (1e-7 / 3), 0.05, 0.3)) is not None
    assert bench._measured(bench.TRAFFIC_K_WF_BOX_BATCH, (1e-7, 0.02, 0.3)) is None
    assert bench._measured(bench.VALU_FLOPS_K_WF_BOX_BATCH, (1e-7, 0.05, 0.3)) is not None
    tables = (bench.TRAFFIC_K_WF_BOX, bench.TRAFFIC_K_WF_BOX_BATCH, bench.TRAFFIC_K_WF_BOX_STRESS,
              bench.VALU_FLOPS_K_WF_BOX, bench.VALU_FLOPS_K_WF_BOX_BATCH)
    for table in tables:
        for k, v in table.items():
            assert isinstance(k, tuple) and bench._measured(table, k) is not None
            assert (v[0] if isinstance(v, tuple) else v) > 0
    monkeypatch.setattr(bench, "MEASURED_SHA", "0" * 16)
    assert bench._measured(bench.TRAFFIC_K_WF_BOX_BATCH, (1e-7, 0.05, 0.3)) is None


def test_adjoint_measured_tables(monkeypatch):
    """The gradient's recorded counter and traffic figures are returned for
    its own step and checkpoint interval while the adjoint's sources are the
    ones they were measured with, and None otherwise."""
    sys.path.insert(0, ROOT)
    import bench
    src, sha = bench.ADJ_KERNEL_SOURCES, bench._kernel_sha(bench.ADJ_KERNEL_SOURCES)
    monkeypatch.setattr(bench, "ADJ_MEASURED_SHA", sha)
    for table in (bench.TRAFFIC_K_ADJ, bench.VALU_FLOPS_K_ADJ):
        assert bench._measured(table, (1e-3, 64), src, sha) is not None
        assert bench._measured(table, (1e-3, 32), src, sha) is None
        assert bench._measured(table, (1e-3, 64), src, "0" * 16) is None


def test_recorded_batch_search_is_the_timed_choice(monkeypatch):
    """The batch's recorded autotuner search is keyed on the options the
    benchmark times by default (workloads.batch_timed_opts): it passed, its
    choice is one of its candidates, and its record is committed; with other
    kernel sources it is not reported."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1012_5107_amd import workloads as W
    op = W.batch_timed_opts()
    key = (op["rtol"], op["h_max"], op["w_fallback"])
    monkeypatch.setattr(bench, "MEASURED_SHA", bench._kernel_sha())
    rec = bench._measured(bench.AUTOTUNE_BATCH, key)
    assert rec is not None and rec["passed"] is True and 0 <= rec["chosen"] < rec["candidates"]
    assert os.path.isfile(os.path.join(ROOT, rec["record"]))
    monkeypatch.setattr(bench, "MEASURED_SHA", "0" * 16)
    assert bench._measured(bench.AUTOTUNE_BATCH, key) is None
