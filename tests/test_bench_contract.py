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
