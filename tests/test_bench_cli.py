"""The bench's command-line contract where it needs no GPU: it measures one
GPU and refuses any other count (or a multi-rank launch) before touching a
device, with a message and exit status 2, printing no JSON line."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    return subprocess.run([sys.executable, "bench.py", *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=120, env=env)


def test_bench_refuses_more_than_one_gpu():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2, r
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_refuses_a_multi_rank_launch():
    env = dict(os.environ, WORLD_SIZE="4")
    r = _run(["--gpus", "1"], env=env)
    assert r.returncode == 2, r
    assert "one GPU" in r.stderr
    assert r.stdout == ""
