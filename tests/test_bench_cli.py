"""bench.py's command line on the CPU: it runs on one GPU only and says so
for more, before touching a device; its help lists every mode."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          cwd=ROOT, capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""          # no JSON line


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="4")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], cwd=ROOT,
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_help_lists_the_modes_and_workloads():
    r = run("--help")
    assert r.returncode == 0
    for word in ("batch", "serve", "reduce", "tune", "srad", "batch-64x1080p",
                 "uneven-512", "single-8192-k7", "band-1024x8192-k7"):
        assert word in r.stdout, word
