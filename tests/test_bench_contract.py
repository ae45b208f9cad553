"""The benchmark's command-line contract, checked without a GPU: one GPU
only (a request for more exits with a message and no JSON line), and the
arguments the driver passes are accepted."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "8", "--steps", "3", "--warmup", "1")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_world_size_above_one_exits_too():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True,
                       text=True, timeout=300, cwd=ROOT, env=env)
    assert r.returncode == 2 and r.stdout.strip() == ""


def test_help_lists_the_driver_arguments():
    r = _run("--help")
    assert r.returncode == 0
    for a in ("--gpus", "--steps", "--warmup"):
        assert a in r.stdout
