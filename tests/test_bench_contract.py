"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message (the library has no multi-GPU path), also when a
launcher sets WORLD_SIZE."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=e,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_launcher_world_size_is_refused():
    r = _run(["--gpus", "1"], env={"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
