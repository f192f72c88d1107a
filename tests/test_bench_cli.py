"""bench.py command line on the CPU: more than one GPU is refused with a message and no
JSON line, before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT, env=env)


def test_more_than_one_gpu_is_refused():
    p = _run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert p.returncode == 2
    assert "one MI355X" in p.stderr
    assert p.stdout.strip() == ""


def test_launcher_world_size_is_refused():
    env = dict(os.environ, WORLD_SIZE="2", RANK="0", LOCAL_RANK="0")
    p = _run("--gpus", "1", env=env)
    assert p.returncode == 2
    assert p.stdout.strip() == ""


def test_help():
    p = _run("--help")
    assert p.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup"):
        assert opt in p.stdout
