"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a device (this library has no multi-GPU
path), also when a launcher sets WORLD_SIZE above one."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.pop("WORLD_SIZE", None)
    if env_extra:
        env.update(env_extra)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=env, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_world_size_above_one_is_refused():
    r = _run(["--gpus", "1"], {"WORLD_SIZE": "8"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
