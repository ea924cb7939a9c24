"""bench.py's command line on the CPU: it measures one GPU only and refuses
more (argument check before any GPU work)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=env, timeout=120, cwd=ROOT)


@pytest.mark.parametrize("args", [["--gpus", "2"], ["--gpus", "8", "--steps", "3"], ["--gpus", "2", "--only",
                                                                                         "sweep-f64"]])
def test_more_than_one_gpu_is_refused(args):
    r = _run(args)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_launcher_world_size_is_refused():
    r = _run([], {"WORLD_SIZE": "2", "RANK": "0", "LOCAL_RANK": "0"})
    assert r.returncode == 2 and "one GPU only" in r.stderr
