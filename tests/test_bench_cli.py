"""bench.py measures one GPU: asked for more (--gpus N with N > 1, or started as
one rank of several), it exits with status 2 and says why, before it touches
a device, so these run on the CPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=300)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None), (["--gpus", "8"], None),
                                      (["--gpus", "1"], {"WORLD_SIZE": "2"})])
def test_bench_refuses_more_than_one_gpu(args, env):
    r = _bench(args, env)
    assert r.returncode == 2, r.stderr[-2000:]
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line
