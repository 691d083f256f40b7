"""CPU: the benchmark's command-line contract where no GPU is needed.

`bench.py` measures one GPU: asked for more (by flag or by a launcher's WORLD_SIZE) it exits with
status 2 and says why, before it imports torch.  Without a GPU it stops with an error instead of
timing anything on the host, and so does the smoke check of the package entry module.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT, env=e)


@pytest.mark.parametrize("args,env", [(("--gpus", "2"), None), (("--gpus", "8", "--steps", "1"), None),
                                      ((), {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = _bench(*args, env=env)
    assert r.returncode == 2, (r.returncode, r.stderr[-500:])
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no result line


def test_no_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _bench("--steps", "1", "--warmup", "0", "--no-cpu-baseline")
    assert r.returncode != 0
    assert "needs a GPU" in r.stderr
    assert r.stdout == ""

    r = subprocess.run([sys.executable, "-c", "import __graft_entry__ as g; g.smoke()"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "needs a GPU" in r.stderr
    assert "smoke ok" not in r.stdout
