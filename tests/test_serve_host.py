"""Host-side test of the serving loop's scheduler (serve.cpp and the C ABI in
api.cpp), built with g++ against a mock HIP runtime (tests/mock_hip) under
AddressSanitizer and UndefinedBehaviorSanitizer.

The mock turns kernel launches into host work that writes a job-specific
pattern, makes events complete a few polls after they are recorded, and counts
live streams, events and graphs.  The driver submits jobs on meshes of uneven
size, waits in and out of order, polls, lets arrivals trickle in, hits
budget-bound admission (one job at a time, then several), submits empty jobs,
and destroys the server with jobs still pending; every job's output must be its
own and nothing may leak.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOCK = os.path.join(ROOT, "tests", "mock_hip")
CSRC = os.path.join(ROOT, "paper_2412_18379_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("serve") / "serve_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", MOCK, "-I", os.path.join(ROOT, "include"),
           os.path.join(MOCK, "serve_driver.cpp"), os.path.join(MOCK, "mock_kernels.cpp"),
           os.path.join(CSRC, "serve.cpp"), os.path.join(CSRC, "api.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


# precision (0 F32, 1 BF16), budget bytes, max_inflight, meshes, jobs, seed
CASES = [
    (1, 4 << 30, 8, 64, 512, 1),   # roomy budget, eight jobs in flight
    (1, 3 << 20, 2, 64, 300, 2),   # the budget admits few jobs at once
    (0, 40 << 20, 3, 64, 300, 3),  # FP32 activations in the footprint
    (1, 2200000, 1, 20, 100, 4),   # one job at a time, the largest grids barely fit
]


@pytest.mark.parametrize("case", CASES)
def test_scheduler_under_sanitizers(driver, case):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               CNNSNS_ENABLE_SERVING="1")
    r = subprocess.run([driver, *map(str, case)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "0 failures" in r.stdout
