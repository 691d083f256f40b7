"""The library's real host code under sanitizers, on the CPU.

Every product source (api.cpp, serve.cpp and the host halves of the .hip
files, compiled with --offload-host-only) is linked against a mock HIP
runtime (tests/host_sanitize/mock_hip_runtime.cpp) in place of libamdhip64:
device memory is host memory, copies and launches run asynchronously on a
mock device thread in stream order, stream capture and graphs follow the
runtime's rules (forks must join, no waits across captures, no device-wide
synchronisation during a capture), and the kernels do nothing.  The driver
(tests/host_sanitize/host_driver.cpp) replays the call sequences of the
served-mix benchmark's pass without a server (64 meshes, BF16 predict,
CNN-SNS and plain locate), of the serving tests, of concurrent predicts on
one mesh, and of the 3D calls, once under AddressSanitizer + UBSan and once
under ThreadSanitizer.  Any sanitizer report, mock-runtime failure, leaked
device allocation or handle fails the test.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_2412_18379_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
PRODUCT = ["mesh.hip", "sns_walk.hip", "cnn.hip", "cnn_bf16.hip", "cnn_fp8.hip", "mesh3d.hip", "cnn3d.hip", "classifier.hip",
           "api.cpp", "serve.cpp"]
SANITIZERS = {"asan": ["address", "undefined"], "tsan": ["thread"]}


def _build(kind, outdir):
    san = []
    for s in SANITIZERS[kind]:
        san += ["-Xarch_host", f"-fsanitize={s}"]
    common = ["--offload-arch=gfx950", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
              "-I", os.path.join(ROOT, "include"), *san, "-x", "hip", "-c"]
    srcs = [os.path.join(CSRC, f) for f in PRODUCT] + [os.path.join(HERE, "mock_hip_runtime.cpp"),
                                                       os.path.join(HERE, "host_driver.cpp")]

    def compile_one(src):
        obj = os.path.join(outdir, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC, *common, src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, f"{src}:\n{r.stderr[-4000:]}"
        return obj

    with ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, srcs))
    # the device images of a host-only build are not linked in: stand-ins for their symbols
    nm = subprocess.run(["nm", "-u", *objs], capture_output=True, text=True, check=True).stdout
    fat = sorted({line.split()[-1] for line in nm.splitlines() if "__hip_fatbin" in line})
    stub = os.path.join(outdir, "fatbin_stubs.c")
    with open(stub, "w") as f:
        for name in fat:
            f.write(f"const char {name}[16] = {{0}};\n")
    exe = os.path.join(outdir, "host_driver")
    flags = ["-fsanitize=" + ",".join(SANITIZERS[kind])]
    r = subprocess.run([CLANGXX, *flags, *objs, "-x", "c", stub, "-o", exe, "-lpthread", "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.fixture(scope="module", params=sorted(SANITIZERS))
def driver(request, tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("hipcc / clang++ not available")
    return request.param, _build(request.param, str(tmp_path_factory.mktemp(request.param)))


SCENARIOS = [
    ("c5ref", "64", "16", "5"),
    ("serve", "1"),
    ("serve", "2"),
    ("predict_mt", "150"),
    ("mesh3d",),
    ("noalloc",),
    ("classify",),
]


@pytest.mark.parametrize("scenario", SCENARIOS, ids=lambda s: "-".join(s))
def test_host_code_under_sanitizers(driver, scenario):
    kind, exe = driver
    env = dict(os.environ, CNNSNS_ENABLE_SERVING="1",
               ASAN_OPTIONS="detect_leaks=1:detect_stack_use_after_return=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = subprocess.run([exe, *scenario], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert " 0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "WARNING: ThreadSanitizer" not in r.stderr
