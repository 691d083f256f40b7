"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before touching the GPU (no compute call is made here)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cnnsns.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cnnsns_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2412_18379_amd import cnnsns
    if not os.path.exists(cnnsns.LIB_PATH):
        pytest.skip("libcnnsns.so not built")
    return cnnsns.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 11
    from paper_2412_18379_amd import cnnsns
    assert set(names) == set(cnnsns.EXPORTS)
    for name in names:
        assert hasattr(L, name), name


def test_argument_errors_without_gpu(L):
    from paper_2412_18379_amd import cnnsns as C
    out = ctypes.c_void_p()
    assert L.cnnsns_build_mesh(None, 3, None, 1, 0, None, ctypes.byref(out)) == C.EINVAL
    assert b"NULL" in L.cnnsns_last_error()
    assert L.cnnsns_locate(None, 10, None, None, None, None, 0, None, None, None, None) == C.EINVAL
    assert L.cnnsns_predict(None, None, None, 0, None, None) == C.EINVAL
    assert L.cnnsns_mesh_info(None, None, None, None, None) == C.EINVAL
    assert L.cnnsns_destroy_mesh(None) == C.OK
    assert L.cnnsns_last_error() == b""
    assert L.cnnsns_submit(None, None, None, 0, None, None, None, None, None, None, None) == C.EINVAL
    assert L.cnnsns_server_destroy(None) == C.OK


def test_serving_switched_off_by_default(L):
    """cnnsns_server_create refuses to start the serving loop unless it is asked for explicitly."""
    if os.environ.get("CNNSNS_ENABLE_SERVING") == "1":
        pytest.skip("serving enabled in this environment")
    from paper_2412_18379_amd import cnnsns as C
    cnn = C._Cnn()
    for l in range(4):
        cnn.w[l] = 1
        cnn.b[l] = 1
    out = ctypes.c_void_p()
    assert L.cnnsns_server_create(1 << 20, 2, 8, C.BF16, ctypes.byref(cnn), ctypes.byref(out)) == C.EINVAL
    assert b"switched off" in L.cnnsns_last_error()
    assert not out.value


def test_binding_rejects_malformed_nets_and_host_tensors():
    """The kernels read every weight at a fixed offset, so the binding accepts only exact layer shapes
    (a wrong input-channel count or a short bias would otherwise be read past its end), and passes
    only device tensors (weights on the host would reach the kernels as host pointers)."""
    import numpy as np
    import torch
    from paper_2412_18379_amd import cnnsns as C

    def net(shapes):
        return [np.zeros(s, np.float32) for s in shapes], [np.zeros(s[0], np.float32) for s in shapes]

    ws, bs = net(C.CNN_SHAPES)
    W = C.Weights(ws, bs, device="cpu")  # shapes are checked before any device is touched
    assert W.device.type == "cpu"
    bad = list(ws)
    bad[1] = np.zeros((32, 16, 3, 3), np.float32)  # the second layer's input channels
    with pytest.raises(ValueError, match="expected"):
        C.Weights(bad, bs, device="cpu")
    with pytest.raises(ValueError, match="expected"):
        C.Weights(ws, bs[:3] + [np.zeros(1, np.float32)], device="cpu")  # a short last bias
    with pytest.raises(ValueError, match="expected"):
        C.Weights(ws[:3], bs[:3], device="cpu")
    ws3, bs3 = net(C.CNN3_SHAPES)
    C.Weights3D(ws3, bs3, device="cpu")
    bad3 = list(ws3)
    bad3[3] = np.zeros((3, 16, 3, 3, 3), np.float32)
    with pytest.raises(ValueError, match="expected"):
        C.Weights3D(bad3, bs3, device="cpu")
    wc, bc = net(C.CLS_SHAPES)
    C.ClsWeights(wc, bc, device="cpu")
    with pytest.raises(ValueError, match="expected"):
        C.ClsWeights(wc, bc[:5] + [np.zeros(80, np.float32)], device="cpu")
    with pytest.raises(ValueError, match="device tensor"):
        C._on(0, ("weights", W.w[0]))
    C._on(0, ("absent", None))
    with pytest.raises(ValueError, match="device tensor"):
        C._ptr(torch.zeros(4))


def test_missing_library_raises(tmp_path):
    """Without the built library the loader that every entry point of the binding goes through
raises, every time it is asked: there is no host fallback."""
    prog = f"""
from paper_2412_18379_amd import cnnsns as C
C.LIB_PATH = {str(tmp_path / 'libcnnsns.so')!r}
C._lib = None
for _ in range(2):
    try:
        C.lib()
    except RuntimeError as e:
        assert "is not built" in str(e), e
    else:
        raise SystemExit("no error")
print("raised")
"""
    r = subprocess.run([sys.executable, "-c", prog], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-1500:]
    assert r.stdout.strip() == "raised"
