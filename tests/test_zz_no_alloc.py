"""GPU test of cnnsns_predict_noalloc, the forward pass that allocates nothing
(its workspace is the library's preallocated per-GPU array).

Through the C ABI it must give what cnnsns_predict gives on the same inputs
(the same kernels: bitwise equal), on two calls in a row, the second with a
smaller overlay, in every precision; an FP32 overlay beyond the array's size
and an unknown precision are refused.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18379_amd import cnnsns
    cnnsns.lib()
    return cnnsns


def _case(C, wl, n_side, G, seed):
    w = wl.build(n_side=n_side, seed=seed, field="fourier", field_seed=seed + 7, U=1.0, k=10.0, origins="nodes", G=G)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=G)
    return mesh, torch.from_numpy(w.vel).cuda()


@pytest.mark.parametrize("precision", ["bf16", "f32", "fp8"])
def test_noalloc_equals_predict(C, wl, precision):
    ws, bs = wl.random_weights(11)
    W = C.Weights(ws, bs)
    big, vel_big = _case(C, wl, 200, 512, 41)    # FP32: exactly the array's size
    small, vel_small = _case(C, wl, 40, 97, 42)  # a smaller, ragged overlay next
    for mesh, vel in ((big, vel_big), (small, vel_small)):
        ref = C.predict(mesh, vel, W, precision)
        got = torch.full_like(ref, float("nan"))
        C.predict_noalloc(mesh, vel, W, got, precision)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), f"G={mesh.G}: differs from cnnsns_predict"
    big.close()
    small.close()


def test_noalloc_limits(C, wl):
    ws, bs = wl.random_weights(12)
    W = C.Weights(ws, bs)
    mesh, vel = _case(C, wl, 30, 1024, 43)
    disp = torch.empty((2, 1024, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(C.CnnsnsError) as e:
        C.predict_noalloc(mesh, vel, W, disp, "f32")
    assert e.value.code == C.EINVAL
    with pytest.raises(C.CnnsnsError) as e:
        C.predict_noalloc(mesh, vel, W, disp, 7)
    assert e.value.code == C.EINVAL
    for precision in ("bf16", "fp8"):  # they need only packed weights (and scales): any G
        ref = C.predict(mesh, vel, W, precision)
        C.predict_noalloc(mesh, vel, W, disp, precision)
        torch.cuda.synchronize()
        assert torch.equal(disp, ref)
    mesh.close()
