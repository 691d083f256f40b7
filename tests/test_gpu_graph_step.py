"""One CNN-SNS step (Alg. 2: cnnsns_predict_noalloc, then cnnsns_locate from the predicted
displacement) captured in a HIP graph through torch's graph API, and replayed: every replay equals
the eager step bit for bit.  Neither call allocates or clears device memory, so the step can be
captured; the no-allocation pass keeps its workspace in the library's per-device array (set up by
an eager call before the capture).  Eager work (a fill of the outputs) runs between the replays.
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,precision", [("c1", "f32"), ("c1", "bf16"), ("c2", "bf16"), ("c2", "fp8")])
def test_captured_step_replays_equal_eager(C, wl, name, precision):
    print(f"[graph step] {name} {precision}", flush=True)
    w = wl.build(name)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    W = C.Weights(*wl.he_weights(200))
    vel, xp, origin = _dev(w.vel), _dev(w.xp), _dev(w.origins)
    n, G = xp.shape[0], mesh.G
    # eager step (also sets up the per-device workspace before any capture)
    disp_e = torch.empty((2, G, G), dtype=torch.float32, device="cuda")
    C.predict_noalloc(mesh, vel, W, disp_e, precision=precision)
    host_e, it_e, st_e = C.locate(mesh, xp, origin=origin, disp=disp_e)
    torch.cuda.synchronize()
    # static buffers of the captured step
    disp = torch.empty_like(disp_e)
    host = torch.empty_like(host_e)
    iters = torch.empty_like(it_e)
    status = torch.empty_like(st_e)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # a warm-up on the capture's stream, as torch recommends
        C.predict_noalloc(mesh, vel, W, disp, precision=precision)
        C.locate(mesh, xp, origin=origin, disp=disp, host=host, iters=iters, status=status)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        C.predict_noalloc(mesh, vel, W, disp, precision=precision)
        C.locate(mesh, xp, origin=origin, disp=disp, host=host, iters=iters, status=status)
    for rep in range(3):
        disp.fill_(float("nan"))
        host.fill_(-7)
        iters.fill_(-7)
        status.fill_(255)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(disp, disp_e), rep
        assert torch.equal(host, host_e) and torch.equal(iters, it_e) and torch.equal(status, st_e), rep
    assert (st_e == C.FOUND).all()
    del g
    mesh.close()
