"""GPU parity of the FP8 e4m3 forward pass (cnnsns_predict with CNNSNS_FP8E4M3) against the FP64
oracle.

* A constructed net whose every weight is a power of two and whose every activation is an integer of
  magnitude <= 16 (exactly representable in e4m3 at any power-of-two scale), with integer velocities:
  the FP8 pass must then equal the oracle exactly.  Its sparse random weights touch all nine taps and
  mix channels, so the operand layouts, the channel interleave, the scales, the biases and the last
  layer's tap sums are all pinned.
* He-initialised nets on random and smooth velocities: the error against the oracle is reported and
  held to the bar below.
* CNN-SNS from the FP8 displacement: hosts equal plain SNS (oracle) off the edges.
* cnnsns_predict_noalloc in FP8 equals cnnsns_predict bit for bit.
"""
import numpy as np
import pytest
import torch

from exact import edge_distances

pytestmark = pytest.mark.gpu

# FP8 bar: e4m3 keeps 3 mantissa bits (unit roundoff 2^-4, 32 times BF16's), so a layer's result
# moves by a few per cent of its scale; the test allows 25% of the channel maximum per element and
# 4% on average over the four layers.
FP8_MAX, FP8_MEAN = 0.25, 0.04


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18379_amd import cnnsns
    cnnsns.lib()
    return cnnsns


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _square_mesh(C, G):
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float64)
    tri = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return C.Mesh(xy, tri, overlay_side=G)


def exact_net(seed):
    """Sparse +-1 weights (layers 1-3: one or two per output channel at a random input channel and
    tap; layer 4: +-1/2 at four random entries per output), small integer biases."""
    rng = np.random.default_rng(seed)
    shapes = [(32, 2, 3, 3), (32, 32, 3, 3), (32, 32, 3, 3), (2, 32, 3, 3)]
    ws = [np.zeros(s, np.float32) for s in shapes]
    bs = [rng.integers(0, 2, 32).astype(np.float32), rng.integers(-1, 2, 32).astype(np.float32),
          rng.integers(-1, 2, 32).astype(np.float32), np.array([0.25, -1.5], np.float32)]
    for l, nz in ((0, 2), (1, 2), (2, 1)):
        for o in range(32):
            for _ in range(rng.integers(1, nz + 1)):
                ws[l][o, rng.integers(0, shapes[l][1]), rng.integers(0, 3), rng.integers(0, 3)] = rng.choice([-1, 1])
    for o in range(2):
        for _ in range(4):
            ws[3][o, rng.integers(0, 32), rng.integers(0, 3), rng.integers(0, 3)] = rng.choice([-0.5, 0.5])
    return ws, bs


def _activations(vel, ws, bs):
    """Layer-by-layer float64 activations (the constructed case's precondition only)."""
    x = torch.from_numpy(vel.astype(np.float64))[None]
    out = []
    for l in range(3):
        x = torch.relu(torch.nn.functional.conv2d(x, torch.from_numpy(ws[l].astype(np.float64)),
                                                  torch.from_numpy(bs[l].astype(np.float64)), padding=1))
        out.append(x[0].numpy())
    return out


@pytest.mark.parametrize("G,seed", [(7, 1), (45, 2), (97, 3), (250, 4)])
def test_fp8_exact_on_representable_net(C, oracle_mod, G, seed):
    print(f"[cnn fp8 exact] G={G} seed={seed}", flush=True)
    rng = np.random.default_rng(100 + seed)
    vel = rng.integers(-3, 4, size=(2, G, G)).astype(np.float32)
    ws, bs = exact_net(seed)
    for a in _activations(vel, ws, bs):  # integers of magnitude <= 16: exact in e4m3 at any 2^k scale
        assert np.all(a == np.round(a)) and np.abs(a).max() <= 16
    mesh = _square_mesh(C, G)
    disp = C.predict(mesh, _dev(vel), C.Weights(ws, bs), "fp8").cpu().numpy()
    ref = oracle_mod.cnn_forward(vel, ws, bs)
    assert np.array_equal(disp.astype(np.float64), ref)
    mesh.close()


def _errors(got, ref):
    scale = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1).reshape(-1, *([1] * (ref.ndim - 1)))
    e = np.abs(np.asarray(got, np.float64) - ref) / scale
    return float(e.max()), float(e.mean())


@pytest.mark.parametrize("G,seed", [(1, 1), (5, 2), (37, 4), (131, 7), (601, 8)])
def test_fp8_random_net(C, oracle_mod, wl, G, seed):
    print(f"[cnn fp8] G={G} seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    vel = rng.standard_normal((2, G, G)).astype(np.float32)
    ws, bs = wl.random_weights(seed)
    mesh = _square_mesh(C, G)
    disp = C.predict(mesh, _dev(vel), C.Weights(ws, bs), "fp8").cpu().numpy()
    ref = oracle_mod.cnn_forward(vel, ws, bs)
    emax, emean = _errors(disp, ref)
    print(f"  fp8 error: max {emax:.4f} mean {emean:.5f} of the channel maximum", flush=True)
    assert emax <= FP8_MAX and emean <= FP8_MEAN, (emax, emean)
    mesh.close()


def test_fp8_smooth_field_he_net(C, oracle_mod, wl):
    G = 256
    fld = wl.FourierVortices(30, norm_G=G)
    vel = wl.overlay_velocity(fld, G)
    ws, bs = wl.he_weights(200)
    mesh = _square_mesh(C, G)
    W = C.Weights(ws, bs)
    d8 = C.predict(mesh, _dev(vel), W, "fp8").cpu().numpy()
    db = C.predict(mesh, _dev(vel), W, "bf16").cpu().numpy()
    ref = oracle_mod.cnn_forward(vel, ws, bs)
    e8, eb = _errors(d8, ref), _errors(db, ref)
    print(f"  smooth field, He net: fp8 max {e8[0]:.4f} mean {e8[1]:.5f}; bf16 max {eb[0]:.4f} mean {eb[1]:.5f}",
          flush=True)
    assert e8[0] <= FP8_MAX and e8[1] <= FP8_MEAN
    assert e8[1] > eb[1]  # the coarser format is the less accurate one
    # the no-allocation entry point runs the same kernels on its own workspace
    d8n = C.predict_noalloc(mesh, _dev(vel), W, torch.empty((2, G, G), dtype=torch.float32, device="cuda"),
                            precision="fp8").cpu().numpy()
    assert np.array_equal(d8n, d8)
    mesh.close()


def test_cnnsns_fp8_hosts_unchanged(C, oracle_mod, wl):
    """The FP8 CNN can only move the start: hosts equal plain SNS (oracle) for every point off the edges."""
    from paper_2412_18379_amd import train as T
    w = wl.build("c2")
    tr = T.load("c2")
    ws, bs = tr if tr is not None else wl.he_weights(200)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    disp = C.predict(mesh, _dev(w.vel), C.Weights(ws, bs), "fp8")
    h, it, st = C.locate(mesh, _dev(w.xp), origin=_dev(w.origins), disp=disp)
    h, it, st = h.cpu().numpy(), it.cpu().numpy(), st.cpu().numpy()
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    ph, pi, ps = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    far = edge_distances(w.xy, tc, ph, w.xp) > 1e-9
    assert np.all(st == C.FOUND)
    assert np.array_equal(h[far], ph[far])
    near = np.nonzero(~far)[0]
    if len(near):
        assert np.all(oracle_mod.brute_force(w.xy, tc, w.xp[near]) >= 0)
    assert it.mean() < 0.2 * pi.mean()
    mesh.close()
