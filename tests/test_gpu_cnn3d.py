"""GPU parity of the 3D displacement CNN (cnnsns_predict3d, Sec. 2.3 with 3 x 3 x 3 kernels)
and of the 3D CNN-SNS walk (cnnsns_locate3d with origin and displacement, Alg. 2) against
the FP64 CPU oracle, through the C ABI.

Bars: the FP32 forward pass within the FP32 tolerance per output channel c,
|y - y_ref| <= 1e-5 |y_ref| + 1e-5 max_c |y_ref| (the 2D bar); a constructed
pass-through net gives -dt u exactly (one rounding of one product); the BF16 pass within
the BF16 bar of the 2D path (every element within 3% of its channel's largest magnitude,
the mean within 0.5%); starts, hosts, path lengths and statuses of the walk bit for bit,
given the same displacement grid.
"""
import numpy as np
import pytest
import torch

from test_oracle_cnn3d import constructed_net

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


def he_net(seed):
    rng = np.random.default_rng(seed)
    ch = (3, 32, 32, 32, 3)
    ws = [(rng.standard_normal((ch[l + 1], ch[l], 3, 3, 3)) * np.sqrt(2.0 / (27 * ch[l]))).astype(np.float32)
          for l in range(4)]
    bs = [(0.1 * rng.standard_normal(ch[l + 1])).astype(np.float32) for l in range(4)]
    return ws, bs


def _cube_mesh(C, G):
    """A one-cube mesh (six Kuhn tetrahedra) whose overlay has side G: predict3d only needs G."""
    from paper_2412_18379_amd import workload as W
    xyz, tet = W.kuhn_mesh(2, seed=0, jitter=0.0)
    return C.Mesh3D(xyz, tet, overlay_side=G)


def _within_bar(got, ref):
    scale = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1).reshape(-1, *([1] * (ref.ndim - 1)))
    ratio = np.abs(got - ref) / (1e-5 * np.abs(ref) + 1e-5 * scale + 1e-30)
    return float(ratio.max())


@pytest.mark.parametrize("G", [1, 2, 3, 5, 8, 17, 33])
def test_forward_full_grid(C, oracle_mod, G):
    rng = np.random.default_rng(100 + G)
    vel = rng.standard_normal((3, G, G, G)).astype(np.float32)
    ws, bs = he_net(G)
    mesh = _cube_mesh(C, G)
    got = C.predict3d(mesh, _dev(vel), C.Weights3D(ws, bs)).cpu().numpy().astype(np.float64)
    ref = oracle_mod.cnn3_forward(vel, ws, bs)
    r = _within_bar(got, ref)
    print(f"[cnn3d] G={G}: worst error / tolerance {r:.4f}", flush=True)
    assert r <= 1.0


@pytest.mark.parametrize("G", [70, 128])
def test_forward_windows(C, oracle_mod, wl, G):
    """Sides with a ragged 64-cell row segment (70) and the 5.8M-tetrahedron mesh's overlay (128):
    the whole grid on the GPU, windows at the faces, edges and inside by the oracle."""
    vel = wl.overlay_velocity_3d(wl.ABCFlow(), G)
    ws, bs = he_net(7)
    mesh = _cube_mesh(C, G)
    got = C.predict3d(mesh, _dev(vel), C.Weights3D(ws, bs)).cpu().numpy().astype(np.float64)
    for o, s in [((0, 0, 0), (1, G, G)), ((G - 1, 0, 0), (1, G, G)), ((G // 2, G - 3, 0), (2, 3, G)),
                 ((5, 60, 60), (4, 8, 10))]:
        ref = oracle_mod.cnn3_window(vel, ws, bs, o, s)
        win = got[:, o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]
        r = _within_bar(win, ref)
        print(f"[cnn3d] G={G} window {o}+{s}: worst error / tolerance {r:.4f}", flush=True)
        assert r <= 1.0


def test_constructed_net_is_exact(C):
    G = 40
    rng = np.random.default_rng(9)
    vel = rng.standard_normal((3, G, G, G)).astype(np.float32)
    dt = 0.0123
    ws, bs = constructed_net(dt)
    mesh = _cube_mesh(C, G)
    got = C.predict3d(mesh, _dev(vel), C.Weights3D(ws, bs)).cpu().numpy()
    assert np.array_equal(got, np.float32(-dt) * vel)
    # twice on the same mesh (the workspace is reused) and into a given output
    out = torch.empty((3, G, G, G), dtype=torch.float32, device="cuda")
    C.predict3d(mesh, _dev(vel), C.Weights3D(ws, bs), disp=out)
    assert np.array_equal(out.cpu().numpy(), got)


@pytest.mark.parametrize("name,net", [("t1", "he"), ("t2", "constructed")])
def test_cnnsns3_bitwise(C, oracle_mod, wl, name, net):
    w = wl.build_3d(name)
    print(f"[cnnsns3d] {name}: {w.n_tet} tetrahedra, {w.n_points} points, G={w.G}, {net} weights", flush=True)
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    lk = oracle_mod.lookup3(w.xyz, tp, w.G)
    vel = wl.overlay_velocity_3d(w.flow, w.G)
    ws, bs = he_net(3) if net == "he" else constructed_net(w.dt)
    # the displacement grid both walks start from, made on the CPU: the oracle's FP64 forward pass (small
    # grid), or the constructed net's exact result -dt u (the oracle's pins show the net computes it)
    ref = oracle_mod.cnn3_forward(vel, ws, bs) if net == "he" else -w.dt * vel.astype(np.float64)
    d32 = ref.astype(np.float32)
    got = C.predict3d(mesh, _dev(vel), C.Weights3D(ws, bs)).cpu().numpy().astype(np.float64)
    scale = np.abs(ref).reshape(3, -1).max(axis=1)[:, None, None, None]
    assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-5 * np.abs(ref))
    h, it, st = (t.cpu().numpy() for t in C.locate3d(mesh, _dev(w.xp), start=_dev(w.start), origin=_dev(w.xyz),
                                                       disp=_dev(d32)))
    _, rh, rit, rst = oracle_mod.cnnsns3(w.xyz, tp, nbr, lk, w.xyz, w.xp, d32.astype(np.float64), fallback=w.start)
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
    assert np.all(st == C.FOUND)
    if net == "constructed":
        plain = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)[1]
        print(f"[cnnsns3d] mean path {it.mean():.2f} vs plain {plain.mean():.2f}", flush=True)
        assert it.mean() < 0.25 * plain.mean()


def test_fallback_and_errors(C, oracle_mod, wl):
    w = wl.build_3d("t1")
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    lk = oracle_mod.lookup3(w.xyz, tp, w.G)
    G = w.G
    # displacements that push every point far outside clamp to the cube's corner cells
    big = np.full((3, G, G, G), 4.0, np.float32)
    for sign in (1.0, -1.0):
        d = _dev(sign * big)
        h, it, st = (t.cpu().numpy() for t in C.locate3d(mesh, _dev(w.xp), origin=_dev(w.xyz), disp=d))
        _, rh, rit, rst = oracle_mod.cnnsns3(w.xyz, tp, nbr, lk, w.xyz, w.xp, sign * big.astype(np.float64))
        assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
    lib = C.lib()
    ws, bs = he_net(1)
    W = C.Weights3D(ws, bs)
    vel = torch.zeros((3, G, G, G), dtype=torch.float32, device="cuda")
    disp = torch.empty_like(vel)
    assert lib.cnnsns_predict3d(mesh.handle, vel.data_ptr(), W.struct, C.PRECISIONS["fp8"], disp.data_ptr(),
                                None) == C.EINVAL
    assert lib.cnnsns_predict3d(None, vel.data_ptr(), W.struct, 0, disp.data_ptr(), None) == C.EINVAL
    assert lib.cnnsns_predict3d(mesh.handle, None, W.struct, 0, disp.data_ptr(), None) == C.EINVAL
    xp = _dev(w.xp[:10])
    host = torch.empty(10, dtype=torch.int32, device="cuda")
    assert lib.cnnsns_locate3d(mesh.handle, 10, xp.data_ptr(), None, None, disp.data_ptr(), 0, host.data_ptr(),
                               None, None, None) == C.EINVAL  # disp without origin
    with pytest.raises(ValueError):
        C.Weights3D([x[:, :, :, :, :2] for x in ws], bs)


def _within_bf16_bar(got, ref):
    """The BF16 bar (no tolerance is stated for the lower precision): per output channel, every
    element within 3% of the channel's largest magnitude and the mean error within 0.5%."""
    scale = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)
    err = np.abs(got - ref).reshape(ref.shape[0], -1)
    return float((err.max(axis=1) / scale).max()), float((err.mean(axis=1) / scale).max())


# 1-3: grids smaller than one block's column; 33 and 70: ragged z-sweep blocks in every dimension
# (8 x 32 cells and 32 planes per block)
@pytest.mark.parametrize("G", [1, 2, 3, 5, 17, 33, 70])
def test_bf16_forward_full_grid(C, oracle_mod, G):
    rng = np.random.default_rng(200 + G)
    vel = rng.standard_normal((3, G, G, G)).astype(np.float32)
    ws, bs = he_net(G + 1)
    mesh = _cube_mesh(C, G)
    got = C.predict3d(mesh, _dev(vel), C.Weights3D(ws, bs), "bf16").cpu().numpy().astype(np.float64)
    worst, mean = _within_bf16_bar(got, oracle_mod.cnn3_forward(vel, ws, bs))
    print(f"[cnn3d bf16] G={G}: worst {worst:.4f}, mean {mean:.5f} of the channel maximum", flush=True)
    assert worst <= 0.03 and mean <= 0.005


def test_bf16_forward_windows_and_walk(C, oracle_mod, wl):
    """The 623K-tetrahedron mesh's overlay (G = 128): windows against the oracle, and the CNN-SNS
    walk from the BF16 displacement bit for bit against the oracle's walk from the same grid."""
    w = wl.build_3d("t2")
    G = w.G
    vel = wl.overlay_velocity_3d(w.flow, G)
    ws, bs = he_net(11)
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=G)
    got = C.predict3d(mesh, _dev(vel), C.Weights3D(ws, bs), "bf16").cpu().numpy().astype(np.float64)
    for o, s in [((0, 0, 0), (1, G, G)), ((G // 2, 5, 0), (2, 3, G))]:
        ref = oracle_mod.cnn3_window(vel, ws, bs, o, s)
        worst, mean = _within_bf16_bar(got[:, o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]], ref)
        assert worst <= 0.03 and mean <= 0.005
    wc, bc = constructed_net(w.dt)
    disp = C.predict3d(mesh, _dev(vel), C.Weights3D(wc, bc), "bf16")
    h, it, st = (t.cpu().numpy() for t in C.locate3d(mesh, _dev(w.xp), start=_dev(w.start), origin=_dev(w.xyz),
                                                       disp=disp))
    # the BF16 displacement only moves the starts: the hosts are the oracle's plain-SNS hosts
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    rh, _, _ = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)
    assert np.all(st == C.FOUND)
    same = h == rh
    assert same.mean() > 0.9  # the rest lie on faces shared by both elements (many are clamped onto the cube)
    # elsewhere both elements hold the point (it lies on their common boundary, e.g. a clipped point)
    for k in np.nonzero(~same)[0]:
        for t in (h[k], rh[k]):
            V = w.xyz[tp[t]]
            lam = np.linalg.solve(np.vstack([V.T, np.ones(4)]), np.append(w.xp[k], 1.0))
            assert lam.min() >= -1e-12


def test_deterministic_and_on_a_side_stream(C, wl):
    """The 3D CNN (both precisions) and the CNN-SNS walk give the same bits on a second stream and
    when repeated (no atomics or order-dependent reductions in their results)."""
    w = wl.build_3d("t1")
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    vel = _dev(wl.overlay_velocity_3d(w.flow, w.G))
    net = C.Weights3D(*he_net(4))
    xp, st, org = _dev(w.xp), _dev(w.start), _dev(w.xyz)
    for prec in ("f32", "bf16"):
        d0 = C.predict3d(mesh, vel, net, prec)
        h0, i0, s0 = C.locate3d(mesh, xp, start=st, origin=org, disp=d0)
        torch.cuda.synchronize()  # calls on one mesh share its CNN workspace and must not overlap
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            d1 = C.predict3d(mesh, vel, net, prec, stream=side)
            h1, i1, s1 = C.locate3d(mesh, xp, start=st, origin=org, disp=d1, stream=side)
        side.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(d0, d1) and torch.equal(h0, h1) and torch.equal(i0, i1) and torch.equal(s0, s1)
        d2 = C.predict3d(mesh, vel, net, prec)
        assert torch.equal(d0, d2)
