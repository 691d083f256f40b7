"""The in-loop training harness's data preparation (paper_2412_18379_amd.online), pinned on the CPU
against the oracle: labels from SNS hosts (Sec. 2.3's B'_l), the pooled ASG grid and the classifier's
inputs, and the displacement targets on a hand-made case."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_labels_pool_and_features_match_the_oracle(oracle_mod, wl):
    from paper_2412_18379_amd import online as O
    w = wl.build(n_side=40, seed=3, field="fourier", field_seed=5, U=1.0, k=6.0, origins="nodes", G=32)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    host, _, _ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    host[::97] = -1  # not an element: no label
    xy, tri = torch.from_numpy(w.xy), torch.from_numpy(w.tri)
    cent = O.centroids_by_id(xy, tri)
    lab = O.class_labels(cent, torch.from_numpy(w.xp), torch.from_numpy(host), w.G).numpy()
    assert np.array_equal(lab, oracle_mod.cls_label(w.xp, w.G, w.xy, w.tri, host))
    pool = O.pooled_grid(cent, w.G)
    opool = oracle_mod.cls_pool(w.xy, w.tri, w.G)
    assert np.allclose(pool.numpy(), opool, rtol=0, atol=1e-15)
    feat, xoff = O.class_features(torch.from_numpy(w.xp), pool)
    ofeat, oxoff = oracle_mod.cls_features(w.xp, opool)
    assert np.allclose(feat.numpy(), ofeat, rtol=1e-6, atol=1e-6) and np.array_equal(xoff.numpy(), oxoff)


def test_displacement_targets_hand_case():
    from paper_2412_18379_amd import online as O
    # two triangles; centroids (0.2, 0.1) and (0.7, 0.6) (node ids ascending in each)
    xy = torch.tensor([[0.0, 0.0], [0.6, 0.0], [0.0, 0.3], [0.6, 0.3], [0.9, 0.9], [0.6, 0.6]], dtype=torch.float64)
    tri = torch.tensor([[0, 1, 2], [3, 4, 5]], dtype=torch.int32)
    cent = O.centroids_by_id(xy, tri)
    assert torch.allclose(cent, torch.tensor([[0.2, 0.1], [0.7, 0.6]], dtype=torch.float64))
    G = 4
    origins = torch.tensor([[0.1, 0.1], [0.2, 0.15], [0.9, 0.9], [0.6, 0.1]], dtype=torch.float64)
    host = torch.tensor([1, 0, 1, -1], dtype=torch.int32)  # the last one is left out
    t, m = O.displacement_targets(cent, origins, host, G)
    # cell (0, 0) holds the first two origins: mean of (0.6, 0.5) and (0.0, -0.05); cell (3, 3) the third
    assert m.sum() == 2 and bool(m[0, 0]) and bool(m[3, 3])
    assert np.allclose(t[:, 0, 0].numpy(), [0.3, 0.225]) and np.allclose(t[:, 3, 3].numpy(), [-0.2, -0.3])
    assert float(t[:, m.logical_not()].abs().sum()) == 0.0


def test_displacement_targets_3d_hand_case():
    from paper_2412_18379_amd import online as O
    # two tetrahedra with centroids (0.1, 0.1, 0.1) and (0.7, 0.65, 0.6); the second lists its nodes out
    # of id order, the centroid sums them in ascending id
    xyz = torch.tensor([[0.0, 0.0, 0.0], [0.4, 0.0, 0.0], [0.0, 0.4, 0.0], [0.0, 0.0, 0.4],
                        [0.7, 0.65, 0.6], [0.9, 0.65, 0.6], [0.7, 0.85, 0.6], [0.5, 0.45, 0.6]],
                       dtype=torch.float64)
    tet = torch.tensor([[0, 1, 2, 3], [7, 5, 6, 4]], dtype=torch.int32)
    cent = O.centroids3_by_id(xyz, tet)
    assert torch.allclose(cent, torch.tensor([[0.1, 0.1, 0.1], [0.7, 0.65, 0.6]], dtype=torch.float64))
    G = 4
    origins = torch.tensor([[0.05, 0.1, 0.2], [0.2, 0.2, 0.1], [0.9, 0.9, 0.9], [0.5, 0.1, 0.9]],
                           dtype=torch.float64)
    host = torch.tensor([1, 0, 1, 5], dtype=torch.int32)  # the last host is not an element: left out
    t, m = O.displacement_targets_3d(cent, origins, host, G)
    # cell (z, y, x) = (0, 0, 0) holds the first two origins, (3, 3, 3) the third
    assert m.sum() == 2 and bool(m[0, 0, 0]) and bool(m[3, 3, 3])
    want0 = ((cent[1] - origins[0]) + (cent[0] - origins[1])) / 2
    assert np.allclose(t[:, 0, 0, 0].numpy(), want0.numpy())
    assert np.allclose(t[:, 3, 3, 3].numpy(), (cent[1] - origins[2]).numpy())
    assert float(t[:, m.logical_not()].abs().sum()) == 0.0


def test_displacement_targets_3d_match_a_loop():
    """Random origins and hosts on a small grid: the scatter-mean equals a per-cell Python loop; the
    cell of a coordinate is min(G - 1, floor(x G))."""
    from paper_2412_18379_amd import online as O
    rng = np.random.default_rng(4)
    G, n, n_el = 5, 400, 30
    cent = torch.from_numpy(rng.uniform(0, 1, size=(n_el, 3)))
    origins = rng.uniform(0, 1, size=(n, 3))
    origins[:7] = 1.0  # on the far faces: the last cell
    host = rng.integers(-1, n_el, size=n).astype(np.int32)
    t, m = O.displacement_targets_3d(cent, torch.from_numpy(origins), torch.from_numpy(host), G)
    sums, cnt = {}, {}
    for i in range(n):
        if host[i] < 0:
            continue
        c = tuple(min(G - 1, int(np.floor(origins[i, a] * G))) for a in (2, 1, 0))
        sums[c] = sums.get(c, 0) + (cent[host[i]].numpy() - origins[i])
        cnt[c] = cnt.get(c, 0) + 1
    assert int(m.sum()) == len(cnt)
    for c, v in sums.items():
        assert bool(m[c]) and np.allclose(t[(slice(None),) + c].numpy(), v / cnt[c], atol=1e-6)


def test_unsteady_abc_flow():
    from paper_2412_18379_amd import workload as W
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, size=(50, 3))
    f0, f = W.ABCFlow(), W.UnsteadyABC(5, drift=0.15)
    assert np.array_equal(np.array(f0(*x.T)), np.array(f.at(0)(*x.T)))
    # a phase shift of the flow equals a shift of the coordinates
    g = f.at(3)
    u = np.array(g(*x.T))
    shift = np.array([g.px, g.py, g.pz]) / (2 * np.pi)
    assert np.allclose(u, np.array(f0(*(x + shift).T)), atol=1e-12)
    # divergence-free: each component is independent of its own coordinate
    h = 1e-6
    for a in range(3):
        xe = x.copy()
        xe[:, a] += h
        assert np.allclose(np.array(g(*xe.T))[a], u[a], atol=1e-12)


def test_gemm_convolution_and_crops_match_the_full_grid():
    """The harness's 3D layer equals torch's conv3d (float64), and the net on a crop gives the full grid's
    outputs on the crop's valid range (inner sides lose four cells, sides on the grid's boundary none)."""
    from paper_2412_18379_amd import online as O
    torch.manual_seed(0)
    x = torch.randn(2, 3, 6, 7, 5, dtype=torch.float64)
    w, b = torch.randn(4, 3, 3, 3, 3, dtype=torch.float64), torch.randn(4, dtype=torch.float64)
    assert torch.allclose(O.conv3d_gemm(x, w, b), torch.nn.functional.conv3d(x, w, b, padding=1), atol=1e-12)
    net = O.DispNet3D().double()
    G, C = 20, 13
    v = torch.randn(1, 3, G, G, G, dtype=torch.float64)
    with torch.no_grad():
        full = net(v)
        for z0, y0, x0 in [(0, 0, 0), (7, 3, 0), (4, 7, 7)]:
            out = net(v[:, :, z0:z0 + C, y0:y0 + C, x0:x0 + C])
            (zl, zh), (yl, yh), (xl, xh) = (O.crop_valid_range(a, C, G) for a in (z0, y0, x0))
            assert zh - zl == C - 4 * ((z0 > 0) + (z0 + C < G))
            a = out[:, :, zl - z0:zh - z0, yl - y0:yh - y0, xl - x0:xh - x0]
            assert torch.allclose(a, full[:, :, zl:zh, yl:yh, xl:xh], atol=1e-12)
            # one cell further in from an inner side differs
            if z0 > 0:
                assert not torch.allclose(out[:, :, zl - z0 - 1], full[:, :, zl - 1, y0:y0 + C, x0:x0 + C])
