"""Pins of the oracle's classifier CNN (Sec. 2.3, eq. 7-8; the prediction step of Alg. 2), in 2D.

cls_pool against exact rational means; cls_features by closed forms on
structured grids; cls_forward against the same network written with torch's
float64 library layers and against hand-built nets with closed-form classes;
cls_start and cls_label on hand-made cases; and end to end, that a walk from
the classifier's start finds the plain walk's host.
"""
from fractions import Fraction

import numpy as np
import pytest
from exact import edge_distances

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _mesh(wl, n_side=12, seed=4, jitter=0.25):
    xy, tri = wl.mesh(n_side, seed, jitter=jitter)
    return xy, tri


def _weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    from oracle import CLS_SHAPES
    ws, bs = [], []
    for s in CLS_SHAPES:
        fan_in = int(np.prod(s[1:]))
        ws.append((rng.standard_normal(s) * np.sqrt(2.0 / fan_in) * scale).astype(np.float32))
        bs.append((0.1 * rng.standard_normal(s[0])).astype(np.float32))
    return ws, bs


# ----------------------------------------------------------------------------- pooling

def test_pool_exact_means(oracle_mod, wl):
    xy, tri = _mesh(wl)
    G = 8
    pool = oracle_mod.cls_pool(xy, tri, G)
    sums, counts = {}, {}
    for t in range(tri.shape[0]):
        c = [sum(Fraction(float(xy[v, k])) for v in tri[t]) / 3 for k in range(2)]
        cell = tuple(min(G - 1, int(c[k] * G)) for k in (1, 0))  # exact floor of a non-negative rational
        sums.setdefault(cell, [Fraction(0), Fraction(0)])
        sums[cell][0] += c[0]
        sums[cell][1] += c[1]
        counts[cell] = counts.get(cell, 0) + 1
    for cy in range(G):
        for cx in range(G):
            if (cy, cx) in counts:
                want = [float(s / counts[(cy, cx)]) for s in sums[(cy, cx)]]
                assert np.allclose(pool[cy, cx], want, rtol=0, atol=4e-16)
            else:
                assert pool[cy, cx, 0] == (cx + 0.5) / G and pool[cy, cx, 1] == (cy + 0.5) / G


def test_pool_empty_cells_and_node_order(oracle_mod, wl):
    xy, tri = _mesh(wl, n_side=4)  # 18 triangles under 64 x 64 cells: most are empty
    G = 64
    pool = oracle_mod.cls_pool(xy, tri, G)
    cent = oracle_mod.element_centroids(xy, tri)
    cells = {(min(G - 1, int(np.floor(c[1] * G))), min(G - 1, int(np.floor(c[0] * G)))) for c in cent}
    assert len(cells) <= tri.shape[0]
    for cy in range(G):
        for cx in range(G):
            if (cy, cx) not in cells:
                assert tuple(pool[cy, cx]) == ((cx + 0.5) / G, (cy + 0.5) / G)
    # each triangle's nodes in another order: the centroid sums its vertices in node-id order
    rng = np.random.default_rng(3)
    xy2, tri2 = _mesh(wl, n_side=20, seed=9)
    perm = np.array([rng.permutation(3) for _ in range(tri2.shape[0])])
    shuffled = np.take_along_axis(tri2, perm, axis=1)
    assert np.array_equal(oracle_mod.cls_pool(xy2, tri2, 16), oracle_mod.cls_pool(xy2, shuffled, 16))


# ----------------------------------------------------------------------------- features

def test_features_closed_forms(oracle_mod, wl):
    xy, tri = _mesh(wl, n_side=33, seed=2)
    G = 16
    pool = oracle_mod.cls_pool(xy, tri, G)
    # a point at a pooled centroid sees zero in the centre cell
    xp = np.array([pool[7, 5], pool[0, 0], pool[15, 15]])
    feat, xoff = oracle_mod.cls_features(xp, pool)
    assert np.all(feat[:, :, 4, 4] == 0.0)
    # the cell offset: a cell centre gives 0, a cell corner -1/2
    xp = np.array([[(5 + 0.5) / G, (7 + 0.5) / G], [3 / G, 9 / G]])
    _, xoff = oracle_mod.cls_features(xp, pool)
    assert np.array_equal(xoff, np.array([[0.0, 0.0], [-0.5, -0.5]], np.float32))
    # one cell to the right: the window moves by one column and channel 0 drops by exactly 1
    p = np.array([[0.40625, 0.53125]])  # dyadic: p and p + 1/G are exact and in the interior
    f0, _ = oracle_mod.cls_features(p, pool)
    f1, _ = oracle_mod.cls_features(p + np.array([[1.0 / G, 0.0]]), pool)
    assert np.allclose(f1[0, 0, :, :-1], f0[0, 0, :, 1:] - 1.0, atol=2e-6)
    assert np.allclose(f1[0, 1, :, :-1], f0[0, 1, :, 1:], atol=2e-6)
    # at the corner cell the window is extended by replication (padding layer)
    fc, _ = oracle_mod.cls_features(np.array([[0.01, 0.02]]), pool)
    for k in range(4):
        assert np.array_equal(fc[0, :, :, k], fc[0, :, :, 4])
        assert np.array_equal(fc[0, :, k, :], fc[0, :, 4, :])
    # the definition at a random point, computed independently in exact rationals
    q = np.array([[0.3141592653589793, 0.7071067811865476]])
    fq, _ = oracle_mod.cls_features(q, pool)
    cx, cy = int(q[0, 0] * G), int(q[0, 1] * G)
    for dy in range(-4, 5):
        for dx in range(-4, 5):
            r, c = min(max(cy + dy, 0), G - 1), min(max(cx + dx, 0), G - 1)
            want = (Fraction(float(pool[r, c, 0])) - Fraction(float(q[0, 0]))) * G
            assert abs(float(fq[0, 0, dy + 4, dx + 4]) - float(want)) <= 1e-6 * max(1.0, abs(float(want)))


# ----------------------------------------------------------------------------- the network

def _torch_forward(feat, xoff, ws, bs):
    t = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64))
    W = [t(w) for w in ws]
    B = [t(b) for b in bs]
    x = t(feat)
    y = F.relu(F.conv2d(x, W[0], B[0], padding=1))
    y = F.relu(F.conv2d(y, W[1], B[1], padding=1))
    y = F.avg_pool2d(y, 2).reshape(x.shape[0], -1)
    m = F.relu(F.linear(t(xoff), W[2], B[2]))
    m = F.relu(F.linear(m, W[3], B[3]))
    h = F.relu(F.linear(torch.cat([y, m], dim=1), W[4], B[4]))
    H = F.linear(h, W[5], B[5])
    return H.numpy(), torch.softmax(H, dim=1).numpy()


def test_forward_equals_torch_float64(oracle_mod):
    rng = np.random.default_rng(7)
    n = 300
    feat = rng.uniform(-5, 5, size=(n, 2, 9, 9)).astype(np.float32)
    xoff = rng.uniform(-0.5, 0.5, size=(n, 2)).astype(np.float32)
    ws, bs = _weights(11)
    logits, prob, cls = oracle_mod.cls_forward(feat, xoff, ws, bs)
    H, P = _torch_forward(feat, xoff, ws, bs)
    assert np.allclose(logits, H, rtol=1e-12, atol=1e-12 * np.abs(H).max())
    assert np.allclose(prob, P, rtol=1e-12, atol=1e-15)
    assert np.array_equal(cls, np.argmax(H, axis=1))


def _zero_net():
    from oracle import CLS_SHAPES
    return [np.zeros(s, np.float32) for s in CLS_SHAPES], [np.zeros(s[0], np.float32) for s in CLS_SHAPES]


def test_hand_built_nets(oracle_mod):
    rng = np.random.default_rng(2)
    n = 64
    feat = rng.uniform(-3, 3, size=(n, 2, 9, 9)).astype(np.float32)
    xoff = rng.uniform(-0.5, 0.5, size=(n, 2)).astype(np.float32)
    # bias only: the largest bias wins, ties to the lowest class
    ws, bs = _zero_net()
    bs[5][[17, 60]] = 3.0
    bs[5][5] = 2.5
    _, prob, cls = oracle_mod.cls_forward(feat, xoff, ws, bs)
    assert np.all(cls == 17)
    assert np.allclose(prob[:, 17], prob[:, 60])
    # module 2 path: relu(x offset) carried through to class 41 (one cell right) when it exceeds 1/4
    ws, bs = _zero_net()
    ws[2][0, 0] = 1.0          # m1[0] = relu(xoff_x)
    ws[3][0, 0] = 1.0          # m2[0] = m1[0]
    ws[4][0, 256] = 1.0        # h[0] = m2[0] (module 2 follows the 256 conv features)
    bs[5][40] = 10.0
    bs[5][41] = 9.75
    ws[5][41, 0] = 1.0         # H_41 = 9.75 + relu(xoff_x)
    xo = np.array([[-0.5, 0.0], [0.1, 0.3], [0.25, -0.2], [0.2500001, 0.0], [0.49, 0.4]], np.float32)
    _, _, cls = oracle_mod.cls_forward(np.zeros((5, 2, 9, 9), np.float32), xo, ws, bs)
    assert cls.tolist() == [40, 40, 40, 41, 41]  # exactly 1/4 ties and goes to the lower class
    # module 1 path: class 1 wins by the 2 x 2 average of relu(channel 0) over the top-left cells
    ws, bs = _zero_net()
    ws[0][0, 0, 1, 1] = 1.0    # conv1 channel 0 = relu(feat channel 0)
    ws[1][0, 0, 1, 1] = 1.0    # conv2 channel 0 = conv1 channel 0
    ws[4][0, 0] = 1.0          # h[0] = pooled (0, 0, 0)
    ws[5][1, 0] = 1.0
    bs[5][0] = 0.5
    logits, _, cls = oracle_mod.cls_forward(feat, xoff, ws, bs)
    pooled = np.maximum(feat[:, 0, :2, :2].astype(np.float64), 0).mean(axis=(1, 2))
    assert np.allclose(logits[:, 1], pooled, atol=1e-15)
    assert np.array_equal(cls, np.where(pooled > 0.5, 1, 0))


# ----------------------------------------------------------------------------- start and label

def test_start_and_label(oracle_mod):
    G = 10
    lk = np.arange(G * G, dtype=np.int32).reshape(G, G)
    lk[0, 0] = -1
    xp = np.array([[0.55, 0.35], [0.05, 0.05], [0.95, 0.95]])
    cls = np.array([40, 0, 80], np.int32)
    st = oracle_mod.cls_start(xp, lk, cls, fallback=np.array([7, 8, 9], np.int32))
    # class 40: the point's own cell (5, 3); class 0: four cells left and down, clamped to (0, 0): empty, so the
    # fallback; class 80: four right and up, clamped to (9, 9)
    assert st.tolist() == [3 * G + 5, 8, 99]
    assert oracle_mod.cls_start(xp[1:2], lk, cls[1:2]).tolist() == [0]
    # labels: the window cell of the host's centroid, clamped to the window
    xy = np.array([[0.0, 0.0], [0.36, 0.0], [0.0, 0.36], [0.93, 0.93], [0.63, 0.93], [0.93, 0.63]])
    tri = np.array([[0, 1, 2], [3, 4, 5]], np.int32)  # centroids (0.12, 0.12), cell (1, 1), and (0.83, 0.83)
    lab = oracle_mod.cls_label(np.array([[0.15, 0.12], [0.35, 0.15], [0.05, 0.05]]), G, xy, tri,
                               np.array([0, 0, 1], np.int32))
    # same cell; two cells left of the point's cell (3, 1); eight right and up, clamped to four
    assert lab.tolist() == [40, 4 * 9 + 2, 80]
    assert oracle_mod.cls_label(xp[:1], G, xy, tri, np.array([-1], np.int32)).tolist() == [-1]


def test_walk_from_classifier_start_finds_the_host(oracle_mod, wl):
    w = wl.build(n_side=40, seed=6, field="fourier", field_seed=8, U=1.0, k=6.0, origins="nodes", G=64)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, w.G)
    ws, bs = _weights(5)
    cls, start, _ = oracle_mod.cls_classify(w.xy, w.tri, lk, w.xp, ws, bs, fallback=w.start)
    h, it, st = oracle_mod.sns(w.xy, tc, nbr, w.xp, start)
    hp, _, _ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    assert np.all(st == oracle_mod.FOUND)
    # the host is unique away from edges; on an edge (a departure point at a node of the boundary,
    # say) the element the walk reaches must contain it
    far = edge_distances(w.xy, tc, hp, w.xp) > 1e-9
    assert np.array_equal(h[far], hp[far]) and far.mean() > 0.5  # clamped points lie on the boundary
    exact_hosts = oracle_mod.brute_force(w.xy, tc, w.xp[~far])
    assert np.all(exact_hosts >= 0)
    assert cls.min() >= 0 and cls.max() < 81
