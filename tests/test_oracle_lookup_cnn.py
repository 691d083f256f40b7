"""Pins of the oracle's ASG overlay lookup, CNN forward pass and CNN-SNS start.

Lookup: exhaustive exact-rational containment of every cell centre (Sec. 1 /
Alg. 2, the auxiliary structured grid).  CNN: an independent library routine
(torch conv2d in float64), impulse responses, zero and constant inputs and
constructed weights with a closed-form output (Sec. 2.3 layers).  Start
selection (Alg. 2): special cases whose answer follows from the lookup pin.
"""
import numpy as np
import pytest
import torch

from exact import containing_sets, edge_distances


@pytest.mark.parametrize("G", [8, 21, 64])
def test_lookup_exact_brute_force(oracle_mod, wl, G):
    xy, tri = wl.mesh(14, 6, graded=True)
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    lk = oracle_mod.lookup(xy, tc, G)
    c = (np.arange(G) + 0.5) / G
    X, Y = np.meshgrid(c, c, indexing="xy")
    centres = np.stack([X.ravel(), Y.ravel()], 1)
    sets = containing_sets(xy, tc, centres)
    assert np.array_equal(lk.ravel(), [s[0] for s in sets])


def test_lookup_uncovered_cells(oracle_mod):
    # a mesh covering only the lower-left quarter of the unit square
    xy = np.array([[0, 0], [0.5, 0], [0.5, 0.5], [0, 0.5]], dtype=np.float64)
    tri = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    tc, _ = oracle_mod.prepare_mesh(xy, tri)
    lk = oracle_mod.lookup(xy, tc, 4)
    assert np.all(lk[2:, :] == -1) and np.all(lk[:, 2:] == -1)
    # centres (1/8, 1/8), (3/8, 3/8) lie on the diagonal: both triangles contain them, the min id wins
    assert lk[0, 0] == 0 and lk[1, 1] == 0 and lk[0, 1] == 0 and lk[1, 0] == 1


def _torch_cnn(vel, ws, bs):
    x = torch.from_numpy(vel.astype(np.float64))[None]
    for l in range(4):
        x = torch.nn.functional.conv2d(x, torch.from_numpy(ws[l].astype(np.float64)),
                                       torch.from_numpy(bs[l].astype(np.float64)), padding=1)
        if l < 3:
            x = torch.relu(x)
    return x[0].numpy()


@pytest.mark.parametrize("G,seed", [(5, 1), (37, 2), (64, 3)])
def test_cnn_equals_torch_conv2d_fp64(oracle_mod, wl, G, seed):
    rng = np.random.default_rng(seed)
    vel = rng.standard_normal((2, G, G)).astype(np.float32)
    ws, bs = wl.random_weights(seed)
    y = oracle_mod.cnn_forward(vel, ws, bs)
    ref = _torch_cnn(vel, ws, bs)
    assert np.abs(y - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_cnn_windows_equal_full_forward(oracle_mod, wl):
    G = 40
    rng = np.random.default_rng(9)
    vel = rng.standard_normal((2, G, G)).astype(np.float32)
    ws, bs = wl.random_weights(4)
    full = oracle_mod.cnn_forward(vel, ws, bs)
    for (r0, c0, h, w) in [(0, 0, 3, 5), (10, 17, 7, 4), (36, 30, 4, 10), (0, 39, 40, 1)]:
        part = oracle_mod.cnn_window(vel, ws, bs, r0, c0, h, w)
        assert np.array_equal(part, full[:, r0:r0 + h, c0:c0 + w])
    px = oracle_mod.cnn_pixels(vel, ws, bs, [0, 39, 20], [39, 0, 20])
    assert np.array_equal(px, full[:, [0, 39, 20], [39, 0, 20]].T)


def _passthrough_net(w1, b1=None):
    """A net whose output is the *linear* response of one conv layer w1 [1][cin][3][3]:
    conv1 splits the response into positive and negative parts (ReLU), conv2/3
    copy them, conv4 subtracts them."""
    cin = w1.shape[1]
    W1 = np.zeros((2, cin, 3, 3), np.float32)
    W1[0] = w1[0]
    W1[1] = -w1[0]
    eye = np.zeros((2, 2, 3, 3), np.float32)
    eye[0, 0, 1, 1] = eye[1, 1, 1, 1] = 1
    W4 = np.zeros((1, 2, 3, 3), np.float32)
    W4[0, 0, 1, 1], W4[0, 1, 1, 1] = 1, -1
    z = lambda k: np.zeros(k, np.float32)
    return [W1, eye, eye.copy(), W4], [z(2), z(2), z(2), z(1)]


def test_cnn_impulse_response_reads_back_weights(oracle_mod):
    """Cross-correlation convention: an impulse at (r0, c0) in channel i puts
    W[o][i][dy+1][dx+1] at output (r0 - dy, c0 - dx)."""
    G, r0, c0 = 9, 4, 3
    rng = np.random.default_rng(1)
    w1 = rng.standard_normal((1, 2, 3, 3)).astype(np.float32)
    ws, bs = _passthrough_net(w1)
    for i in range(2):
        vel = np.zeros((2, G, G), np.float32)
        vel[i, r0, c0] = 1.0
        y = oracle_mod.cnn_forward(vel, ws, bs)[0]
        expect = np.zeros((G, G))
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                expect[r0 - dy, c0 - dx] = w1[0, i, dy + 1, dx + 1]
        assert np.array_equal(y, expect)


def test_cnn_zero_weights_and_zero_padding_pattern(oracle_mod, wl):
    G = 12
    ws, bs = wl.random_weights(3)
    zw = [np.zeros_like(w) for w in ws]
    vel = np.random.default_rng(0).standard_normal((2, G, G)).astype(np.float32)
    y = oracle_mod.cnn_forward(vel, zw, bs)
    # zero weights: every layer outputs relu(bias) ... the last layer outputs its bias
    assert np.array_equal(y, np.broadcast_to(bs[3][:, None, None].astype(np.float64), y.shape))
    # constant input through an all-ones 3x3 kernel: 9c inside, 6c on edges, 4c at corners
    w1 = np.zeros((1, 2, 3, 3), np.float32)
    w1[0, 0] = 1.0
    ws2, bs2 = _passthrough_net(w1)
    c = 0.375
    vel = np.full((2, G, G), c, np.float32)
    y = oracle_mod.cnn_forward(vel, ws2, bs2)[0]
    expect = np.full((G, G), 9 * c)
    expect[0, :] = expect[-1, :] = expect[:, 0] = expect[:, -1] = 6 * c
    expect[0, 0] = expect[0, -1] = expect[-1, 0] = expect[-1, -1] = 4 * c
    assert np.array_equal(y, expect)


def constructed_weights(dt: float):
    """2->32->32->32->2 weights whose output is -dt * u at every cell."""
    W1 = np.zeros((32, 2, 3, 3), np.float32)
    W1[0, 0, 1, 1], W1[1, 0, 1, 1], W1[2, 1, 1, 1], W1[3, 1, 1, 1] = 1, -1, 1, -1
    Wm = np.zeros((32, 32, 3, 3), np.float32)
    for k in range(4):
        Wm[k, k, 1, 1] = 1
    W4 = np.zeros((2, 32, 3, 3), np.float32)
    W4[0, 0, 1, 1], W4[0, 1, 1, 1] = -dt, dt
    W4[1, 2, 1, 1], W4[1, 3, 1, 1] = -dt, dt
    z = lambda k: np.zeros(k, np.float32)
    return [W1, Wm, Wm.copy(), W4], [z(32), z(32), z(32), z(2)]


def test_cnn_constructed_departure_weights(oracle_mod, wl):
    """Constructed weights make the net output -dt u exactly (products of two FP32 values are exact in FP64)."""
    w = wl.build("c1")
    ws, bs = constructed_weights(w.dt)
    y = oracle_mod.cnn_forward(w.vel, ws, bs)
    expect = np.float64(np.float32(-w.dt)) * w.vel.astype(np.float64)
    assert np.array_equal(y, expect)
    # and on Taylor-Green it is the analytic departure displacement at the cell centres
    u, v = wl.TaylorGreen(1.0).grid(w.G)
    assert np.abs(y[0] + w.dt * u).max() < 1e-6 and np.abs(y[1] + w.dt * v).max() < 1e-6


def test_cnnsns_start_special_cases(oracle_mod, wl):
    xy, tri = wl.mesh(12, 2)
    tc, _ = oracle_mod.prepare_mesh(xy, tri)
    G = 16
    lk = oracle_mod.lookup(xy, tc, G)
    c = (np.arange(G) + 0.5) / G
    X, Y = np.meshgrid(c, c, indexing="xy")
    centres = np.stack([X.ravel(), Y.ravel()], 1)
    sets = containing_sets(xy, tc, centres)
    # zero displacement at the cell centres: the start is the (exact) smallest element holding the centre
    st = oracle_mod.cnnsns_start(centres, np.zeros((2, G, G)), lk)
    assert np.array_equal(st, [s[0] for s in sets])
    # a huge displacement is clamped into the corner cell
    big = np.full((2, G, G), 10.0)
    st = oracle_mod.cnnsns_start(centres[:5], big, lk)
    assert np.all(st == lk[G - 1, G - 1])
    st = oracle_mod.cnnsns_start(centres[:5], -big, lk)
    assert np.all(st == lk[0, 0])
    # origins exactly at 1.0 use the last cell
    st = oracle_mod.cnnsns_start(np.array([[1.0, 1.0], [0.0, 1.0]]), np.zeros((2, G, G)), lk)
    assert st[0] == lk[G - 1, G - 1] and st[1] == lk[G - 1, 0]
    # uncovered cells fall back to the given start, else element 0
    lk2 = lk.copy()
    lk2[:] = -1
    st = oracle_mod.cnnsns_start(centres[:3], np.zeros((2, G, G)), lk2, np.array([5, 6, 7], np.int32))
    assert np.array_equal(st, [5, 6, 7])
    st = oracle_mod.cnnsns_start(centres[:3], np.zeros((2, G, G)), lk2)
    assert np.array_equal(st, [0, 0, 0])


def test_cnnsns_preserves_hosts(oracle_mod, wl):
    """CNN-SNS only moves the start: its hosts equal plain SNS's (Sec. 2.3)."""
    w = wl.build("c1")
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, w.G)
    ws, bs = constructed_weights(w.dt)
    disp = oracle_mod.cnn_forward(w.vel, ws, bs)
    st, h, it, s = oracle_mod.cnnsns(w.xy, tc, nbr, lk, w.origins, w.xp, disp)
    h0, it0, s0 = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    assert np.all(s == 0) and np.all(s0 == 0)
    # the host is unique away from edges; on an edge or node any containing element is right
    far = edge_distances(w.xy, tc, h0, w.xp) > 1e-9
    assert far.mean() > 0.8
    assert np.array_equal(h[far], h0[far])
    sets = containing_sets(w.xy, tc, w.xp[~far])
    assert all(hk in sk for hk, sk in zip(h[~far], sets))
    assert it.mean() < 0.5 * it0.mean()
