"""GPU parity of cnnsns_locate (the SNS walk of Alg. 1 and the CNN-SNS start of
Alg. 2) against the FP64 CPU oracle, through the C ABI.

Bar: host element ids, path lengths and statuses equal the oracle bit for bit
(both sides evaluate the same FP64 expressions without FMA); the contract
itself requires equal hosts only for points farther than 1e-9 from an edge of
the oracle's host and containment within 1e-9 otherwise, checked separately.
"""
import numpy as np
import pytest
import torch

from exact import edge_distances

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


def _contract_hosts(O, xy, tc, got, ref, xp):
    """Equal hosts away from edges; near an edge the GPU element must contain x_p within 1e-9."""
    far = edge_distances(xy, tc, ref, xp) > 1e-9
    assert np.array_equal(got[far], ref[far])
    near = np.nonzero(~far)[0]
    if len(near):
        V = xy[tc[got[near]]]
        p = xp[near]
        for k in range(3):
            a, b = V[:, k], V[:, (k + 1) % 3]
            d = b - a
            cross = d[:, 0] * (p[:, 1] - a[:, 1]) - d[:, 1] * (p[:, 0] - a[:, 0])
            assert np.all(cross / np.hypot(d[:, 0], d[:, 1]) >= -1e-9)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_plain_sns_bitwise(C, oracle_mod, wl, name):
    w = wl.build(name)
    print(f"[plain] {name}: {w.n_tri} triangles, {w.n_points} points", flush=True)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    assert mesh.n_tri == w.n_tri and mesh.G == w.G
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    h, it, st = C.locate(mesh, _dev(w.xp), start=_dev(w.start))
    torch.cuda.synchronize()
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    h, it, st = h.cpu().numpy(), it.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(h, oh)
    assert np.array_equal(it, oi)
    assert np.array_equal(st, os_)
    assert np.all(st == C.FOUND)
    _contract_hosts(oracle_mod, w.xy, tc, h, oh, w.xp)


def test_unordered_points_and_flipped_triangles(C, oracle_mod, wl):
    """Triangles given clockwise and points in random order give the same answers."""
    w = wl.build(n_side=150, seed=8, field="fourier", field_seed=3, k=25.0, origins="nodes")
    rng = np.random.default_rng(1)
    tri = w.tri.copy()
    flip = rng.random(tri.shape[0]) < 0.5
    tri[flip] = tri[flip][:, [0, 2, 1]]
    perm = rng.permutation(w.n_points)
    xp, start = w.xp[perm], w.start[perm]
    mesh = C.Mesh(w.xy, tri, overlay_side=256)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, tri)
    h, it, st = C.locate(mesh, _dev(xp), start=_dev(start))
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, xp, start)
    assert np.array_equal(h.cpu().numpy(), oh) and np.array_equal(it.cpu().numpy(), oi)
    assert np.array_equal(st.cpu().numpy(), os_)


def test_lookup_via_one_iteration_asg(C, oracle_mod, wl):
    """ASG start at the cell centres with one iteration returns the lookup itself."""
    # the last two cases put triangles over hundreds of cells (the block-parallel raster path)
    for n_side, G in [(40, 64), (40, 37), (200, 512), (12, 700), (3, 1024)]:
        xy, tri = wl.mesh(n_side, 4, graded=True)
        mesh = C.Mesh(xy, tri, overlay_side=G)
        tc, nbr = oracle_mod.prepare_mesh(xy, tri)
        lk = oracle_mod.lookup(xy, tc, G)
        c = (np.arange(G) + 0.5) / G
        X, Y = np.meshgrid(c, c, indexing="xy")
        centres = np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()], 1))
        h, it, st = C.locate(mesh, _dev(centres), max_iter=1)
        assert np.array_equal(h.cpu().numpy(), lk.ravel())
        assert np.all(st.cpu().numpy() == C.FOUND) and np.all(it.cpu().numpy() == 1)


def test_asg_mode_equals_oracle(C, oracle_mod, wl):
    w = wl.build("c1")
    mesh = C.Mesh(w.xy, w.tri, overlay_side=64)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, 64)
    zero = np.zeros((2, 64, 64))
    st = oracle_mod.cnnsns_start(w.xp, zero, lk)  # ASG at x_p = zero displacement from x_p
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, w.xp, st)
    h, it, s = C.locate(mesh, _dev(w.xp))
    assert np.array_equal(h.cpu().numpy(), oh) and np.array_equal(it.cpu().numpy(), oi)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_cnnsns_start_bitwise_given_displacement(C, oracle_mod, wl, name):
    """With the same displacement grid on both sides, CNN-SNS starts and walks match exactly."""
    w = wl.build(name)
    G = w.G
    rng = np.random.default_rng(7)
    # a seeded displacement grid: the true displacement field -dt u at the cell centres, perturbed
    disp = (-w.dt * w.vel.astype(np.float64) + rng.normal(0, 2 * w.dbar, size=w.vel.shape)).astype(np.float32)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=G)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, G)
    st, oh, oi, os_ = oracle_mod.cnnsns(w.xy, tc, nbr, lk, w.origins, w.xp, disp.astype(np.float64))
    h, it, s = C.locate(mesh, _dev(w.xp), origin=_dev(w.origins), disp=_dev(disp))
    h, it, s = h.cpu().numpy(), it.cpu().numpy(), s.cpu().numpy()
    assert np.array_equal(h, oh) and np.array_equal(it, oi) and np.array_equal(s, os_)
    # the start only moves the walk: hosts equal plain SNS away from edges
    ph, pi, ps = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    _contract_hosts(oracle_mod, w.xy, tc, h, ph, w.xp)
    assert it.mean() < pi.mean()


def test_statuses_and_edge_cases(C, oracle_mod, wl):
    w = wl.build("c1")
    mesh = C.Mesh(w.xy, w.tri, overlay_side=64)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    # MAXITER with a cap of 1, compared with the oracle
    h, it, s = C.locate(mesh, _dev(w.xp), start=_dev(w.start), max_iter=1)
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start, max_iter=1)
    assert np.array_equal(h.cpu().numpy(), oh) and np.array_equal(s.cpu().numpy(), os_)
    assert (os_ == C.MAXITER).any()
    # BADSTART and OUTSIDE
    xp = w.xp.copy()
    start = w.start.copy()
    start[:4] = [-1, w.n_tri, -5, 2 ** 31 - 1]
    xp[10:14] = [[1.5, 0.5], [-0.25, 0.5], [0.5, 1.75], [0.5, -3.0]]
    h, it, s = C.locate(mesh, _dev(xp), start=_dev(start))
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, xp, start)
    assert np.array_equal(h.cpu().numpy(), oh) and np.array_equal(it.cpu().numpy(), oi)
    assert np.array_equal(s.cpu().numpy(), os_)
    assert np.all(os_[:4] == C.BADSTART) and np.all(os_[10:14] == C.OUTSIDE)
    # optional outputs omitted; n = 0; ragged counts around the wave chunk size
    for n in [0, 1, 63, 64, 65, 255, 256, 257, 511, 512, 513, 1000]:
        hh, _, _ = C.locate(mesh, _dev(w.xp[:n]), start=_dev(w.start[:n]), want_iters=False, want_status=False)
        torch.cuda.synchronize()
        if n:
            assert np.array_equal(hh.cpu().numpy(), oracle_mod.sns(w.xy, tc, nbr, w.xp[:n], w.start[:n])[0])


def test_deterministic_and_stream(C, wl):
    w = wl.build("c2")
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    xp, st = _dev(w.xp), _dev(w.start)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = C.locate(mesh, xp, start=st)
    s.synchronize()
    b = C.locate(mesh, xp, start=st)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_mesh_errors_on_device(C):
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 2]], dtype=np.float64)
    with pytest.raises(C.CnnsnsError) as e:
        C.Mesh(xy, np.array([[0, 1, 4], [0, 3, 4]], np.int32))
    assert e.value.code == C.EMESH
    with pytest.raises(C.CnnsnsError) as e:
        C.Mesh(xy, np.array([[0, 1, 7]], np.int32))
    assert e.value.code == C.EMESH
    xy2 = np.array([[0, 0], [1, 1], [1, -1], [-1, 0], [2, 0.5]], dtype=np.float64)
    with pytest.raises(C.CnnsnsError) as e:
        C.Mesh(xy2, np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]], np.int32))
    assert e.value.code == C.EMESH
    xy3 = np.array([[0, 0], [1, 0], [0, 1], [0.2, 0.5]], dtype=np.float64)
    with pytest.raises(C.CnnsnsError) as e:
        C.Mesh(xy3, np.array([[0, 1, 2], [0, 1, 3]], np.int32))
    assert e.value.code == C.EMESH
    with pytest.raises(C.CnnsnsError) as e:  # a non-finite node
        C.Mesh(np.array([[0, 0], [1, 0], [np.nan, 1]], dtype=np.float64), np.array([[0, 1, 2]], np.int32))
    assert e.value.code == C.EMESH


def test_ragged_counts_lookup_modes(C, oracle_mod, wl):
    """CNN-SNS and ASG starts assign each wave strided 64-point runs: every count around the run
    and chunk sizes (and counts whose waves do not fill the last block) matches the oracle exactly."""
    w = wl.build("c2")
    G = w.G
    rng = np.random.default_rng(3)
    disp = (-w.dt * w.vel.astype(np.float64) + rng.normal(0, 2 * w.dbar, size=w.vel.shape)).astype(np.float32)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=G)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, G)
    zero = np.zeros((2, G, G))
    d_disp = _dev(disp)
    for n in [1, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1000, 2049, 4097, 70001]:
        print(f"[ragged lookup modes] n={n}", flush=True)
        xp, org = w.xp[:n], w.origins[:n]
        _, oh, oi, _ = oracle_mod.cnnsns(w.xy, tc, nbr, lk, org, xp, disp.astype(np.float64))
        h, it, _ = C.locate(mesh, _dev(xp), origin=_dev(org), disp=d_disp)
        assert np.array_equal(h.cpu().numpy(), oh) and np.array_equal(it.cpu().numpy(), oi)
        st = oracle_mod.cnnsns_start(xp, zero, lk)
        ah, ai, _ = oracle_mod.sns(w.xy, tc, nbr, xp, st)
        h, it, _ = C.locate(mesh, _dev(xp))
        assert np.array_equal(h.cpu().numpy(), ah) and np.array_equal(it.cpu().numpy(), ai)


def test_unstructured_delaunay_mesh(C, oracle_mod):
    """Qhull's Delaunay triangulation of 50,000 random points (irregular topology and node order,
    a ragged hull): given, ASG and CNN-SNS starts bit for bit against the oracle, including the
    points outside the hull."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(23)
    pts = rng.uniform(0.0, 1.0, size=(50000, 2))
    tri = Delaunay(pts).simplices.astype(np.int32)
    G = 128
    mesh = C.Mesh(pts, tri, overlay_side=G)
    tc, nbr = oracle_mod.prepare_mesh(pts, tri)
    lk = oracle_mod.lookup(pts, tc, G)
    n = 60000
    q = rng.uniform(0.0, 1.0, size=(n, 2))
    start = rng.integers(0, tri.shape[0], size=n).astype(np.int32)
    h, it, st = C.locate(mesh, _dev(q), start=_dev(start))
    rh, rit, rst = oracle_mod.sns(pts, tc, nbr, q, start)
    assert np.array_equal(h.cpu().numpy(), rh) and np.array_equal(it.cpu().numpy(), rit)
    assert np.array_equal(st.cpu().numpy(), rst) and set(np.unique(rst)) == {C.FOUND, C.OUTSIDE}
    h, it, st = C.locate(mesh, _dev(q))
    a_st = oracle_mod.cnnsns_start(q, np.zeros((2, G, G)), lk)
    rh, rit, rst = oracle_mod.sns(pts, tc, nbr, q, a_st)
    assert np.array_equal(h.cpu().numpy(), rh) and np.array_equal(it.cpu().numpy(), rit)
    origin = np.clip(q + rng.normal(0.0, 0.02, size=q.shape), 0.0, 1.0)
    disp = rng.normal(0.0, 0.01, size=(2, G, G)).astype(np.float32)
    h, it, st = C.locate(mesh, _dev(q), start=_dev(start), origin=_dev(origin), disp=_dev(disp))
    _, rh, rit, rst = oracle_mod.cnnsns(pts, tc, nbr, lk, origin, q, disp.astype(np.float64), fallback=start)
    assert np.array_equal(h.cpu().numpy(), rh) and np.array_equal(it.cpu().numpy(), rit)
    assert np.array_equal(st.cpu().numpy(), rst)


def test_full_size_16m_triangles(C, oracle_mod, wl):
    """The headline configuration: 16M triangles (graded), all 8,003,241 node points, in the launch
    configuration the benchmark times.  Plain SNS from the elements before movement (Alg. 1), CNN-SNS
    (Alg. 2) from one fixed displacement grid, the one-step displacement -dt u at the 4096^2 cell
    centres (an input from the generator, not from the GPU), and the ASG start at x_p: host, I_t and
    status of every point equal the oracle's bit for bit."""
    import time
    t0 = time.perf_counter()
    w = wl.build("c3")
    print(f"[c3] {w.n_tri} triangles, {w.n_points} points, G={w.G} ({time.perf_counter() - t0:.1f}s)", flush=True)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    xp, start = _dev(w.xp), _dev(w.start)
    h, it, st = C.locate(mesh, xp, start=start)
    torch.cuda.synchronize()
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    print(f"[c3] plain: oracle mean I_t {oi.mean():.2f} ({time.perf_counter() - t0:.1f}s)", flush=True)
    assert np.array_equal(h.cpu().numpy(), oh)
    assert np.array_equal(it.cpu().numpy(), oi)
    assert np.array_equal(st.cpu().numpy(), os_)
    assert np.all(os_ == C.FOUND)

    disp = (-w.dt * w.vel.astype(np.float64)).astype(np.float32)
    lk = oracle_mod.lookup(w.xy, tc, w.G)
    h2, it2, st2 = C.locate(mesh, xp, start=start, origin=_dev(w.origins), disp=_dev(disp))
    torch.cuda.synchronize()
    _, oh2, oi2, os2 = oracle_mod.cnnsns(w.xy, tc, nbr, lk, w.origins, w.xp, disp, fallback=w.start)
    print(f"[c3] CNN-SNS: oracle mean I_t {oi2.mean():.2f} ({time.perf_counter() - t0:.1f}s)", flush=True)
    assert np.array_equal(h2.cpu().numpy(), oh2)
    assert np.array_equal(it2.cpu().numpy(), oi2)
    assert np.array_equal(st2.cpu().numpy(), os2)
    assert np.array_equal(oh2, oh)  # the start never changes the host here

    h3, it3, st3 = C.locate(mesh, xp)
    torch.cuda.synchronize()
    _, oh3, oi3, os3 = oracle_mod.cnnsns(w.xy, tc, nbr, lk, w.xp, w.xp, np.zeros_like(disp))
    assert np.array_equal(h3.cpu().numpy(), oh3)
    assert np.array_equal(it3.cpu().numpy(), oi3)
    assert np.array_equal(st3.cpu().numpy(), os3)
    mesh.close()
