"""GPU parity of the tetrahedral walk (Alg. 1 with four faces per element, the
paper's own 3D setting of Sec. 2.2) against the FP64 CPU oracle, through the
C ABI (cnnsns_build_mesh3d, cnnsns_locate3d).

Bar: host, iteration count and status bit for bit.  Both sides compute each
face's determinant with the face's nodes in id order (the sign of that
permutation applied), in FP64 without FMA, and break ties to the lowest index.
The overlay lookup is checked cell by cell: a point at a cell centre, walked
for one iteration from the lookup's element, ends there exactly when the
element holds the centre, so the host is the table entry.
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


def _np(*ts):
    return tuple(t.cpu().numpy() for t in ts)


def _cells(x, G):
    return np.clip(np.floor(x * G), 0, G - 1).astype(np.int64)


def _lookup_starts(lk, xp, G):
    """Starts of the lookup mode: the table entry at the cell holding x_p, element 0 for an empty cell."""
    c = _cells(xp, G)
    s = lk[c[:, 2], c[:, 1], c[:, 0]]
    return np.where(s < 0, 0, s).astype(np.int32)


def _centres(G):
    c = (np.arange(G) + 0.5) / G
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))


@pytest.mark.parametrize("name", ["t1", "t2"])
def test_given_start_bitwise(C, oracle_mod, wl, name):
    w = wl.build_3d(name)
    print(f"[locate3d] {name}: {w.n_tet} tetrahedra, {w.n_points} points, G={w.G}", flush=True)
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    assert mesh.n_tet == w.n_tet and mesh.G == w.G and mesh.device_bytes == (128 + 16) * w.n_tet + 4 * w.G ** 3
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    h, it, st = _np(*C.locate3d(mesh, _dev(w.xp), start=_dev(w.start)))
    rh, rit, rst = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)
    assert np.all(rst == C.FOUND)
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)


@pytest.mark.parametrize("name", ["t1", "t2"])
def test_lookup_start_bitwise(C, oracle_mod, wl, name):
    w = wl.build_3d(name)
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    lk = oracle_mod.lookup3(w.xyz, tp, w.G)
    assert np.all(lk >= 0)
    # the whole table: every cell centre, one iteration
    cen = _centres(w.G)
    h, it, st = _np(*C.locate3d(mesh, _dev(cen), max_iter=1))
    assert np.array_equal(h, lk.ravel()) and np.all(it == 1) and np.all(st == C.FOUND)
    # the departure points walked from the table
    h, it, st = _np(*C.locate3d(mesh, _dev(w.xp)))
    rh, rit, rst = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, _lookup_starts(lk, w.xp, w.G))
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
    assert it.mean() < 0.5 * oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)[1].mean()


def test_unordered_points_ragged_tail_and_statuses(C, oracle_mod, wl):
    w = wl.build_3d("t1")
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=7)  # a side that is not a power of two
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    rng = np.random.default_rng(11)
    n = 3 * 512 + 37  # several wavefront chunks and a ragged tail
    xp = rng.uniform(-0.2, 1.2, size=(n, 3))  # some outside the mesh
    start = rng.integers(0, w.n_tet, size=n).astype(np.int32)
    start[[3, 100, n - 1]] = [-1, w.n_tet, -5]  # not elements: BADSTART
    for max_iter in (0, 3):
        h, it, st = _np(*C.locate3d(mesh, _dev(xp), start=_dev(start), max_iter=max_iter))
        rh, rit, rst = oracle_mod.sns3(w.xyz, tp, nbr, xp, start, max_iter=max_iter)
        assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
        assert set(np.unique(st)) >= ({C.MAXITER, C.BADSTART} if max_iter else {C.FOUND, C.OUTSIDE, C.BADSTART})
    lk = oracle_mod.lookup3(w.xyz, tp, 7)
    h, it, st = _np(*C.locate3d(mesh, _dev(xp)))
    rh, rit, rst = oracle_mod.sns3(w.xyz, tp, nbr, xp, _lookup_starts(lk, xp, 7))
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)


def test_edge_cases(C, wl):
    w = wl.build_3d("t1")
    mesh = C.Mesh3D(w.xyz, w.tet)
    assert mesh.G == 32  # 2^ceil(log2(cbrt(20250)))
    h, it, st = C.locate3d(mesh, _dev(np.zeros((0, 3))))
    assert h.shape == (0,)
    lib = C.lib()
    nulls = (None, None, None, None, 0, None, None, None, None)
    assert lib.cnnsns_locate3d(mesh.handle, -1, *nulls) == C.EINVAL
    assert lib.cnnsns_locate3d(mesh.handle, 4, *nulls) == C.EINVAL
    assert lib.cnnsns_locate3d(None, 0, *nulls) == C.EINVAL
    assert lib.cnnsns_locate3d(mesh.handle, 0, *nulls) == C.OK
    # iters and status may be NULL
    xp = _dev(w.xp[:1000])
    host = torch.empty(1000, dtype=torch.int32, device="cuda")
    assert lib.cnnsns_locate3d(mesh.handle, 1000, xp.data_ptr(), None, None, None, 0, host.data_ptr(), None, None,
                               None) == C.OK
    ref, _, _ = C.locate3d(mesh, xp)
    assert torch.equal(host, ref)


def test_mesh_errors(C):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [2, 2, 2]], np.float64)
    with pytest.raises(C.CnnsnsError) as e:
        C.Mesh3D(xyz, np.array([[0, 1, 2, 7]], np.int32))
    assert e.value.code == C.EMESH
    with pytest.raises(C.CnnsnsError) as e:  # flat
        C.Mesh3D(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float64), np.array([[0, 1, 2, 3]], np.int32))
    assert e.value.code == C.EMESH
    with pytest.raises(C.CnnsnsError) as e:  # a non-finite node
        C.Mesh3D(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [np.nan, 0, 1]], np.float64),
                 np.array([[0, 1, 2, 3]], np.int32))
    assert e.value.code == C.EMESH
    with pytest.raises(C.CnnsnsError) as e:  # one face in three tetrahedra
        C.Mesh3D(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1]], np.float64),
                 np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], np.int32))
    assert e.value.code == C.EMESH
    with pytest.raises(C.CnnsnsError) as e:  # two tetrahedra on the same side of their common face
        C.Mesh3D(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.1, 0.1, 2]], np.float64),
                 np.array([[0, 1, 2, 3], [0, 1, 2, 4]], np.int32))
    assert e.value.code == C.EMESH
    with pytest.raises(C.CnnsnsError) as e:
        C.Mesh3D(xyz, np.array([[0, 1, 2, 3]], np.int32), overlay_side=2000)
    assert e.value.code == C.EINVAL
    with pytest.raises(C.CnnsnsError) as e:
        C.Mesh3D(xyz[:3], np.zeros((0, 4), np.int32))
    assert e.value.code == C.EINVAL


def test_full_size_sampled(C, oracle_mod, wl):
    """5.8M tetrahedra (a 100^3 node grid), all 1M departure points: given starts bit for bit
    against the oracle; lookup starts give the same host wherever it is unique; 48 sampled
    lookup cells checked against brute force."""
    w = wl.build_3d("t3")
    print(f"[locate3d] t3: {w.n_tet} tetrahedra, {w.n_points} points, G={w.G}", flush=True)
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    xp = _dev(w.xp)
    h, it, st = _np(*C.locate3d(mesh, xp, start=_dev(w.start)))
    rh, rit, rst = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
    assert np.all(st == C.FOUND)
    h2, it2, st2 = _np(*C.locate3d(mesh, xp))
    assert np.all(st2 == C.FOUND) and it2.mean() < 0.25 * it.mean()
    # where the two walks disagree, both elements hold the point (closed containment, so it is
    # on their common boundary): points clipped onto the cube's faces, edges and corners
    diff = np.nonzero(h2 != h)[0]
    for hh in (h, h2):
        for k in diff:
            V = w.xyz[tp[hh[k]]]
            lam = np.linalg.solve(np.vstack([V.T, np.ones(4)]), np.append(w.xp[k], 1.0))
            assert lam.min() >= -1e-12
    assert np.all(np.any((w.xp[diff] == 0.0) | (w.xp[diff] == 1.0), axis=1))
    rng = np.random.default_rng(17)
    cells = rng.integers(0, w.G, size=(48, 3))
    cen = (cells + 0.5) / w.G
    hc, itc, stc = _np(*C.locate3d(mesh, _dev(cen), max_iter=1))
    assert np.array_equal(hc, oracle_mod.brute_force3(w.xyz, tp, cen)) and np.all(stc == C.FOUND)


def test_coarse_mesh_under_a_fine_overlay(C, oracle_mod, wl):
    """Tetrahedra whose cell boxes are large (48 tetrahedra under a 64^3 overlay) take the
    block-parallel raster; the whole table still equals the oracle's."""
    xyz, tet = wl.kuhn_mesh(3, seed=5, jitter=0.1)
    G = 64
    mesh = C.Mesh3D(xyz, tet, overlay_side=G)
    tp, _ = oracle_mod.prepare_mesh3(xyz, tet)
    lk = oracle_mod.lookup3(xyz, tp, G)
    h, it, st = _np(*C.locate3d(mesh, _dev(_centres(G)), max_iter=1))
    assert np.array_equal(h, lk.ravel()) and np.all(st == C.FOUND)


def test_unstructured_delaunay_mesh(C, oracle_mod, wl):
    """Qhull's Delaunay tetrahedralisation of 20,000 random points (irregular topology and node
    order, a ragged hull): given, lookup and CNN-SNS starts bit for bit against the oracle,
    including the points outside the hull."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(22)
    pts = rng.uniform(0.0, 1.0, size=(20000, 3))
    tet = Delaunay(pts).simplices.astype(np.int32)
    G = 24
    mesh = C.Mesh3D(pts, tet, overlay_side=G)
    tp, nbr = oracle_mod.prepare_mesh3(pts, tet)
    lk = oracle_mod.lookup3(pts, tp, G)
    n = 50000
    q = rng.uniform(0.0, 1.0, size=(n, 3))
    start = rng.integers(0, tet.shape[0], size=n).astype(np.int32)
    h, it, st = _np(*C.locate3d(mesh, _dev(q), start=_dev(start)))
    rh, rit, rst = oracle_mod.sns3(pts, tp, nbr, q, start)
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
    assert set(np.unique(st)) == {C.FOUND, C.OUTSIDE}
    h, it, st = _np(*C.locate3d(mesh, _dev(q)))
    rh, rit, rst = oracle_mod.sns3(pts, tp, nbr, q, _lookup_starts(lk, q, G))
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
    origin = np.clip(q + rng.normal(0.0, 0.05, size=q.shape), 0.0, 1.0)
    # a displacement grid: the mean step of the points whose origin is in the cell, else 0
    c = np.clip(np.floor(origin * G), 0, G - 1).astype(np.int64)
    flat = (c[:, 2] * G + c[:, 1]) * G + c[:, 0]
    grid = np.zeros((3, G ** 3))
    cnt = np.bincount(flat, minlength=G ** 3)
    for a in range(3):
        grid[a] = np.bincount(flat, weights=q[:, a] - origin[:, a], minlength=G ** 3) / np.maximum(cnt, 1)
    grid = grid.reshape(3, G, G, G).astype(np.float32)
    h, it, st = _np(*C.locate3d(mesh, _dev(q), start=_dev(start), origin=_dev(origin), disp=_dev(grid)))
    _, rh, rit, rst = oracle_mod.cnnsns3(pts, tp, nbr, lk, origin, q, grid.astype(np.float64), fallback=start)
    assert np.array_equal(h, rh) and np.array_equal(it, rit) and np.array_equal(st, rst)
