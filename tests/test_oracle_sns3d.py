"""Pins of the oracle's 3D walk (Alg. 1 on tetrahedra, the paper's own setting).

The host element has a plain definition (a tetrahedron whose closed region
contains x_p, Sec. 2.2); it is checked against barycentric coordinates solved
independently with numpy, against the closed form of an unperturbed Kuhn grid
(the cell from floor(x / h), the tetrahedron from the order of the fractional
coordinates), and the neighbour table against the cube's boundary face count,
symmetry and Euler's formula.  The overlay lookup is its own definition
evaluated by brute force.
"""
import numpy as np
import pytest

PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _bary_all(xyz, tp, pts):
    """Barycentric coordinates of every point in every tetrahedron: [n_pts][n_tet][4] (numpy solve)."""
    V = xyz[tp]                                              # [T][4][3]
    M = np.concatenate([np.ones((tp.shape[0], 1, 4)), V.transpose(0, 2, 1)], axis=1)  # [T][4][4]
    Minv = np.linalg.inv(M)
    rhs = np.concatenate([np.ones((pts.shape[0], 1)), pts], axis=1)  # [n][4]
    return np.einsum("tij,nj->nti", Minv, rhs)


def test_mesh_invariants(oracle_mod, wl):
    w = wl.build_3d("t1")
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    a, b, c, d = (w.xyz[tp[:, k]] for k in range(4))
    assert np.all(np.einsum("ij,ij->i", b - a, np.cross(c - a, d - a)) > 0)
    assert np.array_equal(np.sort(tp, axis=1), np.sort(w.tet, axis=1))
    n = w.n_side
    assert (nbr == -1).sum() == 12 * (n - 1) ** 2          # two triangles per boundary square
    t, j = np.nonzero(nbr >= 0)
    u = nbr[t, j]
    face = lambda tt, jj: np.sort(np.delete(tp[tt], jj))  # noqa: E731
    for k in range(0, len(t), 997):
        back = np.nonzero(nbr[u[k]] == t[k])[0]
        assert len(back) == 1 and np.array_equal(face(t[k], j[k]), face(u[k], back[0]))
    edges = set()
    for p_ in range(4):
        for q_ in range(p_ + 1, 4):
            e = np.sort(tp[:, [p_, q_]], axis=1)
            edges.update(map(tuple, e))
    n_faces = (4 * tp.shape[0] + (nbr == -1).sum()) // 2
    assert w.xyz.shape[0] - len(edges) + n_faces - tp.shape[0] == 1  # a ball


def test_hosts_contain_the_points(oracle_mod, wl):
    w = wl.build_3d("t1")
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    h, it, st = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)
    assert np.all(st == 0)
    rng = np.random.default_rng(0)
    sel = rng.choice(w.n_points, 300, replace=False)
    lam = _bary_all(w.xyz, tp, w.xp[sel])                      # [300][T][4]
    inside = np.all(lam >= -1e-12, axis=2)
    assert np.all(inside[np.arange(len(sel)), h[sel]])         # the host contains x_p
    strict = np.all(lam > 1e-9, axis=2)
    one = strict.sum(axis=1) == 1
    assert np.array_equal(h[sel][one], np.argmax(strict[one], axis=1))
    # start = host: found at once
    h2, it2, _ = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, h)
    assert np.array_equal(h2, h) and np.all(it2 == 1)


def test_closed_form_kuhn_grid(oracle_mod, wl):
    n = 9
    xyz, tet = wl.kuhn_mesh(n, seed=1, jitter=0.0)
    tp, nbr = oracle_mod.prepare_mesh3(xyz, tet)
    rng = np.random.default_rng(2)
    pts = rng.uniform(0.0, 1.0, size=(2000, 3))
    start = rng.integers(0, tp.shape[0], size=2000).astype(np.int32)
    h, it, st = oracle_mod.sns3(xyz, tp, nbr, pts, start)
    assert np.all(st == 0)
    f = pts * (n - 1)
    cell = np.minimum(np.floor(f), n - 2).astype(np.int64)
    frac = f - cell
    order = np.argsort(-frac, axis=1, kind="stable")
    perm = np.array([PERMS.index(tuple(o)) for o in order])
    cid = (cell[:, 2] * (n - 1) + cell[:, 1]) * (n - 1) + cell[:, 0]
    assert np.array_equal(h, (6 * cid + perm).astype(np.int32))


def test_outside_maxiter_badstart(oracle_mod, wl):
    w = wl.build_3d("t1")
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    pts = np.array([[1.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    h, it, st = oracle_mod.sns3(w.xyz, tp, nbr, pts, np.array([0, 0, -1], np.int32))
    assert st[0] == 1 and np.any(nbr[h[0]] == -1)              # OUTSIDE at a boundary tetrahedron
    assert st[1] == 0 and st[2] == 3 and h[2] == -1
    h, it, st = oracle_mod.sns3(w.xyz, tp, nbr, pts[1:2], np.array([0], np.int32), max_iter=2)
    assert st[0] == 2 and it[0] == 2


def test_lookup_is_its_definition(oracle_mod, wl):
    w = wl.build_3d("t1")
    tp, _ = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    G = 12
    lk = oracle_mod.lookup3(w.xyz, tp, G)
    c = (np.arange(G) + 0.5) / G
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    centres = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    assert np.array_equal(lk.ravel(), oracle_mod.brute_force3(w.xyz, tp, centres))
    assert np.all(lk >= 0)


def test_mesh_errors(oracle_mod):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [2, 2, 2]], np.float64)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.canonicalise3(xyz, np.array([[0, 1, 2, 7]], np.int32))
    with pytest.raises(oracle_mod.OracleError):  # flat
        oracle_mod.canonicalise3(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float64),
                                 np.array([[0, 1, 2, 3]], np.int32))
    with pytest.raises(oracle_mod.OracleError):  # one face in three tetrahedra
        tp = oracle_mod.canonicalise3(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1],
                                                [1, 1, 1]], np.float64),
                                      np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], np.int32))
        oracle_mod.neighbours3(tp)


def test_ties_go_to_the_lowest_index(oracle_mod, wl):
    """Points whose two smallest numerators are exactly equal (dyadic coordinates on an
    unperturbed 2 x 2 x 2 Kuhn grid, found and confirmed in exact rational arithmetic): one
    iteration (max_iter = 1) moves across the face of the lower vertex index (eq. 5 read with
    ties to the lowest index)."""
    xyz, tet = wl.kuhn_mesh(3, seed=1, jitter=0.0)
    tp, nbr = oracle_mod.prepare_mesh3(xyz, tet)
    cases = [(0, (0.125, 0.25, 0.375), 2), (1, (0.125, 0.375, 0.25), 4), (2, (0.125, 0.625, 0.25), 13)]
    for t, p, want in cases:
        h, it, st = oracle_mod.sns3(xyz, tp, nbr, np.array([p]), np.array([t], np.int32), max_iter=1)
        assert st[0] == 2 and it[0] == 1 and h[0] == want, (t, p, h[0], want)


def test_unstructured_delaunay_mesh_against_qhull(oracle_mod):
    """An unstructured mesh (Qhull's Delaunay tetrahedralisation of 3000 random points): every
    point inside the hull is found in the simplex Qhull's own point location returns, every point
    outside ends OUTSIDE at a boundary face, whatever the start."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(21)
    pts = rng.uniform(0.0, 1.0, size=(3000, 3))
    d = Delaunay(pts)
    tet = d.simplices.astype(np.int32)
    tp, nbr = oracle_mod.prepare_mesh3(pts, tet)
    q = rng.uniform(0.0, 1.0, size=(20000, 3))
    start = rng.integers(0, tet.shape[0], size=20000).astype(np.int32)
    h, it, st = oracle_mod.sns3(pts, tp, nbr, q, start)
    fs = d.find_simplex(q)
    inside = fs >= 0
    assert np.all(st[inside] == 0) and np.array_equal(h[inside], fs[inside])
    assert np.all(st[~inside] == 1) and np.all(np.any(nbr[h[~inside]] == -1, axis=1))
