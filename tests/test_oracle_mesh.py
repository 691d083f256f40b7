"""Pins of the oracle's mesh preparation and of the input generator.

The neighbour table {m^l} and the element list {K_l} are the SNS inputs of
eq. (6); these tests fix them by invariants (symmetry, hull size, Euler's
formula), by an independent edge matcher, and by an independent library
(scipy / Qhull) for the Delaunay generator.
"""
import numpy as np
import pytest

from exact import orient


def _edge_matcher(tri):
    """Independent neighbour table: dictionary keyed on the sorted vertex pair."""
    edges = {}
    for t, row in enumerate(tri.tolist()):
        for j in range(3):
            key = tuple(sorted((row[(j + 1) % 3], row[(j + 2) % 3])))
            edges.setdefault(key, []).append((t, j))
    nbr = -np.ones_like(tri)
    for key, lst in edges.items():
        assert len(lst) <= 2
        if len(lst) == 2:
            (t1, j1), (t2, j2) = lst
            nbr[t1, j1] = t2
            nbr[t2, j2] = t1
    return nbr


@pytest.mark.parametrize("n,seed,graded", [(8, 11, False), (32, 1, False), (40, 5, True), (120, 9, False),
                                           (90, 4, True)])
def test_generator_is_delaunay_equal_to_qhull(wl, n, seed, graded):
    from scipy.spatial import Delaunay
    xy, tri = wl.mesh(n, seed, graded=graded)
    assert tri.shape == (2 * (n - 1) ** 2, 3)
    ours = {tuple(sorted(t)) for t in tri.tolist()}
    qh = {tuple(sorted(t)) for t in Delaunay(xy).simplices.tolist()}
    assert ours == qh


def test_generator_boundary_and_orientation(wl):
    n = 25
    xy, tri = wl.mesh(n, 2)
    assert xy.min() == 0.0 and xy.max() == 1.0
    on_b = (xy[:, 0] == 0) | (xy[:, 0] == 1) | (xy[:, 1] == 0) | (xy[:, 1] == 1)
    assert on_b.sum() == 4 * (n - 1)
    for row in tri[:200].tolist():
        assert orient(xy[row[0]], xy[row[1]], xy[row[2]]) > 0


def test_generator_local_delaunay_exact(wl):
    """Every interior edge is locally Delaunay (exact incircle), hence the mesh is Delaunay."""
    from fractions import Fraction as F
    xy, tri = wl.mesh(20, 13, graded=True)
    nbr = _edge_matcher(tri)

    def incircle(a, b, c, d):
        m = []
        for p in (a, b, c):
            dx, dy = F(float(p[0])) - F(float(d[0])), F(float(p[1])) - F(float(d[1]))
            m.append((dx, dy, dx * dx + dy * dy))
        (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = m
        return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0)

    for t in range(tri.shape[0]):
        for j in range(3):
            s = nbr[t, j]
            if s < 0:
                continue
            q = [v for v in tri[s] if v not in tri[t]][0]
            a, b, c = (xy[v] for v in tri[t])
            assert incircle(a, b, c, xy[q]) <= 0


def test_canonicalise_orients_and_keeps_ids(oracle_mod, wl):
    xy, tri = wl.mesh(16, 3)
    rng = np.random.default_rng(0)
    flip = rng.random(tri.shape[0]) < 0.5
    bad = tri.copy()
    bad[flip] = bad[flip][:, [0, 2, 1]]
    tc = oracle_mod.canonicalise(xy, bad)
    for t in range(tri.shape[0]):
        assert sorted(tc[t]) == sorted(tri[t])
        assert orient(xy[tc[t, 0]], xy[tc[t, 1]], xy[tc[t, 2]]) > 0
    assert np.array_equal(tc, tri)  # the generator's order is already CCW


def test_neighbours_match_independent_matcher(oracle_mod, wl):
    for n, seed, graded in [(16, 1, False), (33, 2, True)]:
        xy, tri = wl.mesh(n, seed, graded=graded)
        tc, nbr = oracle_mod.prepare_mesh(xy, tri)
        assert np.array_equal(nbr, _edge_matcher(tc))


def test_neighbour_invariants(oracle_mod, wl):
    n = 50
    xy, tri = wl.mesh(n, 7)
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    nt, nv = tc.shape[0], xy.shape[0]
    # symmetry and shared vertices
    for t in range(nt):
        for j in range(3):
            s = nbr[t, j]
            if s >= 0:
                assert t in nbr[s]
                shared = set(tc[t]) & set(tc[s])
                assert shared == {tc[t, (j + 1) % 3], tc[t, (j + 2) % 3]}
    # boundary edges = hull edges of the square grid; Euler: N_t = 2 N_v - h - 2
    n_boundary = int((nbr < 0).sum())
    assert n_boundary == 4 * (n - 1)
    assert nt == 2 * nv - n_boundary - 2


def test_mesh_errors(oracle_mod):
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 2]], dtype=np.float64)
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.canonicalise(xy, np.array([[0, 1, 4], [0, 3, 4]], np.int32))  # 0,3,4 collinear
    assert e.value.code == oracle_mod.EMESH
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.canonicalise(xy, np.array([[0, 1, 5]], np.int32))
    assert e.value.code == oracle_mod.EMESH
    # edge (0,3) in three triangles
    xy2 = np.array([[0, 0], [1, 1], [1, -1], [-1, 0], [2, 0.5]], dtype=np.float64)
    tri = oracle_mod.canonicalise(xy2, np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]], np.int32))
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.neighbours(5, tri)
    assert e.value.code == oracle_mod.EMESH
    # two overlapping triangles traversing their shared edge the same way
    xy3 = np.array([[0, 0], [1, 0], [0, 1], [0.2, 0.5]], dtype=np.float64)
    tri3 = oracle_mod.canonicalise(xy3, np.array([[0, 1, 2], [0, 1, 3]], np.int32))
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.neighbours(4, tri3)
    assert e.value.code == oracle_mod.EMESH
