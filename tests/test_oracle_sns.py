"""Pins of the oracle's SNS walk (Alg. 1) and its host-element result.

The host element has a plain definition (the element whose closed region
contains x_p, Sec. 2.2), so the walk's result is pinned by exhaustive
exact-rational containment.  The path length I_t follows Alg. 1 and is pinned
by closed forms (strips, hand-derived walks), the dual-graph distance bound and
special cases.
"""
import collections
import os

import numpy as np
import pytest

from exact import containing_sets, edge_distances

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_square4():
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], dtype=np.float64)
    tri = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], dtype=np.int32)
    rows = np.loadtxt(os.path.join(GOLDEN, "square4_walks.txt"), comments="#")
    return xy, tri, rows


def test_golden_square4_walks(oracle_mod):
    xy, tri, rows = _load_square4()
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    assert np.array_equal(nbr, [[1, 3, -1], [2, 0, -1], [3, 1, -1], [0, 2, -1]])
    h, it, st = oracle_mod.sns(xy, tc, nbr, rows[:, :2], rows[:, 2].astype(np.int32))
    assert np.array_equal(h, rows[:, 3].astype(np.int32))
    assert np.array_equal(it, rows[:, 4].astype(np.int32))
    assert np.array_equal(st, rows[:, 5].astype(np.uint8))


def _strip(m):
    """Strip of 2m triangles over [0,m]x[0,1]: T_2i = (b_i, b_i+1, t_i), T_2i+1 = (b_i+1, t_i+1, t_i)."""
    b = [(float(i), 0.0) for i in range(m + 1)]
    t = [(float(i), 1.0) for i in range(m + 1)]
    xy = np.array(b + t, dtype=np.float64)
    B = lambda i: i
    T = lambda i: m + 1 + i
    tri = []
    for i in range(m):
        tri.append([B(i), B(i + 1), T(i)])
        tri.append([B(i + 1), T(i + 1), T(i)])
    return xy, np.array(tri, dtype=np.int32)


@pytest.mark.parametrize("m", [1, 2, 3, 7])
def test_strip_closed_form(oracle_mod, m):
    """Along a straight strip the walk visits every triangle in order: I_t = host + 1."""
    xy, tri = _strip(m)
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    pts, expect = [], []
    for k in range(m):
        pts.append((k + 0.25, 0.5))   # below the diagonal x + y = k + 1 of cell k: T_2k
        expect.append(2 * k)
        pts.append((k + 0.75, 0.6))   # above it: T_2k+1
        expect.append(2 * k + 1)
    pts = np.array(pts)
    h, it, st = oracle_mod.sns(xy, tc, nbr, pts, np.zeros(len(pts), np.int32))
    assert np.array_equal(h, expect)
    assert np.array_equal(it, np.array(expect) + 1)
    assert np.all(st == oracle_mod.FOUND)
    # beyond the right end: reaches the last triangle, whose right edge is a boundary
    h, it, st = oracle_mod.sns(xy, tc, nbr, np.array([[m + 0.5, 0.5]]), np.zeros(1, np.int32))
    assert (h[0], it[0], st[0]) == (2 * m - 1, 2 * m, oracle_mod.OUTSIDE)


def test_structured_grid_closed_form(oracle_mod, wl):
    """Unperturbed grid: the host follows from floor(x/h), floor(y/h) and the diagonal side (Sec. 2.1)."""
    n = 17  # h = 1/16, exact in binary
    xy = wl.jittered_grid(n, 0, jitter=0.0)
    tri = wl.triangulate_grid(n, xy)  # cocircular quads keep the main diagonal p00-p11
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    rng = np.random.default_rng(5)
    pts = rng.random((4000, 2))
    h = 1.0 / (n - 1)
    i = np.floor(pts[:, 0] / h).astype(int)
    j = np.floor(pts[:, 1] / h).astype(int)
    fx, fy = pts[:, 0] / h - i, pts[:, 1] / h - j
    keep = (np.abs(fx - fy) > 1e-6) & (fx > 1e-6) & (fy > 1e-6) & (fx < 1 - 1e-6) & (fy < 1 - 1e-6)
    pts, i, j, fx, fy = pts[keep], i[keep], j[keep], fx[keep], fy[keep]
    expect = 2 * (j * (n - 1) + i) + (fy > fx)
    starts = rng.integers(0, tri.shape[0], size=len(pts)).astype(np.int32)
    host, it, st = oracle_mod.sns(xy, tc, nbr, pts, starts)
    assert np.array_equal(host, expect)
    assert np.all(st == oracle_mod.FOUND)


@pytest.mark.parametrize("n,seed,graded,npts", [(12, 3, False, 400), (32, 1, False, 1024), (30, 8, True, 600)])
def test_host_equals_exact_brute_force(oracle_mod, wl, n, seed, graded, npts):
    """Host = an element whose closed region contains x_p, by exact rational tests over all elements."""
    xy, tri = wl.mesh(n, seed, graded=graded)
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    rng = np.random.default_rng(seed)
    pts = rng.random((npts, 2))
    # hard cases: mesh nodes (in several elements) and exact boundary points
    pts[: n] = xy[rng.integers(0, xy.shape[0], size=n)]
    pts[n: n + 8] = [[0, 0], [1, 1], [0, 0.3], [0.7, 0], [1, 0.5], [0.25, 1], [1, 0], [0, 1]]
    starts = rng.integers(0, tri.shape[0], size=npts).astype(np.int32)
    host, it, st = oracle_mod.sns(xy, tc, nbr, pts, starts)
    sets = containing_sets(xy, tc, pts)
    assert all(len(s) >= 1 for s in sets)
    for k in range(npts):
        assert st[k] == oracle_mod.FOUND
        assert host[k] in sets[k], (k, pts[k], host[k], sets[k])
    # the oracle's own exhaustive search returns the smallest exact containing id
    bf = oracle_mod.brute_force(xy, tc, pts)
    assert np.array_equal(bf, [s[0] for s in sets])


def _dual_bfs(nbr, src):
    dist = np.full(nbr.shape[0], -1)
    dist[src] = 0
    q = collections.deque([src])
    while q:
        t = q.popleft()
        for s in nbr[t]:
            if s >= 0 and dist[s] < 0:
                dist[s] = dist[t] + 1
                q.append(s)
    return dist


def test_path_length_bounds_and_special_cases(oracle_mod, wl):
    w = wl.build("c1")
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    host, it, st = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    assert np.all(st == oracle_mod.FOUND)  # Delaunay: the walk never cycles
    # I_t - 1 hops can never beat the dual-graph distance from start to host
    for k in range(0, w.n_points, 7):
        d = _dual_bfs(nbr, int(w.start[k]))
        assert it[k] - 1 >= d[host[k]]
    # starting in the host: one iteration, same host (idempotent)
    h2, it2, st2 = oracle_mod.sns(w.xy, tc, nbr, w.xp, host)
    assert np.array_equal(h2, host) and np.all(it2 == 1)
    # the mean walk is several elements long for a ~3-diameter displacement
    assert 3.0 < it.mean() < 30.0


def test_maxiter_and_badstart(oracle_mod, wl):
    w = wl.build("c1")
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    host, it, st = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    h1, it1, st1 = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start, max_iter=1)
    moved = it > 1
    assert np.all(st1[moved] == oracle_mod.MAXITER) and np.all(it1 == 1)
    assert np.all(st1[~moved] == oracle_mod.FOUND)
    # MAXITER returns the element just moved to: a neighbour of the start
    for k in np.nonzero(moved)[0][:50]:
        assert h1[k] in nbr[w.start[k]]
    bad = w.start.copy()
    bad[:3] = [-1, w.n_tri, -7]
    h2, it2, st2 = oracle_mod.sns(w.xy, tc, nbr, w.xp, bad)
    assert np.all(st2[:3] == oracle_mod.BADSTART) and np.all(h2[:3] == -1) and np.all(it2[:3] == 0)


def test_outside_points(oracle_mod, wl):
    xy, tri = wl.mesh(20, 4)
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    pts = np.array([[1.5, 0.5], [-0.2, 0.3], [0.5, 2.0], [0.4, -1e-3]])
    host, it, st = oracle_mod.sns(xy, tc, nbr, pts, np.full(4, tri.shape[0] // 2, np.int32))
    assert np.all(st == oracle_mod.OUTSIDE)
    for k in range(4):
        assert (nbr[host[k]] < 0).any()  # stopped in a boundary element


def test_agrees_with_qhull_at_scale(oracle_mod, wl):
    """An independent point-location routine (scipy / Qhull find_simplex) finds the same elements."""
    from scipy.spatial import Delaunay
    w = wl.build(n_side=300, seed=21, field="fourier", field_seed=4, k=20.0, origins="nodes", with_overlay=False)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    host, it, st = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    assert np.all(st == oracle_mod.FOUND)
    d = Delaunay(w.xy)
    simp = d.find_simplex(w.xp)
    key = {tuple(sorted(t)): k for k, t in enumerate(w.tri.tolist())}
    qh = np.array([key[tuple(sorted(d.simplices[s]))] for s in simp])
    far = edge_distances(w.xy, w.tri, host, w.xp) > 1e-9
    assert far.mean() > 0.8  # departure points clamped onto the square's boundary lie on an edge
    assert np.array_equal(host[far], qh[far])
    # plain SNS walks are long for a ~20-diameter displacement
    assert it.mean() > 15
