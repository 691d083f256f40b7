"""Pins of the oracle's interpolation at the departure point in a tetrahedron (Sec. 2.1 after
eq. 4, with the nodal basis of Sec. 2.2: the four barycentric coordinates).

Fixed without any reference output: fields linear in x, y, z are reproduced (to rounding),
constants are reproduced (the coordinates sum to one), a node's own value is returned at the
node, coordinates solved independently from the 4x4 homogeneous system give the same value,
a convex field is over-estimated by at most the squared longest edge, and the value does not
depend on the order the element lists its vertices in.
"""
import numpy as np
import pytest


def _setup(oracle_mod, wl, n=3000, seed=0):
    w = wl.build_3d("t1")
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    rng = np.random.default_rng(seed)
    xp = rng.uniform(0.0, 1.0, size=(n, 3))
    host, _, st = oracle_mod.sns3(w.xyz, tp, nbr, xp, np.zeros(n, np.int32))
    assert np.all(st == 0)
    return w, tp, host, xp


def test_linear_fields_are_reproduced(oracle_mod, wl):
    w, tp, host, xp = _setup(oracle_mod, wl)
    rng = np.random.default_rng(1)
    a, B = rng.standard_normal(3), rng.standard_normal((3, 3))
    got = oracle_mod.interpolate3(w.xyz, tp, a[None, :] + w.xyz @ B.T, xp, host)
    assert np.max(np.abs(got - (a[None, :] + xp @ B.T))) <= 1e-13


def test_constants_are_reproduced(oracle_mod, wl):
    w, tp, host, xp = _setup(oracle_mod, wl)
    nodal = np.tile([3.25, -0.5, 7.0], (w.xyz.shape[0], 1))
    got = oracle_mod.interpolate3(w.xyz, tp, nodal, xp, host)
    assert np.max(np.abs(got - nodal[0])) <= 16 * np.finfo(np.float64).eps * 7.0


def test_node_values_at_nodes(oracle_mod, wl):
    w = wl.build_3d("t1")
    tp, _ = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    rng = np.random.default_rng(2)
    nodal = rng.standard_normal((w.xyz.shape[0], 3))
    t = np.repeat(np.arange(0, tp.shape[0], 7, dtype=np.int32), 4)
    nodes = tp[t, np.tile(np.arange(4), len(t) // 4)]  # every vertex of every 7th tetrahedron
    got = oracle_mod.interpolate3(w.xyz, tp, nodal, w.xyz[nodes], t)
    assert np.all(np.abs(got - nodal[nodes]) <= 8 * np.finfo(np.float64).eps * np.abs(nodal[nodes]) + 1e-300)


def test_against_an_independent_solve(oracle_mod, wl):
    w, tp, host, xp = _setup(oracle_mod, wl, n=1500, seed=3)
    rng = np.random.default_rng(4)
    nodal = rng.standard_normal((w.xyz.shape[0], 3))
    got = oracle_mod.interpolate3(w.xyz, tp, nodal, xp, host)
    v = w.xyz[tp[host]]                                       # [n][4][3]
    M = np.concatenate([np.ones((len(host), 1, 4)), v.transpose(0, 2, 1)], axis=1)
    rhs = np.concatenate([np.ones((len(host), 1)), xp], axis=1)
    lam = np.linalg.solve(M, rhs[:, :, None])[:, :, 0]
    want = np.einsum("nj,njc->nc", lam, nodal[tp[host]])
    assert np.max(np.abs(got - want)) <= 1e-11


def test_convex_field_bound(oracle_mod, wl):
    """f = |x|^2: the P1 interpolant of a convex function lies above it, by at most the squared
    longest edge (sum_j lambda_j |n_j - p|^2 <= max_j |n_j - p|^2)."""
    w, tp, host, xp = _setup(oracle_mod, wl, seed=5)
    f = (w.xyz ** 2).sum(axis=1)
    got = oracle_mod.interpolate3(w.xyz, tp, np.stack([f, -f, 2 * f], axis=1), xp, host)
    over = got[:, 0] - (xp ** 2).sum(axis=1)
    v = w.xyz[tp[host]]
    h2 = np.max([((v[:, a] - v[:, b]) ** 2).sum(axis=1) for a in range(4) for b in range(a + 1, 4)], axis=0)
    assert np.all(over >= -1e-15) and np.all(over <= h2 + 1e-15)
    assert np.array_equal(got[:, 1], -got[:, 0]) and np.array_equal(got[:, 2], 2 * got[:, 0])


def test_vertex_order_does_not_matter_and_invalid_hosts(oracle_mod, wl):
    w, tp, host, xp = _setup(oracle_mod, wl, n=500, seed=6)
    rng = np.random.default_rng(7)
    nodal = rng.standard_normal((w.xyz.shape[0], 3))
    got = oracle_mod.interpolate3(w.xyz, tp, nodal, xp, host)
    # an even permutation of every element's vertices keeps it positive
    tq = np.ascontiguousarray(tp[:, [1, 2, 0, 3]])
    assert np.array_equal(oracle_mod.interpolate3(w.xyz, tq, nodal, xp, host), got)
    bad = oracle_mod.interpolate3(w.xyz, tp, nodal, xp[:3], np.array([-1, tp.shape[0], 0], np.int32))
    assert np.all(np.isnan(bad[:2])) and np.all(np.isfinite(bad[2]))
    with pytest.raises(ValueError):
        oracle_mod.interpolate3(w.xyz, tp, nodal[:-1], xp, host)
