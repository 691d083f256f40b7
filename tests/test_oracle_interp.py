"""Pins of the oracle's interpolation at the departure point (Sec. 2.1, after eq. 4).

The value at x_p is the P1 interpolant in the host element: its nodal basis
functions are the barycentric coordinates of Sec. 2.2.  That fixes it without
any reference output: fields linear in x and y are reproduced (to rounding),
constants are reproduced (the coordinates sum to one), a node's own value is
returned at the node, the coordinates solved independently from the 3x3
homogeneous system give the same value, and a convex field is never
under-estimated, by at most the squared element size.
"""
import numpy as np
import pytest


def _mesh_and_points(oracle_mod, wl, name="c1", n=4000, seed=0):
    w = wl.build(name, with_overlay=False) if name != "c1" else wl.build("c1")
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    rng = np.random.default_rng(seed)
    xp = rng.uniform(0.0, 1.0, size=(n, 2))
    host = oracle_mod.brute_force(w.xy, tc, xp) if w.n_tri < 5000 else None
    if host is None:
        start = np.zeros(n, np.int32)
        host, _, st = oracle_mod.sns(w.xy, tc, nbr, xp, start)
        assert np.all(st == 0)
    return w, tc, np.asarray(host, np.int32), xp


def test_linear_fields_are_reproduced(oracle_mod, wl):
    w, tc, host, xp = _mesh_and_points(oracle_mod, wl)
    rng = np.random.default_rng(1)
    a = rng.standard_normal(2)
    B = rng.standard_normal((2, 2))
    nodal = a[None, :] + w.xy @ B.T
    got = oracle_mod.interpolate(w.xy, tc, nodal, xp, host)
    want = a[None, :] + xp @ B.T
    assert np.max(np.abs(got - want)) <= 1e-13


def test_constants_are_reproduced(oracle_mod, wl):
    w, tc, host, xp = _mesh_and_points(oracle_mod, wl)
    nodal = np.tile([3.25, -0.5], (w.xy.shape[0], 1))
    got = oracle_mod.interpolate(w.xy, tc, nodal, xp, host)
    assert np.max(np.abs(got - nodal[0])) <= 8 * np.finfo(np.float64).eps * 3.25


def test_node_values_at_nodes(oracle_mod, wl):
    """At a node of the host element its own basis function is 1 and the others are exactly 0."""
    w = wl.build("c1")
    tc, _ = oracle_mod.prepare_mesh(w.xy, w.tri)
    rng = np.random.default_rng(2)
    nodal = rng.standard_normal((w.xy.shape[0], 2))
    t = np.repeat(np.arange(tc.shape[0], dtype=np.int32), 3)
    nodes = tc.reshape(-1)
    got = oracle_mod.interpolate(w.xy, tc, nodal, w.xy[nodes], t)
    want = nodal[nodes]
    # the node's own coordinate is |S_0| evaluated in another vertex order: 1 within an ulp or two
    assert np.all(np.abs(got - want) <= 4 * np.finfo(np.float64).eps * np.abs(want))
    first = np.arange(0, 3 * tc.shape[0], 3)  # vertex 0: the same expression as |S_0|, exactly 1
    assert np.array_equal(got[first], want[first])


def test_against_an_independent_solve(oracle_mod, wl):
    """Barycentric coordinates from numpy's solve of [1 1 1; x; y] lambda = [1; px; py]."""
    w, tc, host, xp = _mesh_and_points(oracle_mod, wl, n=1500, seed=3)
    rng = np.random.default_rng(4)
    nodal = rng.standard_normal((w.xy.shape[0], 2))
    got = oracle_mod.interpolate(w.xy, tc, nodal, xp, host)
    v = w.xy[tc[host]]                                   # [n][3][2]
    M = np.stack([np.ones((len(host), 3)), v[:, :, 0], v[:, :, 1]], axis=1)
    rhs = np.stack([np.ones(len(host)), xp[:, 0], xp[:, 1]], axis=1)
    lam = np.linalg.solve(M, rhs[:, :, None])[:, :, 0]
    want = np.einsum("nj,njc->nc", lam, nodal[tc[host]])
    assert np.max(np.abs(got - want)) <= 1e-11


def test_convex_field_bounds(oracle_mod, wl):
    """f = x^2 + y^2: the P1 interpolant of a convex function lies above it, by at most the
    squared longest edge of the element (sum_j lambda_j |n_j - p|^2 <= max_j |n_j - p|^2)."""
    w, tc, host, xp = _mesh_and_points(oracle_mod, wl, seed=5)
    f = (w.xy ** 2).sum(axis=1)
    nodal = np.stack([f, -f], axis=1)
    got = oracle_mod.interpolate(w.xy, tc, nodal, xp, host)
    exact = (xp ** 2).sum(axis=1)
    v = w.xy[tc[host]]
    hmax2 = np.max([((v[:, (j + 1) % 3] - v[:, j]) ** 2).sum(axis=1) for j in range(3)], axis=0)
    over = got[:, 0] - exact
    assert np.all(over >= -1e-15) and np.all(over <= hmax2 + 1e-15)
    assert np.array_equal(got[:, 1], -got[:, 0])


def test_invalid_hosts_give_nan(oracle_mod, wl):
    w = wl.build("c1")
    tc, _ = oracle_mod.prepare_mesh(w.xy, w.tri)
    nodal = np.ones((w.xy.shape[0], 2))
    xp = np.full((3, 2), 0.5)
    got = oracle_mod.interpolate(w.xy, tc, nodal, xp, np.array([-1, tc.shape[0], 0], np.int32))
    assert np.all(np.isnan(got[:2])) and np.all(np.isfinite(got[2]))
    with pytest.raises(ValueError):
        oracle_mod.interpolate(w.xy, tc, nodal[:-1], xp, np.zeros(3, np.int32))
