"""GPU parity of cnnsns_interpolate3d (the P1 interpolation at x_p in its host tetrahedron,
Sec. 2.1 after eq. 4) against the FP64 CPU oracle, through the C ABI.

Bar: bit for bit.  Both sides evaluate the same FP64 expressions without FMA: the walk's face
numerators, six times the volume with the nodes in ascending id, four quotients and the sum over
the nodes in ascending id.
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


def _nodal(w):
    u, v, x = w.flow(w.xyz[:, 0], w.xyz[:, 1], w.xyz[:, 2])
    return np.ascontiguousarray(np.stack([u, v, x], axis=1), dtype=np.float64)


@pytest.mark.parametrize("name", ["t1", "t2"])
def test_velocity_at_departure_points_bitwise(C, oracle_mod, wl, name):
    w = wl.build_3d(name)
    print(f"[interp3d] {name}: {w.n_tet} tetrahedra, {w.n_points} points", flush=True)
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    oh, _, os_ = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)  # the oracle's hosts, given to both sides
    xp = _dev(w.xp)
    nodal = _nodal(w)
    out = C.interpolate3d(mesh, xp, _dev(oh), _dev(nodal)).cpu().numpy()
    ref = oracle_mod.interpolate3(w.xyz, tp, nodal, w.xp, oh)
    assert np.all(os_ == C.FOUND)
    assert np.array_equal(out, ref)
    # and it is the flow itself up to the P1 error of a smooth field on elements of size dbar
    u, v, x = w.flow(w.xp[:, 0], w.xp[:, 1], w.xp[:, 2])
    assert np.max(np.abs(out - np.stack([u, v, x], axis=1))) < 0.1 * np.max(np.abs(nodal))


def test_random_fields_ragged_and_invalid_hosts(C, oracle_mod, wl):
    w = wl.build_3d("t1")
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    tp, _ = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    rng = np.random.default_rng(8)
    n = 3 * 256 + 41
    xp = rng.uniform(0.0, 1.0, size=(n, 3))
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    lk = oracle_mod.lookup3(w.xyz, tp, w.G)
    _, hh, _, _ = oracle_mod.cnnsns3(w.xyz, tp, nbr, lk, xp, xp, np.zeros((3, w.G, w.G, w.G)))
    hh = hh.copy()
    hh[[0, 9, n - 1]] = [-1, w.n_tet, -3]
    nodal = rng.standard_normal((w.xyz.shape[0], 3))
    out = C.interpolate3d(mesh, _dev(xp), _dev(hh), _dev(nodal)).cpu().numpy()
    ref = oracle_mod.interpolate3(w.xyz, tp, nodal, xp, hh)
    assert np.array_equal(out, ref, equal_nan=True)
    assert np.all(np.isnan(out[[0, 9, n - 1]])) and np.all(np.isfinite(np.delete(out, [0, 9, n - 1], axis=0)))
    lib = C.lib()
    assert lib.cnnsns_interpolate3d(mesh.handle, -1, None, None, None, None, None) == C.EINVAL
    assert lib.cnnsns_interpolate3d(mesh.handle, 4, None, None, None, None, None) == C.EINVAL
    assert lib.cnnsns_interpolate3d(None, 0, None, None, None, None, None) == C.EINVAL
    assert lib.cnnsns_interpolate3d(mesh.handle, 0, None, None, None, None, None) == C.OK
    with pytest.raises(ValueError):
        C.interpolate3d(mesh, _dev(xp), _dev(hh), _dev(nodal[:-1]))


def test_full_size_sampled(C, oracle_mod, wl):
    """5.8M tetrahedra, all 1M departure points interpolated; 20,000 sampled against the oracle."""
    w = wl.build_3d("t3")
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    tp, nbr = oracle_mod.prepare_mesh3(w.xyz, w.tet)
    oh, _, _ = oracle_mod.sns3(w.xyz, tp, nbr, w.xp, w.start)  # the oracle's hosts of all points
    xp = _dev(w.xp)
    nodal = _nodal(w)
    out = C.interpolate3d(mesh, xp, _dev(oh), _dev(nodal)).cpu().numpy()
    rng = np.random.default_rng(14)
    idx = np.concatenate([rng.integers(0, w.n_points, 20000), [0, w.n_points - 1]])
    ref = oracle_mod.interpolate3(w.xyz, tp, nodal, w.xp[idx], oh[idx])
    assert np.array_equal(out[idx], ref)
