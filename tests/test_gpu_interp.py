"""GPU parity of cnnsns_interpolate (the P1 interpolation at x_p in its host
element, Sec. 2.1 after eq. 4) against the FP64 CPU oracle, through the C ABI.

Bar: bit for bit.  Both sides evaluate the same FP64 expressions without FMA
(barycentric numerators, doubled area, three quotients, the sum in node order)
on the same counter-clockwise vertex order.  The host elements given to both
sides are the oracle's (its walks), never the GPU's.  The same holds for
cnnsns_locate_interpolate, which fuses the interpolation into the walk's last
iteration: its hosts, path lengths and statuses equal the oracle's walk, and
its values the oracle's interpolation in those hosts.
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
    u, v = w.flow(w.xy[:, 0], w.xy[:, 1])
    return np.ascontiguousarray(np.stack([u, v], axis=1), dtype=np.float64)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_velocity_at_departure_points_bitwise(C, oracle_mod, wl, name):
    w = wl.build(name)
    print(f"[interp] {name}: {w.n_tri} triangles, {w.n_points} points", flush=True)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    xp = _dev(w.xp)
    nodal = _nodal(w)
    out = C.interpolate(mesh, xp, _dev(oh), _dev(nodal)).cpu().numpy()
    ref = oracle_mod.interpolate(w.xy, tc, nodal, w.xp, oh)
    assert np.all(os_ == C.FOUND)
    assert np.array_equal(out, ref)
    # fused into the walk
    h, it, st, fo = C.locate_interpolate(mesh, xp, _dev(nodal), start=_dev(w.start))
    assert np.array_equal(h.cpu().numpy(), oh) and np.array_equal(it.cpu().numpy(), oi)
    assert np.array_equal(st.cpu().numpy(), os_) and np.array_equal(fo.cpu().numpy(), ref)
    # and it is the flow itself up to the P1 error (a smooth field, elements of size dbar)
    u, v = w.flow(w.xp[:, 0], w.xp[:, 1])
    assert np.max(np.abs(out - np.stack([u, v], axis=1))) < 0.05 * np.max(np.hypot(u, v))


def test_random_fields_unordered_points_and_invalid_hosts(C, oracle_mod, wl):
    w = wl.build("c1")
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    tc, _ = oracle_mod.prepare_mesh(w.xy, w.tri)
    rng = np.random.default_rng(7)
    n = 3 * 1024 + 37  # several blocks and a ragged tail
    xp = rng.uniform(0.0, 1.0, size=(n, 2))
    lk = oracle_mod.lookup(w.xy, tc, w.G)
    _, hh, _, _ = oracle_mod.cnnsns(w.xy, tc, oracle_mod.neighbours(w.xy.shape[0], tc), lk, xp, xp,
                                    np.zeros((2, w.G, w.G)))  # the oracle's lookup-started walks
    hh = hh.copy()
    hh[[0, 5, n - 1]] = [-1, w.n_tri, -7]  # not elements: NaN
    nodal = rng.standard_normal((w.xy.shape[0], 2))
    out = C.interpolate(mesh, _dev(xp), _dev(hh), _dev(nodal)).cpu().numpy()
    ref = oracle_mod.interpolate(w.xy, tc, nodal, xp, hh)
    assert np.array_equal(out, ref, equal_nan=True)
    assert np.all(np.isnan(out[[0, 5, n - 1]])) and np.all(np.isfinite(np.delete(out, [0, 5, n - 1], axis=0)))


def test_edge_cases(C, wl):
    w = wl.build("c1")
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    nodal = _dev(np.ones((w.xy.shape[0], 2)))
    empty = C.interpolate(mesh, _dev(np.zeros((0, 2))), _dev(np.zeros(0, np.int32)), nodal)
    assert empty.shape == (0, 2)
    with pytest.raises(ValueError):  # nodal must cover every node
        C.interpolate(mesh, _dev(np.zeros((4, 2))), _dev(np.zeros(4, np.int32)), nodal[:-1].contiguous())
    lib = C.lib()
    assert lib.cnnsns_interpolate(mesh.handle, -1, None, None, None, None, None) == C.EINVAL
    assert lib.cnnsns_interpolate(mesh.handle, 4, None, None, None, None, None) == C.EINVAL
    assert lib.cnnsns_interpolate(None, 0, None, None, None, None, None) == C.EINVAL
    assert lib.cnnsns_interpolate(mesh.handle, 0, None, None, None, None, None) == C.OK


def test_full_size_sampled(C, oracle_mod, wl):
    """16M triangles, all 8M departure points interpolated; 20,000 sampled against the oracle."""
    w = wl.build("c3", with_overlay=False)
    print(f"[interp] c3: {w.n_tri} triangles, {w.n_points} points", flush=True)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=0)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    oh, oi, os_ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)  # the oracle's hosts of all points
    xp = _dev(w.xp)
    nodal = _nodal(w)
    out = C.interpolate(mesh, xp, _dev(oh), _dev(nodal)).cpu().numpy()
    rng = np.random.default_rng(13)
    idx = np.concatenate([rng.integers(0, w.n_points, 20000), [0, w.n_points - 1]])
    ref = oracle_mod.interpolate(w.xy, tc, nodal, w.xp[idx], oh[idx])
    assert np.array_equal(out[idx], ref)
    # fused into the walk, in the launch configuration of the benchmark's plain leg
    h, it, st, fo = C.locate_interpolate(mesh, xp, _dev(nodal), start=_dev(w.start))
    assert np.array_equal(h.cpu().numpy(), oh) and np.array_equal(it.cpu().numpy(), oi)
    assert np.array_equal(st.cpu().numpy(), os_) and np.array_equal(fo.cpu().numpy()[idx], ref)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fused_walk_and_interpolation_all_start_modes(C, oracle_mod, wl, name):
    """CNN-SNS from a fixed displacement grid, the ASG start, given starts with invalid ids, a small
    iteration cap (MAXITER: the value is taken in the element moved to), a ragged count."""
    w = wl.build(name)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, w.G)
    nodal = np.random.default_rng(3).standard_normal((w.xy.shape[0], 2))
    n = w.n_points - 13
    xp, org, start = w.xp[:n], w.origins[:n], w.start[:n].copy()
    disp = (-w.dt * w.vel.astype(np.float64)).astype(np.float32)
    cases = [
        ("cnn", dict(start=_dev(start), origin=_dev(org), disp=_dev(disp)),
         lambda: oracle_mod.cnnsns(w.xy, tc, nbr, lk, org, xp, disp, fallback=start)[1:]),
        ("asg", dict(), lambda: oracle_mod.cnnsns(w.xy, tc, nbr, lk, xp, xp, np.zeros_like(disp))[1:]),
    ]
    bad = start.copy()
    bad[[1, 7, n - 2]] = [-1, w.n_tri, -5]
    cases.append(("given-bad", dict(start=_dev(bad)), lambda: oracle_mod.sns(w.xy, tc, nbr, xp, bad)))
    cases.append(("maxiter", dict(start=_dev(start), max_iter=3),
                  lambda: oracle_mod.sns(w.xy, tc, nbr, xp, start, max_iter=3)))
    for label, kw, ref_fn in cases:
        oh, oi, os_ = ref_fn()
        h, it, st, fo = C.locate_interpolate(mesh, _dev(xp), _dev(nodal), **kw)
        assert np.array_equal(h.cpu().numpy(), oh), label
        assert np.array_equal(it.cpu().numpy(), oi) and np.array_equal(st.cpu().numpy(), os_), label
        ref = oracle_mod.interpolate(w.xy, tc, nodal, xp, oh)
        assert np.array_equal(fo.cpu().numpy(), ref, equal_nan=True), label
        if label == "maxiter":
            assert np.any(os_ == C.MAXITER)
        if label == "given-bad":
            assert np.all(np.isnan(fo.cpu().numpy()[[1, 7, n - 2]]))
