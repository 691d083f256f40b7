"""GPU tests of the serving loop (cnnsns_server_* / cnnsns_submit).

Each job's result (host elements and path lengths) must be bitwise the same
when the job runs alone (cnnsns_predict + cnnsns_locate) and when it runs
inside a mix of jobs on meshes of uneven size that are admitted by device
footprint and overlap on the GPU.
"""
import numpy as np
import pytest
import torch

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the serving loop is switched off: GPU runs of it (this test once, the 64-mesh "
                            "served-mix benchmark once) ended in a host segmentation fault whose cause has not "
                            "been found"),
]


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18379_amd import cnnsns
    cnnsns.lib()
    return cnnsns


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def mix(C, wl):
    """Six meshes of 1.6k to 160k triangles, each with its own flow; CNN weights He-initialised."""
    specs = [(30, 31, 1.0), (90, 32, 2.5), (150, 33, 0.7), (60, 34, 4.0), (283, 35, 1.5), (45, 36, 3.0)]
    out = []
    for n_side, seed, U in specs:
        w = wl.build(n_side=n_side, seed=seed, field="fourier", field_seed=seed + 100, U=U, k=20.0, origins="nodes")
        mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
        out.append(dict(w=w, mesh=mesh, xp=_dev(w.xp), origin=_dev(w.origins), vel=_dev(w.vel)))
    ws, bs = wl.random_weights(9)
    return out, C.Weights(ws, bs)


def _alone(C, job, W, precision):
    disp = C.predict(job["mesh"], job["vel"], W, precision)
    h, it, _ = C.locate(job["mesh"], job["xp"], origin=job["origin"], disp=disp)
    torch.cuda.synchronize()
    return h.cpu().numpy(), it.cpu().numpy()


@pytest.mark.parametrize("precision,budget_mb,inflight", [("bf16", 256, 4), ("bf16", 3, 2), ("f32", 40, 3)])
def test_alone_equals_mix(C, mix, precision, budget_mb, inflight):
    jobs, W = mix
    ref = [_alone(C, j, W, precision) for j in jobs]
    srv = C.Server(W, hbm_budget_bytes=budget_mb << 20, max_inflight=inflight, queue_depth=4096, precision=precision)
    order = [k % len(jobs) for k in range(30)]
    outs, ids = [], []
    for k in order:
        j = jobs[k]
        h = torch.full((j["w"].n_points,), -7, dtype=torch.int32, device="cuda")
        it = torch.zeros(j["w"].n_points, dtype=torch.int32, device="cuda")
        ids.append(srv.submit(j["mesh"], j["vel"], j["xp"], j["origin"], h, it))
        outs.append((k, h, it))
    lat = [srv.wait(i) for i in ids]
    srv.close()
    assert all(l > 0 for l in lat)
    for k, h, it in outs:
        assert np.array_equal(h.cpu().numpy(), ref[k][0])
        assert np.array_equal(it.cpu().numpy(), ref[k][1])


def test_poll_and_errors(C, mix):
    jobs, W = mix
    j = jobs[4]
    G = j["mesh"].G
    # a job whose displacement grid alone exceeds the budget can never be admitted
    srv = C.Server(W, hbm_budget_bytes=2 * 4 * G * G - 1, max_inflight=1, queue_depth=8, precision="bf16")
    h = torch.empty(j["w"].n_points, dtype=torch.int32, device="cuda")
    with pytest.raises(C.CnnsnsError) as e:
        srv.submit(j["mesh"], j["vel"], j["xp"], j["origin"], h)
    assert e.value.code == C.ENOMEM
    srv.close()
    # a full queue refuses submissions with EBUSY; accepted jobs still complete
    srv = C.Server(W, hbm_budget_bytes=64 << 20, max_inflight=1, queue_depth=1, precision="bf16")
    accepted, busy = [], 0
    for _ in range(40):
        h = torch.empty(j["w"].n_points, dtype=torch.int32, device="cuda")
        try:
            accepted.append((srv.submit(j["mesh"], j["vel"], j["xp"], j["origin"], h), h))
        except C.CnnsnsError as err:
            assert err.code == C.EBUSY
            busy += 1
    assert busy > 0 and len(accepted) > 0
    for jid, h in accepted:
        while srv.poll(jid) is None:
            pass
    srv.close()
    # invalid arguments
    with pytest.raises(C.CnnsnsError) as e:
        C.Server(W, hbm_budget_bytes=0)
    assert e.value.code == C.EINVAL
    with pytest.raises(C.CnnsnsError) as e:
        C.Server(W, hbm_budget_bytes=1 << 20, precision="fp8")
    assert e.value.code == C.EINVAL
