"""In-loop training of the 3D displacement CNN from the tetrahedral walk's own output (Sec. 2.3's SNS
labels with Adam; Sec. 3.1: train on the first n_t = 3 steps, then predict) on the GPU: a drifting ABC
flow on a 48^3-node Kuhn mesh (623K tetrahedra), 5 steps, G = 64.

The trained net changes only where walks start: in a predicted step the CNN-SNS hosts equal the oracle's
plain-SNS hosts wherever the host is unique, and otherwise are tetrahedra that contain x_p; the walks are
far shorter than plain SNS."""
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


def test_in_loop_training_3d(C, oracle_mod, wl):
    from paper_2412_18379_amd import online as O
    rep = O.run3d(C, "t2", G=64, n_steps=5, n_t=3, disp_steps=1500, log=lambda m: print(m, flush=True))
    later = [s for s in rep["steps"] if s["step"] >= 3]
    assert len(later) == 2
    for s in later:
        assert s["cnn_sns_mean_path"] < 0.25 * s["plain_mean_path"]
        assert s["cnn_sns_bf16_mean_path"] < 0.25 * s["plain_mean_path"]
    # the last step's hosts from the trained net's starts against the oracle's plain walk
    cfg = wl.CONFIGS_3D["t2"]
    xyz, tet = wl.kuhn_mesh(cfg["n_side"], cfg["seed"])
    G, dt = rep["G"], rep["dt"]
    f = wl.UnsteadyABC(5, drift=0.15).at(4)
    u = np.stack(f(xyz[:, 0], xyz[:, 1], xyz[:, 2]), axis=1)
    xp = np.ascontiguousarray(np.clip(xyz - dt * u, 0.0, 1.0))
    start = wl.node_start_tets(xyz.shape[0], tet)
    mesh = C.Mesh3D(xyz, tet, overlay_side=G)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    disp = C.predict3d(mesh, dev(wl.overlay_velocity_3d(f, G)), C.Weights3D(*rep["weights"]["displacement"]), "f32")
    h, it, st = C.locate3d(mesh, dev(xp), start=dev(start), origin=dev(xyz), disp=disp)
    h, st = h.cpu().numpy(), st.cpu().numpy()
    tp, nbr = oracle_mod.prepare_mesh3(xyz, tet)
    oh, _, ost = oracle_mod.sns3(xyz, tp, nbr, xp, start)
    assert np.all(st == C.FOUND) and np.all(ost == C.FOUND)
    diff = np.nonzero(h != oh)[0]
    assert len(diff) < 0.05 * len(h)
    for hh in (h, oh):  # both contain x_p: it lies on their common boundary
        for k in diff:
            V = xyz[tp[hh[k]]]
            lam = np.linalg.solve(np.vstack([V.T, np.ones(4)]), np.append(xp[k], 1.0))
            assert lam.min() >= -1e-12
    mesh.close()
