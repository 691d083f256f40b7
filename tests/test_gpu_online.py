"""In-loop training from the walk's own output on the GPU (Sec. 2.3 labels and Adam; Sec. 3.1: train on
the first n_t = 3 steps, then predict): a time-dependent flow on a 45K-triangle mesh, 6 steps.

The trained predictors change only where walks start, never the hosts: in the predicted steps the hosts
of CNN-SNS with either trained net equal the oracle's plain-SNS hosts (away from edges bit for bit, on
an edge an element containing x_p), and both shorten the walks well below plain SNS."""
import numpy as np
import pytest
import torch

from exact import edge_distances

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18379_amd import cnnsns
    cnnsns.lib()
    return cnnsns


def test_in_loop_training(C, oracle_mod, wl):
    from paper_2412_18379_amd import online as O
    rep = O.run(C, n_side=150, seed=4, field_seed=31, k=12.0, G=128, n_steps=6, n_t=3, disp_steps=300,
                cls_steps=600, log=lambda m: print(m, flush=True))
    later = [s for s in rep["steps"] if s["step"] >= 3]
    assert len(later) == 3
    for s in later:
        assert s["cnn_sns_mean_path"] < 0.5 * s["plain_mean_path"]
        assert s["classifier_mean_path"] < 0.5 * s["plain_mean_path"]
    # hosts at the last step against the oracle, from the trained nets' starts
    xy, tri = wl.mesh(150, 4)
    G = rep["G"]
    f = wl.UnsteadyFourier(31, U=1.0, norm_G=G, drift=0.15).at(5)
    xp = wl.departure_points(xy, f, rep["dt"])
    start = wl.node_start_elements(xy.shape[0], tri)
    mesh = C.Mesh(xy, tri, overlay_side=G)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    disp = C.predict(mesh, dev(wl.overlay_velocity(f, G)), C.Weights(*rep["weights"]["displacement"]), "f32")
    hd, _, _ = C.locate(mesh, dev(xp), start=dev(start), origin=dev(xy), disp=disp)
    st, _, _ = C.classify(mesh, dev(xp), C.ClsWeights(*rep["weights"]["classifier"]), fallback=dev(start))
    hc, _, _ = C.locate(mesh, dev(xp), start=st)
    tc, nbr = oracle_mod.prepare_mesh(xy, tri)
    oh, _, _ = oracle_mod.sns(xy, tc, nbr, xp, start)
    far = edge_distances(xy, tc, oh, xp) > 1e-9
    for h in (hd.cpu().numpy(), hc.cpu().numpy()):
        assert np.array_equal(h[far], oh[far])
        near = np.nonzero(~far)[0]
        if len(near):
            assert np.all(oracle_mod.brute_force(xy, tc, xp[near]) >= 0)
    mesh.close()
