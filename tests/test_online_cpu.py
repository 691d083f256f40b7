"""The in-loop training harness's data preparation (paper_2412_18379_amd.online), pinned on the CPU
against the oracle: labels from SNS hosts (Sec. 2.3's B'_l), the pooled ASG grid and the classifier's
inputs, and the displacement targets on a hand-made case."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_labels_pool_and_features_match_the_oracle(oracle_mod, wl):
    from paper_2412_18379_amd import online as O
    w = wl.build(n_side=40, seed=3, field="fourier", field_seed=5, U=1.0, k=6.0, origins="nodes", G=32)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    host, _, _ = oracle_mod.sns(w.xy, tc, nbr, w.xp, w.start)
    host[::97] = -1  # not an element: no label
    xy, tri = torch.from_numpy(w.xy), torch.from_numpy(w.tri)
    cent = O.centroids_by_id(xy, tri)
    lab = O.class_labels(cent, torch.from_numpy(w.xp), torch.from_numpy(host), w.G).numpy()
    assert np.array_equal(lab, oracle_mod.cls_label(w.xp, w.G, w.xy, w.tri, host))
    pool = O.pooled_grid(cent, w.G)
    opool = oracle_mod.cls_pool(w.xy, w.tri, w.G)
    assert np.allclose(pool.numpy(), opool, rtol=0, atol=1e-15)
    feat, xoff = O.class_features(torch.from_numpy(w.xp), pool)
    ofeat, oxoff = oracle_mod.cls_features(w.xp, opool)
    assert np.allclose(feat.numpy(), ofeat, rtol=1e-6, atol=1e-6) and np.array_equal(xoff.numpy(), oxoff)


def test_displacement_targets_hand_case():
    from paper_2412_18379_amd import online as O
    # two triangles; centroids (0.2, 0.1) and (0.7, 0.6) (node ids ascending in each)
    xy = torch.tensor([[0.0, 0.0], [0.6, 0.0], [0.0, 0.3], [0.6, 0.3], [0.9, 0.9], [0.6, 0.6]], dtype=torch.float64)
    tri = torch.tensor([[0, 1, 2], [3, 4, 5]], dtype=torch.int32)
    cent = O.centroids_by_id(xy, tri)
    assert torch.allclose(cent, torch.tensor([[0.2, 0.1], [0.7, 0.6]], dtype=torch.float64))
    G = 4
    origins = torch.tensor([[0.1, 0.1], [0.2, 0.15], [0.9, 0.9], [0.6, 0.1]], dtype=torch.float64)
    host = torch.tensor([1, 0, 1, -1], dtype=torch.int32)  # the last one is left out
    t, m = O.displacement_targets(cent, origins, host, G)
    # cell (0, 0) holds the first two origins: mean of (0.6, 0.5) and (0.0, -0.05); cell (3, 3) the third
    assert m.sum() == 2 and bool(m[0, 0]) and bool(m[3, 3])
    assert np.allclose(t[:, 0, 0].numpy(), [0.3, 0.225]) and np.allclose(t[:, 3, 3].numpy(), [-0.2, -0.3])
    assert float(t[:, m.logical_not()].abs().sum()) == 0.0
