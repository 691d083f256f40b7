"""GPU parity of cnnsns_classify, the paper's classifier CNN (Sec. 2.3, eq. 7-8: the prediction step of
Alg. 2), against the FP64 oracle, through the C ABI.

The network's inputs are formed in FP64 and rounded to FP32 on both sides by
the same operations; the network runs in FP32 on the GPU.  Bars:
  * logits: per point, |H_gpu - H_oracle| <= 2e-5 max_l |H_oracle,l| (FP32
    accumulation over at most 512 terms in five layers; the measured error is
    about a tenth of this);
  * class: the oracle's argmax of the softmax, except where the oracle's two
    largest logits are within twice the logit bar of each other: there the
    GPU class must be one of the classes within that margin of the maximum
    (a decision FP32 cannot make the same way as FP64);
  * start: where the classes agree, the oracle's start bit for bit; elsewhere
    the overlay lookup element of the GPU class's cell (its definition);
  * the walk from the classifier's starts finds the plain walk's host (away
    from edges, bitwise; on an edge, an element that contains x_p).
"""
import numpy as np
import pytest
import torch

from exact import edge_distances

pytestmark = pytest.mark.gpu

BAR = 2e-5


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18379_amd import cnnsns
    cnnsns.lib()
    return cnnsns


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _weights(seed):
    from oracle import CLS_SHAPES
    rng = np.random.default_rng(seed)
    ws = [(rng.standard_normal(s) * np.sqrt(2.0 / np.prod(s[1:]))).astype(np.float32) for s in CLS_SHAPES]
    bs = [(0.1 * rng.standard_normal(s[0])).astype(np.float32) for s in CLS_SHAPES]
    return ws, bs


def _check(C, oracle_mod, w, xp, ws, bs, fallback=None, G=None):
    G = G or w.G
    mesh = C.Mesh(w.xy, w.tri, overlay_side=G)
    tc, nbr = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, G)
    W = C.ClsWeights(ws, bs)
    fb = None if fallback is None else _dev(fallback)
    st, cls, lg = C.classify(mesh, _dev(xp), W, fallback=fb, want_logits=True)
    torch.cuda.synchronize()
    st, cls, lg = st.cpu().numpy(), cls.cpu().numpy(), lg.cpu().numpy().astype(np.float64)
    ocls, ost, olg = oracle_mod.cls_classify(w.xy, w.tri, lk, xp, ws, bs, fallback=fallback)
    scale = np.abs(olg).max(axis=1, keepdims=True)
    err = np.abs(lg - olg) / scale
    print(f"[cls] {len(xp)} points, G={G}: logit error max {err.max():.2e} mean {err.mean():.2e} (bar {BAR})",
          flush=True)
    assert np.all(err <= BAR)
    top = np.sort(olg, axis=1)
    close = (top[:, -1] - top[:, -2]) <= 2 * BAR * scale[:, 0]
    assert np.array_equal(cls[~close], ocls[~close])
    rows = np.nonzero(close)[0]
    assert np.all(olg[rows, cls[rows]] >= top[rows, -1] - 2 * BAR * scale[rows, 0])
    same = cls == ocls
    assert np.array_equal(st[same], ost[same])
    for i in np.nonzero(~same)[0]:  # the definition of the start for the GPU's class
        cx = min(max(int(np.floor(xp[i, 0] * G)), 0), G - 1) + cls[i] % 9 - 4
        cy = min(max(int(np.floor(xp[i, 1] * G)), 0), G - 1) + cls[i] // 9 - 4
        k = lk[min(max(cy, 0), G - 1), min(max(cx, 0), G - 1)]
        assert st[i] == (k if k >= 0 else (fallback[i] if fallback is not None else 0))
    # the walk from these starts finds the host
    h, it, s = C.locate(mesh, _dev(xp), start=_dev(st))
    oh, _, _ = oracle_mod.sns(w.xy, tc, nbr, xp, w.start if fallback is None else fallback)
    h = h.cpu().numpy()
    far = edge_distances(w.xy, tc, oh, xp) > 1e-9
    assert np.array_equal(h[far], oh[far])
    mesh.close()
    return cls, ocls


@pytest.mark.parametrize("name,seed", [("c1", 1), ("c1", 2)])
def test_classifier_small(C, oracle_mod, wl, name, seed):
    w = wl.build(name)
    ws, bs = _weights(seed)
    _check(C, oracle_mod, w, w.xp, ws, bs, fallback=w.start)


def test_classifier_several_chunks(C, oracle_mod, wl):
    """70,001 points: two passes of the 65,536-point chunk, ragged 64-row tiles; a finer overlay."""
    w = wl.build(n_side=265, seed=12, field="fourier", field_seed=9, U=1.0, k=8.0, origins="nodes", G=256)
    n = 70001
    ws, bs = _weights(3)
    _check(C, oracle_mod, w, w.xp[:n], ws, bs, fallback=w.start[:n])


def test_classifier_edges_of_the_grid(C, oracle_mod, wl):
    """Points on the boundary, at the corners and outside the square (cells clamped, windows replicated);
    a coarse mesh under a fine overlay (empty pooled cells, uncovered lookup cells use the fallback)."""
    w = wl.build(n_side=12, seed=5, field="tg", field_seed=None, U=1.0, k=2.0, origins="nodes", G=64)
    extra = np.array([[0.0, 0.0], [1.0, 1.0], [1.0, 0.0], [0.0, 1.0], [-0.2, 0.5], [0.5, 1.3], [0.999, 0.001]])
    xp = np.concatenate([w.xp, extra])
    fb = np.concatenate([w.start, np.zeros(len(extra), np.int32)]).astype(np.int32)
    ws, bs = _weights(4)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=64)
    W = C.ClsWeights(ws, bs)
    st, cls, lg = C.classify(mesh, _dev(xp), W, fallback=_dev(fb), want_logits=True)
    torch.cuda.synchronize()
    tc, _ = oracle_mod.prepare_mesh(w.xy, w.tri)
    lk = oracle_mod.lookup(w.xy, tc, 64)
    ocls, ost, olg = oracle_mod.cls_classify(w.xy, w.tri, lk, xp, ws, bs, fallback=fb)
    lg = lg.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(lg - olg) <= BAR * np.abs(olg).max(axis=1, keepdims=True))
    same = cls.cpu().numpy() == ocls
    assert same.mean() > 0.99 and np.array_equal(st.cpu().numpy()[same], ost[same])
    # nothing to do for no points
    st0, _, _ = C.classify(mesh, _dev(np.zeros((0, 2))), W)
    assert st0.shape == (0,)
    mesh.close()


def test_classifier_same_bits_on_a_side_stream_and_repeated(C, wl):
    w = wl.build("c1")
    ws, bs = _weights(6)
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    W = C.ClsWeights(ws, bs)
    xp = _dev(w.xp)
    a = C.classify(mesh, xp, W, want_logits=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = C.classify(mesh, xp, W, want_logits=True, stream=s)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    mesh.close()
