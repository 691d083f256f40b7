"""Python driver for the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the slow, plain reference that the GPU library is
checked against.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library and never calls it.

Parity status of each function (what pins it, see ``tests/test_oracle_*.py``):
  canonicalise, neighbours  - invariants (symmetry, hull count, Euler formula,
                              orientation), brute-force edge matching
  sns                       - exact-rational brute-force containment over all
                              triangles; closed forms on strips and structured
                              grids; dual-graph BFS lower bound on I_t;
                              scipy/Qhull find_simplex at scale
  lookup                    - brute force over all triangles and cells in exact
                              rationals on small grids
  cnn_window / cnn_forward  - torch.nn.functional.conv2d in float64; impulse
                              responses; constructed pass-through weights
  cnnsns_start              - closed-form cells on hand-made cases
  brute_force               - exact-rational containment
  canonicalise3, neighbours3 - numpy volumes, Kuhn boundary face count,
                              symmetry, Euler characteristic of a ball
  sns3                      - numpy barycentric solve (host contains x_p, the
                              unique strict container); Kuhn closed form; ties
                              found in exact rational arithmetic
  lookup3, brute_force3     - their definitions by brute force
  cnn3_window / cnn3_forward - torch.nn.functional.conv3d in float64; impulse
                              responses; in-grid tap counts of a constant
                              input; constructed pass-through weights
  interpolate3              - linear fields, constants, node values, numpy
                              barycentric solve, convex-field bound
  cnnsns3_start             - zero displacement at cell centres gives the
                              lookup; clamping; x = 1 maps to cell G-1;
                              fallback of empty cells
  cls_pool                  - exact-rational means of the centroids per cell;
                              empty cells give their centre; independent of
                              the node order within a triangle
  cls_features              - closed forms on a structured grid (features of
                              a point at a pooled centroid, one-cell shifts,
                              the window replicated at the boundary)
  cls_forward               - the same network in torch float64 (conv2d,
                              avg_pool2d, linear, softmax); hand-built nets
                              with closed-form classes (ties to the lowest)
  cls_start, cls_label      - closed-form cells on hand-made cases
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "_oracle.so")
_lib = None

OK, EINVAL, ENOMEM, EMESH = 0, -1, -2, -4
FOUND, OUTSIDE, MAXITER, BADSTART = 0, 1, 2, 3
CHANNELS = (2, 32, 32, 32, 2)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no FMA contraction, OpenMP threads."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
                               "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        sig = {
            "orc_set_threads": [ctypes.c_int],
            "orc_canonicalise": [i64, vp, i64, vp, vp],
            "orc_neighbours": [i64, i64, vp, vp],
            "orc_sns": [i64, vp, vp, vp, i64, vp, vp, i32, vp, vp, vp],
            "orc_lookup": [i64, vp, vp, i32, vp],
            "orc_cnn_window": [i32, vp, vp, vp, vp, i64, i64, i64, i64, vp],
            "orc_cnnsns_start": [i64, vp, i32, vp, vp, vp, vp],
            "orc_brute_force": [i64, vp, vp, i64, vp, vp],
            "orc_interp": [i64, vp, vp, vp, i64, vp, vp, vp],
            "orc3_canonicalise": [i64, vp, i64, vp, vp],
            "orc3_neighbours": [i64, vp, vp],
            "orc3_sns": [i64, vp, vp, vp, i64, vp, vp, i32, vp, vp, vp],
            "orc3_lookup": [i64, vp, vp, i32, vp],
            "orc3_brute_force": [i64, vp, vp, i64, vp, vp],
            "orc3_cnn_window": [i32, vp, vp, vp, vp, vp, vp, vp],
            "orc3_interp": [i64, vp, vp, vp, i64, vp, vp, vp],
            "orc3_cnnsns_start": [i64, vp, i32, vp, vp, vp, vp],
            "orc_cls_pool": [i64, vp, i64, vp, i32, vp],
            "orc_cls_features": [i64, vp, i32, vp, vp, vp],
            "orc_cls_forward": [i64, vp, vp, vp, vp, vp, vp, vp],
            "orc_cls_start": [i64, vp, i32, vp, vp, vp, vp],
            "orc_cls_label": [i64, vp, i32, vp, i64, vp, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def set_threads(n: int = 0) -> int:
    """Set the thread count of the oracle's parallel loops (0: query)."""
    return int(_L().orc_set_threads(int(n)))


def canonicalise(xy, tri):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    out = np.empty_like(tri)
    _check(_L().orc_canonicalise(xy.shape[0], _p(xy), tri.shape[0], _p(tri), _p(out)), "canonicalise")
    return out


def neighbours(n_nodes: int, tri_ccw):
    tri_ccw = np.ascontiguousarray(tri_ccw, dtype=np.int32)
    nbr = np.empty_like(tri_ccw)
    _check(_L().orc_neighbours(int(n_nodes), tri_ccw.shape[0], _p(tri_ccw), _p(nbr)), "neighbours")
    return nbr


def prepare_mesh(xy, tri):
    """(counter-clockwise triangles, neighbour table) of a mesh."""
    tc = canonicalise(xy, tri)
    return tc, neighbours(np.asarray(xy).shape[0], tc)


def sns(xy, tri_ccw, nbr, xp, start, max_iter: int = 0):
    """Alg. 1 for every point: (host, iters, status)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    start = np.ascontiguousarray(start, dtype=np.int32)
    n = xp.shape[0]
    host = np.empty(n, np.int32)
    iters = np.empty(n, np.int32)
    status = np.empty(n, np.uint8)
    _check(_L().orc_sns(tri_ccw.shape[0], _p(xy), _p(tri_ccw), _p(nbr), n, _p(xp), _p(start), int(max_iter),
                        _p(host), _p(iters), _p(status)), "sns")
    return host, iters, status


def interpolate(xy, tri_ccw, nodal, xp, host):
    """P1 interpolation of a two-component nodal field at xp in the host elements (Sec. 2.1,
    after eq. 4): FP64 [n][2], NaN where the host id is not an element."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri_ccw = np.ascontiguousarray(tri_ccw, dtype=np.int32)
    nodal = np.ascontiguousarray(nodal, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    host = np.ascontiguousarray(host, dtype=np.int32)
    if nodal.shape != (xy.shape[0], 2) or xp.ndim != 2 or xp.shape[1] != 2 or host.shape != (xp.shape[0],):
        raise ValueError("interpolate: nodal [n_nodes][2], xp [n][2] and host [n] expected")
    out = np.empty((xp.shape[0], 2), np.float64)
    _check(_L().orc_interp(tri_ccw.shape[0], _p(xy), _p(tri_ccw), _p(nodal), xp.shape[0], _p(xp), _p(host),
                           _p(out)), "interpolate")
    return out


def lookup(xy, tri_ccw, G: int):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    out = np.empty((G, G), np.int32)
    _check(_L().orc_lookup(tri_ccw.shape[0], _p(xy), _p(tri_ccw), int(G), _p(out)), "lookup")
    return out


def cnn_window(vel, ws, bs, r0: int, c0: int, h: int, w: int):
    """Four-layer CNN output on rows [r0, r0+h) x cols [c0, c0+w): FP64 [C_out][h][w]."""
    vel = np.ascontiguousarray(vel, dtype=np.float32)
    G = vel.shape[-1]
    ws = [np.ascontiguousarray(x, dtype=np.float32) for x in ws]
    bs = [np.ascontiguousarray(x, dtype=np.float32) for x in bs]
    chan = np.array([ws[0].shape[1]] + [x.shape[0] for x in ws], dtype=np.int32)
    wp = (ctypes.c_void_p * 4)(*[x.ctypes.data for x in ws])
    bp = (ctypes.c_void_p * 4)(*[x.ctypes.data for x in bs])
    out = np.empty((chan[4], h, w), np.float64)
    _check(_L().orc_cnn_window(G, _p(vel), _p(chan), wp, bp, r0, c0, h, w, _p(out)), "cnn_window")
    return out


def cnn_forward(vel, ws, bs):
    G = vel.shape[-1]
    return cnn_window(vel, ws, bs, 0, 0, G, G)


def cnn_pixels(vel, ws, bs, rows, cols):
    """CNN output at individual pixels: FP64 [len(rows)][C_out]."""
    out = np.empty((len(rows), ws[-1].shape[0]), np.float64)
    for k, (r, c) in enumerate(zip(rows, cols)):
        out[k] = cnn_window(vel, ws, bs, int(r), int(c), 1, 1)[:, 0, 0]
    return out


def cnnsns_start(origin, disp, lookup_grid, fallback=None):
    """Alg. 2 start element from the predicted displacement (FP64 [2][G][G])."""
    origin = np.ascontiguousarray(origin, dtype=np.float64)
    disp = np.ascontiguousarray(disp, dtype=np.float64)
    lk = np.ascontiguousarray(lookup_grid, dtype=np.int32)
    fb = None if fallback is None else np.ascontiguousarray(fallback, dtype=np.int32)
    n = origin.shape[0]
    out = np.empty(n, np.int32)
    _check(_L().orc_cnnsns_start(n, _p(origin), lk.shape[0], _p(disp), _p(lk), _p(fb), _p(out)), "cnnsns_start")
    return out


def brute_force(xy, tri_ccw, xp):
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    host = np.empty(xp.shape[0], np.int32)
    _check(_L().orc_brute_force(tri_ccw.shape[0], _p(xy), _p(tri_ccw), xp.shape[0], _p(xp), _p(host)),
           "brute_force")
    return host


def cnnsns(xy, tri_ccw, nbr, lookup_grid, origin, xp, disp, fallback=None, max_iter: int = 0):
    """Alg. 2 end to end from a given displacement grid: (start, host, iters, status)."""
    st = cnnsns_start(origin, disp, lookup_grid, fallback)
    h, it, s = sns(xy, tri_ccw, nbr, xp, st, max_iter)
    return st, h, it, s


# ---------------------------------------------------------------------------- metrics

def element_centroids(xy, tri):
    xy = np.asarray(xy)
    return (xy[tri[:, 0]] + xy[tri[:, 1]] + xy[tri[:, 2]]) / 3.0


def err_metric(xy, tri, start, host):
    """Distance between the centroids of the start element and the host (Sec. 3.1)."""
    c = element_centroids(xy, tri)
    return np.hypot(*(c[host] - c[start]).T)


def opt(c_sns: float, c_cnnsns: float) -> float:
    """Optimisation rate (C(SNS) - C(CNN-SNS)) / C(SNS) (Sec. 3.1)."""
    return (c_sns - c_cnnsns) / c_sns


# ----------------------------------------------------------------------------- 3D (tetrahedra)

def canonicalise3(xyz, tet):
    """Tetrahedra in positive orientation (3rd and 4th vertex swapped where negative)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tet = np.ascontiguousarray(tet, dtype=np.int32)
    out = np.empty_like(tet)
    _check(_L().orc3_canonicalise(xyz.shape[0], _p(xyz), tet.shape[0], _p(tet), _p(out)), "canonicalise3")
    return out


def neighbours3(tet_pos):
    tet_pos = np.ascontiguousarray(tet_pos, dtype=np.int32)
    nbr = np.empty_like(tet_pos)
    _check(_L().orc3_neighbours(tet_pos.shape[0], _p(tet_pos), _p(nbr)), "neighbours3")
    return nbr


def prepare_mesh3(xyz, tet):
    """(positively oriented tetrahedra, neighbour table) of a tetrahedral mesh."""
    tp = canonicalise3(xyz, tet)
    return tp, neighbours3(tp)


def sns3(xyz, tet_pos, nbr, xp, start, max_iter: int = 0):
    """Alg. 1 on a tetrahedral mesh for every point: (host, iters, status)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    start = np.ascontiguousarray(start, dtype=np.int32)
    n = xp.shape[0]
    host, iters, status = np.empty(n, np.int32), np.empty(n, np.int32), np.empty(n, np.uint8)
    _check(_L().orc3_sns(tet_pos.shape[0], _p(xyz), _p(tet_pos), _p(nbr), n, _p(xp), _p(start), int(max_iter),
                         _p(host), _p(iters), _p(status)), "sns3")
    return host, iters, status


def lookup3(xyz, tet_pos, G: int):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    out = np.empty((G, G, G), np.int32)
    _check(_L().orc3_lookup(tet_pos.shape[0], _p(xyz), _p(tet_pos), int(G), _p(out)), "lookup3")
    return out


def brute_force3(xyz, tet_pos, xp):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    host = np.empty(xp.shape[0], np.int32)
    _check(_L().orc3_brute_force(tet_pos.shape[0], _p(xyz), _p(tet_pos), xp.shape[0], _p(xp), _p(host)),
           "brute_force3")
    return host


def cnn3_window(vel, ws, bs, origin3, size3):
    """Four-layer 3D CNN output on the window [z0, z0+d) x [y0, y0+h) x [x0, x0+w) of the G^3 grid:
    FP64 [C_out][d][h][w].  vel FP32 [C_in][G][G][G]; ws[l] FP32 [C_out][C_in][3][3][3]."""
    vel = np.ascontiguousarray(vel, dtype=np.float32)
    G = vel.shape[-1]
    ws = [np.ascontiguousarray(x, dtype=np.float32) for x in ws]
    bs = [np.ascontiguousarray(x, dtype=np.float32) for x in bs]
    chan = np.array([ws[0].shape[1]] + [x.shape[0] for x in ws], dtype=np.int32)
    wp = (ctypes.c_void_p * 4)(*[x.ctypes.data for x in ws])
    bp = (ctypes.c_void_p * 4)(*[x.ctypes.data for x in bs])
    o3 = np.ascontiguousarray(origin3, dtype=np.int64)
    s3 = np.ascontiguousarray(size3, dtype=np.int64)
    out = np.empty((chan[4], *[int(v) for v in s3]), np.float64)
    _check(_L().orc3_cnn_window(G, _p(vel), _p(chan), wp, bp, _p(o3), _p(s3), _p(out)), "cnn3_window")
    return out


def cnn3_forward(vel, ws, bs):
    G = vel.shape[-1]
    return cnn3_window(vel, ws, bs, (0, 0, 0), (G, G, G))


def cnnsns3_start(origin, disp, lookup_grid, fallback=None):
    """Alg. 2 start element in 3D from the predicted displacement (FP64 [3][G][G][G])."""
    origin = np.ascontiguousarray(origin, dtype=np.float64)
    disp = np.ascontiguousarray(disp, dtype=np.float64)
    lk = np.ascontiguousarray(lookup_grid, dtype=np.int32)
    fb = None if fallback is None else np.ascontiguousarray(fallback, dtype=np.int32)
    n = origin.shape[0]
    out = np.empty(n, np.int32)
    _check(_L().orc3_cnnsns_start(n, _p(origin), lk.shape[0], _p(disp), _p(lk), _p(fb), _p(out)), "cnnsns3_start")
    return out


def cnnsns3(xyz, tet_pos, nbr, lookup_grid, origin, xp, disp, fallback=None, max_iter: int = 0):
    """Alg. 2 end to end on tetrahedra from a given displacement grid: (start, host, iters, status)."""
    st = cnnsns3_start(origin, disp, lookup_grid, fallback)
    h, it, s = sns3(xyz, tet_pos, nbr, xp, st, max_iter)
    return st, h, it, s


def interpolate3(xyz, tet_pos, nodal, xp, host):
    """P1 interpolation of a nodal field FP64 [n_nodes][3] at the points in their host tetrahedra."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    nodal = np.ascontiguousarray(nodal, dtype=np.float64)
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    host = np.ascontiguousarray(host, dtype=np.int32)
    if nodal.shape != (xyz.shape[0], 3):
        raise ValueError("nodal must be [n_nodes][3]")
    out = np.empty((xp.shape[0], 3), np.float64)
    _check(_L().orc3_interp(tet_pos.shape[0], _p(xyz), _p(tet_pos), _p(nodal), xp.shape[0], _p(xp), _p(host),
                            _p(out)), "interpolate3")
    return out


# ---------------------------------------------------------------------------- the classifier CNN (Sec. 2.3)

CLS_W, CLS_NA = 9, 81
CLS_SHAPES = [(16, 2, 3, 3), (16, 16, 3, 3), (256, 2), (256, 256), (512, 512), (81, 512)]


def cls_pool(xy, tri, G: int):
    """Average-pooled ASG grid [G][G][2]: per overlay cell the mean centroid of the elements whose centroid
    lies in it (ascending element id), or the cell centre."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    out = np.empty((G, G, 2), np.float64)
    _check(_L().orc_cls_pool(xy.shape[0], _p(xy), tri.shape[0], _p(tri), int(G), _p(out)), "cls_pool")
    return out


def cls_features(xp, pool):
    """Network inputs: feat FP32 [n][2][9][9] (G (pooled centroid - x_p) over the 9 x 9 window) and xoff FP32
    [n][2] (x_p's offset in its cell)."""
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    pool = np.ascontiguousarray(pool, dtype=np.float64)
    n, G = xp.shape[0], pool.shape[0]
    feat = np.empty((n, 2, CLS_W, CLS_W), np.float32)
    xoff = np.empty((n, 2), np.float32)
    _check(_L().orc_cls_features(n, _p(xp), int(G), _p(pool), _p(feat), _p(xoff)), "cls_features")
    return feat, xoff


def cls_forward(feat, xoff, ws, bs):
    """(logits FP64 [n][81], probabilities FP64 [n][81], class int32 [n])."""
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    xoff = np.ascontiguousarray(xoff, dtype=np.float32)
    ws = [np.ascontiguousarray(x, dtype=np.float32) for x in ws]
    bs = [np.ascontiguousarray(x, dtype=np.float32) for x in bs]
    if [tuple(w.shape) for w in ws] != CLS_SHAPES or [b.shape[0] for b in bs] != [s[0] for s in CLS_SHAPES]:
        raise ValueError("cls_forward: weights of the 2-16-16 conv / 2-256-256 / 512-512-81 net expected")
    n = feat.shape[0]
    wp = (ctypes.c_void_p * 6)(*[x.ctypes.data for x in ws])
    bp = (ctypes.c_void_p * 6)(*[x.ctypes.data for x in bs])
    logits = np.empty((n, CLS_NA), np.float64)
    prob = np.empty((n, CLS_NA), np.float64)
    cls = np.empty(n, np.int32)
    _check(_L().orc_cls_forward(n, _p(feat), _p(xoff), wp, bp, _p(logits), _p(prob), _p(cls)), "cls_forward")
    return logits, prob, cls


def cls_start(xp, lookup_grid, cls, fallback=None):
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    lk = np.ascontiguousarray(lookup_grid, dtype=np.int32)
    cls = np.ascontiguousarray(cls, dtype=np.int32)
    fb = None if fallback is None else np.ascontiguousarray(fallback, dtype=np.int32)
    out = np.empty(xp.shape[0], np.int32)
    _check(_L().orc_cls_start(xp.shape[0], _p(xp), lk.shape[0], _p(lk), _p(cls), _p(fb), _p(out)), "cls_start")
    return out


def cls_label(xp, G: int, xy, tri, host):
    """Training labels from SNS hosts: the window class of the cell holding the host's centroid."""
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    host = np.ascontiguousarray(host, dtype=np.int32)
    out = np.empty(xp.shape[0], np.int32)
    _check(_L().orc_cls_label(xp.shape[0], _p(xp), int(G), _p(xy), tri.shape[0], _p(tri), _p(host), _p(out)),
           "cls_label")
    return out


def cls_classify(xy, tri, lookup_grid, xp, ws, bs, fallback=None):
    """The classifier's prediction step of Alg. 2 end to end: (class, K_p, logits)."""
    G = lookup_grid.shape[0]
    feat, xoff = cls_features(xp, cls_pool(xy, tri, G))
    logits, _, cls = cls_forward(feat, xoff, ws, bs)
    return cls, cls_start(xp, lookup_grid, cls, fallback), logits
