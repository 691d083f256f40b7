"""Seeded synthetic workloads for 2D CNN-SNS particle location.

The paper runs its tracker inside an L-G flow solver on 3D tetrahedral meshes
(Sec. 3); none of those meshes, flows or trained networks are available, so
every input here is synthetic and seeded: a Delaunay triangulation of a
jittered point grid on the unit square (optionally graded toward the centre),
an analytic divergence-free velocity field, departure points from the
first-order trajectory step of eq. (3) and the start elements the plain SNS
method uses (the host element before movement, Sec. 2.2).

This module only *makes inputs*.  It holds none of the point-location
arithmetic (barycentric tests, walk, overlay lookup, CNN) and is shared by the
GPU library's callers and by the checker alike.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field as dc_field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "meshgen.c")
_SO = os.path.join(_HERE, "_meshgen.so")
_lib = None


def build_meshgen(force: bool = True) -> str:
    """Compile the mesh-generation helper with gcc (host code only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _meshgen():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_meshgen(force=True)
        lib = ctypes.CDLL(_SO)
        lib.mg_triangulate_grid.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        lib.mg_triangulate_grid.restype = ctypes.c_int
        lib.mg_lawson.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_int64)]
        lib.mg_lawson.restype = ctypes.c_int
        _lib = lib
    return _lib


# ----------------------------------------------------------------------------- meshes

def jittered_grid(n: int, seed: int, jitter: float = 0.25, graded: bool = False) -> np.ndarray:
    """n*n points on [0,1]^2, node (i, j) at index j*n + i (x index i).

    Interior points move by U(-jitter*h, +jitter*h) per axis (h = 1/(n-1));
    points on an edge of the square move only along that edge; corners stay.
    With ``graded`` the points are then pushed through the L-infinity radial
    map rho' = 0.4 rho + 1.2 rho^2 about the centre (rho = |x - 1/2|_inf), which
    keeps the square's boundary and makes the spacing 0.4x at the centre and
    1.6x at the edge: a linear density ratio of 4 between centre and edge.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    g = np.arange(n, dtype=np.float64) * h
    X, Y = np.meshgrid(g, g, indexing="xy")  # X[j, i] = i*h
    jx = rng.uniform(-jitter, jitter, size=(n, n)) * h
    jy = rng.uniform(-jitter, jitter, size=(n, n)) * h
    jx[:, 0] = 0.0
    jx[:, -1] = 0.0
    jy[0, :] = 0.0
    jy[-1, :] = 0.0
    X = X + jx
    Y = Y + jy
    # exact boundary values
    X[:, 0] = 0.0
    X[:, -1] = 1.0
    Y[0, :] = 0.0
    Y[-1, :] = 1.0
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    if graded:
        d = xy - 0.5
        rho = np.max(np.abs(d), axis=1)
        scale = np.ones_like(rho)
        nz = rho > 0
        scale[nz] = (0.4 * rho[nz] + 1.2 * rho[nz] ** 2) / rho[nz]
        on_x0, on_x1 = X.ravel() == 0.0, X.ravel() == 1.0
        on_y0, on_y1 = Y.ravel() == 0.0, Y.ravel() == 1.0
        xy = 0.5 + d * scale[:, None]
        # keep boundary points exactly on the boundary
        xy[on_x0, 0] = 0.0
        xy[on_x1, 0] = 1.0
        xy[on_y0, 1] = 0.0
        xy[on_y1, 1] = 1.0
    return np.ascontiguousarray(xy)


def triangulate_grid(n: int, xy: np.ndarray, delaunay: bool = True) -> np.ndarray:
    """CCW triangles of the n x n point grid, made Delaunay by Lawson flips."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    nt = 2 * (n - 1) ** 2
    tri = np.empty((nt, 3), dtype=np.int32)
    lib = _meshgen()
    rc = lib.mg_triangulate_grid(n, xy.ctypes.data, tri.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"mg_triangulate_grid failed ({rc})")
    if delaunay:
        nflips = ctypes.c_int64(0)
        rc = lib.mg_lawson(xy.shape[0], xy.ctypes.data, nt, tri.ctypes.data, ctypes.byref(nflips))
        if rc != 0:
            raise RuntimeError(f"mg_lawson failed ({rc})")
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    if not np.all(area2 > 0):
        raise RuntimeError("generated triangulation has non-positive triangles")
    return tri


def mesh(n: int, seed: int, graded: bool = False, jitter: float = 0.25):
    xy = jittered_grid(n, seed, jitter=jitter, graded=graded)
    tri = triangulate_grid(n, xy)
    return xy, tri


def longest_edges(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    e = np.stack([np.hypot(*(b - a).T), np.hypot(*(c - b).T), np.hypot(*(a - c).T)], axis=1)
    return e.max(axis=1)


def mean_diameter(xy: np.ndarray, tri: np.ndarray) -> float:
    """Mean over triangles of the longest edge (the element diameter)."""
    return float(longest_edges(xy, tri).mean())


def centroids(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray((xy[tri[:, 0]] + xy[tri[:, 1]] + xy[tri[:, 2]]) / 3.0)


def node_start_elements(n_nodes: int, tri: np.ndarray) -> np.ndarray:
    """For every node, the smallest id of a triangle incident to it (-1 if none)."""
    big = np.iinfo(np.int32).max
    s = np.full(n_nodes, big, dtype=np.int64)
    ids = np.repeat(np.arange(tri.shape[0], dtype=np.int64), 3)
    np.minimum.at(s, tri.ravel().astype(np.int64), ids)
    s[s == big] = -1
    return s.astype(np.int32)


# ----------------------------------------------------------------------------- velocity fields

class TaylorGreen:
    """u = U sin(pi x) cos(pi y), v = -U cos(pi x) sin(pi y)."""

    def __init__(self, U: float = 1.0):
        self.U = float(U)

    def __call__(self, x, y):
        u = self.U * np.sin(np.pi * x) * np.cos(np.pi * y)
        v = -self.U * np.cos(np.pi * x) * np.sin(np.pi * y)
        return u, v

    def grid(self, G: int):
        c = (np.arange(G, dtype=np.float64) + 0.5) / G
        sx, cx = np.sin(np.pi * c), np.cos(np.pi * c)
        u = self.U * cx[:, None] * sx[None, :]  # [y, x]: sin(pi x) cos(pi y)
        v = -self.U * sx[:, None] * cx[None, :]
        return u, v


class FourierVortices:
    """Stream function psi = sum_k a_k sin(pi m_k x + phi_k) sin(pi n_k y + theta_k),
    u = d psi / dy, v = -d psi / dx (divergence-free), with m_k, n_k in {1..4},
    a_k ~ N(0,1), phases ~ U[0, 2 pi).  The field is scaled so that the maximum
    speed over the cell centres of a ``norm_G`` x ``norm_G`` grid equals U."""

    def __init__(self, seed: int, U: float = 1.0, n_modes: int = 8, norm_G: int = 1024):
        rng = np.random.default_rng(seed)
        self.a = rng.standard_normal(n_modes)
        self.m = rng.integers(1, 5, size=n_modes).astype(np.float64)
        self.n = rng.integers(1, 5, size=n_modes).astype(np.float64)
        self.phi = rng.uniform(0, 2 * np.pi, size=n_modes)
        self.theta = rng.uniform(0, 2 * np.pi, size=n_modes)
        self.scale = 1.0
        u, v = self.grid(norm_G)
        self.scale = float(U) / float(np.sqrt(u * u + v * v).max())

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        u = np.zeros(np.broadcast(x, y).shape)
        v = np.zeros_like(u)
        for a, m, n, p, t in zip(self.a, self.m, self.n, self.phi, self.theta):
            X = np.pi * m * x + p
            Y = np.pi * n * y + t
            u += a * np.sin(X) * (np.pi * n) * np.cos(Y)
            v -= a * (np.pi * m) * np.cos(X) * np.sin(Y)
        return u * self.scale, v * self.scale

    def grid(self, G: int):
        c = (np.arange(G, dtype=np.float64) + 0.5) / G
        u = np.zeros((G, G))
        v = np.zeros((G, G))
        for a, m, n, p, t in zip(self.a, self.m, self.n, self.phi, self.theta):
            sX, cX = np.sin(np.pi * m * c + p), np.cos(np.pi * m * c + p)
            sY, cY = np.sin(np.pi * n * c + t), np.cos(np.pi * n * c + t)
            u += a * (np.pi * n) * np.outer(cY, sX)  # [y, x]
            v -= a * (np.pi * m) * np.outer(sY, cX)
        return u * self.scale, v * self.scale


class UnsteadyFourier:
    """A time-dependent flow: the Fourier vortices of FourierVortices(seed) whose phases drift by
    omega_k * drift radians per time step (omega_k ~ U[0.5, 1.5], drawn from seed + 1), with the
    normalisation of step 0 kept (so the speed scale stays near U)."""

    def __init__(self, seed: int, U: float = 1.0, norm_G: int = 1024, drift: float = 0.15):
        self.base = FourierVortices(seed, U=U, norm_G=norm_G)
        rng = np.random.default_rng(seed + 1)
        n = len(self.base.a)
        self.w_phi = rng.uniform(0.5, 1.5, size=n) * drift
        self.w_theta = rng.uniform(0.5, 1.5, size=n) * drift

    def at(self, step: int) -> "FourierVortices":
        f = FourierVortices.__new__(FourierVortices)
        f.a, f.m, f.n, f.scale = self.base.a, self.base.m, self.base.n, self.base.scale
        f.phi = self.base.phi + self.w_phi * step
        f.theta = self.base.theta + self.w_theta * step
        return f


def overlay_velocity(field, G: int) -> np.ndarray:
    """(u, v) at the cell centres ((cx+1/2)/G, (cy+1/2)/G), float32 [2][G][G] (channel, y, x)."""
    u, v = field.grid(G)
    return np.ascontiguousarray(np.stack([u, v]).astype(np.float32))


def departure_points(origins: np.ndarray, field, dt: float) -> np.ndarray:
    """First-order departure point x - dt u(x) (eq. 3), clamped into the unit square."""
    u, v = field(origins[:, 0], origins[:, 1])
    xp = np.stack([origins[:, 0] - dt * u, origins[:, 1] - dt * v], axis=1)
    return np.ascontiguousarray(np.clip(xp, 0.0, 1.0))


def overlay_side_for(n_tri: int) -> int:
    return 1 << int(math.ceil(math.log2(math.sqrt(n_tri))))


# ----------------------------------------------------------------------------- configurations

@dataclass
class Workload:
    name: str
    n_side: int
    xy: np.ndarray          # float64 [N_v][2]
    tri: np.ndarray         # int32 [N_t][3] (CCW as generated)
    origins: np.ndarray     # float64 [n][2]  x_i (positions before movement)
    xp: np.ndarray          # float64 [n][2]  departure points x_p
    start: np.ndarray       # int32 [n]       K_m, the host element before movement
    G: int                  # overlay side
    vel: Optional[np.ndarray]  # float32 [2][G][G]
    dt: float
    dbar: float             # mean element diameter
    flow: object = None
    seeds: dict = dc_field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return int(self.xp.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])


CONFIGS = {
    # name: (n_side, mesh seed, graded, field kind, field seed, U, k diameters, origins, G)
    "c1": dict(n_side=32, seed=1, graded=False, field="tg", field_seed=None, U=1.0, k=3.0,
               origins="nodes", G=64),
    "c2": dict(n_side=708, seed=2, graded=False, field="fourier", field_seed=20, U=1.0, k=20.0,
               origins="centroids", G=1024),
    "c3": dict(n_side=2829, seed=3, graded=True, field="fourier", field_seed=30, U=1.0, k=150.0,
               origins="nodes", G=4096),
}
CONFIGS["c4"] = dict(CONFIGS["c2"])


def make_field(kind: str, field_seed, U: float, G: int):
    if kind == "tg":
        return TaylorGreen(U)
    return FourierVortices(field_seed, U=U, norm_G=G)


def build(name: str = None, *, n_side: int = None, seed: int = None, graded: bool = False,
          field: str = "fourier", field_seed: int = 0, U: float = 1.0, k: float = 20.0,
          origins: str = "nodes", G: int = None, with_overlay: bool = True) -> Workload:
    """Build one workload, either a named configuration or from explicit knobs."""
    if name is not None:
        cfg = dict(CONFIGS[name])
        n_side, seed, graded = cfg["n_side"], cfg["seed"], cfg["graded"]
        field, field_seed, U, k = cfg["field"], cfg["field_seed"], cfg["U"], cfg["k"]
        origins, G = cfg["origins"], cfg["G"]
    xy, tri = mesh(n_side, seed, graded=graded)
    if G is None:
        G = overlay_side_for(tri.shape[0])
    fld = make_field(field, field_seed, U, G)
    if origins == "nodes":
        org = xy
        start = node_start_elements(xy.shape[0], tri)
    elif origins == "centroids":
        org = centroids(xy, tri)
        start = np.arange(tri.shape[0], dtype=np.int32)
    else:
        raise ValueError(origins)
    dbar = mean_diameter(xy, tri)
    u, v = fld(org[:, 0], org[:, 1])
    dt = k * dbar / float(np.mean(np.hypot(u, v)))
    xp = departure_points(org, fld, dt)
    vel = overlay_velocity(fld, G) if with_overlay else None
    return Workload(name=name or "custom", n_side=n_side, xy=xy, tri=tri, origins=np.ascontiguousarray(org),
                    xp=xp, start=start, G=G, vel=vel, dt=dt, dbar=dbar, flow=fld,
                    seeds=dict(mesh=seed, field=field_seed))


def served_mix_specs(n_meshes: int = 64, seed: int = 5, lo: float = 1e4, hi: float = 4e6):
    """Per-mesh knobs of the served mix: triangle counts log-uniform in [lo, hi],
    speed scale U ~ U[0.5, 4], mesh seed 5000+k, field seed 6000+k."""
    rng = np.random.default_rng(seed)
    nts = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_meshes))
    Us = rng.uniform(0.5, 4.0, size=n_meshes)
    specs = []
    for k_, (nt, U) in enumerate(zip(nts, Us)):
        n_side = int(round(math.sqrt(nt / 2.0))) + 1
        specs.append(dict(n_side=n_side, seed=5000 + k_, graded=False, field="fourier",
                          field_seed=6000 + k_, U=float(U), origins="nodes",
                          G=overlay_side_for(2 * (n_side - 1) ** 2)))
    return specs


def build_served(spec: dict) -> Workload:
    """One served-mix mesh: dt = 20 dbar / mean|u| of the U = 1 field, so that the
    displacement grows with U (about 10 to 80 element diameters).

    Meshes of the mix have different time steps, so the overlay input of a
    served job is the displacement over one step, dt u, sampled at the cell
    centres (FP32 [2][G][G]); one shared network maps it to the start
    displacement whatever the mesh."""
    xy, tri = mesh(spec["n_side"], spec["seed"])
    G = spec["G"]
    fld1 = FourierVortices(spec["field_seed"], U=1.0, norm_G=G)
    fld = FourierVortices(spec["field_seed"], U=spec["U"], norm_G=G)
    dbar = mean_diameter(xy, tri)
    u, v = fld1(xy[:, 0], xy[:, 1])
    dt = 20.0 * dbar / float(np.mean(np.hypot(u, v)))
    xp = departure_points(xy, fld, dt)
    start = node_start_elements(xy.shape[0], tri)
    vel = np.ascontiguousarray((overlay_velocity(fld, G).astype(np.float64) * dt).astype(np.float32))
    return Workload(name=f"mix{spec['seed']}", n_side=spec["n_side"], xy=xy, tri=tri, origins=xy, xp=xp,
                    start=start, G=G, vel=vel, dt=dt, dbar=dbar, flow=fld,
                    seeds=dict(mesh=spec["seed"], field=spec["field_seed"]))


def he_weights(seed: int = 200, channels=(2, 32, 32, 32, 2)):
    """He-normal conv weights (std sqrt(2 / (9 C_in))), zero bias, OIHW float32."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    for cin, cout in zip(channels[:-1], channels[1:]):
        std = math.sqrt(2.0 / (9 * cin))
        ws.append(np.ascontiguousarray((rng.standard_normal((cout, cin, 3, 3)) * std).astype(np.float32)))
        bs.append(np.zeros(cout, dtype=np.float32))
    return ws, bs


def classifier_he_weights(seed: int = 300):
    """He-normal weights of the classifier CNN (Sec. 2.3; PyTorch layouts, FP32), bias 0."""
    shapes = [(16, 2, 3, 3), (16, 16, 3, 3), (256, 2), (256, 256), (512, 512), (81, 512)]
    rng = np.random.default_rng(seed)
    ws = [(rng.standard_normal(s) * math.sqrt(2.0 / float(np.prod(s[1:])))).astype(np.float32) for s in shapes]
    bs = [np.zeros(s[0], np.float32) for s in shapes]
    return ws, bs


def random_weights(seed: int, channels=(2, 32, 32, 32, 2), bias_scale: float = 0.1):
    """He-normal weights with non-zero random biases (exercises the bias path)."""
    ws, _ = he_weights(seed, channels)
    rng = np.random.default_rng(seed + 1)
    bs = [np.ascontiguousarray((rng.standard_normal(w.shape[0]) * bias_scale).astype(np.float32)) for w in ws]
    return ws, bs


# ----------------------------------------------------------------------------- 3D (tetrahedra)

def kuhn_mesh(n: int, seed: int, jitter: float = 0.15):
    """Tetrahedral mesh of [0,1]^3: an n x n x n point grid (node (i, j, k) at index (k n + j) n + i),
    interior points moved by U(-jitter h, +jitter h) per axis (h = 1/(n-1)), points on a face of
    the cube only within that face, and every cell split into the six tetrahedra of its Kuhn
    (Freudenthal) subdivision along the main diagonal, which conforms across cells.  With
    jitter <= 0.15 no tetrahedron can invert (a Kuhn tetrahedron's heights are >= h / sqrt(2)).
    Returns (xyz float64 [n^3][3], tet int32 [6 (n-1)^3][4])."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    g = np.linspace(0.0, 1.0, n)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")  # X[k, j, i] = i h
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    J = rng.uniform(-jitter, jitter, size=P.shape) * h
    J[(P == 0.0) | (P == 1.0)] = 0.0  # points on a face of the cube stay on it
    P = P + J
    i, j, k = np.meshgrid(np.arange(n - 1), np.arange(n - 1), np.arange(n - 1), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()

    def node(di, dj, dk):
        return ((k + dk) * n + (j + dj)) * n + (i + di)

    tets = []
    unit = {0: (1, 0, 0), 1: (0, 1, 0), 2: (0, 0, 1)}
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        c = [0, 0, 0]
        vs = [node(*c)]
        for axis in perm:
            c = [c[a] + unit[axis][a] for a in range(3)]
            vs.append(node(*c))
        tets.append(np.stack(vs, axis=1))
    # cell-major order: the six tetrahedra of a cell are consecutive
    tet = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    order = np.argsort(np.repeat((k * (n - 1) + j) * (n - 1) + i, 6), kind="stable")
    return np.ascontiguousarray(P), np.ascontiguousarray(tet[order])


class ABCFlow:
    """Arnold-Beltrami-Childress flow on the unit cube (divergence-free):
    u = A sin(2 pi z + p_z) + C cos(2 pi y + p_y), v = B sin(2 pi x + p_x) + A cos(2 pi z + p_z),
    w = C sin(2 pi y + p_y) + B cos(2 pi x + p_x), with phases p = (p_x, p_y, p_z) (zero by default)."""

    def __init__(self, A: float = 1.0, B: float = 0.8, C: float = 0.6, phase=(0.0, 0.0, 0.0)):
        self.A, self.B, self.C = A, B, C
        self.px, self.py, self.pz = (float(p) for p in phase)

    def __call__(self, x, y, z):
        t = 2.0 * np.pi
        ax, ay, az = t * x + self.px, t * y + self.py, t * z + self.pz
        u = self.A * np.sin(az) + self.C * np.cos(ay)
        v = self.B * np.sin(ax) + self.A * np.cos(az)
        w = self.C * np.sin(ay) + self.B * np.cos(ax)
        return u, v, w


class UnsteadyABC:
    """A time-dependent ABC flow: the phases drift by omega_a * drift radians per time step
    (omega_a ~ U[0.5, 1.5] per axis, drawn from seed); step 0 is ABCFlow()."""

    def __init__(self, seed: int, drift: float = 0.15):
        self.w = np.random.default_rng(seed).uniform(0.5, 1.5, size=3) * drift

    def at(self, step: int) -> ABCFlow:
        return ABCFlow(phase=tuple(self.w * step))


def overlay_velocity_3d(flow, G: int) -> np.ndarray:
    """A 3D flow sampled at the centres ((c + 1/2) / G per axis) of a G^3 overlay: FP32 [3][G][G][G]
    (component, z, y, x)."""
    c = (np.arange(G) + 0.5) / G
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    u, v, w = flow(X, Y, Z)
    return np.ascontiguousarray(np.stack([u, v, w]).astype(np.float32))


def passthrough_weights_3d(dt: float):
    """3D CNN weights (3 -> 32 -> 32 -> 32 -> 3, 3x3x3, OIDHW) whose output is -dt u at every cell:
    layer 1 puts relu(u_a) and relu(-u_a) in channels 2a and 2a+1, layers 2 and 3 pass them on,
    layer 4 forms -dt (u+ - u-).  A constructed stand-in for a trained net: the displacement of
    one explicit step with the velocity of the origin's cell."""
    w1 = np.zeros((32, 3, 3, 3, 3), np.float32)
    w4 = np.zeros((3, 32, 3, 3, 3), np.float32)
    for a in range(3):
        w1[2 * a, a, 1, 1, 1] = 1.0
        w1[2 * a + 1, a, 1, 1, 1] = -1.0
        w4[a, 2 * a, 1, 1, 1] = -dt
        w4[a, 2 * a + 1, 1, 1, 1] = dt
    ident = np.zeros((32, 32, 3, 3, 3), np.float32)
    for k in range(32):
        ident[k, k, 1, 1, 1] = 1.0
    ws = [w1, ident, ident.copy(), w4]
    bs = [np.zeros(c, np.float32) for c in (32, 32, 32, 3)]
    return ws, bs


def tet_longest_edges(xyz: np.ndarray, tet: np.ndarray) -> np.ndarray:
    best = np.zeros(tet.shape[0])
    for a in range(4):
        for b in range(a + 1, 4):
            best = np.maximum(best, np.linalg.norm(xyz[tet[:, b]] - xyz[tet[:, a]], axis=1))
    return best


def node_start_tets(n_nodes: int, tet: np.ndarray) -> np.ndarray:
    """The smallest id of a tetrahedron incident to each node."""
    start = np.full(n_nodes, np.iinfo(np.int32).max, dtype=np.int64)
    ids = np.repeat(np.arange(tet.shape[0], dtype=np.int64), 4)
    np.minimum.at(start, tet.reshape(-1), ids)
    return start.astype(np.int32)


def overlay_side_for_3d(n_tet: int) -> int:
    return 1 << int(math.ceil(math.log2(n_tet ** (1.0 / 3.0))))


@dataclass
class Workload3D:
    name: str
    n_side: int
    xyz: np.ndarray     # float64 [N_v][3]
    tet: np.ndarray     # int32 [N_t][4] (orientation as generated)
    xp: np.ndarray      # float64 [n][3] departure points
    start: np.ndarray   # int32 [n] K_m
    G: int              # overlay side (G^3 cells)
    dt: float
    dbar: float
    flow: object = None

    @property
    def n_points(self) -> int:
        return int(self.xp.shape[0])

    @property
    def n_tet(self) -> int:
        return int(self.tet.shape[0])


CONFIGS_3D = {
    # name: grid side, mesh seed, displacement in mean element diameters
    "t1": dict(n_side=16, seed=41, k=4.0),
    "t2": dict(n_side=48, seed=42, k=10.0),
    # the 1M-point mesh takes an overlay of about two cells per point (the default side for its
    # 5.8M tetrahedra would be 256, 16.8M cells for the 3D CNN)
    "t3": dict(n_side=100, seed=43, k=10.0, G=128),
}


def build_3d(name: str) -> Workload3D:
    """Nodes of a jittered Kuhn mesh advected backwards one step in the ABC flow
    (x_p = clamp(x_i - dt u(x_i), 0, 1)), starting from their smallest incident tetrahedron."""
    cfg = CONFIGS_3D[name]
    xyz, tet = kuhn_mesh(cfg["n_side"], cfg["seed"])
    fl = ABCFlow()
    dbar = float(tet_longest_edges(xyz, tet).mean())
    u, v, w = fl(xyz[:, 0], xyz[:, 1], xyz[:, 2])
    dt = cfg["k"] * dbar / float(np.mean(np.sqrt(u * u + v * v + w * w)))
    xp = np.clip(xyz - dt * np.stack([u, v, w], axis=1), 0.0, 1.0)
    return Workload3D(name=name, n_side=cfg["n_side"], xyz=xyz, tet=tet, xp=np.ascontiguousarray(xp),
                      start=node_start_tets(xyz.shape[0], tet), G=cfg.get("G", overlay_side_for_3d(tet.shape[0])), dt=dt,
                      dbar=dbar, flow=fl)
