"""Thin ctypes binding of libcnnsns.so (the C ABI in include/cnnsns.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (``tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcnnsns.so")

OK, EINVAL, ENOMEM, EHIP, EMESH, EBUSY = 0, -1, -2, -3, -4, -5
FOUND, OUTSIDE, MAXITER, BADSTART = 0, 1, 2, 3
F32, BF16, FP8E4M3 = 0, 1, 2
PRECISIONS = {"f32": F32, "bf16": BF16, "fp8": FP8E4M3}

EXPORTS = (
    "cnnsns_build_mesh", "cnnsns_mesh_info", "cnnsns_destroy_mesh", "cnnsns_predict", "cnnsns_predict_noalloc",
    "cnnsns_locate", "cnnsns_classify", "cnnsns_locate_interpolate",
    "cnnsns_interpolate", "cnnsns_build_mesh3d", "cnnsns_mesh3d_info", "cnnsns_destroy_mesh3d", "cnnsns_predict3d",
    "cnnsns_locate3d", "cnnsns_interpolate3d",
    "cnnsns_server_create", "cnnsns_submit", "cnnsns_poll", "cnnsns_wait", "cnnsns_server_destroy",
    "cnnsns_last_error",
)

_lib = None


class CnnsnsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Cnn(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p * 4), ("b", ctypes.c_void_p * 4)]


class _Cls(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p * 6), ("b", ctypes.c_void_p * 6)]


def lib():
    """Load libcnnsns.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2412_18379_amd.build first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        sig = {
            "cnnsns_build_mesh": [vp, i64, vp, i64, i32, vp, ctypes.POINTER(vp)],
            "cnnsns_mesh_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                 ctypes.POINTER(ctypes.c_double)],
            "cnnsns_destroy_mesh": [vp],
            "cnnsns_predict": [vp, vp, ctypes.POINTER(_Cnn), i32, vp, vp],
            "cnnsns_predict_noalloc": [vp, vp, ctypes.POINTER(_Cnn), i32, vp, vp],
            "cnnsns_locate": [vp, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp],
            "cnnsns_classify": [vp, i64, vp, ctypes.POINTER(_Cls), vp, vp, vp, vp, vp],
            "cnnsns_locate_interpolate": [vp, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp],
            "cnnsns_interpolate": [vp, i64, vp, vp, vp, vp, vp],
            "cnnsns_build_mesh3d": [vp, i64, vp, i64, i32, vp, ctypes.POINTER(vp)],
            "cnnsns_mesh3d_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64)],
            "cnnsns_destroy_mesh3d": [vp],
            "cnnsns_predict3d": [vp, vp, ctypes.POINTER(_Cnn), i32, vp, vp],
            "cnnsns_locate3d": [vp, i64, vp, vp, vp, vp, i32, vp, vp, vp, vp],
            "cnnsns_interpolate3d": [vp, i64, vp, vp, vp, vp, vp],
            "cnnsns_server_create": [i64, i32, i32, i32, ctypes.POINTER(_Cnn), ctypes.POINTER(vp)],
            "cnnsns_submit": [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)],
            "cnnsns_poll": [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)],
            "cnnsns_wait": [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)],
            "cnnsns_server_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.cnnsns_last_error.argtypes = []
        L.cnnsns_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise CnnsnsError(rc, lib().cnnsns_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream, device: Optional[int] = None) -> ctypes.c_void_p:
    """The given stream, else the current stream of `device` (default: the current device)."""
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _on(device: int, *named):
    """Every given device tensor must be on the GPU the mesh was built on: the library takes raw
    pointers of that device."""
    for name, t in named:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError(f"{name}: device tensor expected")
        if t.device.index != device:
            raise ValueError(f"{name}: on cuda:{t.device.index}, but the mesh is on cuda:{device}")


CNN_SHAPES = [(32, 2, 3, 3), (32, 32, 3, 3), (32, 32, 3, 3), (2, 32, 3, 3)]
CNN3_SHAPES = [(32, 3, 3, 3, 3), (32, 32, 3, 3, 3), (32, 32, 3, 3, 3), (3, 32, 3, 3, 3)]


def _check_layers(ws, bs, shapes, what):
    """The kernels read every weight and bias at fixed offsets: all shapes must be exact."""
    gw, gb = [tuple(w.shape) for w in ws], [tuple(b.shape) for b in bs]
    if gw != list(shapes) or gb != [(sh[0],) for sh in shapes]:
        raise ValueError(f"{what}: weights of shapes {list(shapes)} and biases of sizes "
                         f"{[sh[0] for sh in shapes]} expected, got {gw} and {gb}")


def _need(t: Optional[torch.Tensor], dtype, shape=None, name="tensor"):
    if t is None:
        return
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


class Mesh:
    """A device-resident mesh (cnnsns_build_mesh).  xy, tri are host numpy arrays."""

    def __init__(self, xy, tri, overlay_side: int = 0, stream=None):
        import numpy as np
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        if xy.ndim != 2 or xy.shape[1] != 2 or tri.ndim != 2 or tri.shape[1] != 3:
            raise ValueError("xy must be [n,2] and tri [m,3]")
        h = ctypes.c_void_p()
        self.device = torch.cuda.current_device()  # the library builds on the current device
        _check(lib().cnnsns_build_mesh(xy.ctypes.data, xy.shape[0], tri.ctypes.data, tri.shape[0],
                                       int(overlay_side), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.n_nodes = int(xy.shape[0])
        n_tri, G, nbytes, diam = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().cnnsns_mesh_info(h, ctypes.byref(n_tri), ctypes.byref(G), ctypes.byref(nbytes),
                                      ctypes.byref(diam)))
        self.n_tri, self.G, self.device_bytes, self.mean_diam = n_tri.value, G.value, nbytes.value, diam.value

    def close(self):
        if self.handle:
            _check(lib().cnnsns_destroy_mesh(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Weights:
    """CNN weights as device tensors (FP32 OIHW + bias), kept alive with the struct."""

    def __init__(self, ws: Sequence, bs: Sequence, device="cuda"):
        self.w = [torch.as_tensor(w, dtype=torch.float32).to(device).contiguous() for w in ws]
        self.b = [torch.as_tensor(b, dtype=torch.float32).to(device).contiguous() for b in bs]
        _check_layers(self.w, self.b, CNN_SHAPES, "a 2-32-32-32-2 net of 3x3 kernels")
        self.device = self.w[0].device
        self.struct = _Cnn()
        for l in range(4):
            self.struct.w[l] = self.w[l].data_ptr()
            self.struct.b[l] = self.b[l].data_ptr()


def predict(mesh: Mesh, vel: torch.Tensor, weights: Weights, precision="f32", disp: torch.Tensor = None,
            stream=None) -> torch.Tensor:
    G = mesh.G
    _need(vel, torch.float32, (2, G, G), "vel")
    if disp is None:
        disp = torch.empty((2, G, G), dtype=torch.float32, device=vel.device)
    _need(disp, torch.float32, (2, G, G), "disp")
    _on(mesh.device, ("vel", vel), ("disp", disp), ("weights", weights.w[0]))
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().cnnsns_predict(mesh.handle, _ptr(vel), ctypes.byref(weights.struct), p, _ptr(disp),
                                _stream(stream, mesh.device)))
    return disp


def predict_noalloc(mesh: Mesh, vel: torch.Tensor, weights: Weights, disp: torch.Tensor, precision="bf16",
                    stream=None) -> torch.Tensor:
    """The forward pass with the library's preallocated per-GPU workspace (cnnsns_predict_noalloc):
    no device allocation; calls overlapping on one GPU race.  `disp` is caller-allocated."""
    G = mesh.G
    _need(vel, torch.float32, (2, G, G), "vel")
    _need(disp, torch.float32, (2, G, G), "disp")
    _on(mesh.device, ("vel", vel), ("disp", disp), ("weights", weights.w[0]))
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().cnnsns_predict_noalloc(mesh.handle, _ptr(vel), ctypes.byref(weights.struct), p, _ptr(disp),
                                        _stream(stream, mesh.device)))
    return disp


def locate(mesh: Mesh, xp: torch.Tensor, start: torch.Tensor = None, origin: torch.Tensor = None,
           disp: torch.Tensor = None, max_iter: int = 0, host: torch.Tensor = None, iters: torch.Tensor = None,
           status: torch.Tensor = None, want_iters=True, want_status=True, stream=None):
    n = xp.shape[0]
    _need(xp, torch.float64, (n, 2), "xp")
    _need(start, torch.int32, (n,), "start")
    _need(origin, torch.float64, (n, 2), "origin")
    _need(disp, torch.float32, (2, mesh.G, mesh.G), "disp")
    dev = xp.device
    if host is None:
        host = torch.empty(n, dtype=torch.int32, device=dev)
    if iters is None and want_iters:
        iters = torch.empty(n, dtype=torch.int32, device=dev)
    if status is None and want_status:
        status = torch.empty(n, dtype=torch.uint8, device=dev)
    _need(host, torch.int32, (n,), "host")
    _need(iters, torch.int32, (n,), "iters")
    _need(status, torch.uint8, (n,), "status")
    _on(mesh.device, ("xp", xp), ("start", start), ("origin", origin), ("disp", disp), ("host", host),
        ("iters", iters), ("status", status))
    _check(lib().cnnsns_locate(mesh.handle, n, _ptr(xp), _ptr(start), _ptr(origin), _ptr(disp), int(max_iter),
                               _ptr(host), _ptr(iters), _ptr(status), _stream(stream, mesh.device)))
    return host, iters, status


CLS_SHAPES = [(16, 2, 3, 3), (16, 16, 3, 3), (256, 2), (256, 256), (512, 512), (81, 512)]


class ClsWeights:
    """Weights of the classifier CNN as device tensors (FP32, PyTorch layouts), kept alive with the struct."""

    def __init__(self, ws: Sequence, bs: Sequence, device="cuda"):
        self.w = [torch.as_tensor(w, dtype=torch.float32).to(device).contiguous() for w in ws]
        self.b = [torch.as_tensor(b, dtype=torch.float32).to(device).contiguous() for b in bs]
        _check_layers(self.w, self.b, CLS_SHAPES, "the classifier")
        self.device = self.w[0].device
        self.struct = _Cls()
        for l in range(6):
            self.struct.w[l] = self.w[l].data_ptr()
            self.struct.b[l] = self.b[l].data_ptr()


def classify(mesh: Mesh, xp: torch.Tensor, weights: ClsWeights, fallback: torch.Tensor = None,
             start: torch.Tensor = None, want_class=True, want_logits=False, stream=None):
    """The classifier's prediction step of Alg. 2 (cnnsns_classify): (start K_p, class, logits)."""
    n = xp.shape[0]
    _need(xp, torch.float64, (n, 2), "xp")
    _need(fallback, torch.int32, (n,), "fallback")
    if start is None:
        start = torch.empty(n, dtype=torch.int32, device=xp.device)
    _need(start, torch.int32, (n,), "start")
    cls = torch.empty(n, dtype=torch.int32, device=xp.device) if want_class else None
    logits = torch.empty((n, 81), dtype=torch.float32, device=xp.device) if want_logits else None
    _on(mesh.device, ("xp", xp), ("fallback", fallback), ("start", start), ("weights", weights.w[0]))
    _check(lib().cnnsns_classify(mesh.handle, n, _ptr(xp), ctypes.byref(weights.struct), _ptr(fallback),
                                 _ptr(start), _ptr(cls), _ptr(logits), _stream(stream, mesh.device)))
    return start, cls, logits


def locate_interpolate(mesh: Mesh, xp: torch.Tensor, nodal: torch.Tensor, start: torch.Tensor = None,
                       origin: torch.Tensor = None, disp: torch.Tensor = None, max_iter: int = 0,
                       host: torch.Tensor = None, iters: torch.Tensor = None, status: torch.Tensor = None,
                       out: torch.Tensor = None, want_iters=True, want_status=True, stream=None):
    """cnnsns_locate with the P1 interpolation of `nodal` at x_p fused into the walk's last step:
    (host, iters, status, out)."""
    n = xp.shape[0]
    _need(xp, torch.float64, (n, 2), "xp")
    _need(start, torch.int32, (n,), "start")
    _need(origin, torch.float64, (n, 2), "origin")
    _need(disp, torch.float32, (2, mesh.G, mesh.G), "disp")
    _need(nodal, torch.float64, (mesh.n_nodes, 2), "nodal")
    dev = xp.device
    host = torch.empty(n, dtype=torch.int32, device=dev) if host is None else host
    if iters is None and want_iters:
        iters = torch.empty(n, dtype=torch.int32, device=dev)
    if status is None and want_status:
        status = torch.empty(n, dtype=torch.uint8, device=dev)
    out = torch.empty((n, 2), dtype=torch.float64, device=dev) if out is None else out
    _need(host, torch.int32, (n,), "host")
    _need(iters, torch.int32, (n,), "iters")
    _need(status, torch.uint8, (n,), "status")
    _need(out, torch.float64, (n, 2), "out")
    _on(mesh.device, ("xp", xp), ("start", start), ("origin", origin), ("disp", disp), ("host", host),
        ("iters", iters), ("status", status), ("nodal", nodal), ("out", out))
    _check(lib().cnnsns_locate_interpolate(mesh.handle, n, _ptr(xp), _ptr(start), _ptr(origin), _ptr(disp),
                                           int(max_iter), _ptr(host), _ptr(iters), _ptr(status), _ptr(nodal),
                                           _ptr(out), _stream(stream, mesh.device)))
    return host, iters, status, out


class Mesh3D:
    """A device-resident tetrahedral mesh (cnnsns_build_mesh3d).  xyz, tet are host numpy arrays."""

    def __init__(self, xyz, tet, overlay_side: int = 0, stream=None):
        import numpy as np
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or tet.ndim != 2 or tet.shape[1] != 4:
            raise ValueError("xyz must be [n,3] and tet [m,4]")
        h = ctypes.c_void_p()
        self.device = torch.cuda.current_device()
        _check(lib().cnnsns_build_mesh3d(xyz.ctypes.data, xyz.shape[0], tet.ctypes.data, tet.shape[0],
                                         int(overlay_side), _stream(stream), ctypes.byref(h)))
        self.handle = h
        n_tet, G, nbytes = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().cnnsns_mesh3d_info(h, ctypes.byref(n_tet), ctypes.byref(G), ctypes.byref(nbytes)))
        self.n_tet, self.G, self.device_bytes = n_tet.value, G.value, nbytes.value
        self.n_nodes = int(xyz.shape[0])

    def close(self):
        if self.handle:
            _check(lib().cnnsns_destroy_mesh3d(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Weights3D:
    """3D CNN weights as device tensors (FP32 OIDHW + bias, 3-32-32-32-3 with 3x3x3 kernels)."""

    def __init__(self, ws: Sequence, bs: Sequence, device="cuda"):
        self.w = [torch.as_tensor(w, dtype=torch.float32).to(device).contiguous() for w in ws]
        self.b = [torch.as_tensor(b, dtype=torch.float32).to(device).contiguous() for b in bs]
        _check_layers(self.w, self.b, CNN3_SHAPES, "a 3-32-32-32-3 net of 3x3x3 kernels")
        self.device = self.w[0].device
        self.struct = _Cnn()
        for l in range(4):
            self.struct.w[l] = self.w[l].data_ptr()
            self.struct.b[l] = self.b[l].data_ptr()


def predict3d(mesh: Mesh3D, vel: torch.Tensor, weights: Weights3D, precision="f32", disp: torch.Tensor = None,
              stream=None) -> torch.Tensor:
    """The 3D displacement CNN on the mesh's G^3 overlay (cnnsns_predict3d, FP32 or BF16)."""
    G = mesh.G
    _need(vel, torch.float32, (3, G, G, G), "vel")
    if disp is None:
        disp = torch.empty((3, G, G, G), dtype=torch.float32, device=vel.device)
    _need(disp, torch.float32, (3, G, G, G), "disp")
    _on(mesh.device, ("vel", vel), ("disp", disp), ("weights", weights.w[0]))
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().cnnsns_predict3d(mesh.handle, _ptr(vel), ctypes.byref(weights.struct), p, _ptr(disp),
                                  _stream(stream, mesh.device)))
    return disp


def locate3d(mesh: Mesh3D, xp: torch.Tensor, start: torch.Tensor = None, origin: torch.Tensor = None,
             disp: torch.Tensor = None, max_iter: int = 0, host: torch.Tensor = None, iters: torch.Tensor = None,
             status: torch.Tensor = None, stream=None):
    """Alg. 1 on a tetrahedral mesh (cnnsns_locate3d): (host, iters, status).  Starts: `start`, or
    CNN-SNS from `origin` and `disp` (Alg. 2), or the overlay lookup of x_p."""
    n = xp.shape[0]
    _need(xp, torch.float64, (n, 3), "xp")
    _need(start, torch.int32, (n,), "start")
    _need(origin, torch.float64, (n, 3), "origin")
    _need(disp, torch.float32, (3, mesh.G, mesh.G, mesh.G), "disp")
    dev = xp.device
    host = torch.empty(n, dtype=torch.int32, device=dev) if host is None else host
    iters = torch.empty(n, dtype=torch.int32, device=dev) if iters is None else iters
    status = torch.empty(n, dtype=torch.uint8, device=dev) if status is None else status
    _need(host, torch.int32, (n,), "host")
    _need(iters, torch.int32, (n,), "iters")
    _need(status, torch.uint8, (n,), "status")
    _on(mesh.device, ("xp", xp), ("start", start), ("origin", origin), ("disp", disp), ("host", host),
        ("iters", iters), ("status", status))
    _check(lib().cnnsns_locate3d(mesh.handle, n, _ptr(xp), _ptr(start), _ptr(origin), _ptr(disp), int(max_iter),
                                 _ptr(host), _ptr(iters), _ptr(status), _stream(stream, mesh.device)))
    return host, iters, status


def interpolate3d(mesh: Mesh3D, xp: torch.Tensor, host: torch.Tensor, nodal: torch.Tensor, out: torch.Tensor = None,
                  stream=None) -> torch.Tensor:
    """P1 interpolation of a nodal field (FP64 [n_nodes][3]) at points in their host tetrahedra
    (cnnsns_interpolate3d)."""
    n = xp.shape[0]
    _need(xp, torch.float64, (n, 3), "xp")
    _need(host, torch.int32, (n,), "host")
    _need(nodal, torch.float64, (mesh.n_nodes, 3), "nodal")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=xp.device)
    _need(out, torch.float64, (n, 3), "out")
    _on(mesh.device, ("xp", xp), ("host", host), ("nodal", nodal), ("out", out))
    _check(lib().cnnsns_interpolate3d(mesh.handle, n, _ptr(xp), _ptr(host), _ptr(nodal), _ptr(out),
                                      _stream(stream, mesh.device)))
    return out


def interpolate(mesh: Mesh, xp: torch.Tensor, host: torch.Tensor, nodal: torch.Tensor, out: torch.Tensor = None,
                stream=None) -> torch.Tensor:
    """P1 interpolation of a nodal field (FP64 [n_nodes][2]) at the points xp in their host
    elements (cnnsns_interpolate)."""
    n = xp.shape[0]
    _need(xp, torch.float64, (n, 2), "xp")
    _need(host, torch.int32, (n,), "host")
    _need(nodal, torch.float64, (mesh.n_nodes, 2), "nodal")
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float64, device=xp.device)
    _need(out, torch.float64, (n, 2), "out")
    _on(mesh.device, ("xp", xp), ("host", host), ("nodal", nodal), ("out", out))
    _check(lib().cnnsns_interpolate(mesh.handle, n, _ptr(xp), _ptr(host), _ptr(nodal), _ptr(out),
                                    _stream(stream, mesh.device)))
    return out


class Server:
    """Serving loop (cnnsns_server_*)."""

    def __init__(self, weights: Weights, hbm_budget_bytes: int, max_inflight: int = 4, queue_depth: int = 1024,
                 precision="bf16"):
        self.weights = weights
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        _check(lib().cnnsns_server_create(int(hbm_budget_bytes), int(max_inflight), int(queue_depth), p,
                                          ctypes.byref(weights.struct), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, mesh: Mesh, vel, xp, origin, host, iters=None, start=None, stream=None) -> int:
        """Queue a CNN-SNS job; it runs after the work enqueued on `stream` (default: the current
        stream) before this call.  The mesh and the buffers are kept alive until it completes."""
        n = xp.shape[0]
        G = mesh.G
        _need(vel, torch.float32, (2, G, G), "vel")
        _need(xp, torch.float64, (n, 2), "xp")
        _need(origin, torch.float64, (n, 2), "origin")
        _need(host, torch.int32, (n,), "host")
        _need(iters, torch.int32, (n,), "iters")
        _need(start, torch.int32, (n,), "start")
        _on(mesh.device, ("vel", vel), ("xp", xp), ("origin", origin), ("host", host), ("iters", iters),
            ("start", start), ("weights", self.weights.w[0]))
        jid = ctypes.c_uint64()
        _check(lib().cnnsns_submit(self.handle, mesh.handle, _ptr(vel), n, _ptr(xp), _ptr(origin),
                                   _ptr(start), _ptr(host), _ptr(iters), _stream(stream, mesh.device),
                                   ctypes.byref(jid)))
        self._keep[jid.value] = (mesh, vel, xp, origin, host, iters, start)
        return jid.value

    def poll(self, job_id: int):
        done, lat = ctypes.c_int32(), ctypes.c_double()
        _check(lib().cnnsns_poll(self.handle, job_id, ctypes.byref(done), ctypes.byref(lat)))
        if done.value:
            self._keep.pop(job_id, None)
            return lat.value
        return None

    def wait(self, job_id: int) -> float:
        lat = ctypes.c_double()
        _check(lib().cnnsns_wait(self.handle, job_id, ctypes.byref(lat)))
        self._keep.pop(job_id, None)
        return lat.value

    def close(self):
        if self.handle:
            _check(lib().cnnsns_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
