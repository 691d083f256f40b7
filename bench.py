"""Benchmark: points located per second, CNN-SNS vs plain SNS, on one MI355X.

One step is one pass of the CNN-SNS hot path over the whole workload with all
inputs resident in device memory: the CNN forward pass over the overlay grid
(cnnsns_predict) followed by the CNN-SNS walk of every point
(cnnsns_locate with the displacement grid).  The plain SNS walk from the
element before movement, and the ASG start (overlay lookup at x_p), are timed
beside it on the same inputs.

Default workload: the 16M-triangle radially graded mesh with 8M departure
points at ~150 element diameters and a 4096 x 4096 overlay, FP32 CNN.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c4] [--precision f32|bf16|fp8]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import faulthandler
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm_GBps": 8000.0, "f32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0, "fp8_TFLOPs": 5000.0}
CNN_MACS_PER_PIXEL = 2 * 32 * 9 + 32 * 32 * 9 * 2 + 32 * 2 * 9  # 19,584
# Winograd F(2x2,3x3) multiplies per output pixel and channel pair: 16 per 2 x 2 block; the MACs it
# saves are not counted as useful work
WINO_USEFUL_MACS_PER_PIXEL = 2 * 32 * 9 + 2 * 32 * 32 * 4 + 32 * 2 * 9  # 9,344


def _cdiv(a, b):
    return -(-a // b)


def conv34_tiles(G: int, cus: int) -> int:
    """Tiles the FP32 conv34 kernel runs over a G x G overlay: column strips 30 outputs wide, cut into
    segments of 14 + 16 kb rows (a first tile of 14 output rows, then kb tiles of 16 that reuse the two
    region rows above them), kb chosen as the kernel's host code chooses it for `cus` compute units."""
    tx, gmax = _cdiv(G, 30), max(8, _cdiv(cus, 8) * 8)
    best = None
    for kb in range(65):
        seg = 14 + 16 * kb
        nseg = tx * _cdiv(G, seg)
        grid = max(8, _cdiv(nseg, 8) * 8) if nseg < gmax else gmax
        cost = _cdiv(nseg, grid) * (kb + 1)
        if best is None or cost <= best[0]:
            best = (cost, kb)
        if seg >= G:
            break
    seg = 14 + 16 * best[1]
    tiles = 0
    for sy in range(_cdiv(G, seg)):
        ylim, n = min((sy + 1) * seg, G), 1
        while sy * seg + 14 + 16 * (n - 1) < ylim:
            n += 1
        tiles += n
    return tx * tiles


def _cus() -> int:
    """Compute units of GPU 0 (the MI355X's 256 when no GPU is visible)."""
    import torch
    if not torch.cuda.is_available():
        return 256
    return torch.cuda.get_device_properties(0).multi_processor_count


def cnn_issued_macs(G: int, precision: str) -> float:
    """Matrix-core MACs one forward pass issues over a G x G overlay, padding and recomputed halos
    included (per tile, as the kernels are written)."""
    cdiv = _cdiv
    if precision == "f32":
        regions12 = cdiv(G, 32) * cdiv(G, 16)  # 16 x 32 regions: conv1 (K 18 -> 20) on the 39 M-blocks of
        tiles34 = conv34_tiles(G, _cus())      # the 18 x 34 input tile, then conv2 as Winograd F(2x2,3x3);
        # conv34 tiles: conv3 as Winograd on a 16 x 32 region, conv4 as 16 matrix columns
        return (regions12 * (624 * 20 * 32 + 128 * 16 * 32 * 32) +
                tiles34 * (128 * 16 * 32 * 32 + 512 * 32 * 16))
    if precision == "bf16":
        tiles = cdiv(G, 30) * cdiv(G, 14)  # fused 14 x 30 output tiles: conv1 (K 32) on 20 x 36 pixels,
        # conv2 on 40 M-blocks (18 x 34 pixels), conv3 on 32 (16 x 32), conv4 as 32 columns of K 32
        return tiles * (720 * 32 * 32 + 640 * 288 * 32 + 512 * 288 * 32 + 512 * 32 * 32)
    raise ValueError(precision)


# the classifier CNN (Sec. 2.3) per point: matrix-core MACs issued (conv1 on 96 rows of 16 x 20, conv2 on
# 96 rows of 16 x 144, the FC layers 256 x 256, 512 x 512 and 512 x 128 with the 81 logits padded to two
# 64-column tiles) and the products the network needs (module 2's first layer runs on the vector ALUs)
CLS_ISSUED_MACS = 96 * 20 * 16 + 96 * 144 * 16 + 256 * 256 + 512 * 512 + 512 * 128  # 645,120
CLS_USEFUL_MACS = 81 * 18 * 16 + 81 * 144 * 16 + 2 * 256 + 256 * 256 + 512 * 512 + 512 * 81  # 579,616
REC_BYTES = 60  # algorithmic bytes of one element record: 6 FP64 coordinates + 3 int32 neighbours
# one tetrahedron record: 12 FP64 coordinates, 4 int32 neighbours and the 4 int32 node ids that put
# each face's nodes in a fixed order
TET_REC_BYTES = 128
CNN3_MACS_PER_CELL = 3 * 32 * 27 + 2 * 32 * 32 * 27 + 32 * 3 * 27  # 60,480


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _traffic_entry(group: str, workload: str):
    from paper_2412_18379_amd import profiling as P

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        db = json.load(f)
    e = db.get(f"{group}@{workload}")
    if not e or e.get("source_sha") != P.source_sha(*P.SOURCES[group]):
        return None
    return e


def traffic_for(group: str, workload: str):
    """HBM bytes per launch of a kernel group, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of the
    current source of its kernels (scaled by a copy of known size), else None."""
    e = _traffic_entry(group, workload)
    return None if e is None else e.get("hbm_bytes_per_launch")


def traffic_by_request_size(group: str, workload: str, ms: float):
    """The same launch's HBM bytes with the read side taken from the TCC read requests counted by
    size (no copy scale), and the rate they give over the launch time ms; None if not measured."""
    e = _traffic_entry(group, workload)
    if e is None or "hbm_bytes_per_launch_by_request_size" not in e:
        return None
    b = e["hbm_bytes_per_launch_by_request_size"]
    return {"bytes": b, "GBps": round(b / (ms / 1e3) / 1e9, 1), "frac": round(b / (ms / 1e3) / 1e9 / PEAK["hbm_GBps"], 4)}


def copy_probe(nbytes: int, reps: int = 3):
    """A device-to-device copy of nbytes (the calibration run for the HBM byte counters)."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def gather_probe(nbytes: int, reps: int = 3):
    """A gather of nbytes of 64-byte rows in a seeded random order (each row read once, the int64 row
    ids streamed, the rows written in order): the second calibration run for the HBM byte counters,
    with the access size of the walk's element records rather than a copy's streaming lines."""
    import torch

    rows = nbytes // 64
    g = torch.Generator().manual_seed(7)
    perm = torch.randperm(rows, generator=g).to("cuda")
    src = torch.ones((rows, 16), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.index_select(src, 0, perm, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"gather_probe_rows": rows, "row_bytes": 64, "index_bytes": 8, "reps": reps}), flush=True)


def copy_bandwidth(nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Device-to-device copy rate in GB/s (bytes read + bytes written per second): the
    streaming bandwidth this GPU reaches in practice, a second denominator for HBM-bound
    kernels beside the published peak."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbps


def _off_edge(w, host, pts, eps=1e-9):
    """Points farther than eps from every edge of their (oracle) host element."""
    V = w.xy[w.tri[host]]
    best = np.full(len(pts), np.inf)
    for k in range(3):
        a, b = V[:, k], V[:, (k + 1) % 3]
        d = b - a
        t = np.clip(np.einsum("ij,ij->i", pts - a, d) / np.einsum("ij,ij->i", d, d), 0.0, 1.0)
        best = np.minimum(best, np.hypot(*(a + t[:, None] * d - pts).T))
    return best > eps


def pct(a, q):
    return float(np.percentile(a, q))


def cpu_baseline_3d(w, ws, bs, vel, d32, slab: int = 8):
    """The FP64 oracle beside the 3D legs on a bounded sample of the same workload (host cores):
    the plain walk of all points, and the 3D CNN on `slab` overlay planes plus the CNN-SNS start
    and walk of the points whose origin lies in them.  Also the timed FP32 3D CNN output on that
    slab against the oracle (the 1e-5 bar per channel)."""
    import oracle as O

    threads = O.set_threads(0)
    G = w.G
    t = time.perf_counter()
    tp, nbr = O.prepare_mesh3(w.xyz, w.tet)
    lk = O.lookup3(w.xyz, tp, G)
    setup_s = time.perf_counter() - t
    z0 = max(0, G // 2 - slab // 2)
    z1 = min(G, z0 + slab)
    cz = np.clip(np.floor(w.xyz[:, 2] * G), 0, G - 1).astype(np.int64)
    sel = np.nonzero((cz >= z0) & (cz < z1))[0]
    t = time.perf_counter()
    ref = O.cnn3_window(vel, ws, bs, (z0, 0, 0), (z1 - z0, G, G))
    t_cnn = time.perf_counter() - t
    disp = np.zeros((3, G, G, G))
    disp[:, z0:z1] = ref
    t = time.perf_counter()
    s0 = O.cnnsns3_start(w.xyz[sel], disp, lk, w.start[sel])
    _, it, _ = O.sns3(w.xyz, tp, nbr, w.xp[sel], s0)
    t_walk = time.perf_counter() - t
    t = time.perf_counter()
    _, pit, _ = O.sns3(w.xyz, tp, nbr, w.xp, w.start)
    t_plain = time.perf_counter() - t
    got = d32[:, z0:z1].astype(np.float64)
    scale = np.abs(ref).reshape(3, -1).max(axis=1)[:, None, None, None]
    ratio = float((np.abs(got - ref) / (1e-5 * np.abs(ref) + 1e-5 * scale + 1e-30)).max())
    n = len(sel)
    return {
        "value": n / (t_cnn + t_walk), "unit": "points/s", "cores": threads, "kind": "oracle",
        "sample": (f"overlay planes z in [{z0},{z1}) of {G}: FP64 3D CNN on them ({t_cnn:.2f}s) + CNN-SNS start and "
                   f"walk of the {n} points whose origin lies in them ({t_walk:.2f}s); mesh prep and lookup untimed "
                   f"({setup_s:.1f}s)"),
        "plain_sns_value": w.n_points / t_plain, "plain_sns_s": t_plain, "plain_sns_sample": "all points",
        "mean_path_cnn_sns": float(it.mean()), "mean_path_plain": float(pit.mean()),
        "f32_parity_on_slab": {"worst_error_over_tolerance": round(ratio, 4), "pass": ratio <= 1.0},
    }


def walk3d_leg(name: str, K: int, warmup: int, copy_gbps: float, with_cpu: bool = True):
    """Alg. 1 on a tetrahedral mesh (the walk of Sec. 2.2 with four faces per element): the
    departure points of a jittered Kuhn mesh advected in the ABC flow, walked from the element
    before movement and from the overlay lookup, on the same GPU."""
    import torch

    from paper_2412_18379_amd import cnnsns as C
    from paper_2412_18379_amd import workload as W

    t0 = time.perf_counter()
    w = W.build_3d(name)
    mesh = C.Mesh3D(w.xyz, w.tet, overlay_side=w.G)
    torch.cuda.synchronize()
    log(f"3D workload {name}: {w.n_tet} tetrahedra, {w.n_points} points, G={w.G}, "
        f"{mesh.device_bytes / 2**20:.0f} MiB resident ({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    n = w.n_points
    xp = torch.from_numpy(w.xp).to(dev)
    start = torch.from_numpy(w.start).to(dev)
    host = torch.empty(n, dtype=torch.int32, device=dev)
    iters = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(n, dtype=torch.uint8, device=dev)

    def timed(**kw):
        for _ in range(warmup):
            C.locate3d(mesh, xp, host=host, iters=iters, status=status, **kw)
        torch.cuda.synchronize()
        e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for k in range(K):
            e[k][0].record(stream)
            C.locate3d(mesh, xp, host=host, iters=iters, status=status, **kw)
            e[k][1].record(stream)
        torch.cuda.synchronize()
        return (np.array([a.elapsed_time(b) for a, b in e]), iters.cpu().numpy(), status.cpu().numpy(),
                host.cpu().numpy())

    plain_ms, it_p, st_p, host_p = timed(start=start)
    asg_ms, it_a, st_a, host_a = timed()
    # CNN-SNS in 3D: the 3D CNN on the G^3 overlay, then the walk from its start (Alg. 2).  The
    # weights are the constructed pass-through net (displacement -dt u of the origin's cell), a
    # stand-in for a trained net.
    ws, bs = W.passthrough_weights_3d(w.dt)
    wts = C.Weights3D(ws, bs, device=dev)
    vel = torch.from_numpy(W.overlay_velocity_3d(w.flow, w.G)).to(dev)
    origin = torch.from_numpy(w.xyz).to(dev)
    disp = torch.empty((3, w.G, w.G, w.G), dtype=torch.float32, device=dev)
    for _ in range(warmup):
        C.predict3d(mesh, vel, wts, disp=disp)
        C.locate3d(mesh, xp, start=start, origin=origin, disp=disp, host=host, iters=iters, status=status)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    for k in range(K):
        ev[k][0].record(stream)
        C.predict3d(mesh, vel, wts, disp=disp)
        ev[k][1].record(stream)
        C.locate3d(mesh, xp, start=start, origin=origin, disp=disp, host=host, iters=iters, status=status)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    p3_ms = np.array([a.elapsed_time(b) for a, b, _ in ev])
    l3_ms = np.array([b.elapsed_time(c) for _, b, c in ev])
    it_c, st_c, host_c = iters.cpu().numpy(), status.cpu().numpy(), host.cpu().numpy()
    log(f"3D CNN-SNS: predict {p3_ms.mean():.3f} ms, locate {l3_ms.mean():.3f} ms, mean I_t {it_c.mean():.2f}")
    cnn3_flops = 2.0 * CNN3_MACS_PER_CELL * w.G ** 3
    cnn3_tf = cnn3_flops / (p3_ms.mean() / 1e3) / 1e12
    d32 = disp.cpu().numpy()
    # the same step with the BF16 3D CNN (precision variant)
    for _ in range(warmup):
        C.predict3d(mesh, vel, wts, "bf16", disp=disp)
    torch.cuda.synchronize()
    eb = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    for k in range(K):
        eb[k][0].record(stream)
        C.predict3d(mesh, vel, wts, "bf16", disp=disp)
        eb[k][1].record(stream)
        C.locate3d(mesh, xp, start=start, origin=origin, disp=disp, host=host, iters=iters, status=status)
        eb[k][2].record(stream)
    torch.cuda.synchronize()
    pb_ms = np.array([a.elapsed_time(b) for a, b, _ in eb])
    lb_ms = np.array([b.elapsed_time(c) for _, b, c in eb])
    it_b = iters.cpu().numpy()
    log(f"3D CNN-SNS, BF16 CNN: predict {pb_ms.mean():.3f} ms, locate {lb_ms.mean():.3f} ms, mean I_t {it_b.mean():.2f}")
    cnn3_tf_b = cnn3_flops / (pb_ms.mean() / 1e3) / 1e12
    # the step after location: the velocity at x_p, P1-interpolated in the host tetrahedron
    fu, fv, fw = w.flow(w.xyz[:, 0], w.xyz[:, 1], w.xyz[:, 2])
    nodal = torch.from_numpy(np.ascontiguousarray(np.stack([fu, fv, fw], axis=1))).to(dev)
    u_xp = torch.empty((n, 3), dtype=torch.float64, device=dev)
    for _ in range(warmup):
        C.interpolate3d(mesh, xp, host, nodal, out=u_xp)
    torch.cuda.synchronize()
    ei = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for k in range(K):
        ei[k][0].record(stream)
        C.interpolate3d(mesh, xp, host, nodal, out=u_xp)
        ei[k][1].record(stream)
    torch.cuda.synchronize()
    i3_ms = np.array([a.elapsed_time(b) for a, b in ei])
    # x_p 24 + host 4 + vertices 96 and orientation 4 + node ids 16 + four nodal values 96 + result 24
    b_i3 = n * (24 + 4 + 96 + 4 + 16 + 96 + 24)
    g_i3 = b_i3 / (i3_ms.mean() / 1e3) / 1e9
    log(f"3D plain SNS: {plain_ms.mean():.3f} ms, mean I_t {it_p.mean():.2f}; "
        f"3D lookup start: {asg_ms.mean():.3f} ms, mean I_t {it_a.mean():.2f}")
    # one 128-byte element record per iteration; per point x_p 24 B, the start (or lookup entry)
    # 4 B and host, iteration count and status 9 B
    per_point = 24 + 4 + 9
    b_plain = TET_REC_BYTES * float(it_p.sum()) + n * per_point
    b_asg = TET_REC_BYTES * float(it_a.sum()) + n * per_point
    g_plain = b_plain / (plain_ms.mean() / 1e3) / 1e9
    g_asg = b_asg / (asg_ms.mean() / 1e3) / 1e9
    out = {
        "workload": f"{w.n_side}^3-node jittered Kuhn mesh, {w.n_tet} tetrahedra, {n} node points advected "
                    f"{W.CONFIGS_3D[name]['k']:g} mean element diameters in the ABC flow, G={w.G}",
        "plain_sns": {"ms": round(float(plain_ms.mean()), 4), "points_per_s": round(n / (plain_ms.mean() / 1e3), 1),
                      "mean_path_length": round(float(it_p.mean()), 3),
                      "path_length_p50_p99_max": [pct(it_p, 50), pct(it_p, 99), int(it_p.max())],
                      "found_frac": float(np.mean(st_p == C.FOUND))},
        "lookup_start": {"ms": round(float(asg_ms.mean()), 4), "points_per_s": round(n / (asg_ms.mean() / 1e3), 1),
                         "mean_path_length": round(float(it_a.mean()), 3),
                         "path_length_p50_p99_max": [pct(it_a, 50), pct(it_a, 99), int(it_a.max())],
                         "found_frac": float(np.mean(st_a == C.FOUND)),
                         "host_agreement_with_plain": float(np.mean(host_a == host_p))},
        "cnn_sns": {"weights": ("constructed pass-through (-dt u of the origin's cell); the forward pass costs the "
                                "same for any weights, and the net trained in the loop is timed and walked in "
                                "online_training_3d_leg"),
                    "predict_ms": round(float(p3_ms.mean()), 4), "locate_ms": round(float(l3_ms.mean()), 4),
                    "step_ms": round(float((p3_ms + l3_ms).mean()), 4),
                    "points_per_s": round(n / ((p3_ms + l3_ms).mean() / 1e3), 1),
                    "speedup_vs_plain_sns": round(float(plain_ms.mean() / (p3_ms + l3_ms).mean()), 4),
                    "mean_path_length": round(float(it_c.mean()), 3),
                    "path_length_p50_p99_max": [pct(it_c, 50), pct(it_c, 99), int(it_c.max())],
                    "found_frac": float(np.mean(st_c == C.FOUND)),
                    "host_agreement_with_plain": float(np.mean(host_c == host_p)),
                    "cnn_roofline": {"kernel": "3D cnn forward (k3c_zconv1 + 2 x k3c_conv32 + k3c_zconv4_f32)",
                                     "bound": "mfma", "achieved": round(cnn3_tf, 3), "peak": PEAK["f32_TFLOPs"],
                                     "unit": "TFLOP/s", "frac": round(cnn3_tf / PEAK["f32_TFLOPs"], 4),
                                     "traffic": traffic_for("cnn3_forward_f32", name),
                                     "algorithmic_per_launch": f"{cnn3_flops:.4e} FLOP (2 x 60480 MAC x G^3, "
                                                               f"G={w.G})"}},
        "cnn_sns_bf16": {"predict_ms": round(float(pb_ms.mean()), 4), "locate_ms": round(float(lb_ms.mean()), 4),
                         "step_ms": round(float((pb_ms + lb_ms).mean()), 4),
                         "speedup_vs_plain_sns": round(float(plain_ms.mean() / (pb_ms + lb_ms).mean()), 4),
                         "mean_path_length": round(float(it_b.mean()), 3),
                         "cnn_roofline": {"achieved": round(cnn3_tf_b, 3), "peak": PEAK["bf16_TFLOPs"],
                                          "unit": "TFLOP/s", "frac": round(cnn3_tf_b / PEAK["bf16_TFLOPs"], 4),
                                          "traffic": traffic_for("cnn3_forward_bf16", name)}},
        "interp_leg": {"kernel": "k3_interp (P1 velocity at x_p in its host tetrahedron)",
                       "ms": round(float(i3_ms.mean()), 4), "points_per_s": round(n / (i3_ms.mean() / 1e3), 1),
                       "bound": "hbm", "achieved": round(g_i3, 1), "unit": "GB/s",
                       "frac": round(g_i3 / PEAK["hbm_GBps"], 4), "traffic": traffic_for("k3_interp", name),
                       "algorithmic_per_launch": f"{b_i3:.4e} B (264 B x n)"},
        "roofline": {"kernel": "k3_locate (plain SNS leg)", "bound": "hbm", "achieved": round(g_plain, 1),
                     "peak": PEAK["hbm_GBps"], "unit": "GB/s", "frac": round(g_plain / PEAK["hbm_GBps"], 4),
                     "frac_of_measured_copy": round(g_plain / copy_gbps, 4),
                     "traffic": traffic_for("k3_locate_plain", name),
                     "traffic_by_request_size": traffic_by_request_size("k3_locate_plain", name, plain_ms.mean()),
                     "algorithmic_per_launch": f"{b_plain:.4e} B (128 B x sum I_t + {per_point} B x n)",
                     "lookup_start_leg": {"achieved": round(g_asg, 1), "frac": round(g_asg / PEAK["hbm_GBps"], 4),
                                          "traffic": traffic_for("k3_locate_lookup", name)}},
    }
    if with_cpu:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline_3d(w, ws, bs, W.overlay_velocity_3d(w.flow, w.G), d32)
        log(f"3D cpu baseline: {out['cpu_baseline']['value']:.0f} points/s CNN-SNS, "
            f"{out['cpu_baseline']['plain_sns_value']:.0f} points/s plain ({time.perf_counter() - t0:.1f}s)")
    mesh.close()
    return out


def cpu_baseline(w, ws, bs, band_rows: int):
    """The FP64 oracle on a bounded band of the same workload (host cores)."""
    import oracle as O

    threads = O.set_threads(0)
    G = w.G
    t = time.perf_counter()
    tc, nbr = O.prepare_mesh(w.xy, w.tri)
    lk = O.lookup(w.xy, tc, G)
    setup_s = time.perf_counter() - t
    r0 = max(0, G // 2 - band_rows // 2)
    r1 = min(G, r0 + band_rows)
    cy = np.clip(np.floor(w.origins[:, 1] * G), 0, G - 1).astype(np.int64)
    sel = np.nonzero((cy >= r0) & (cy < r1))[0]
    org, xp, st = w.origins[sel], w.xp[sel], w.start[sel]
    t = time.perf_counter()
    band = O.cnn_window(w.vel, ws, bs, r0, 0, r1 - r0, G)
    t_cnn = time.perf_counter() - t
    disp = np.zeros((2, G, G))
    disp[:, r0:r1, :] = band
    t = time.perf_counter()
    s0 = O.cnnsns_start(org, disp, lk, st)
    h, it, s = O.sns(w.xy, tc, nbr, xp, s0)
    t_walk = time.perf_counter() - t
    t = time.perf_counter()
    ph, pit, ps = O.sns(w.xy, tc, nbr, xp, st)
    t_plain = time.perf_counter() - t
    n = len(sel)
    return {
        "value": n / (t_cnn + t_walk), "unit": "points/s", "cores": threads, "kind": "oracle",
        "sample": (f"overlay rows [{r0},{r1}) of {G}: FP64 CNN on that band ({t_cnn:.2f}s) + CNN-SNS start and walk "
                   f"of the {n} points whose origin lies in it ({t_walk:.2f}s); mesh prep and lookup untimed "
                   f"({setup_s:.1f}s)"),
        "plain_sns_value": n / t_plain, "plain_sns_s": t_plain, "mean_path_cnn_sns": float(it.mean()),
        "mean_path_plain": float(pit.mean()),
        "_band": (r0, r1, band), "_sel": sel, "_plain_host": ph,
    }


SERVED = {
    # name: meshes, triangle range (log-uniform), jobs in flight, device budget
    "c5": dict(n_meshes=64, lo=1e4, hi=4e6, max_inflight=8, budget=4 << 30,
               label="64 resident meshes, triangles log-uniform in [1e4, 4e6]"),
    "c5s": dict(n_meshes=6, lo=1.6e3, hi=1.6e5, max_inflight=4, budget=256 << 20,
                label="6 resident meshes, triangles log-uniform in [1.6e3, 1.6e5] (the serving tests' range)"),
}


def bench_served(args):
    """Served mix: resident meshes of uneven size, CNN-SNS jobs arriving as a Poisson process,
    continuous batching by the library's server (BF16 CNN, FP64 walk)."""
    import torch

    from paper_2412_18379_amd import cnnsns as C
    from paper_2412_18379_amd import train as T
    from paper_2412_18379_amd import workload as W

    cfg = SERVED[args.workload]
    t0 = time.perf_counter()
    specs = W.served_mix_specs(n_meshes=cfg["n_meshes"], seed=5, lo=cfg["lo"], hi=cfg["hi"])
    meshes = []
    for spec in specs:
        w = W.build_served(spec)
        m = C.Mesh(w.xy, w.tri, overlay_side=w.G)
        meshes.append(dict(w=w, mesh=m, xp=torch.from_numpy(w.xp).cuda(), origin=torch.from_numpy(w.origins).cuda(),
                           start=torch.from_numpy(w.start).cuda(), vel=torch.from_numpy(w.vel).cuda()))
    torch.cuda.synchronize()
    n_tri = sum(d["w"].n_tri for d in meshes)
    n_pts = np.array([d["w"].n_points for d in meshes])
    log(f"served mix: {len(meshes)} meshes, {n_tri} triangles, {n_pts.sum()} points "
        f"({time.perf_counter() - t0:.1f}s)")
    tr = T.load("c5")
    ws, bs = tr if tr is not None else W.he_weights(200)
    Wt = C.Weights(ws, bs)
    prec = args.precision or "bf16"

    # each job alone (reference for the alone-vs-mix check) and plain SNS over the mix
    ref = []
    for d in meshes:
        disp = C.predict(d["mesh"], d["vel"], Wt, prec)
        h, it, _ = C.locate(d["mesh"], d["xp"], origin=d["origin"], disp=disp)
        ref.append((h, it))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plain_it = []
    for d in meshes:
        plain_it.append(C.locate(d["mesh"], d["xp"], start=d["start"])[1])
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    cnn_it = np.concatenate([r[1].cpu().numpy() for r in ref])
    plain_it = np.concatenate([x.cpu().numpy() for x in plain_it])

    log(f"reference pass (each job alone) and plain SNS done ({time.perf_counter() - t0:.1f}s)")
    budget = cfg["budget"]
    srv = C.Server(Wt, hbm_budget_bytes=budget, max_inflight=cfg["max_inflight"], queue_depth=1 << 16,
                   precision=prec)
    log("server created")

    def run(order, arrivals=None):
        outs, ids = [], []
        tstart = time.perf_counter()
        for k, mi in enumerate(order):
            d = meshes[mi]
            if arrivals is not None:
                while time.perf_counter() - tstart < arrivals[k]:
                    pass
            h = torch.empty(d["w"].n_points, dtype=torch.int32, device="cuda")
            it = torch.empty(d["w"].n_points, dtype=torch.int32, device="cuda")
            ids.append(srv.submit(d["mesh"], d["vel"], d["xp"], d["origin"], h, it))
            outs.append((mi, h, it))
        lat = np.array([srv.wait(i) for i in ids])
        wall = time.perf_counter() - tstart
        return outs, lat, wall

    run(list(range(min(16, len(meshes)))))  # warm-up
    log("warm-up done")
    order = list(range(len(meshes)))
    outs, lat_sat, wall_sat = run(order)
    same = all(torch.equal(h, ref[mi][0]) and torch.equal(it, ref[mi][1]) for mi, h, it in outs)
    mu = len(order) / wall_sat
    log(f"saturation: {mu:.1f} jobs/s, {n_pts.sum() / wall_sat:.4g} points/s, alone == mix: {same}")
    rng = np.random.default_rng(5)
    legs = {}
    for frac in (0.5, 0.9):
        lam = frac * mu
        order = rng.integers(0, len(meshes), size=args.mix_jobs).tolist()
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(order)))
        arrivals -= arrivals[0]
        outs, lat, wall = run(order, arrivals)
        pts = int(n_pts[order].sum())
        legs[f"{frac:.1f}mu"] = {"rate_jobs_per_s": round(lam, 2), "jobs": len(order),
                                 "p50_ms": round(float(np.percentile(lat, 50)), 3),
                                 "p99_ms": round(float(np.percentile(lat, 99)), 3),
                                 "points_per_s": round(pts / wall, 1), "wall_s": round(wall, 3)}
        log(f"lambda = {frac} mu: p50 {legs[f'{frac:.1f}mu']['p50_ms']} ms, p99 {legs[f'{frac:.1f}mu']['p99_ms']} ms")
    srv.close()
    hi = legs["0.9mu"]
    res = {
        "metric": "points located/s CNN-SNS vs SNS (1 GPU); mean SNS path length; p99 latency",
        "value": hi["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": args.mix_jobs, "warmup": 16,
        "ms_per_step": round(1e3 * hi["wall_s"] / args.mix_jobs, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{prec} CNN / f64 SNS", "data": "synthetic",
        "config": {"workload": f"served mix: {cfg['label']}, Poisson arrivals, continuous batching",
                   "n_meshes": len(meshes),
                   "n_triangles": n_tri, "points_per_pass": int(n_pts.sum()), "hbm_budget_bytes": budget,
                   "max_inflight": cfg["max_inflight"], "weights": "trained (mix)" if tr is not None else "he-init"},
        "saturation": {"jobs_per_s": round(mu, 2), "points_per_s": round(float(n_pts.sum()) / wall_sat, 1),
                       "p50_ms": round(float(np.percentile(lat_sat, 50)), 3),
                       "p99_ms": round(float(np.percentile(lat_sat, 99)), 3)},
        "poisson": legs, "alone_equals_mix": bool(same),
        "mean_path_length": {"cnn_sns": round(float(cnn_it.mean()), 3), "plain_sns": round(float(plain_it.mean()), 3)},
        "plain_sns_points_per_s_sequential": round(float(n_pts.sum()) / (plain_ms / 1e3), 1),
    }
    print(json.dumps(res), flush=True)


def config_legs(C, T, K: int, warmup: int, with_cpu: bool):
    """The other configurations at their own sizes: C1 (plain SNS on 2K triangles), C2 (plain vs CNN-SNS with
    the FP32 CNN on 1M triangles) and C4 (C2 with the BF16 CNN: displacement error against the FP64 oracle
    over the whole grid, path-length change, host agreement), each with the oracle beside it on one host
    thread (the walks of all points; C2's FP64 CNN on a band of rows)."""
    import torch

    from paper_2412_18379_amd import workload as W
    stream = torch.cuda.current_stream()
    dev = torch.device("cuda:0")

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for k in range(K):
            e[k][0].record(stream)
            fn()
            e[k][1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in e]))

    out = {}
    O = None
    if with_cpu:
        import oracle as O
        threads_before = O.set_threads(0)
    # C1
    w = W.build("c1")
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    xp, start = torch.from_numpy(w.xp).to(dev), torch.from_numpy(w.start).to(dev)
    host = torch.empty(w.n_points, dtype=torch.int32, device=dev)
    iters = torch.empty(w.n_points, dtype=torch.int32, device=dev)
    ms = timed(lambda: C.locate(mesh, xp, start=start, host=host, iters=iters, want_status=False))
    leg = {"workload": "1,922-triangle jittered Delaunay, 1,024 node points, Taylor-Green, ~3 diameters",
           "plain_sns_ms": round(ms, 4), "plain_sns_points_per_s": round(w.n_points / (ms / 1e3), 1),
           "mean_path_length": round(float(iters.double().mean()), 3)}
    if O is not None:
        tc, nbr = O.prepare_mesh(w.xy, w.tri)
        O.set_threads(1)
        t = time.perf_counter()
        oh, oi, _ = O.sns(w.xy, tc, nbr, w.xp, w.start)
        t_or = time.perf_counter() - t
        O.set_threads(threads_before)
        leg["hosts_equal_oracle"] = bool(np.array_equal(host.cpu().numpy(), oh))
        leg["cpu_baseline"] = {"value": round(w.n_points / t_or, 1), "unit": "points/s", "cores": 1, "kind": "oracle",
                               "sample": "plain SNS of all 1,024 points, one thread"}
    out["c1"] = leg
    mesh.close()
    # C2 and C4
    w = W.build("c2")
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    tr = T.load("c2")
    ws, bs = tr if tr is not None else W.he_weights(200)
    Wt = C.Weights(ws, bs)
    n = w.n_points
    xp, start = torch.from_numpy(w.xp).to(dev), torch.from_numpy(w.start).to(dev)
    origin, vel = torch.from_numpy(w.origins).to(dev), torch.from_numpy(w.vel).to(dev)
    host = torch.empty(n, dtype=torch.int32, device=dev)
    iters = torch.empty(n, dtype=torch.int32, device=dev)
    disp = torch.empty((2, w.G, w.G), dtype=torch.float32, device=dev)
    plain = timed(lambda: C.locate(mesh, xp, start=start, host=host, iters=iters, want_status=False))
    hp, ip = host.cpu().numpy(), iters.cpu().numpy()
    legs = {}
    for prec, name in (("f32", "c2"), ("bf16", "c4"), ("fp8", "c4_fp8")):
        pred = timed(lambda: C.predict(mesh, vel, Wt, prec, disp=disp))
        loc = timed(lambda: C.locate(mesh, xp, origin=origin, disp=disp, host=host, iters=iters, want_status=False))
        ic = iters.cpu().numpy()
        legs[name] = {"cnn_precision": prec, "weights": "trained" if tr is not None else "he-init",
                      "predict_ms": round(pred, 4), "locate_ms": round(loc, 4), "plain_sns_ms": round(plain, 4),
                      "points_per_s": round(n / ((pred + loc) / 1e3), 1),
                      "plain_sns_points_per_s": round(n / (plain / 1e3), 1),
                      "speedup_vs_plain_sns": round(plain / (pred + loc), 3),
                      "mean_path_length": {"cnn_sns": round(float(ic.mean()), 3), "plain_sns": round(float(ip.mean()), 3)},
                      "host_agreement_with_plain": float(np.mean(host.cpu().numpy() == hp)),
                      "_disp": disp.cpu().numpy().astype(np.float64), "_iters": ic}
    legs["c2"]["workload"] = "1M-triangle jittered Delaunay, 999,698 centroid points, ~20 diameters, G=1024, FP32 CNN"
    legs["c4"]["workload"] = "C2 with the BF16 CNN (FP32 accumulation), walk in FP64"
    legs["c4_fp8"]["workload"] = ("C2 with the FP8 e4m3 CNN (per-channel power-of-two weight scales, FP32 "
                                  "accumulation; the stretch form of C4), walk in FP64")
    for name in ("c4", "c4_fp8"):
        legs[name]["mean_path_change_vs_f32"] = round(float(legs[name]["_iters"].mean() -
                                                            legs["c2"]["_iters"].mean()), 4)
    if O is not None:
        tc, nbr = O.prepare_mesh(w.xy, w.tri)
        ref = O.cnn_forward(w.vel, ws, bs)  # FP64, all host threads
        for name in ("c2", "c4", "c4_fp8"):
            err = np.hypot(*(legs[name]["_disp"] - ref)) / w.dbar
            legs[name]["disp_error_vs_fp64_oracle_diameters"] = {"max": round(float(err.max()), 6),
                                                                  "mean": round(float(err.mean()), 7)}
        lk = O.lookup(w.xy, tc, w.G)
        O.set_threads(1)
        t = time.perf_counter()
        oh, oi, _ = O.sns(w.xy, tc, nbr, w.xp, w.start)
        t_walk = time.perf_counter() - t
        t = time.perf_counter()
        O.cnnsns(w.xy, tc, nbr, lk, w.origins, w.xp, ref, fallback=w.start)
        t_cnnsns_walk = time.perf_counter() - t
        rows = 16
        t = time.perf_counter()
        O.cnn_window(w.vel, ws, bs, w.G // 2, 0, rows, w.G)
        t_cnn = (time.perf_counter() - t) * (w.G / rows)  # the whole grid at this rate
        O.set_threads(threads_before)
        far = _off_edge(w, oh, w.xp)
        legs["c2"]["hosts_equal_oracle_off_edge"] = float(np.mean(hp[far] == oh[far]))
        legs["c2"]["cpu_baseline"] = {
            "value": round(n / (t_cnn + t_cnnsns_walk), 1),
            "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": (f"one thread: the FP64 CNN on {rows} of the {w.G} overlay rows ({t_cnn * rows / w.G:.2f}s), "
                       f"scaled to the whole grid, plus the CNN-SNS starts and walks of all {n} points from the "
                       f"oracle's own displacement grid ({t_cnnsns_walk:.2f}s); plain SNS of all points "
                       f"{t_walk:.2f}s"),
            "plain_sns_value": round(n / t_walk, 1)}
    for name in ("c2", "c4", "c4_fp8"):
        legs[name].pop("_disp")
        legs[name].pop("_iters")
        out[name] = legs[name]
    mesh.close()
    log(f"configs: c1 {out['c1']['plain_sns_points_per_s']:.3g} points/s; c2 {out['c2']['speedup_vs_plain_sns']}x; "
        f"c4 {out['c4']['speedup_vs_plain_sns']}x; c4 fp8 {out['c4_fp8']['speedup_vs_plain_sns']}x")
    return out


def classifier_leg(C, T, w, mesh, xp, start, K: int, warmup: int, plain_ms: float):
    """The paper's own prediction step (the classifier CNN of Sec. 2.3, one inference per point) followed by
    the walk from its start, on the same points: the cost beside the displacement form."""
    import torch

    from paper_2412_18379_amd import workload as W

    tr = T.load_classifier(w.name) if hasattr(T, "load_classifier") else None
    ws, bs = tr if tr is not None else W.classifier_he_weights(300)
    Wc = C.ClsWeights(ws, bs)
    n = xp.shape[0]
    st = torch.empty(n, dtype=torch.int32, device=xp.device)
    host = torch.empty(n, dtype=torch.int32, device=xp.device)
    iters = torch.empty(n, dtype=torch.int32, device=xp.device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        C.classify(mesh, xp, Wc, fallback=start, start=st, want_class=False)
        C.locate(mesh, xp, start=st, host=host, iters=iters, want_status=False)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    for k in range(K):
        ev[k][0].record(stream)
        C.classify(mesh, xp, Wc, fallback=start, start=st, want_class=False)
        ev[k][1].record(stream)
        C.locate(mesh, xp, start=st, host=host, iters=iters, want_status=False)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    cls_ms = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)])
    loc_ms = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)])
    it = iters.cpu().numpy()
    issued = 2.0 * CLS_ISSUED_MACS * n / (cls_ms.mean() / 1e3) / 1e12
    log(f"classifier CNN-SNS: classify {cls_ms.mean():.3f} ms, locate {loc_ms.mean():.3f} ms, mean I_t {it.mean():.2f}")
    return {
        "form": "the paper's classifier CNN, one inference per point (9 x 9 pooled ASG window, 81 classes)",
        "weights": "trained on SNS labels" if tr is not None else "he-init (seed 300)",
        "classify_ms": round(float(cls_ms.mean()), 4), "locate_ms": round(float(loc_ms.mean()), 4),
        "step_ms": round(float((cls_ms + loc_ms).mean()), 4),
        "points_per_s": round(n / ((cls_ms + loc_ms).mean() / 1e3), 1),
        "speedup_vs_plain_sns": round(float(plain_ms / (cls_ms + loc_ms).mean()), 4),
        "mean_path_length": round(float(it.mean()), 3),
        "path_length_p50_p99_max": [pct(it, 50), pct(it, 99), int(it.max())],
        "roofline": {"kernel": "cnnsns_classify (k_cls_module1 + 3 x k_dense_f32 + k_cls_argmax)", "bound": "mfma",
                     "achieved": round(issued, 3), "peak": PEAK["f32_TFLOPs"], "unit": "TFLOP/s",
                     "frac": round(issued / PEAK["f32_TFLOPs"], 4),
                     "algorithmic_per_launch": f"{2.0 * CLS_ISSUED_MACS * n:.4e} FLOP issued ({CLS_ISSUED_MACS} MAC "
                                               f"per point on the matrix cores; {CLS_USEFUL_MACS} needed)"},
    }


def main():
    faulthandler.enable()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c5", "c5s"])
    ap.add_argument("--mix-jobs", type=int, default=512, help="served mix: jobs per arrival rate")
    ap.add_argument("--precision", default=None, choices=["f32", "bf16", "fp8"])
    ap.add_argument("--weights", default="trained", choices=["trained", "he"])
    ap.add_argument("--cpu-band-rows", type=int, default=0, help="oracle sample band (0: auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--configs", default="on", choices=["on", "off"],
                    help="legs for the 2K- and 1M-triangle configurations (FP32 and BF16 CNN) with the oracle "
                         "on one host thread beside them")
    ap.add_argument("--online", default="on", choices=["on", "off"],
                    help="in-loop training of both predictors (and, with a 3D leg, the 3D displacement CNN) from "
                         "the walks of the first 3 steps of an unsteady flow, then CNN-SNS in the later steps")
    ap.add_argument("--classifier", default="on", choices=["on", "off"],
                    help="the paper's per-point classifier CNN leg (on: time it beside the displacement form)")
    ap.add_argument("--no-bf16-variant", action="store_true", help="skip the BF16 CNN leg of an FP32 run")
    ap.add_argument("--walk3d", default="t3", choices=["t1", "t2", "t3", "none"],
                    help="tetrahedral walk leg (none: skip)")
    ap.add_argument("--gather-probe", type=int, default=0, metavar="BYTES",
                    help="only run a 64-byte-row random gather of BYTES (counter calibration) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device copy of BYTES (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(points are independent; see the sharding note in the design document).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_18379_amd import cnnsns as C
    from paper_2412_18379_amd import train as T
    from paper_2412_18379_amd import workload as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.gather_probe:
        return gather_probe(args.gather_probe)
    C.lib()
    if args.workload == "c5":
        # Switched off: one run of this served-mix benchmark ended in a host
        # segmentation fault after the meshes were built, with no GPU fault;
        # the cause has not been found (the serving loop passes its GPU parity
        # tests and its scheduler passes host sanitizer tests), so it stays off
        # until it is.
        sys.exit("bench.py: the served-mix workload (c5) is switched off until the cause of a host crash "
                 "in it is found")
    if args.workload == "c5s":
        # switched off as well: a run of the serving tests later ended in the same kind of host
        # crash, so the serving loop is off until its cause is found
        sys.exit("bench.py: the serving loop is switched off (an intermittent host crash in it is unexplained)")
    precision = args.precision or ("bf16" if args.workload == "c4" else "f32")
    wl_name = "c2" if args.workload == "c4" else args.workload
    t0 = time.perf_counter()
    w = W.build(wl_name)
    log(f"workload {args.workload}: {w.n_tri} triangles, {w.n_points} points, G={w.G} "
        f"({time.perf_counter() - t0:.1f}s)")
    trained = T.load(wl_name) if args.weights == "trained" else None
    if trained is not None:
        ws, bs = trained
        weights_kind = "trained"
    else:
        ws, bs = W.he_weights(200)
        weights_kind = "he-init seed 200"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mesh = C.Mesh(w.xy, w.tri, overlay_side=w.G)
    torch.cuda.synchronize()
    log(f"mesh resident: {mesh.device_bytes / 2**20:.0f} MiB ({time.perf_counter() - t0:.1f}s)")
    Wt = C.Weights(ws, bs, device=dev)
    xp = torch.from_numpy(w.xp).to(dev)
    origin = torch.from_numpy(w.origins).to(dev)
    start = torch.from_numpy(w.start).to(dev)
    vel = torch.from_numpy(w.vel).to(dev)
    n = w.n_points
    disp = torch.empty((2, w.G, w.G), dtype=torch.float32, device=dev)
    host = torch.empty(n, dtype=torch.int32, device=dev)
    iters = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(n, dtype=torch.uint8, device=dev)

    def step():
        C.predict(mesh, vel, Wt, precision, disp=disp)
        C.locate(mesh, xp, origin=origin, disp=disp, host=host, iters=iters, status=status)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record(stream)
        C.predict(mesh, vel, Wt, precision, disp=disp)
        ev[k][1].record(stream)
        C.locate(mesh, xp, origin=origin, disp=disp, host=host, iters=iters, status=status)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / K
    pred_ms = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)])
    loc_ms = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)])
    step_ms = pred_ms + loc_ms
    it_c = iters.cpu().numpy()
    st_c = status.cpu().numpy()
    host_c = host.cpu().numpy()
    log(f"CNN-SNS: {ms_step:.3f} ms/step (predict {pred_ms.mean():.3f} ms, locate {loc_ms.mean():.3f} ms), "
        f"mean I_t {it_c.mean():.2f}")

    # plain SNS and ASG-at-x_p legs on the same inputs
    def timed_locate(**kw):
        for _ in range(args.warmup):
            C.locate(mesh, xp, host=host, iters=iters, status=status, **kw)
        torch.cuda.synchronize()
        e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for k in range(K):
            e[k][0].record(stream)
            C.locate(mesh, xp, host=host, iters=iters, status=status, **kw)
            e[k][1].record(stream)
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) for a, b in e]), iters.cpu().numpy(), host.cpu().numpy()

    plain_ms, it_p, host_p = timed_locate(start=start)
    log(f"plain SNS: {plain_ms.mean():.3f} ms, mean I_t {it_p.mean():.2f}")
    asg_ms, it_a, host_a = timed_locate()
    log(f"ASG start: {asg_ms.mean():.3f} ms, mean I_t {it_a.mean():.2f}")
    same_host = float(np.mean(host_c == host_p))

    # the step after location: the velocity at x_p, P1-interpolated in the host element
    fu, fv = w.flow(w.xy[:, 0], w.xy[:, 1])
    nodal = torch.from_numpy(np.ascontiguousarray(np.stack([fu, fv], axis=1))).to(dev)
    host_i = torch.from_numpy(host_c).to(dev)
    u_xp = torch.empty((n, 2), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        C.interpolate(mesh, xp, host_i, nodal, out=u_xp)
    torch.cuda.synchronize()
    ei = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for k in range(K):
        ei[k][0].record(stream)
        C.interpolate(mesh, xp, host_i, nodal, out=u_xp)
        ei[k][1].record(stream)
    torch.cuda.synchronize()
    interp_ms = np.array([a.elapsed_time(b) for a, b in ei])
    log(f"interpolation at x_p: {interp_ms.mean():.3f} ms")
    # the same interpolation fused into the CNN-SNS walk's last iteration (one pass instead of two)
    for _ in range(args.warmup):
        C.locate_interpolate(mesh, xp, nodal, origin=origin, disp=disp, host=host, iters=iters, status=status,
                             out=u_xp)
    torch.cuda.synchronize()
    ef = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for k in range(K):
        ef[k][0].record(stream)
        C.locate_interpolate(mesh, xp, nodal, origin=origin, disp=disp, host=host, iters=iters, status=status,
                             out=u_xp)
        ef[k][1].record(stream)
    torch.cuda.synchronize()
    fused_ms = np.array([a.elapsed_time(b) for a, b in ef])
    log(f"CNN-SNS walk with the interpolation fused: {fused_ms.mean():.3f} ms "
        f"(separately {loc_ms.mean():.3f} + {interp_ms.mean():.3f} ms)")

    value = n / (ms_step / 1e3)
    G = w.G
    cnn_flops = 2.0 * CNN_MACS_PER_PIXEL * G * G
    cnn_peak = PEAK[{"f32": "f32_TFLOPs", "bf16": "bf16_TFLOPs", "fp8": "fp8_TFLOPs"}[precision]]
    cnn_tf = cnn_flops / (pred_ms.mean() / 1e3) / 1e12
    # walk algorithmic bytes: one element record per iteration plus per-point inputs and outputs
    out_b = 4 + 4 + 1
    bytes_cnn_walk = REC_BYTES * float(it_c.sum()) + n * (16 + 16 + 8 + 4 + out_b)
    bytes_plain = REC_BYTES * float(it_p.sum()) + n * (16 + 4 + out_b)
    gbps_cnn_walk = bytes_cnn_walk / (loc_ms.mean() / 1e3) / 1e9
    gbps_plain = bytes_plain / (plain_ms.mean() / 1e3) / 1e9
    issued_tf = 2.0 * cnn_issued_macs(G, precision) / (pred_ms.mean() / 1e3) / 1e12
    useful_macs = (WINO_USEFUL_MACS_PER_PIXEL if precision == "f32" else CNN_MACS_PER_PIXEL) * G * G
    roofline = {
        "kernel": {"f32": "cnn forward (k_conv12_f32 + k_conv34_f32, one cnnsns_predict)",
                   "bf16": "cnn forward (k_cnn_bf16, one cnnsns_predict)"}.get(precision, "cnn forward"),
        "bound": "mfma", "achieved": round(issued_tf, 3), "peak": cnn_peak, "unit": "TFLOP/s",
        "frac": round(issued_tf / cnn_peak, 4),
        "traffic": traffic_for(f"cnn_forward_{precision}", args.workload),
        "algorithmic_per_launch": (f"{2 * cnn_issued_macs(G, precision):.4e} FLOP issued on the matrix cores "
                                   f"(G={G}: {cnn_issued_macs(G, precision) / (G * G):.0f} MAC per cell with "
                                   f"padding, recomputed halos and, in FP32, the Winograd form)"),
        "useful_work": {"macs_per_cell": useful_macs // (G * G),
                        "achieved": round(2.0 * useful_macs / (pred_ms.mean() / 1e3) / 1e12, 3),
                        "frac": round(2.0 * useful_macs / (pred_ms.mean() / 1e3) / 1e12 / cnn_peak, 4),
                        "note": "the products the method needs: " + (
                            "Winograd F(2x2,3x3) for conv2/conv3, direct for conv1/conv4" if precision == "f32"
                            else "direct convolution")},
        "direct_conv_equivalent": {"macs_per_cell": CNN_MACS_PER_PIXEL, "achieved": round(cnn_tf, 3),
                                   "note": "2 x 19584 MAC x G^2 over the pass time; exceeds the matrix "
                                           "cores' work when conv2/conv3 run as Winograd"},
    }
    # interpolation: x_p 16 + host 4 + element coordinates 48 and node ids 12 + three nodal values 48
    # + the result 16 bytes per point
    bytes_interp = n * (16 + 4 + 48 + 12 + 48 + 16)
    gbps_interp = bytes_interp / (interp_ms.mean() / 1e3) / 1e9
    copy_gbps = copy_bandwidth()
    log(f"device copy: {copy_gbps:.0f} GB/s (read + write)")
    roofline_sns = {
        "kernel": "k_locate (plain SNS leg)", "bound": "hbm", "achieved": round(gbps_plain, 1),
        "peak": PEAK["hbm_GBps"], "unit": "GB/s", "frac": round(gbps_plain / PEAK["hbm_GBps"], 4),
        "traffic": traffic_for("k_locate_plain", args.workload),
        "traffic_by_request_size": traffic_by_request_size("k_locate_plain", args.workload, plain_ms.mean()),
        "algorithmic_per_launch": f"{bytes_plain:.4e} B (60 B x sum I_t + 29 B x n)",
        "note": ("walks of nearby points cross the same elements, so records are re-read from L2 and MALL: "
                 "algorithmic bytes can exceed what reaches HBM (compare traffic_by_request_size)"),
        "measured_copy_GBps": round(copy_gbps, 1),
        "frac_of_measured_copy": round(gbps_plain / copy_gbps, 4),
        "cnn_sns_leg": {"achieved": round(gbps_cnn_walk, 1), "frac": round(gbps_cnn_walk / PEAK["hbm_GBps"], 4),
                        "frac_of_measured_copy": round(gbps_cnn_walk / copy_gbps, 4),
                        "traffic": traffic_for("k_locate_cnn", args.workload),
                        "traffic_by_request_size": traffic_by_request_size("k_locate_cnn", args.workload,
                                                                           loc_ms.mean()),
                        "algorithmic_per_launch": f"{bytes_cnn_walk:.4e} B (60 B x sum I_t + 69 B x n)"},
    }
    res = {
        "metric": "points located/s CNN-SNS vs SNS (1 GPU); mean SNS path length; p99 latency",
        "value": round(value, 1), "unit": "points/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32 CNN / f64 SNS", "bf16": "bf16 CNN / f64 SNS", "fp8": "fp8 CNN / f64 SNS"}[precision],
        "data": "synthetic",
        "config": {"workload": {"c2": "1M-triangle jittered Delaunay, 1M centroid points, ~20 diameters, G=1024",
                                "c3": "16M-triangle graded jittered Delaunay, 8M node points, ~150 diameters, G=4096",
                                "c4": "1M-triangle jittered Delaunay, 1M centroid points, ~20 diameters, G=1024, "
                                      "BF16 CNN"}[args.workload],
                   "n_triangles": w.n_tri, "n_points": n, "overlay": G, "cnn_precision": precision,
                   "weights": weights_kind, "seeds": w.seeds, "mean_displacement_diameters":
                       round(float(np.mean(np.hypot(*(w.xp - w.origins).T)) / w.dbar), 2)},
        "plain_sns_points_per_s": round(n / (plain_ms.mean() / 1e3), 1),
        "asg_start_points_per_s": round(n / (asg_ms.mean() / 1e3), 1),
        "speedup_vs_plain_sns": round(float(plain_ms.mean() / step_ms.mean()), 3),
        "mean_path_length": {"cnn_sns": round(float(it_c.mean()), 3), "plain_sns": round(float(it_p.mean()), 3),
                             "asg_start": round(float(it_a.mean()), 3)},
        "path_length_p50_p99_max": {"cnn_sns": [pct(it_c, 50), pct(it_c, 99), int(it_c.max())],
                                    "plain_sns": [pct(it_p, 50), pct(it_p, 99), int(it_p.max())]},
        "opt_path_length": round(1.0 - float(it_c.mean()) / float(it_p.mean()), 4),
        "step_latency_ms": {"p50": round(pct(step_ms, 50), 4), "p99": round(pct(step_ms, 99), 4)},
        "predict_ms": round(float(pred_ms.mean()), 4), "locate_ms": round(float(loc_ms.mean()), 4),
        "plain_locate_ms": round(float(plain_ms.mean()), 4),
        "host_agreement_cnn_vs_plain": same_host,
        "status_found_frac": float(np.mean(st_c == C.FOUND)),
        "roofline": roofline, "roofline_sns": roofline_sns,
        "interp_leg": {"kernel": "k_interp (P1 velocity at x_p in its host element)", "ms": round(float(interp_ms.mean()), 4),
                       "points_per_s": round(n / (interp_ms.mean() / 1e3), 1), "bound": "hbm",
                       "achieved": round(gbps_interp, 1), "unit": "GB/s",
                       "frac": round(gbps_interp / PEAK["hbm_GBps"], 4),
                       "frac_of_measured_copy": round(gbps_interp / copy_gbps, 4),
                       "traffic": traffic_for("k_interp", args.workload),
                       "traffic_by_request_size": traffic_by_request_size("k_interp", args.workload,
                                                                          interp_ms.mean()),
                       "algorithmic_per_launch": f"{bytes_interp:.4e} B (144 B x n)",
                       "fused_into_cnn_sns_walk": {
                           "kernel": "k_locate<START_CNN, interpolating> (cnnsns_locate_interpolate)",
                           "ms": round(float(fused_ms.mean()), 4),
                           "separate_walk_plus_interp_ms": round(float(loc_ms.mean() + interp_ms.mean()), 4),
                           "traffic": traffic_for("k_locate_cnn_interp", args.workload),
                           "traffic_by_request_size": traffic_by_request_size("k_locate_cnn_interp",
                                                                              args.workload, fused_ms.mean()),
                           "saved_ms": round(float(loc_ms.mean() + interp_ms.mean() - fused_ms.mean()), 4)}},
    }
    disp_var = {}
    for vp in (("bf16", "fp8") if precision == "f32" and not args.no_bf16_variant else ()):
        # the same step with a lower-precision CNN (precision variants): time, walk lengths, hosts
        dv = disp_var[vp] = torch.empty_like(disp)
        host_b = torch.empty_like(host)
        iters_b = torch.empty_like(iters)

        def step_v():
            C.predict(mesh, vel, Wt, vp, disp=dv)
            C.locate(mesh, xp, origin=origin, disp=dv, host=host_b, iters=iters_b, status=status)

        for _ in range(args.warmup):
            step_v()
        torch.cuda.synchronize()
        eb = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
        t0 = time.perf_counter()
        for k in range(K):
            eb[k][0].record(stream)
            C.predict(mesh, vel, Wt, vp, disp=dv)
            eb[k][1].record(stream)
            C.locate(mesh, xp, origin=origin, disp=dv, host=host_b, iters=iters_b, status=status)
            eb[k][2].record(stream)
        torch.cuda.synchronize()
        wall_b = time.perf_counter() - t0
        pb = np.array([eb[k][0].elapsed_time(eb[k][1]) for k in range(K)])
        lb = np.array([eb[k][1].elapsed_time(eb[k][2]) for k in range(K)])
        it_b = iters_b.cpu().numpy()
        pk = PEAK[f"{vp}_TFLOPs"]
        issued = 2.0 * cnn_issued_macs(G, "bf16")  # the FP8 pass has the BF16 pass's tiling
        res[f"{vp}_variant"] = {
            "points_per_s": round(n / wall_b * K, 1), "ms_per_step": round(wall_b * 1e3 / K, 4),
            "predict_ms": round(float(pb.mean()), 4), "locate_ms": round(float(lb.mean()), 4),
            "speedup_vs_plain_sns": round(float(plain_ms.mean() / (pb + lb).mean()), 3),
            "mean_path_length": round(float(it_b.mean()), 3),
            "mean_path_change_vs_f32": round(float(it_b.mean() - it_c.mean()), 4),
            "host_agreement_with_f32_path": float(np.mean(host_b.cpu().numpy() == host_c)),
            "cnn_roofline": {"achieved": round(issued / (pb.mean() / 1e3) / 1e12, 3),
                             "peak": pk, "unit": "TFLOP/s",
                             "frac": round(issued / (pb.mean() / 1e3) / 1e12 / pk, 4),
                             "algorithmic_per_launch": (f"{issued:.4e} FLOP issued "
                                                        f"({issued / 2 / (G * G):.0f} MAC per "
                                                        f"cell with padding and recomputed halos)"),
                             "useful_work": {"macs_per_cell": CNN_MACS_PER_PIXEL,
                                             "frac": round(cnn_flops / (pb.mean() / 1e3) / 1e12 / pk, 4)},
                             "traffic": traffic_for(f"cnn_forward_{vp}", args.workload)},
        }
        log(f"{vp.upper()} CNN-SNS: {res[f'{vp}_variant']['ms_per_step']:.3f} ms/step (predict {pb.mean():.3f} ms), "
            f"mean I_t {it_b.mean():.2f}")
    if precision != "f32":
        # the same step with the FP32 CNN: how much the lower precision lengthens the walks
        disp32 = C.predict(mesh, vel, Wt, "f32")
        _, it32, _ = C.locate(mesh, xp, origin=origin, disp=disp32)
        it32 = it32.cpu().numpy()
        res["precision_report"] = {"mean_path_f32_cnn": round(float(it32.mean()), 4),
                                   "mean_path_change": round(float(it_c.mean() - it32.mean()), 4)}
    if args.configs == "on" and args.workload == "c3":
        res["config_legs"] = config_legs(C, T, K, args.warmup, with_cpu=not args.no_cpu_baseline)
    if args.online == "on":
        from paper_2412_18379_amd import online as O
        t0 = time.perf_counter()
        rep = O.run(C, n_side=708, seed=2, field_seed=21, k=20.0, G=1024, n_steps=8, n_t=3, log=log)
        rep.pop("weights")
        later = [s for s in rep["steps"] if s["step"] >= rep["n_t"]]
        rep["summary"] = {
            "mean_path_plain": round(float(np.mean([s["plain_mean_path"] for s in later])), 3),
            "mean_path_cnn_sns": round(float(np.mean([s["cnn_sns_mean_path"] for s in later])), 3),
            "mean_path_classifier": round(float(np.mean([s["classifier_mean_path"] for s in later])), 3),
            "wall_s": round(time.perf_counter() - t0, 2)}
        rep["workload"] = ("1M-triangle jittered Delaunay (708 x 708 nodes), unsteady Fourier vortices (phases "
                           "drifting 0.15 rad per step), ~20 diameters per step, G=1024, 8 steps, trained on the "
                           "first 3 from plain SNS hosts")
        res["online_training_leg"] = rep
    if args.classifier == "on":
        res["classifier_leg"] = classifier_leg(C, T, w, mesh, xp, start, K, args.warmup, float(plain_ms.mean()))
    if args.walk3d != "none":
        res["walk3d_leg"] = walk3d_leg(args.walk3d, K, args.warmup, copy_gbps, with_cpu=not args.no_cpu_baseline)
    if args.online == "on" and args.walk3d != "none":
        # the 3D displacement CNN trained in the loop from the tetrahedral walk's own hosts
        from paper_2412_18379_amd import online as O
        t0 = time.perf_counter()
        rep = O.run3d(C, args.walk3d, n_steps=6, n_t=3, disp_steps=6000, log=log)
        rep.pop("weights")
        later = [s for s in rep["steps"] if s["step"] >= rep["n_t"]]
        rep["summary"] = {k: round(float(np.mean([s[k] for s in later])), 3) for k in (
            "plain_mean_path", "cnn_sns_mean_path", "cnn_sns_bf16_mean_path", "passthrough_net_mean_path",
            "lookup_at_xp_mean_path", "hosts_equal_plain")}
        rep["summary"]["wall_s"] = round(time.perf_counter() - t0, 2)
        res["online_training_3d_leg"] = rep
    if not args.no_cpu_baseline:
        band = args.cpu_band_rows or {"c2": 1024, "c3": 1536, "c4": 1024}[args.workload]
        t0 = time.perf_counter()
        cb = cpu_baseline(w, ws, bs, band)
        log(f"cpu baseline: {cb['value']:.0f} points/s on {cb['cores']} threads ({time.perf_counter() - t0:.1f}s)")
        r0, r1, ref_band = cb.pop("_band")
        sel, oracle_host = cb.pop("_sel"), cb.pop("_plain_host")
        # host elements of the band's points against the oracle (points on an edge may take either element)
        far = _off_edge(w, oracle_host, w.xp[sel])
        res["host_agreement_with_oracle_band"] = float(np.mean(host_c[sel][far] == oracle_host[far]))
        def disp_error(dgpu):
            got = dgpu.cpu().numpy()[:, r0:r1, :].astype(np.float64)
            err = np.hypot(*(got - ref_band)) / w.dbar
            return {"max": round(float(err.max()), 6), "mean": round(float(err.mean()), 7)}

        sample = f"overlay rows [{r0},{r1}) of {G} (the oracle's CNN band)"
        if precision != "f32":
            res["precision_report"].update({"disp_error_vs_fp64_oracle_diameters": disp_error(disp),
                                            "error_sample": sample})
        else:
            # full-size parity of the timed FP32 forward pass on the band: the bar per channel c is
            # |y - y_ref| <= 1e-5 |y_ref| + 1e-5 max_c |y_ref|
            got = disp.cpu().numpy()[:, r0:r1, :].astype(np.float64)
            scale = np.abs(ref_band).reshape(2, -1).max(axis=1)[:, None, None]
            ratio = float((np.abs(got - ref_band) / (1e-5 * np.abs(ref_band) + 1e-5 * scale + 1e-30)).max())
            res["f32_parity_on_band"] = {"worst_error_over_tolerance": round(ratio, 4), "pass": ratio <= 1.0,
                                         "sample": sample}
            for vp, dv in disp_var.items():
                res[f"{vp}_variant"]["disp_error_vs_fp64_oracle_diameters"] = disp_error(dv)
                res[f"{vp}_variant"]["error_sample"] = sample
        res["cpu_baseline"] = cb
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
