"""In-loop training of the start predictors from the walk's own output (triangular and tetrahedral
meshes).

After Sec. 2.3 (training data from SNS: the host K_t the walk finds is the
label, cross-entropy, Adam) and Sec. 3.1 (train on the first n_t = 3 time steps,
then predict in the later ones).  A time-dependent flow advances step by step;
in every step each mesh node is moved back along the flow, x_p = x_i - dt
u_s(x_i) (eq. 3, clamped into the domain), and located.  In the first n_t steps
the points are located by plain SNS from the element before movement
(cnnsns_locate), and its output hosts become the training data:

* the displacement CNN (2 -> 32 -> 32 -> 32 -> 2): per overlay cell, the mean
  over the cell's origins x_i of centroid(K_t) - x_i, a masked mean-squared
  error over the whole grid (its zero padding as in the library);
* the classifier CNN (Sec. 2.3): per point, the class of the window cell
  holding the centroid of K_t (B'_l = 1 for that class), softmax
  cross-entropy.

Both train with Adam on the GPU (PyTorch autograd: this is the training
harness, not the located-point path), and the trained FP32 weights are then
used by the library's own calls (cnnsns_predict, cnnsns_classify) on the
resident mesh for the later steps, whose walks start from their predictions.
"""
from __future__ import annotations

import os
import time

# the convolution layers' first call would otherwise search MIOpen's algorithms exhaustively (about a
# minute for the full-grid shapes); training takes the first applicable one
os.environ.setdefault("MIOPEN_FIND_MODE", "FAST")

import numpy as np
import torch

from . import workload as W

CLS_SHAPES = [(16, 2, 3, 3), (16, 16, 3, 3), (256, 2), (256, 256), (512, 512), (81, 512)]


def centroids_by_id(xy: torch.Tensor, tri: torch.Tensor) -> torch.Tensor:
    """Element centroids with the vertices summed in ascending node id (FP64 [n_tri][2])."""
    ids, _ = torch.sort(tri.long(), dim=1)
    v = xy[ids]  # [n_tri][3][2]
    return ((v[:, 0] + v[:, 1]) + v[:, 2]) / 3.0


def cell_of(x: torch.Tensor, G: int) -> torch.Tensor:
    """min(G - 1, floor(x G)), 0 for negative values and NaN."""
    f = torch.floor(x * G)
    f = torch.where(f >= 0, f, torch.zeros_like(f))
    return torch.clamp(f, max=G - 1).long()


def displacement_targets(cent: torch.Tensor, origins: torch.Tensor, host: torch.Tensor, G: int):
    """Per overlay cell the mean of centroid(host) - x_i over the origins x_i in it, and the mask of cells
    that hold one ([2][G][G] FP32, [G][G] bool).  Points whose host is not an element are left out."""
    ok = (host >= 0) & (host < cent.shape[0])
    o, h = origins[ok], host[ok].long()
    d = cent[h] - o
    cell = cell_of(o[:, 1], G) * G + cell_of(o[:, 0], G)
    cnt = torch.zeros(G * G, dtype=torch.float64, device=o.device).index_add_(0, cell, torch.ones_like(d[:, 0]))
    t = torch.zeros((2, G * G), dtype=torch.float64, device=o.device)
    t[0].index_add_(0, cell, d[:, 0])
    t[1].index_add_(0, cell, d[:, 1])
    mask = cnt > 0
    t[:, mask] /= cnt[mask]
    return t.reshape(2, G, G).float(), mask.reshape(G, G)


def class_labels(cent: torch.Tensor, xp: torch.Tensor, host: torch.Tensor, G: int) -> torch.Tensor:
    """The class of the window cell holding the centroid of each point's host, its offset from the cell of
    x_p clamped to the 9 x 9 window; -1 where the host is not an element."""
    ok = (host >= 0) & (host < cent.shape[0])
    c = cent[torch.where(ok, host, torch.zeros_like(host)).long()]
    dx = torch.clamp(cell_of(c[:, 0], G) - cell_of(xp[:, 0], G), -4, 4)
    dy = torch.clamp(cell_of(c[:, 1], G) - cell_of(xp[:, 1], G), -4, 4)
    return torch.where(ok, (dy + 4) * 9 + (dx + 4), torch.full_like(dx, -1))


def pooled_grid(cent: torch.Tensor, G: int) -> torch.Tensor:
    """Per overlay cell the mean centroid of the elements whose centroid lies in it, or the cell centre
    (FP64 [G][G][2])."""
    cell = cell_of(cent[:, 1], G) * G + cell_of(cent[:, 0], G)
    cnt = torch.zeros(G * G, dtype=torch.float64, device=cent.device).index_add_(0, cell, torch.ones_like(cent[:, 0]))
    s = torch.zeros((G * G, 2), dtype=torch.float64, device=cent.device).index_add_(0, cell, cent)
    c = (torch.arange(G, dtype=torch.float64, device=cent.device) + 0.5) / G
    centre = torch.stack([c.repeat(G), c.repeat_interleave(G)], dim=1)
    pool = torch.where(cnt[:, None] > 0, s / cnt.clamp(min=1)[:, None], centre)
    return pool.reshape(G, G, 2)


def class_features(xp: torch.Tensor, pool: torch.Tensor):
    """The classifier's inputs: G (pooled value - x_p) over the 9 x 9 window (FP32 [n][2][9][9]) and x_p's
    offset in its cell (FP32 [n][2])."""
    G = pool.shape[0]
    cx, cy = cell_of(xp[:, 0], G), cell_of(xp[:, 1], G)
    off = torch.arange(-4, 5, device=xp.device)
    rows = torch.clamp(cy[:, None] + off[None], 0, G - 1)  # [n][9]
    cols = torch.clamp(cx[:, None] + off[None], 0, G - 1)
    q = pool[rows[:, :, None], cols[:, None, :]]  # [n][9][9][2]
    feat = ((q - xp[:, None, None, :]) * G).float().permute(0, 3, 1, 2).contiguous()
    xoff = torch.stack([xp[:, 0] * G - (cx.double() + 0.5), xp[:, 1] * G - (cy.double() + 0.5)], dim=1).float()
    return feat, xoff


class ClsNet(torch.nn.Module):
    """The classifier of Sec. 2.3 as the library computes it (layouts of cnnsns_cls)."""

    def __init__(self):
        super().__init__()
        self.c1 = torch.nn.Conv2d(2, 16, 3, padding=1)
        self.c2 = torch.nn.Conv2d(16, 16, 3, padding=1)
        self.x1 = torch.nn.Linear(2, 256)
        self.x2 = torch.nn.Linear(256, 256)
        self.f1 = torch.nn.Linear(512, 512)
        self.f2 = torch.nn.Linear(512, 81)

    def forward(self, feat, xoff):
        y = torch.relu(self.c2(torch.relu(self.c1(feat))))
        y = torch.nn.functional.avg_pool2d(y, 2).flatten(1)
        m = torch.relu(self.x2(torch.relu(self.x1(xoff))))
        return self.f2(torch.relu(self.f1(torch.cat([y, m], dim=1))))

    def export(self):
        layers = [self.c1, self.c2, self.x1, self.x2, self.f1, self.f2]
        ws = [np.ascontiguousarray(l.weight.detach().float().cpu().numpy()) for l in layers]
        bs = [np.ascontiguousarray(l.bias.detach().float().cpu().numpy()) for l in layers]
        return ws, bs


class DispNet(torch.nn.Module):
    """The displacement CNN (2 -> 32 -> 32 -> 32 -> 2, 3x3, zero padding, ReLU between layers)."""

    def __init__(self):
        super().__init__()
        ch = (2, 32, 32, 32, 2)
        self.convs = torch.nn.ModuleList(torch.nn.Conv2d(a, b, 3, padding=1) for a, b in zip(ch[:-1], ch[1:]))
        for c in self.convs:
            torch.nn.init.kaiming_normal_(c.weight, nonlinearity="relu")
            torch.nn.init.zeros_(c.bias)

    def forward(self, x):
        for k, c in enumerate(self.convs):
            x = c(x)
            if k < 3:
                x = torch.relu(x)
        return x

    def export(self, out_scale: float):
        ws, bs = [], []
        for k, c in enumerate(self.convs):
            w = c.weight.detach().double().cpu().numpy()
            b = c.bias.detach().double().cpu().numpy()
            if k == 3:  # the net learns the displacement / out_scale: fold the scale into the last layer
                w, b = w * out_scale, b * out_scale
            ws.append(np.ascontiguousarray(w.astype(np.float32)))
            bs.append(np.ascontiguousarray(b.astype(np.float32)))
        return ws, bs


def train_displacement(vels, targets, masks, out_scale: float, steps: int = 400, lr: float = 3e-3, seed: int = 0):
    """Masked mean-squared error over whole grids (the first n_t steps), Adam with a cosine schedule."""
    torch.manual_seed(seed)
    dev = vels[0].device
    net = DispNet().to(dev)
    x = torch.stack(vels)                    # [n_t][2][G][G]
    y = torch.stack(targets) / out_scale
    m = torch.stack(masks).float()[:, None]  # [n_t][1][G][G]
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    for _ in range(steps):
        loss = (((net(x) - y) ** 2) * m).sum() / (2 * m.sum())
        opt.zero_grad()
        loss.backward()
        opt.step()
        sched.step()
    return net.export(out_scale), float(loss.item())


def train_classifier(feat, xoff, labels, steps: int = 1500, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
    """Softmax cross-entropy against the one-hot SNS labels (Sec. 2.3), Adam."""
    torch.manual_seed(seed)
    dev = feat.device
    keep = labels >= 0
    feat, xoff, labels = feat[keep], xoff[keep], labels[keep]
    net = ClsNet().to(dev)
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    g = torch.Generator(device=dev).manual_seed(seed)
    for _ in range(steps):
        idx = torch.randint(0, feat.shape[0], (batch,), device=dev, generator=g)
        loss = torch.nn.functional.cross_entropy(net(feat[idx], xoff[idx]), labels[idx])
        opt.zero_grad()
        loss.backward()
        opt.step()
        sched.step()
    with torch.no_grad():
        acc = float((net(feat[:65536], xoff[:65536]).argmax(1) == labels[:65536]).float().mean())
    return net.export(), float(loss.item()), acc


def run(C, n_side: int = 708, seed: int = 2, field_seed: int = 21, k: float = 20.0, G: int = 0, n_steps: int = 8,
        n_t: int = 3, drift: float = 0.15, disp_steps: int = 400, cls_steps: int = 1500, log=print):
    """One time-dependent run: n_t training steps of plain SNS, in-loop training of both predictors from the
    hosts the walk found, then CNN-SNS with each trained predictor in the remaining steps (plain SNS beside).
    Returns per-step path lengths, times and agreement of hosts."""
    dev = torch.device("cuda")
    xy, tri = W.mesh(n_side, seed)
    G = G or W.overlay_side_for(tri.shape[0])
    flow = W.UnsteadyFourier(field_seed, U=1.0, norm_G=G, drift=drift)
    dbar = W.mean_diameter(xy, tri)
    u0, v0 = flow.at(0)(xy[:, 0], xy[:, 1])
    dt = k * dbar / float(np.mean(np.hypot(u0, v0)))
    start = torch.from_numpy(W.node_start_elements(xy.shape[0], tri)).to(dev)
    mesh = C.Mesh(xy, tri, overlay_side=G)
    xy_t, tri_t = torch.from_numpy(xy).to(dev), torch.from_numpy(tri).to(dev)
    cent = centroids_by_id(xy_t, tri_t)
    pool = pooled_grid(cent, G)
    origins = xy_t
    steps = []
    train_vel, train_tgt, train_mask, feats, xoffs, labels = [], [], [], [], [], []
    disp_w = cls_w = None
    t_train = {}
    for s in range(n_steps):
        f = flow.at(s)
        vel = torch.from_numpy(W.overlay_velocity(f, G)).to(dev)
        xp = torch.from_numpy(W.departure_points(xy, f, dt)).to(dev)
        hp, ip, _ = C.locate(mesh, xp, start=start)
        rec = {"step": s, "plain_mean_path": float(ip.double().mean())}
        if s < n_t:  # the walk's own output becomes training data
            t, m = displacement_targets(cent, origins, hp, G)
            train_vel.append(vel)
            train_tgt.append(t)
            train_mask.append(m)
            fe, xo = class_features(xp, pool)
            feats.append(fe)
            xoffs.append(xo)
            labels.append(class_labels(cent, xp, hp, G))
            rec["training"] = True
        else:
            if disp_w is None:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                disp_w, disp_loss = train_displacement(train_vel, train_tgt, train_mask, out_scale=dt,
                                                        steps=disp_steps)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                cls_w, cls_loss, cls_acc = train_classifier(torch.cat(feats), torch.cat(xoffs), torch.cat(labels),
                                                            steps=cls_steps)
                torch.cuda.synchronize()
                t_train = {"displacement_s": round(t1 - t0, 3), "classifier_s": round(time.perf_counter() - t1, 3),
                           "displacement_final_loss": disp_loss, "classifier_final_loss": cls_loss,
                           "classifier_train_accuracy": round(cls_acc, 4)}
                log(f"in-loop training from the first {n_t} steps' walks: {t_train}")
                Wd, Wc = C.Weights(*disp_w), C.ClsWeights(*cls_w)
            disp = C.predict(mesh, vel, Wd, "f32")
            hd, idp, _ = C.locate(mesh, xp, start=start, origin=origins, disp=disp)
            st, _, _ = C.classify(mesh, xp, Wc, fallback=start, want_class=False)
            hc, ic, _ = C.locate(mesh, xp, start=st)
            rec.update({"cnn_sns_mean_path": float(idp.double().mean()),
                        "classifier_mean_path": float(ic.double().mean()),
                        "hosts_equal_plain": float(((hd == hp) & (hc == hp)).double().mean())})
        steps.append(rec)
        log(f"step {s}: " + ", ".join(f"{k_}={v:.4g}" if isinstance(v, float) else f"{k_}={v}"
                                       for k_, v in rec.items() if k_ != "step"))
    mesh.close()
    return {"n_steps": n_steps, "n_t": n_t, "G": G, "n_triangles": int(tri.shape[0]), "n_points": int(xy.shape[0]),
            "dt": dt, "mean_displacement_diameters": k, "training": t_train, "steps": steps,
            "weights": {"displacement": disp_w, "classifier": cls_w}}


# ----------------------------------------------------------------------------- tetrahedral meshes
#
# The same in-loop training for the 3D displacement CNN (3 -> 32 -> 32 -> 32 -> 3, 3x3x3 kernels) on the
# G^3 overlay: the first n_t steps of a time-dependent ABC flow are located by plain SNS on the
# tetrahedral mesh, the per-cell mean of centroid(K_t) - x_i is the target, and the trained weights drive
# cnnsns_predict3d in the later steps.

def centroids3_by_id(xyz: torch.Tensor, tet: torch.Tensor) -> torch.Tensor:
    """Tetrahedron centroids with the vertices summed in ascending node id (FP64 [n_tet][3])."""
    ids, _ = torch.sort(tet.long(), dim=1)
    v = xyz[ids]  # [n_tet][4][3]
    return (((v[:, 0] + v[:, 1]) + v[:, 2]) + v[:, 3]) / 4.0


def displacement_targets_3d(cent: torch.Tensor, origins: torch.Tensor, host: torch.Tensor, G: int,
                            xp: torch.Tensor = None):
    """Per overlay cell (z, y, x) the mean of centroid(host) - x_i over the origins x_i in it, and the
    mask of cells that hold one ([3][G][G][G] FP32, [G][G][G] bool); hosts that are not elements are
    left out, and so, given the departure points xp, are points whose x_p lies on the cube's boundary:
    their departure point was clamped into the domain, a step the start rule takes again on the
    predicted point, so the net should learn the displacement before the clamp."""
    ok = (host >= 0) & (host < cent.shape[0])
    if xp is not None:
        ok &= ((xp > 0.0) & (xp < 1.0)).all(dim=1)
    o, h = origins[ok], host[ok].long()
    d = cent[h] - o
    cell = (cell_of(o[:, 2], G) * G + cell_of(o[:, 1], G)) * G + cell_of(o[:, 0], G)
    cnt = torch.zeros(G ** 3, dtype=torch.float64, device=o.device).index_add_(0, cell, torch.ones_like(d[:, 0]))
    t = torch.zeros((3, G ** 3), dtype=torch.float64, device=o.device)
    for a in range(3):
        t[a].index_add_(0, cell, d[:, a])
    mask = cnt > 0
    t[:, mask] /= cnt[mask]
    return t.reshape(3, G, G, G).float(), mask.reshape(G, G, G)


def conv3d_gemm(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """3x3x3 convolution with zero padding 1 as one matrix product over the 27 shifted views (the
    training harness's 3D layer: library GEMMs, no per-shape kernel search or compilation)."""
    N, Ci, D, H, Wd = x.shape
    xp = torch.nn.functional.pad(x, (1, 1, 1, 1, 1, 1))
    cols = torch.stack([xp[:, :, a:a + D, c:c + H, e:e + Wd] for a in range(3) for c in range(3) for e in range(3)],
                       dim=2)  # [N][Ci][27][D][H][W]: the (ci, kz, ky, kx) order of an OIDHW weight
    y = torch.matmul(w.reshape(w.shape[0], Ci * 27), cols.reshape(N, Ci * 27, D * H * Wd))
    return (y + b[None, :, None]).reshape(N, w.shape[0], D, H, Wd)


class DispNet3D(torch.nn.Module):
    """The 3D displacement CNN (3 -> 32 -> 32 -> 32 -> 3, 3x3x3, zero padding, ReLU between layers)."""

    def __init__(self):
        super().__init__()
        ch = (3, 32, 32, 32, 3)
        self.convs = torch.nn.ModuleList(torch.nn.Conv3d(a, b, 3, padding=1) for a, b in zip(ch[:-1], ch[1:]))
        for c in self.convs:
            torch.nn.init.kaiming_normal_(c.weight, nonlinearity="relu")
            torch.nn.init.zeros_(c.bias)
        # the two 32 -> 32 layers start near the identity (a centre tap per channel, small noise), so
        # the untrained net passes layer 1's features straight to layer 4
        with torch.no_grad():
            for c in self.convs[1:3]:
                torch.nn.init.dirac_(c.weight)
                c.weight.add_(0.01 * torch.randn_like(c.weight))

    def forward(self, x):
        for k, c in enumerate(self.convs):
            x = conv3d_gemm(x, c.weight, c.bias)
            if k < 3:
                x = torch.relu(x)
        return x

    export = DispNet.export


def point_targets_3d(cent: torch.Tensor, host: torch.Tensor):
    """Per point the centroid of its host (FP64 [n][3]) and whether the host is an element."""
    ok = (host >= 0) & (host < cent.shape[0])
    return cent[torch.where(ok, host, torch.zeros_like(host)).long()], ok


def crop_valid_range(z0: int, C: int, G: int, halo: int = 4):
    """Cells [lo, hi) of a crop [z0, z0 + C) of a G-cell axis whose outputs equal the full grid's: the
    net sees 'halo' cells each way (four 3x3x3 layers), and a crop side inside the grid pads with
    zeros where the grid has values; a side on the grid's own boundary pads exactly as the grid does."""
    lo = z0 + (halo if z0 > 0 else 0)
    hi = z0 + C - (halo if z0 + C < G else 0)
    return lo, hi


def train_displacement_3d(vels, origins, cents, oks, out_scale: float, steps: int = 3000, lr: float = 1e-3,
                          crop: int = 48, seed: int = 0, log=None):
    """The net's displacement D at the cell of each origin x_i is scored where the start rule uses it:
    the squared distance between clamp(x_i + D, 0, 1) and the centroid of the host K_t the walk found,
    over the points of the first n_t steps (in units of out_scale), Adam with a cosine schedule.  (The
    departure points are clamped into the cube, so a label taken before the clamp would teach the net
    shrunken displacements near the faces.)  Each step runs the net on one random crop^3 block of the
    grid of one of the n_t steps (drawn at random) and scores the points whose origin cell lies where the
    crop's output equals the full grid's."""
    torch.manual_seed(seed)
    dev = vels[0].device
    G = vels[0].shape[-1]
    C = min(crop, G)
    g = torch.Generator().manual_seed(seed)
    net = DispNet3D().to(dev)
    x = torch.stack(vels)  # [n_t][3][G][G][G]
    o = origins.float()
    cz, cy, cx = cell_of(origins[:, 2], G), cell_of(origins[:, 1], G), cell_of(origins[:, 0], G)
    c = torch.stack(cents).float()            # [n_t][n][3]
    w = torch.stack(oks).float()[..., None]   # [n_t][n][1]
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    loss = torch.zeros(())
    for _ in range(steps):
        # per axis the crop sits on the low face, on the high face or anywhere, a third each: the cells
        # next to the faces (where the zero padding enters the net) are as well trained as the rest
        side = torch.randint(0, 3, (3,), generator=g)
        anywhere = torch.randint(0, G - C + 1, (3,), generator=g)
        z0, y0, x0 = (0 if int(sd) == 0 else (G - C if int(sd) == 1 else int(a)) for sd, a in zip(side, anywhere))
        (zl, zh), (yl, yh), (xl, xh) = (crop_valid_range(a, C, G) for a in (z0, y0, x0))
        sel = torch.nonzero((cz >= zl) & (cz < zh) & (cy >= yl) & (cy < yh) & (cx >= xl) & (cx < xh)).squeeze(1)
        if sel.numel() == 0:
            continue
        t = int(torch.randint(0, x.shape[0], (1,), generator=g))
        out = net(x[t:t + 1, :, z0:z0 + C, y0:y0 + C, x0:x0 + C].contiguous())[0]
        flat = ((cz[sel] - z0) * C + (cy[sel] - y0)) * C + (cx[sel] - x0)
        d = out.flatten(1)[:, flat].t() * out_scale  # [m][3]
        p = torch.clamp(o[sel] + d, 0.0, 1.0)
        ws = w[t, sel]
        loss = (((p - c[t, sel]) / out_scale) ** 2 * ws).sum() / (3 * ws.sum().clamp(min=1.0))
        opt.zero_grad()
        loss.backward()
        opt.step()
        sched.step()
        if log is not None and (_ + 1) % 250 == 0:
            log(f"3D training step {_ + 1}: loss {float(loss.detach()):.5f}")
    return net.export(out_scale), float(loss.item())


def run3d(C, name: str = "t3", n_steps: int = 6, n_t: int = 3, drift: float = 0.15, flow_seed: int = 5,
          disp_steps: int = 3000, G: int = 0, log=print):
    """One time-dependent run on the tetrahedral workload `name`'s mesh and overlay: n_t steps of plain
    SNS whose hosts train the 3D displacement CNN, then CNN-SNS with the trained net in the remaining
    steps, beside plain SNS, the constructed -dt u net and the overlay lookup at x_p."""
    dev = torch.device("cuda")
    cfg = W.CONFIGS_3D[name]
    xyz, tet = W.kuhn_mesh(cfg["n_side"], cfg["seed"])
    G = G or cfg.get("G", W.overlay_side_for_3d(tet.shape[0]))
    flow = W.UnsteadyABC(flow_seed, drift=drift)
    dbar = float(W.tet_longest_edges(xyz, tet).mean())
    u0 = np.stack(flow.at(0)(xyz[:, 0], xyz[:, 1], xyz[:, 2]), axis=1)
    dt = cfg["k"] * dbar / float(np.mean(np.linalg.norm(u0, axis=1)))
    start = torch.from_numpy(W.node_start_tets(xyz.shape[0], tet)).to(dev)
    mesh = C.Mesh3D(xyz, tet, overlay_side=G)
    xyz_t, tet_t = torch.from_numpy(xyz).to(dev), torch.from_numpy(tet).to(dev)
    cent = centroids3_by_id(xyz_t, tet_t)
    origins = xyz_t
    Wp = C.Weights3D(*W.passthrough_weights_3d(dt))
    steps, tv, tt, tm = [], [], [], []
    disp_w, t_train, Wd = None, {}, None
    for s in range(n_steps):
        f = flow.at(s)
        vel = torch.from_numpy(W.overlay_velocity_3d(f, G)).to(dev)
        u = np.stack(f(xyz[:, 0], xyz[:, 1], xyz[:, 2]), axis=1)
        xp = torch.from_numpy(np.ascontiguousarray(np.clip(xyz - dt * u, 0.0, 1.0))).to(dev)
        hp, ip, _ = C.locate3d(mesh, xp, start=start)
        rec = {"step": s, "plain_mean_path": float(ip.double().mean())}
        if s < n_t:
            c, ok = point_targets_3d(cent, hp)
            tv.append(vel)
            tt.append(c)
            tm.append(ok)
            rec["training"] = True
        else:
            if Wd is None:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                disp_w, loss = train_displacement_3d(tv, origins, tt, tm, out_scale=dt, steps=disp_steps, log=log)
                torch.cuda.synchronize()
                t_train = {"displacement_s": round(time.perf_counter() - t0, 3), "displacement_final_loss": loss}
                log(f"3D in-loop training from the first {n_t} steps' walks: {t_train}")
                Wd = C.Weights3D(*disp_w)
            disp = C.predict3d(mesh, vel, Wd, "f32")
            hd, idp, _ = C.locate3d(mesh, xp, start=start, origin=origins, disp=disp)
            dbf = C.predict3d(mesh, vel, Wd, "bf16")
            hb, ib, _ = C.locate3d(mesh, xp, start=start, origin=origins, disp=dbf)
            dpass = C.predict3d(mesh, vel, Wp, "f32")
            _, ipass, _ = C.locate3d(mesh, xp, start=start, origin=origins, disp=dpass)
            hl, il, _ = C.locate3d(mesh, xp)
            rec.update({"cnn_sns_mean_path": float(idp.double().mean()),
                        "cnn_sns_bf16_mean_path": float(ib.double().mean()),
                        "passthrough_net_mean_path": float(ipass.double().mean()),
                        "lookup_at_xp_mean_path": float(il.double().mean()),
                        "hosts_equal_plain": float(((hd == hp) & (hb == hp)).double().mean())})
        steps.append(rec)
        log(f"3D step {s}: " + ", ".join(f"{k_}={v:.4g}" if isinstance(v, float) else f"{k_}={v}"
                                          for k_, v in rec.items() if k_ != "step"))
    mesh.close()
    return {"workload": name, "n_steps": n_steps, "n_t": n_t, "G": G, "n_tetrahedra": int(tet.shape[0]),
            "n_points": int(xyz.shape[0]), "dt": dt, "mean_displacement_diameters": cfg["k"],
            "flow": f"ABC, phases drifting {drift} rad x U[0.5,1.5] per axis per step (seed {flow_seed})",
            "training": t_train, "steps": steps, "weights": {"displacement": disp_w}}
