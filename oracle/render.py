"""FP64 reference renderer: RGB, mean depth and raw C-ToF quads, with gradients.

TEST INFRASTRUCTURE ONLY (see the package header).

What is computed (paper §3):

* Eq. 2 (RGB):     c(x) = c_bg T_final + sum_k c_k alpha_k T_k
* Eq. 4 (quads):   q_j(x) = q_bg,j T_final^p + sum_k (s r_k / d_k^2) sin(psi_k + phi_j) alpha_k T_k^2
                   with psi_k = 4 pi f d_k / c, evaluated directly per offset phi_j
                   (for phi = 0, pi/2, pi, 3pi/2 this is the list sin, cos, -sin, -cos).
* Eq. 5 (depth):   d(x) = sum_k d_k alpha_k T_k      (no background, T not squared)

with alpha_k = min(alpha_max, o_k G_k(x)), G_k the projected 2D Gaussian, and
T_k = prod_{l<k} (1 - alpha_l) over the Gaussians composited before k.
d_k is the distance from the Gaussian centre to the optical centre.
T_final is the product over *all* composited Gaussians and p = bg_T_power
(1 literally; 2 optional).

Readings where the paper is silent (rasterizer constants, "based on 3DGS"):
a pixel takes the Gaussians of its tile in ascending (depth key, index) order
(oracle.binning); a Gaussian with alpha < alpha_min is skipped; the walk stops
before the first Gaussian whose compositing would take T (1 - alpha) below
T_min; n_contrib = 1 + position of the last composited Gaussian in the tile
list (0 if none).  Pixel (i, j) is sampled at (i + 0.5, j + 0.5).

Gradients are the exact derivatives of this piecewise-smooth function with the
discrete decisions (skip, stop, clamp, tile lists, order) held fixed, obtained
by torch autograd in float64.  The per-pixel visiting decisions are taken in
a first pass without gradients; the differentiable pass then evaluates the
same sums in closed form (T_k as an exclusive cumulative product).

Pins: tests/test_oracle_render.py (single-Gaussian closed form, phase of an
equal-range shell, telescoping identities, monotone transmittance, brute
force, recursion S2/S3, central finite differences).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binning, sh

C_LIGHT = 299_792_458.0
FIELDS = ("mean", "vel", "acc", "scale", "quat", "omega", "opacity_logit", "rgb", "albedo")
SH_FIELDS = ("sh_rgb", "sh_albedo")   # optional view-dependent colour / reflectivity (§3)
OPTIONAL = SH_FIELDS + ("delta",)     # + per-frame centre offsets [F, 3, N] (§4 network)


def fields_of(g):
    """The parameter fields a Gaussian set carries (optional ones when present)."""
    return FIELDS + tuple(k for k in OPTIONAL if getattr(g, k, None) is not None)


def _w(x):
    """Inputs are float32 values widened exactly (Python scalars are rounded
    to float32 first, as the device receives them); float64 numpy arrays
    (finite-difference probes in the tests) are taken as they are."""
    if isinstance(x, np.ndarray) and x.dtype == np.float64:
        return x
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _s(x):
    return float(_w(x))


def _t(x, requires_grad=False):
    return torch.tensor(_w(x), dtype=torch.float64, requires_grad=requires_grad)


def params_to_torch(g, requires_grad=False):
    return {k: _t(getattr(g, k), requires_grad) for k in fields_of(g)}


def _quat_rotation(q):
    """Rotation matrices [N,3,3] of unit quaternions q = (w, x, y, z) [4,N]."""
    w, x, y, z = q
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], dim=-1)
    return r.reshape(-1, 3, 3)


def gaussian_quantities(p, frame, cfg, f=0):
    """Differentiable per-Gaussian screen-space quantities for one frame.

    p: dict of float64 tensors (FIELDS).  Returns a dict of tensors over N:
    u, v (pixel centre), A, B, C (conic = inverse 2D covariance, with the
    off-diagonal B), o (opacity), d (range to the optical centre), amp
    (s r / d^2), psi [n_freq, N], rgb [3, N].
    """
    t = _s(frame.time)
    tlo, thi = _s(getattr(frame, "t_lo", 0.0)), _s(getattr(frame, "t_hi", 0.0))
    if thi > tlo:
        # Eq. 7: straight line between the positions at the two anchors
        w1, w2 = (thi - t) / (thi - tlo), (t - tlo) / (thi - tlo)
        mu = (w1 * (p["mean"] + p["vel"] * tlo + 0.5 * p["acc"] * (tlo * tlo))
              + w2 * (p["mean"] + p["vel"] * thi + 0.5 * p["acc"] * (thi * thi)))
    else:
        mu = p["mean"] + p["vel"] * t + 0.5 * p["acc"] * (t * t)        # [3,N]
    if "delta" in p:
        mu = mu + p["delta"][f]        # deformation-network offset of frame f (§4)
    q0 = p["quat"]
    om = p["omega"]
    # (0, omega) (x) q0 = (-omega . v0, w0 omega + omega x v0)
    w0, v0 = q0[0], q0[1:]
    dq = torch.cat([-(om * v0).sum(0, keepdim=True),
                    w0[None] * om + torch.cross(om, v0, dim=0)], 0)
    q = q0 + 0.5 * t * dq
    qn = q / torch.linalg.norm(q, dim=0, keepdim=True)
    Rq = _quat_rotation(qn)                                             # [N,3,3]
    s2 = p["scale"].T ** 2                                              # [N,3]
    Sig = (Rq * s2[:, None, :]) @ Rq.transpose(1, 2)                    # [N,3,3]

    W = torch.tensor(_w(frame.R).reshape(3, 3))
    tc = torch.tensor(_w(frame.t))
    pc = W @ mu + tc[:, None]                                            # [3,N]
    X, Y, Z = pc
    fx, fy = _s(frame.fx), _s(frame.fy)
    cx, cy = _s(frame.cx), _s(frame.cy)
    zero = torch.zeros_like(Z)
    J = torch.stack([torch.stack([fx / Z, zero, -fx * X / Z ** 2], -1),
                     torch.stack([zero, fy / Z, -fy * Y / Z ** 2], -1)], 1)  # [N,2,3]
    T = J @ W
    S2 = T @ Sig @ T.transpose(1, 2)
    dil = _s(cfg.dilation)
    a = S2[:, 0, 0] + dil
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + dil
    det = a * c - b * b
    A, B, Cc = c / det, -b / det, a / det

    u = fx * X / Z + cx
    v = fy * Y / Z + cy
    centre = -(W.T @ tc)                                                 # optical centre
    d = torch.linalg.norm(mu - centre[:, None], dim=0)
    o = torch.sigmoid(p["opacity_logit"])
    rgb, albedo = p["rgb"], p["albedo"]
    if p.get("sh_rgb") is not None or p.get("sh_albedo") is not None:
        # view-dependent colour and reflectivity (§3): spherical harmonics at
        # the direction from the optical centre to the Gaussian centre
        direc = (mu - centre[:, None]) / d
        if p.get("sh_rgb") is not None:
            rgb = sh.colour(p["sh_rgb"], direc, _degree(p["sh_rgb"].shape[0]))
        if p.get("sh_albedo") is not None:
            albedo = sh.colour(p["sh_albedo"][:, None, :], direc, _degree(p["sh_albedo"].shape[0]))[0]
    s_int = _s(cfg.source_intensity)
    amp = s_int * albedo / d ** 2
    psi = torch.stack([4.0 * math.pi * _s(f) * d / C_LIGHT for f in cfg.freqs])
    return dict(u=u, v=v, A=A, B=B, C=Cc, o=o, d=d, amp=amp, psi=psi, rgb=rgb)


def _degree(n_coeffs):
    return {v: k for k, v in sh.N_COEFFS.items()}[int(n_coeffs)]


QKEYS = ("u", "v", "A", "B", "C", "o", "d", "amp", "psi", "rgb")


def _raw_alpha(q, sel, px, py):
    """o_k G_k(x) for the entries `sel` (rows) at pixel centres px, py (cols)."""
    dx = px[None, :] - q["u"][sel][:, None]
    dy = py[None, :] - q["v"][sel][:, None]
    power = -0.5 * (q["A"][sel][:, None] * dx * dx + q["C"][sel][:, None] * dy * dy) \
        - q["B"][sel][:, None] * dx * dy
    return q["o"][sel][:, None] * torch.exp(power)


def visit_pass(q, sel, px, py, inside, cfg, flag_rel=(1e-5, 1e-4), chunk=1024, counts=None):
    """Per-pixel walk over one tile list without gradients.

    Returns (active [K,P] bool, K, n_contrib [P], flagged [P]).  K is the list
    length actually needed: every entry at or beyond K is inert for every
    pixel.  `flagged` marks pixels where some skip / clamp / stop predicate
    lies within the relative window flag_rel = (alpha window, T window) of
    its threshold, i.e. where a float32 evaluation may legitimately decide
    differently.  With a dict `counts`, counts["n_evaluated"] [P] is the
    number of entries whose alpha each pixel evaluates: every entry up to and
    including the one that stops it (the whole list if none does).
    """
    amin, amax, tmin = _s(cfg.alpha_min), _s(cfg.alpha_max), _s(cfg.T_min)
    ea, et = flag_rel
    P = px.numel()
    L = int(sel.numel())
    T = np.ones(P)
    done = ~inside.copy()
    ncontrib = np.zeros(P, np.int64)
    n_eval = np.zeros(P, np.int64)
    flagged = np.zeros(P, bool)
    active_rows = []
    K = 0
    with torch.no_grad():
        for c0 in range(0, L, chunk):
            raw = _raw_alpha(q, sel[c0:c0 + chunk], px, py).numpy()
            alpha = np.minimum(raw, amax)
            for r in range(raw.shape[0]):
                k = c0 + r
                a = alpha[r]
                live = ~done
                n_eval += live
                flagged |= live & (np.abs(a - amin) <= ea * amin) & (amin > 0)
                flagged |= live & (np.abs(raw[r] - amax) <= ea * amax)
                cons = live & (a >= amin)
                testT = T * (1.0 - a)
                if tmin > 0:
                    flagged |= cons & (np.abs(testT - tmin) <= et * tmin)
                term = cons & (testT < tmin)
                comp = cons & ~term
                done |= term
                T = np.where(comp, testT, T)
                ncontrib = np.where(comp, k + 1, ncontrib)
                active_rows.append(comp)
                K = k + 1
                if done.all():
                    break
            if done.all():
                break
    active = np.stack(active_rows) if active_rows else np.zeros((0, P), bool)
    if counts is not None:
        counts["n_evaluated"] = n_eval
    return active, K, ncontrib, flagged


def composite_tile(q, sel, px, py, active, frame, cfg, bg_rgb, bg_quad):
    """Differentiable closed-form sums of Eqs. 2, 4, 5 over one tile.

    sel [K] entry Gaussian indices, active [K,P] mask from `visit_pass`.
    Returns rgb [3,P], quad [NQ,P], depth [P], T_final [P], alpha [K,P].
    """
    K = int(sel.numel())
    P = px.numel()
    if K == 0:
        Tf = torch.ones(P, dtype=torch.float64)
        rgb = bg_rgb[:, None] * Tf[None]
        quad = bg_quad.reshape(-1)[:, None] * (Tf[None] ** cfg.bg_T_power)
        return rgb, quad, torch.zeros(P, dtype=torch.float64), Tf, torch.zeros(0, P)
    raw = _raw_alpha(q, sel, px, py)
    alpha = torch.clamp(raw, max=_s(cfg.alpha_max))
    A = alpha * torch.from_numpy(active.astype(np.float64))
    om = 1.0 - A
    cp = torch.cumprod(om, 0)
    T = torch.cat([torch.ones(1, P, dtype=torch.float64), cp[:-1]], 0)
    Tf = cp[-1]
    w = A * T
    w2 = w * T
    rgb = q["rgb"][:, sel] @ w + bg_rgb[:, None] * Tf[None]
    depth = q["d"][sel] @ w
    quads = []
    for fi in range(cfg.n_freq):
        for ph in cfg.phases:
            val = q["amp"][sel] * torch.sin(q["psi"][fi][sel] + _s(ph))
            quads.append(val @ w2)
    quad = torch.stack(quads) + bg_quad.reshape(-1)[:, None] * (Tf[None] ** cfg.bg_T_power)
    return rgb, quad, depth, Tf, A


def render(g, frames, cfg, tiles=None, upstream=None, flag_rel=(1e-5, 1e-4),
           keep_tile_data=False):
    """Render a batch of frames; optionally back-propagate an upstream gradient.

    g: scenes.Gaussians (float32); frames: list of scenes.Frame; cfg: RenderConfig.
    tiles: None for every tile, or a list (per frame) of tile ids to evaluate.
    upstream: None or dict(rgb [F,3,H,W], quad [F,NQ,H,W], depth [F,H,W]).

    Returns dict of float64 numpy arrays: rgb, quad, depth, T_final,
    n_contrib (int64), n_evaluated and n_composited (int64: entries whose
    alpha the pixel evaluates / that it composites), flagged (bool),
    computed (bool), pairs (binning), E (sum of n_contrib over computed
    pixels) and, with `upstream`, grads
    (per parameter field), grad_bg_rgb [F,3], grad_bg_quad [F,NQ] and
    grad2d (per frame dict of per-Gaussian screen-space gradients).
    """
    F = len(frames)
    H, Wd = cfg.height, cfg.width
    ntx, nty = cfg.tiles_x, cfg.tiles_y
    n_tiles = ntx * nty
    NQ = cfg.n_quad
    # every tile: all pairs of the batch; a tile subset: only those tiles' lists
    pairs = binning.sorted_pairs(g, frames, cfg) if tiles is None else None
    out = dict(rgb=np.full((F, 3, H, Wd), np.nan), quad=np.full((F, NQ, H, Wd), np.nan),
               depth=np.full((F, H, Wd), np.nan), T_final=np.full((F, H, Wd), np.nan),
               n_contrib=np.full((F, H, Wd), -1, np.int64),
               n_evaluated=np.full((F, H, Wd), -1, np.int64),
               n_composited=np.full((F, H, Wd), -1, np.int64),
               flagged=np.zeros((F, H, Wd), bool), computed=np.zeros((F, H, Wd), bool),
               pairs=pairs)
    want_grad = upstream is not None
    params = params_to_torch(g, requires_grad=want_grad)
    grad_bg_rgb = np.zeros((F, 3))
    grad_bg_quad = np.zeros((F, NQ))
    grad2d = []
    tile_data = []
    ly, lx = np.meshgrid(np.arange(cfg.tile_h), np.arange(cfg.tile_w), indexing="ij")
    ly, lx = ly.ravel(), lx.ravel()
    for f, frame in enumerate(frames):
        q_graph = gaussian_quantities(params, frame, cfg, f)
        leaves = {k: q_graph[k].detach().clone().requires_grad_(want_grad) for k in QKEYS}
        bgr = torch.tensor(_w(frame.bg_rgb), requires_grad=want_grad)
        bq_np = np.zeros(NQ) if frame.bg_quad is None else _w(frame.bg_quad).reshape(-1)
        bgq = torch.tensor(bq_np, requires_grad=want_grad)
        if tiles is None:
            lists = binning.tile_lists(pairs, f, n_tiles)
            tile_ids = range(n_tiles)
        else:
            tile_ids = tiles[f]
            lists = binning.lists_for_tiles(binning.project(g, frame, cfg, f), cfg, tile_ids)
        for tid in tile_ids:
            ty, tx = divmod(int(tid), ntx)
            gx = tx * cfg.tile_w + lx
            gy = ty * cfg.tile_h + ly
            inside = (gx < Wd) & (gy < H)
            px = torch.from_numpy(gx + 0.5)
            py = torch.from_numpy(gy + 0.5)
            sel_all = torch.from_numpy(lists[tid])
            counts = {}
            active, K, ncontrib, flagged = visit_pass(leaves, sel_all, px, py, inside, cfg,
                                                      flag_rel, counts=counts)
            sel = sel_all[:K]
            rgb, quad, depth, Tf, A = composite_tile(leaves, sel, px, py, active, frame, cfg,
                                                     bgr, bgq)
            ii = inside
            yy, xx = gy[ii], gx[ii]
            out["rgb"][f][:, yy, xx] = rgb.detach().numpy()[:, ii]
            out["quad"][f][:, yy, xx] = quad.detach().numpy()[:, ii]
            out["depth"][f][yy, xx] = depth.detach().numpy()[ii]
            out["T_final"][f][yy, xx] = Tf.detach().numpy()[ii]
            out["n_contrib"][f][yy, xx] = ncontrib[ii]
            out["n_evaluated"][f][yy, xx] = counts["n_evaluated"][ii]
            out["n_composited"][f][yy, xx] = active.sum(axis=0)[ii]
            out["flagged"][f][yy, xx] = flagged[ii]
            out["computed"][f][yy, xx] = True
            if keep_tile_data:
                tile_data.append(dict(frame=f, tile=int(tid), sel=sel.numpy(), active=active,
                                      inside=inside, px=gx, py=gy))
            if want_grad:
                m = torch.from_numpy(inside.astype(np.float64))
                ur = torch.from_numpy(np.nan_to_num(upstream["rgb"][f][:, gy.clip(0, H - 1),
                                                                      gx.clip(0, Wd - 1)]
                                                    .astype(np.float64)))
                uq = torch.from_numpy(upstream["quad"][f][:, gy.clip(0, H - 1),
                                                          gx.clip(0, Wd - 1)].astype(np.float64))
                ud = torch.from_numpy(upstream["depth"][f][gy.clip(0, H - 1),
                                                           gx.clip(0, Wd - 1)].astype(np.float64))
                loss = ((ur * rgb).sum(0) * m).sum() + ((uq * quad).sum(0) * m).sum() \
                    + (ud * depth * m).sum()
                loss.backward()
        if want_grad:
            outs = [q_graph[k] for k in QKEYS]
            gl = [leaves[k].grad if leaves[k].grad is not None else torch.zeros_like(leaves[k])
                  for k in QKEYS]
            torch.autograd.backward(outs, gl)
            grad2d.append({k: v.detach().numpy().copy() for k, v in zip(QKEYS, gl)})
            grad_bg_rgb[f] = bgr.grad.numpy() if bgr.grad is not None else 0.0
            grad_bg_quad[f] = bgq.grad.numpy() if bgq.grad is not None else 0.0
    comp = out["computed"]
    out["E"] = int(out["n_contrib"][comp].sum())
    if keep_tile_data:
        out["tile_data"] = tile_data
    if want_grad:
        out["grads"] = {k: (params[k].grad.numpy().copy() if params[k].grad is not None
                            else np.zeros(params[k].shape)) for k in params}
        out["grad_bg_rgb"] = grad_bg_rgb
        out["grad_bg_quad"] = grad_bg_quad
        out["grad2d"] = grad2d
    return out


def loss_of(out, upstream):
    """sum(upstream * output) over computed pixels: the scalar whose gradient
    `render(..., upstream=...)` returns (for finite differences)."""
    tot = 0.0
    for f in range(out["rgb"].shape[0]):
        m = out["computed"][f]
        tot += float((upstream["rgb"][f][:, m] * out["rgb"][f][:, m]).sum())
        tot += float((upstream["quad"][f][:, m] * out["quad"][f][:, m]).sum())
        tot += float((upstream["depth"][f][m] * out["depth"][f][m]).sum())
    return tot
