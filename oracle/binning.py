"""FP64 binning: projection, tile rectangle and depth key per (frame, Gaussian).

TEST INFRASTRUCTURE ONLY (see the package header).

Which Gaussians a tile composites, and in what order, is an integer result
decided by floating point.  To make it reproducible bit for bit, the decision
is defined here as one fixed sequence of IEEE-754 binary64 operations: every
statement below is a single correctly rounded +, -, *, / or sqrt (no fused
multiply-add, no transcendental), evaluated left to right exactly as written.
Inputs are the float32 parameters, widened exactly to float64.

The geometric content follows the Gaussian splatting image formation the paper
builds on (§3, "GS image formation model"; §4 "Implementation details"):

* time evaluation (the dynamic stand-in for the deformation MLP, §4):
  x(t) = x0 + v t + a t^2 / 2 and q(t) = q0 + (t/2) (0, omega) (x) q0, the
  first-order constant-rate quaternion step; q(t) is not renormalised because
  the rotation is formed as M(q) / |q|^2, which is exact for any q != 0.
* asynchronous raw quads (§4, Eq. 7): a frame with anchors t_lo < t_hi takes
  the centre on the line between its positions at the two integer timesteps,
  x = w1 x(t_lo) + w2 x(t_hi), w1 = (t_hi - t) / (t_hi - t_lo),
  w2 = (t - t_lo) / (t_hi - t_lo) (for unit spacing these are Eq. 7's
  weights i2 - j and j - i1).  The deformation of the paper offsets positions
  only; here the quaternion stays evaluated at t, which is the same thing as
  interpolating it, because q(t) is affine in t.
* deformation offsets (§4): with per-frame offsets delta [F][3][N] (the
  network's output at the frame's time), frame f's centre is the trajectory
  position plus delta[f].
* camera space p = R x + t; culled unless p_z > near.
* EWA projection: Sigma' = J R Rq S^2 Rq^T R^T J^T + dilation I, with the
  pinhole Jacobian J at p.
* extent: the ellipse (p - c)^T Sigma'^-1 (p - c) <= k^2, k = extent_sigma
  (3 by default), whose axis-aligned bounding box has the half-widths
  hx = k sqrt(Sigma'_xx), hy = k sqrt(Sigma'_yy).
* tile rectangle: the tiles whose pixel centres reach into that box, i.e.
  whose centre range [tx Tw + 1/2, (tx + 1) Tw - 1/2] meets [u - hx, u + hx]:
  x in [max(0, floor((u - hx + 1/2)/Tw)), min(nTx - 1, floor((u + hx - 1/2)/Tw))],
  same for y; culled if empty or det <= 0.  (Unbounded support with k <= 0:
  every tile.)
* depth key: the float32 rounding of p_z, compared as its bit pattern.
* pair order: ascending (frame, tile, depth key, Gaussian index).

Pins: tests/test_oracle_binning.py (closed form for an axis-aligned Gaussian on
the optical axis; sorted lists equal Python's sorted() of tuple keys).
"""
from __future__ import annotations

import numpy as np


def _d(x):
    """Inputs are float32 values widened exactly (Python scalars are rounded
    to float32 first, as the device receives them); float64 numpy arrays
    (finite-difference probes in the tests) are taken as they are."""
    if isinstance(x, np.ndarray) and x.dtype == np.float64:
        return x
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def project(g, frame, cfg, f=0):
    """Binning quantities of every Gaussian for frame f of a batch (float64
    arrays); f selects the frame's row of the optional centre offsets.

    Returns a dict with u, v (pixel centre), S00, S01, S11 (2D covariance incl.
    dilation), det, half (the extent box's half-widths hx, hy), rect (x_lo,
    x_hi, y_lo, y_hi as int64), count
    (tiles covered, 0 if culled), key (uint32 depth bits), pz, valid.
    """
    with np.errstate(all="ignore"):
        t = _d(frame.time)
        x0x, x0y, x0z = _d(g.mean)
        vx, vy, vz = _d(g.vel)
        ax, ay, az = _d(g.acc)
        tt = t * t
        tlo, thi = _d(getattr(frame, "t_lo", 0.0)), _d(getattr(frame, "t_hi", 0.0))
        if thi > tlo:
            # Eq. 7 between the anchors, one IEEE operation per statement
            span = thi - tlo
            w1 = (thi - t) / span
            w2 = (t - tlo) / span
            tl2 = tlo * tlo
            th2 = thi * thi
            mx = w1 * ((x0x + vx * tlo) + (0.5 * ax) * tl2) + w2 * ((x0x + vx * thi) + (0.5 * ax) * th2)
            my = w1 * ((x0y + vy * tlo) + (0.5 * ay) * tl2) + w2 * ((x0y + vy * thi) + (0.5 * ay) * th2)
            mz = w1 * ((x0z + vz * tlo) + (0.5 * az) * tl2) + w2 * ((x0z + vz * thi) + (0.5 * az) * th2)
        else:
            mx = (x0x + vx * t) + (0.5 * ax) * tt
            my = (x0y + vy * t) + (0.5 * ay) * tt
            mz = (x0z + vz * t) + (0.5 * az) * tt
        dl = getattr(g, "delta", None)
        if dl is not None:
            # the deformation network's offset of this frame (§4), added last
            ox_, oy_, oz_ = _d(dl[f])
            mx = mx + ox_
            my = my + oy_
            mz = mz + oz_

        w0, qx0, qy0, qz0 = _d(g.quat)
        ox, oy, oz = _d(g.omega)
        ht = 0.5 * t
        dw = -((ox * qx0 + oy * qy0) + oz * qz0)
        dxq = w0 * ox + (oy * qz0 - oz * qy0)
        dyq = w0 * oy + (oz * qx0 - ox * qz0)
        dzq = w0 * oz + (ox * qy0 - oy * qx0)
        qw = w0 + ht * dw
        qx = qx0 + ht * dxq
        qy = qy0 + ht * dyq
        qz = qz0 + ht * dzq

        ww = qw * qw
        xx = qx * qx
        yy = qy * qy
        zz = qz * qz
        nq = ((ww + xx) + yy) + zz
        M = [[((ww + xx) - yy) - zz, 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy)],
             [2.0 * (qx * qy + qw * qz), ((ww - xx) + yy) - zz, 2.0 * (qy * qz - qw * qx)],
             [2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), ((ww - xx) - yy) + zz]]

        W = _d(frame.R).reshape(3, 3)
        tc = _d(frame.t)
        px = ((W[0, 0] * mx + W[0, 1] * my) + W[0, 2] * mz) + tc[0]
        py = ((W[1, 0] * mx + W[1, 1] * my) + W[1, 2] * mz) + tc[1]
        pz = ((W[2, 0] * mx + W[2, 1] * my) + W[2, 2] * mz) + tc[2]

        near = _d(cfg.near_z)
        in_front = pz > near

        fx = _d(frame.fx)
        fy = _d(frame.fy)
        cx = _d(frame.cx)
        cy = _d(frame.cy)
        iz = 1.0 / pz
        ja = fx * iz
        jb = fy * iz
        jc = -(((fx * px) * iz) * iz)
        jd = -(((fy * py) * iz) * iz)

        # L = R_cam M  (3 x 3)
        L = [[(W[i, 0] * M[0][j] + W[i, 1] * M[1][j]) + W[i, 2] * M[2][j] for j in range(3)]
             for i in range(3)]
        s = _d(g.scale)
        sc = [s[j] / nq for j in range(3)]
        U0 = [(ja * L[0][j] + jc * L[2][j]) * sc[j] for j in range(3)]
        U1 = [(jb * L[1][j] + jd * L[2][j]) * sc[j] for j in range(3)]
        dil = _d(cfg.dilation)
        S00 = ((U0[0] * U0[0] + U0[1] * U0[1]) + U0[2] * U0[2]) + dil
        S01 = (U0[0] * U1[0] + U0[1] * U1[1]) + U0[2] * U1[2]
        S11 = ((U1[0] * U1[0] + U1[1] * U1[1]) + U1[2] * U1[2]) + dil
        det = S00 * S11 - S01 * S01

        u = (fx * px) * iz + cx
        v = (fy * py) * iz + cy

        ntx = cfg.tiles_x
        nty = cfg.tiles_y
        ext = _d(cfg.extent_sigma)
        if ext > 0.0:
            hx = ext * np.sqrt(S00)
            hy = ext * np.sqrt(S11)
            tw = float(cfg.tile_w)
            th = float(cfg.tile_h)
            x_lo = np.maximum(np.floor(((u - hx) + 0.5) / tw), 0.0)
            x_hi = np.minimum(np.floor(((u + hx) - 0.5) / tw), float(ntx - 1))
            y_lo = np.maximum(np.floor(((v - hy) + 0.5) / th), 0.0)
            y_hi = np.minimum(np.floor(((v + hy) - 0.5) / th), float(nty - 1))
        else:  # unbounded support: every tile
            hx = hy = np.full_like(u, np.inf)
            x_lo = np.zeros_like(u)
            x_hi = np.full_like(u, float(ntx - 1))
            y_lo = np.zeros_like(u)
            y_hi = np.full_like(u, float(nty - 1))
        valid = in_front & (det > 0.0) & (x_lo <= x_hi) & (y_lo <= y_hi)
        xl = np.where(valid, x_lo, 0).astype(np.int64)
        xh = np.where(valid, x_hi, -1).astype(np.int64)
        yl = np.where(valid, y_lo, 0).astype(np.int64)
        yh = np.where(valid, y_hi, -1).astype(np.int64)
        count = np.where(valid, (xh - xl + 1) * (yh - yl + 1), 0)
        key = pz.astype(np.float32).view(np.uint32)
        key = np.where(valid, key, np.uint32(0xFFFFFFFF)).astype(np.uint32)
    return dict(u=u, v=v, S00=S00, S01=S01, S11=S11, det=det, half=(hx, hy),
                rect=np.stack([xl, xh, yl, yh]), count=count.astype(np.int64),
                key=key, pz=pz, px=px, py=py, valid=valid)


def frame_pairs(proj, cfg):
    """(tile, key, index) of every covered (tile, Gaussian) pair of one frame,
    in ascending (tile, key, index) order."""
    ntx = cfg.tiles_x
    xl, xh, yl, yh = proj["rect"]
    idx = np.nonzero(proj["valid"])[0]
    cnt = proj["count"][idx]
    rep = np.repeat(idx, cnt)
    # position of each pair inside its Gaussian's rectangle (row-major)
    starts = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(rep.size) - starts
    wdt = (xh - xl + 1)[rep]
    ty = yl[rep] + local // wdt
    tx = xl[rep] + local % wdt
    tile = ty * ntx + tx
    key = proj["key"][rep]
    order = np.lexsort((rep, key, tile))
    return tile[order], key[order], rep[order]


def sorted_pairs(g, frames, cfg):
    """All pairs of a batch, ascending (frame, tile, depth key, index).

    Returns dict(frame, tile, key, index, P, projections)."""
    fr, tl, ky, ix, projs = [], [], [], [], []
    for f, frame in enumerate(frames):
        p = project(g, frame, cfg, f)
        projs.append(p)
        t, k, i = frame_pairs(p, cfg)
        fr.append(np.full(t.size, f, np.int64))
        tl.append(t)
        ky.append(k)
        ix.append(i)
    cat = lambda a: np.concatenate(a) if a else np.zeros(0, np.int64)
    out = dict(frame=cat(fr), tile=cat(tl), key=cat(ky).astype(np.uint32), index=cat(ix),
               projections=projs)
    out["P"] = int(out["tile"].size)
    return out


def tile_lists(pairs, frame, n_tiles):
    """Per-tile Gaussian index lists (sorted) for one frame of `sorted_pairs`."""
    sel = pairs["frame"] == frame
    tile = pairs["tile"][sel]
    idx = pairs["index"][sel]
    bounds = np.searchsorted(tile, np.arange(n_tiles + 1))
    return [idx[bounds[t]:bounds[t + 1]] for t in range(n_tiles)]


def lists_for_tiles(proj, cfg, tiles):
    """Sorted Gaussian lists of selected tiles of one frame, straight from the
    rectangle test: the same lists as `frame_pairs`, for a few tiles of a
    large frame without building every pair."""
    xl, xh, yl, yh = proj["rect"]
    valid = proj["valid"]
    out = {}
    for tid in tiles:
        ty, tx = divmod(int(tid), cfg.tiles_x)
        idx = np.nonzero(valid & (xl <= tx) & (tx <= xh) & (yl <= ty) & (ty <= yh))[0]
        order = np.lexsort((idx, proj["key"][idx]))
        out[int(tid)] = idx[order]
    return out
