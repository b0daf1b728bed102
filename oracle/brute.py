"""Brute-force per-pixel renderer in plain Python floats (tiny scenes only).

TEST INFRASTRUCTURE ONLY (see the package header).

For every pixel: compute every Gaussian's screen-space quantities from the
standard formulas (normalised quaternion rotation, EWA covariance with the
pinhole Jacobian), keep those whose support reaches the pixel's tile (or all
of them with unbounded support: some pixel centre of the tile lies within the
axis-aligned box around the extent ellipse, tested here by the distance from
the centre to the tile's nearest pixel-centre row and column), order them by
(float32 depth bits, index)
and walk them one by one applying Eqs. 2, 4 and 5 of paper §3 with the skip /
clamp / stop rules stated in oracle.render.  No vectorisation, no tiles
shared between pixels: an independent check of oracle.render.
"""
from __future__ import annotations

import math
import struct


def _f32(x):
    return struct.unpack("f", struct.pack("f", float(x)))[0]


def _f32bits(x):
    return struct.unpack("I", struct.pack("f", float(x)))[0]


def gaussian_2d(g, k, frame, cfg):
    t = _f32(frame.time)
    mu = [_f32(g.mean[i, k]) + _f32(g.vel[i, k]) * t + 0.5 * _f32(g.acc[i, k]) * t * t
          for i in range(3)]
    w0, x0, y0, z0 = (_f32(g.quat[i, k]) for i in range(4))
    ox, oy, oz = (_f32(g.omega[i, k]) for i in range(3))
    # q(t) = q0 + t/2 * (0, omega) (x) q0
    w = w0 + 0.5 * t * (-(ox * x0 + oy * y0 + oz * z0))
    x = x0 + 0.5 * t * (w0 * ox + oy * z0 - oz * y0)
    y = y0 + 0.5 * t * (w0 * oy + oz * x0 - ox * z0)
    z = z0 + 0.5 * t * (w0 * oz + ox * y0 - oy * x0)
    n = math.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    R = [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
         [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
         [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]]
    s = [_f32(g.scale[i, k]) for i in range(3)]
    Sig = [[sum(R[i][m] * s[m] * s[m] * R[j][m] for m in range(3)) for j in range(3)]
           for i in range(3)]
    Wc = [[_f32(frame.R[i][j]) for j in range(3)] for i in range(3)]
    tc = [_f32(frame.t[i]) for i in range(3)]
    p = [sum(Wc[i][j] * mu[j] for j in range(3)) + tc[i] for i in range(3)]
    fx, fy, cx, cy = _f32(frame.fx), _f32(frame.fy), _f32(frame.cx), _f32(frame.cy)
    J = [[fx / p[2], 0.0, -fx * p[0] / p[2] ** 2], [0.0, fy / p[2], -fy * p[1] / p[2] ** 2]]
    T = [[sum(J[i][m] * Wc[m][j] for m in range(3)) for j in range(3)] for i in range(2)]
    S2 = [[sum(T[i][a] * Sig[a][b] * T[j][b] for a in range(3) for b in range(3))
           for j in range(2)] for i in range(2)]
    dil = _f32(cfg.dilation)
    a, b, c = S2[0][0] + dil, S2[0][1], S2[1][1] + dil
    det = a * c - b * b
    centre = [-sum(Wc[j][i] * tc[j] for j in range(3)) for i in range(3)]
    d = math.sqrt(sum((mu[i] - centre[i]) ** 2 for i in range(3)))
    mid = 0.5 * (a + c)
    lam = mid + math.sqrt(max(mid * mid - det, 0.0))
    logit = _f32(g.opacity_logit[k])
    return dict(u=fx * p[0] / p[2] + cx, v=fy * p[1] / p[2] + cy,
                A=c / det, B=-b / det, C=a / det, det=det, pz=p[2], lam=lam, d=d,
                S2=[[a, b], [b, c]],
                o=1.0 / (1.0 + math.exp(-logit)),
                rgb=[_f32(g.rgb[i, k]) for i in range(3)],
                amp=_f32(cfg.source_intensity) * _f32(g.albedo[k]) / (d * d),
                psi=[4.0 * math.pi * _f32(f) * d / 299_792_458.0 for f in cfg.freqs])


def render_frame(g, frame, cfg):
    """Returns dict of nested lists: rgb[3][H][W], quad[NQ][H][W],
    depth[H][W], T_final[H][W], n_contrib[H][W], n_evaluated[H][W] (entries
    whose alpha the pixel computes) and n_composited[H][W]."""
    H, W = cfg.height, cfg.width
    gs = [gaussian_2d(g, k, frame, cfg) for k in range(g.n)]
    NQ = cfg.n_quad
    bgq = [0.0] * NQ if frame.bg_quad is None else \
        [_f32(x) for x in list(frame.bg_quad.reshape(-1))]
    bgr = [_f32(x) for x in frame.bg_rgb]
    res = dict(rgb=[[[0.0] * W for _ in range(H)] for _ in range(3)],
               quad=[[[0.0] * W for _ in range(H)] for _ in range(NQ)],
               depth=[[0.0] * W for _ in range(H)], T_final=[[0.0] * W for _ in range(H)],
               n_contrib=[[0] * W for _ in range(H)], n_evaluated=[[0] * W for _ in range(H)],
               n_composited=[[0] * W for _ in range(H)])
    for j in range(H):
        for i in range(W):
            tx, ty = i // cfg.tile_w, j // cfg.tile_h
            cand = []
            for k, q in enumerate(gs):
                if not (q["pz"] > cfg.near_z and q["det"] > 0):
                    continue
                if cfg.extent_sigma > 0:
                    # nearest pixel-centre column / row of the tile to the centre
                    nx = min(max(q["u"], tx * cfg.tile_w + 0.5), (tx + 1) * cfg.tile_w - 0.5)
                    ny = min(max(q["v"], ty * cfg.tile_h + 0.5), (ty + 1) * cfg.tile_h - 0.5)
                    hx = cfg.extent_sigma * math.sqrt(q["S2"][0][0])
                    hy = cfg.extent_sigma * math.sqrt(q["S2"][1][1])
                    if abs(nx - q["u"]) > hx or abs(ny - q["v"]) > hy:
                        continue
                cand.append((_f32bits(q["pz"]), k))
            cand.sort()
            x, y = i + 0.5, j + 0.5
            T = 1.0
            rgb = [0.0] * 3
            dep = 0.0
            quad = [0.0] * NQ
            last = 0
            n_eval = n_comp = 0
            for pos, (_, k) in enumerate(cand):
                q = gs[k]
                n_eval += 1
                dx, dy = x - q["u"], y - q["v"]
                power = -0.5 * (q["A"] * dx * dx + q["C"] * dy * dy) - q["B"] * dx * dy
                alpha = min(cfg.alpha_max, q["o"] * math.exp(power))
                if alpha < cfg.alpha_min:
                    continue
                nt = T * (1.0 - alpha)
                if nt < cfg.T_min:
                    break
                for ch in range(3):
                    rgb[ch] += q["rgb"][ch] * alpha * T
                dep += q["d"] * alpha * T
                m = 0
                for fi in range(cfg.n_freq):
                    for ph in cfg.phases:
                        quad[m] += q["amp"] * math.sin(q["psi"][fi] + _f32(ph)) * alpha * T * T
                        m += 1
                T = nt
                last = pos + 1
                n_comp += 1
            for ch in range(3):
                res["rgb"][ch][j][i] = rgb[ch] + bgr[ch] * T
            for m in range(NQ):
                res["quad"][m][j][i] = quad[m] + bgq[m] * T ** cfg.bg_T_power
            res["depth"][j][i] = dep
            res["T_final"][j][i] = T
            res["n_contrib"][j][i] = last
            res["n_evaluated"][j][i] = n_eval
            res["n_composited"][j][i] = n_comp
    return res
