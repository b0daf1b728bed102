"""Per-pixel opacity gradients by the supplement's back-to-front recursion.

TEST INFRASTRUCTURE ONLY (see the package header).

Supplement C writes the opacity gradient of the composited colour as
dc/dalpha_k = T_k (c_k - acc_k), acc_k = alpha_{k+1} c_{k+1} + (1 - alpha_{k+1}) acc_{k+1}
(Eq. S2) and, for the raw quads whose Gaussian terms carry T_k^2,
dq/dalpha_k = T_k^2 (q_k + 2 (alpha_k - 1) acc^q_k),
acc^q_k = alpha_{k+1} q_{k+1} + (1 - alpha_{k+1})^2 acc^q_{k+1}   (Eq. S3),
both with acc_N = 0.  The supplement drops the background: since the
background is weighted by T_final (RGB) or T_final^p (quads), its derivative
adds -c_bg T_final / (1 - alpha_k) and -p q_bg T_final^p / (1 - alpha_k).
The mean depth of Eq. 5 follows S2 with c_k replaced by d_k and no
background.

This module evaluates those recursions literally, pixel by pixel, for one
tile, so that tests can pin them against autograd of the closed-form sums
(oracle.render) and against finite differences.
"""
from __future__ import annotations

import numpy as np


def alpha_grads(alpha, colors, depths, quadvals, up_rgb, up_depth, up_quad,
                bg_rgb, bg_quad, bg_power=1):
    """dL/dalpha for every (entry, pixel) of one tile.

    alpha    [K, P]  composited opacities in list order (0 for skipped entries)
    colors   [K, 3]  c_k;  depths [K] d_k;  quadvals [K, NQ] q_k,j
    up_*     upstream gradients dL/d(output) per pixel: [3, P], [P], [NQ, P]
    bg_rgb   [3];  bg_quad [NQ]
    Returns [K, P].
    """
    K, P = alpha.shape
    out = np.zeros((K, P))
    for p in range(P):
        a = alpha[:, p]
        T = np.ones(K + 1)
        for k in range(K):
            T[k + 1] = T[k] * (1.0 - a[k])
        Tf = T[K]
        acc_c = np.zeros(3)
        acc_d = 0.0
        acc_q = np.zeros(quadvals.shape[1])
        for k in range(K - 1, -1, -1):
            if k < K - 1:
                an = a[k + 1]
                acc_c = an * colors[k + 1] + (1.0 - an) * acc_c
                acc_d = an * depths[k + 1] + (1.0 - an) * acc_d
                acc_q = an * quadvals[k + 1] + (1.0 - an) ** 2 * acc_q
            if a[k] == 0.0:
                continue  # not composited: its alpha is not a free variable here
            dc = T[k] * (colors[k] - acc_c) - bg_rgb * Tf / (1.0 - a[k])
            dd = T[k] * (depths[k] - acc_d)
            dq = T[k] ** 2 * (quadvals[k] + 2.0 * (a[k] - 1.0) * acc_q) \
                - bg_power * bg_quad * Tf ** bg_power / (1.0 - a[k])
            out[k, p] = up_rgb[:, p] @ dc + up_depth[p] * dd + up_quad[:, p] @ dq
    return out
