"""L2 reconstruction loss and Adam in FP64 (paper §4).

TEST INFRASTRUCTURE ONLY (see the package header).

Loss (paper Eq. 9, L2 part only): L = w_q mean((q - q*)^2) + mean((c - c*)^2)
with the quad weight w_q (the paper's alpha: 1 for synthetic scenes).

Adam (paper §4 hyperparameters): beta = (0.9, 0.999), eps = 1e-15, per-group
learning rates; the bias-corrected update
m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Pins: tests/test_oracle_optim.py (first step equals -lr g / (|g| + eps);
loss gradient by central differences).
"""
from __future__ import annotations

import numpy as np


def l2_loss_grad(pred_rgb, pred_quad, tgt_rgb, tgt_quad, quad_weight=1.0):
    """Returns (loss, d_rgb, d_quad) in float64."""
    pr, pq = np.asarray(pred_rgb, np.float64), np.asarray(pred_quad, np.float64)
    tr, tq = np.asarray(tgt_rgb, np.float64), np.asarray(tgt_quad, np.float64)
    rr, rq = pr - tr, pq - tq
    loss = quad_weight * np.mean(rq * rq) + np.mean(rr * rr)
    return loss, 2.0 * rr / rr.size, quad_weight * 2.0 * rq / rq.size


def decayed_lr(lr, lr_final, decay_steps, step):
    """Exponential learning-rate decay (§4: the network's rate falls from
    8e-4 to 1.6e-6 over 60K iterations): lr at 1-based step 1, lr_final from
    step decay_steps + 1 on, geometric in between; constant without decay."""
    if decay_steps <= 0:
        return lr
    s = min(step - 1, decay_steps) / decay_steps
    return lr * (lr_final / lr) ** s


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-15):
    """One Adam update at 1-based step `step`; returns new (p, m, v)."""
    p, g = np.asarray(p, np.float64), np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
