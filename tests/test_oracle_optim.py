"""Pins for oracle.optim and for the paper's constants (tests/golden)."""
import math
import os

import numpy as np
import pytest

import scenes
from oracle import optim, render

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        out[parts[0]] = parts[1:-1]
    return out


def test_adam_first_step_closed_form():
    # After one bias-corrected step, m_hat = g and v_hat = g^2, so the update is
    # -lr g / (|g| + eps) elementwise.
    g = _golden()
    b1, b2, eps = float(g["adam_beta1"][0]), float(g["adam_beta2"][0]), float(g["adam_eps"][0])
    rng = np.random.default_rng(0)
    p, gr = rng.normal(size=100), rng.normal(size=100) * 1e-3
    lr = float(g["reflectivity_lr"][0])
    p1, m, v = optim.adam_step(p, gr, np.zeros(100), np.zeros(100), 1, lr, b1, b2, eps)
    np.testing.assert_allclose(p1 - p, -lr * gr / (np.abs(gr) + eps), rtol=1e-12)
    # second step with the same gradient: still -lr sign(g) up to eps
    p2, _, _ = optim.adam_step(p1, gr, m, v, 2, lr, b1, b2, eps)
    np.testing.assert_allclose(p2 - p1, -lr * np.sign(gr), rtol=1e-9)


def test_l2_loss_gradient_central_differences():
    rng = np.random.default_rng(1)
    pr, pq = rng.normal(size=(3, 5, 4)), rng.normal(size=(4, 5, 4))
    tr, tq = rng.normal(size=pr.shape), rng.normal(size=pq.shape)
    loss, dr, dq = optim.l2_loss_grad(pr, pq, tr, tq, quad_weight=5.0)
    h = 1e-6
    for arr, grad, which in ((pr, dr, 0), (pq, dq, 1)):
        for idx in [(0, 0, 0), (2, 4, 3), (1, 2, 1)]:
            a2 = arr.copy(); a2[idx] += h
            args = (a2, pq) if which == 0 else (pr, a2)
            lp = optim.l2_loss_grad(*args, tr, tq, 5.0)[0]
            a2[idx] -= 2 * h
            args = (a2, pq) if which == 0 else (pr, a2)
            lm = optim.l2_loss_grad(*args, tr, tq, 5.0)[0]
            assert (lp - lm) / (2 * h) == pytest.approx(grad[idx], rel=1e-6)


def test_l2_loss_closed_forms():
    # Eq. 9's L2 part, w_q mean((q - q*)^2) + mean((c - c*)^2), with the two
    # means taken over tensors of different sizes (3 colour channels, 8 quad
    # channels at two frequencies, unequal frame counts).
    # (a) constant residuals c_r, c_q: L = w_q c_q^2 + c_r^2 whatever the sizes,
    #     and every gradient element is 2 c / (elements of its tensor), the
    #     quad one times w_q
    rng = np.random.default_rng(3)
    tr, tq = rng.normal(size=(2, 3, 7, 5)), rng.normal(size=(3, 8, 6, 4))
    cr, cq, w = 0.375, -1.25, 3.0
    loss, dr, dq = optim.l2_loss_grad(tr + cr, tq + cq, tr, tq, quad_weight=w)
    assert loss == pytest.approx(w * cq * cq + cr * cr, rel=1e-13)
    np.testing.assert_allclose(dr, 2 * cr / tr.size, rtol=1e-13)
    np.testing.assert_allclose(dq, w * 2 * cq / tq.size, rtol=1e-13)
    # (b) one non-zero residual d in each tensor: L = w_q d_q^2 / |q| + d_r^2 / |c|
    pr, pq = tr.copy(), tq.copy()
    pr[1, 2, 3, 4] += 0.5
    pq[2, 7, 0, 1] -= 2.0
    loss, dr, dq = optim.l2_loss_grad(pr, pq, tr, tq, quad_weight=w)
    assert loss == pytest.approx(w * 4.0 / tq.size + 0.25 / tr.size, rel=1e-12)
    assert np.count_nonzero(dr) == 1 and dr[1, 2, 3, 4] == pytest.approx(2 * 0.5 / tr.size, rel=1e-12)
    assert np.count_nonzero(dq) == 1 and dq[2, 7, 0, 1] == pytest.approx(-w * 2 * 2.0 / tq.size, rel=1e-12)
    # (c) zero quad weight: the quads do not enter
    loss, _, dq = optim.l2_loss_grad(tr + cr, tq + cq, tr, tq, quad_weight=0.0)
    assert loss == pytest.approx(cr * cr, rel=1e-13) and not np.any(dq)


def test_paper_constants():
    g = _golden()
    assert [float(eval(x.replace("pi", "*math.pi").lstrip("*") if "pi" in x else x))
            if x != "pi" else math.pi for x in g["phase_offsets"]] == pytest.approx(scenes.QUAD_PHASES)
    du = scenes.SPEED_OF_LIGHT / (2 * 30e6)
    assert du == pytest.approx(float(g["unambiguous_range_m_at_30MHz"][0]), abs=1e-4)
    assert render.C_LIGHT == scenes.SPEED_OF_LIGHT
    # the paper's random background range and initial reflectivity
    assert [float(x) for x in g["random_background_range"]] == [-1.0, 1.0]
    gt, tr, _ = scenes.cfg5_scenes(n=10)
    assert np.all(tr.albedo == np.float32(float(g["initial_reflectivity"][0])))


def test_decayed_learning_rate():
    # §4's network schedule: 8e-4 at the first step, 1.6e-6 from step 60001 on,
    # a constant ratio between consecutive steps in between
    lr0, lr1, S = 8e-4, 1.6e-6, 60_000
    assert optim.decayed_lr(lr0, lr1, S, 1) == lr0
    assert optim.decayed_lr(lr0, lr1, S, S + 1) == pytest.approx(lr1, rel=1e-12)
    assert optim.decayed_lr(lr0, lr1, S, 10 * S) == pytest.approx(lr1, rel=1e-12)
    r = [optim.decayed_lr(lr0, lr1, S, t + 1) / optim.decayed_lr(lr0, lr1, S, t) for t in (1, 500, 59_999)]
    assert r[0] == pytest.approx(r[1], rel=1e-9) and r[1] == pytest.approx(r[2], rel=1e-9)
    assert r[0] == pytest.approx((lr1 / lr0) ** (1 / S), rel=1e-12)
    assert optim.decayed_lr(lr0, lr1, 0, 123) == lr0
