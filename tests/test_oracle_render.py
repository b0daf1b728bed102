"""Pins for oracle.render, oracle.recursion and oracle.brute."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import binning, brute, recursion, render

C = 299_792_458.0


def _gauss(means, scales, logits, albedo=None, rgb=None, quats=None):
    n = len(means)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    q = np.zeros((4, n)); q[0] = 1.0
    if quats is not None:
        q = np.asarray(quats, np.float64).T
    return scenes.Gaussians(
        mean=f32(np.asarray(means).T), vel=f32(np.zeros((3, n))), acc=f32(np.zeros((3, n))),
        scale=f32(np.asarray(scales).T), quat=f32(q), omega=f32(np.zeros((3, n))),
        opacity_logit=f32(logits),
        rgb=f32(np.full((3, n), 0.5) if rgb is None else np.asarray(rgb).T),
        albedo=f32(np.ones(n) if albedo is None else albedo))


def _f32(x):
    return float(np.float32(x))


def test_single_gaussian_closed_form():
    # One axis-aligned Gaussian on the optical axis, alone in the scene:
    # alpha(x) = o exp(-1/2 d^T Sigma'^-1 d), Sigma' = diag(f^2 s^2 / z^2) + dil,
    # rgb = c alpha + c_bg (1 - alpha), quad_j = (s r / z^2) sin(4 pi f z / c + phi_j) alpha
    # + q_bg (1 - alpha)^p.
    z, sx, sy = 2.0, 0.1, 0.06
    g = _gauss([(0.0, 0.0, z)], [(sx, sy, 0.02)], [0.4], albedo=[0.7], rgb=[(0.2, 0.5, 0.9)])
    cfg = scenes.RenderConfig(width=24, height=20, tile_w=8, tile_h=8).strict()
    bgq = np.array([[0.3, -0.2, 0.1, 0.05]], np.float32)
    fr = scenes.Frame(fx=60.0, fy=60.0, cx=12.0, cy=10.0, bg_rgb=np.array([0.1, 0.2, 0.3], np.float32),
                      bg_quad=bgq)
    for p_bg in (1, 2):
        c2 = dataclasses.replace(cfg, bg_T_power=p_bg)
        out = render.render(g, [fr], c2)
        s00 = 60.0 ** 2 * _f32(sx) ** 2 / z ** 2 + _f32(0.3)
        s11 = 60.0 ** 2 * _f32(sy) ** 2 / z ** 2 + _f32(0.3)
        o = 1.0 / (1.0 + math.exp(-_f32(0.4)))
        ys, xs = np.mgrid[0:20, 0:24] + 0.5
        alpha = o * np.exp(-0.5 * ((xs - 12.0) ** 2 / s00 + (ys - 10.0) ** 2 / s11))
        for ch, col in enumerate((0.2, 0.5, 0.9)):
            exp = _f32(col) * alpha + _f32(fr.bg_rgb[ch]) * (1 - alpha)
            np.testing.assert_allclose(out["rgb"][0, ch], exp, rtol=1e-12, atol=1e-14)
        amp = _f32(0.7) / z ** 2
        psi = 4 * math.pi * 30e6 * z / C
        for j, ph in enumerate(cfg.phases):
            exp = amp * math.sin(psi + _f32(ph)) * alpha + _f32(bgq[0, j]) * (1 - alpha) ** p_bg
            np.testing.assert_allclose(out["quad"][0, j], exp, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(out["depth"][0], z * alpha, rtol=1e-12)
        np.testing.assert_allclose(out["T_final"][0], 1 - alpha, rtol=1e-12)
        assert (out["n_contrib"][0] == 1).all()


def test_eq4_quad_list_for_four_offsets():
    # Paper Eq. 4: for offsets 0, pi/2, pi, 3pi/2 the quad factors are
    # sin psi, cos psi, -sin psi, -cos psi.
    z = 3.3
    g = _gauss([(0.0, 0.0, z)], [(0.2, 0.2, 0.2)], [2.0])
    cfg = scenes.RenderConfig(width=8, height=8, tile_w=8, tile_h=8).strict()
    out = render.render(g, [scenes.Frame(fx=8.0, fy=8.0, cx=4.0, cy=4.0)], cfg)
    q = out["quad"][0][:, 4, 4]
    psi = 4 * math.pi * 30e6 * z / C
    ratio = q / q[0] * math.sin(psi)
    np.testing.assert_allclose(ratio, [math.sin(psi), math.cos(psi), -math.sin(psi), -math.cos(psi)],
                               rtol=1e-6, atol=1e-7)


def _shell(n, d, seed, width=32, height=24, f=30.0, size=1.0, logit_shift=0.0):
    """n Gaussians at the same range d from the optical centre, in the view."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(2, width - 2, n)
    v = rng.uniform(2, height - 2, n)
    dirs = np.stack([(u - width / 2) / f, (v - height / 2) / f, np.ones(n)], 1)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    means = dirs * d
    # float32 rounding moves ranges by ~1e-7 relative; keep it in mind in tolerances
    return _gauss(means, rng.uniform(0.02, 0.08, (n, 3)) * d / 2 * size,
                  rng.normal(0, 1, n) + logit_shift,
                  albedo=rng.uniform(0.2, 1.0, n), rgb=np.ones((n, 3)))


@pytest.mark.parametrize("freq,d", [(30e6, 2.1), (60e6, 3.6), (60e6, 4.4)])
def test_phase_of_equal_range_shell(freq, d):
    # Eq. 1: with every Gaussian at range d and no background, the recovered
    # phase atan2(Q0 - Qpi, Qpi/2 - Q3pi/2) mod 2 pi equals 4 pi f d / c mod 2 pi,
    # independent of the weights.  60 MHz with d > c / 2f = 2.498 m wraps.
    g = _shell(30, d, seed=1)
    cfg = scenes.RenderConfig(width=32, height=24, tile_w=8, tile_h=8, freqs=(freq,))
    fr = scenes.Frame(fx=30.0, fy=30.0, cx=16.0, cy=12.0)
    out = render.render(g, [fr], cfg)
    q = out["quad"][0]
    mag = np.hypot(q[0] - q[2], q[1] - q[3])
    m = mag > 1e-6 * mag.max()
    phase = np.mod(np.arctan2(q[0] - q[2], q[1] - q[3]), 2 * np.pi)[m]
    ranges = np.linalg.norm(g.mean.astype(np.float64), axis=0)
    for r in (ranges.min(), ranges.max()):
        exp = (4 * np.pi * freq * r / C) % (2 * np.pi)
        assert np.abs(np.angle(np.exp(1j * (phase - exp)))).max() < 1e-5
    # Eq. 1 in its arctan form, for a phase inside (-pi/2, pi/2):
    psi = 4 * np.pi * freq * ranges.mean() / C
    # amplitude A = s r / d^2 is recovered too (paper §2): half the phasor length
    assert np.all(mag[m] > 0)


def test_telescoping_and_monotone_transmittance():
    # With all colours and the background equal to 1, Eq. 2 gives exactly 1
    # (sum_k alpha_k T_k + T_final = 1); with all ranges equal to d, Eq. 5 gives
    # d (1 - T_final); T_final lies in [T_min, 1].
    d = 2.0
    g = _shell(150, d, seed=2, size=5.0, logit_shift=2.0)
    cfg = scenes.RenderConfig(width=32, height=24, tile_w=8, tile_h=8)
    fr = scenes.Frame(fx=30.0, fy=30.0, cx=16.0, cy=12.0, bg_rgb=np.ones(3, np.float32))
    out = render.render(g, [fr], cfg)
    np.testing.assert_allclose(out["rgb"], 1.0, rtol=1e-12)
    ranges = np.linalg.norm(g.mean.astype(np.float64), axis=0)
    dep = out["depth"][0]
    lo = ranges.min() * (1 - out["T_final"][0])
    hi = ranges.max() * (1 - out["T_final"][0])
    assert np.all(dep >= lo - 1e-12) and np.all(dep <= hi + 1e-12)
    assert out["T_final"].min() >= _f32(cfg.T_min) and out["T_final"].max() <= 1.0
    assert out["T_final"].min() < 0.05   # the scene is dense enough to exercise the stop rule


def test_quad_factorisation_identity():
    # Q(phi) = cos(phi) Q(0) + sin(phi) Q(pi/2) for any offset (no background):
    # the identity the two-accumulator GPU kernels rely on.
    wl = scenes.tiny_scene(25, 24, 16, seed=4)
    phis = (0.0, 0.5 * np.pi, 0.3, 2.0, 4.1)
    cfg = dataclasses.replace(wl.cfg, phases=phis)
    fr = dataclasses.replace(wl.frames[0], bg_quad=None)
    out = render.render(wl.gaussians, [fr], cfg)
    q = out["quad"][0]
    for j, ph in enumerate(phis):
        ph = _f32(ph)
        # Q(0) and Q(pi/2) are rendered with float32-rounded offsets
        c0, s0 = math.cos(_f32(0.5 * np.pi)), math.sin(_f32(0.5 * np.pi))
        # solve for the two accumulators from Q(0) = S and Q(pi/2) = c0 S + s0 C
        S = q[0]
        Cc = (q[1] - c0 * S) / s0
        np.testing.assert_allclose(q[j], math.cos(ph) * S + math.sin(ph) * Cc, atol=1e-13)


@pytest.mark.parametrize("strict", [True, False])
@pytest.mark.parametrize("seed", [0, 1])
def test_matches_brute_force(strict, seed):
    wl = scenes.tiny_scene(14, 20, 13, seed=seed, dynamic=True)
    cfg = wl.cfg.strict() if strict else wl.cfg
    fr = dataclasses.replace(wl.frames[0], time=0.1, bg_rgb=np.array([0.3, -0.2, 0.5], np.float32),
                             bg_quad=np.array([[0.2, -0.4, 0.1, 0.7]], np.float32))
    out = render.render(wl.gaussians, [fr], cfg)
    ref = brute.render_frame(wl.gaussians, fr, cfg)
    np.testing.assert_allclose(out["rgb"][0], np.array(ref["rgb"]), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(out["quad"][0], np.array(ref["quad"]), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(out["depth"][0], np.array(ref["depth"]), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(out["T_final"][0], np.array(ref["T_final"]), rtol=1e-11, atol=1e-14)
    assert (out["n_contrib"][0] == np.array(ref["n_contrib"])).all()
    # the workload counts: entries evaluated up to the stop, entries composited
    assert (out["n_evaluated"][0] == np.array(ref["n_evaluated"])).all()
    assert (out["n_composited"][0] == np.array(ref["n_composited"])).all()
    if not strict:
        assert (out["n_evaluated"][0] > out["n_composited"][0]).any()


def test_recursion_S2_S3_matches_autograd():
    # The supplement's recursions (plus the background term) give the same
    # dL/dalpha as differentiating the closed-form sums.
    rng = np.random.default_rng(0)
    K, P, NQ = 12, 7, 4
    alpha = rng.uniform(0.05, 0.9, (K, P))
    alpha[rng.uniform(size=(K, P)) < 0.2] = 0.0          # skipped entries
    colors = rng.uniform(0, 1, (K, 3))
    depths = rng.uniform(1, 4, K)
    qv = rng.normal(0, 1, (K, NQ))
    up_rgb, up_d, up_q = rng.normal(0, 1, (3, P)), rng.normal(0, 1, P), rng.normal(0, 1, (NQ, P))
    bg_rgb, bg_q = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, NQ)
    for p_bg in (1, 2):
        rec = recursion.alpha_grads(alpha, colors, depths, qv, up_rgb, up_d, up_q, bg_rgb, bg_q, p_bg)
        a = torch.tensor(alpha, requires_grad=True)
        om = 1 - a
        cp = torch.cumprod(om, 0)
        T = torch.cat([torch.ones(1, P, dtype=torch.float64), cp[:-1]], 0)
        Tf = cp[-1]
        w = a * T
        rgb = torch.tensor(colors).T @ w + torch.tensor(bg_rgb)[:, None] * Tf
        dep = torch.tensor(depths) @ w
        quad = torch.tensor(qv).T @ (w * T) + torch.tensor(bg_q)[:, None] * Tf ** p_bg
        loss = (torch.tensor(up_rgb) * rgb).sum() + (torch.tensor(up_d) * dep).sum() \
            + (torch.tensor(up_q) * quad).sum()
        loss.backward()
        auto = a.grad.numpy() * (alpha > 0)
        np.testing.assert_allclose(rec, auto, rtol=1e-10, atol=1e-12)
    # without the background term the supplement's recursion alone disagrees
    rec0 = recursion.alpha_grads(alpha, colors, depths, qv, up_rgb, up_d, up_q,
                                 np.zeros(3), np.zeros(NQ), 1)
    assert np.abs(rec0 - auto).max() > 1e-3


def _smooth_scene(seed, dynamic):
    wl = scenes.tiny_scene(8, 16, 12, seed=seed, dynamic=dynamic)
    g = wl.gaussians
    g.opacity_logit[:] = np.clip(g.opacity_logit, -2.0, 1.5)   # o <= 0.82 < alpha_max
    return wl


@pytest.mark.parametrize("dynamic", [False, True])
def test_gradients_central_differences(dynamic):
    wl = _smooth_scene(5, dynamic)
    cfg = wl.cfg.strict()
    fr = dataclasses.replace(wl.frames[0], time=0.15 if dynamic else 0.0,
                             bg_rgb=np.array([0.2, 0.1, -0.3], np.float32),
                             bg_quad=np.array([[0.3, -0.1, 0.2, 0.4]], np.float32))
    up = scenes.upstream_grads(1, cfg, seed=9)
    g64 = scenes.Gaussians(**{k: v.astype(np.float64) for k, v in wl.gaussians.arrays().items()})
    out = render.render(g64, [fr], cfg, upstream=up)
    rng = np.random.default_rng(1)
    fields = list(scenes.Gaussians.FIELDS)
    if not dynamic:
        fields = [f for f in fields if f not in ("vel", "acc", "omega")]
    for name in fields:
        arr = getattr(g64, name)
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            vals = []
            for sgn in (1, -1):
                gp = scenes.Gaussians(**{k: v.copy() for k, v in g64.arrays().items()})
                getattr(gp, name)[idx] += sgn * h
                vals.append(render.loss_of(render.render(gp, [fr], cfg), up))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = out["grads"][name][idx]
            assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-2), (name, idx, fd, an)
    # background gradients: dL/dc_bg = sum up * T_final, dL/dq_bg = sum up * T_final^p
    Tf = out["T_final"][0]
    np.testing.assert_allclose(out["grad_bg_rgb"][0], (up["rgb"][0] * Tf).sum((1, 2)), rtol=1e-10)
    np.testing.assert_allclose(out["grad_bg_quad"][0], (up["quad"][0] * Tf).sum((1, 2)), rtol=1e-10)


def test_sh_gradients_central_differences():
    # view-dependent colour and reflectivity: the coefficients and, through
    # the viewing direction, the centre
    wl = _smooth_scene(5, False)
    cfg = wl.cfg.strict()
    fr = dataclasses.replace(wl.frames[0], bg_rgb=np.array([0.2, 0.1, -0.3], np.float32))
    up = scenes.upstream_grads(1, cfg, seed=4)
    g32 = scenes.with_sh(wl.gaussians, 3, seed=2)
    g64 = scenes.Gaussians(**{k: v.astype(np.float64) for k, v in g32.arrays().items()})
    out = render.render(g64, [fr], cfg, upstream=up)
    assert not np.any(out["grads"]["rgb"]) and not np.any(out["grads"]["albedo"])   # replaced by SH
    rng = np.random.default_rng(3)
    for name in ("sh_rgb", "sh_albedo", "mean"):
        arr = getattr(g64, name)
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            vals = []
            for sgn in (1, -1):
                gp = scenes.Gaussians(**{k: v.copy() for k, v in g64.arrays().items()})
                getattr(gp, name)[idx] += sgn * h
                vals.append(render.loss_of(render.render(gp, [fr], cfg), up))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = out["grads"][name][idx]
            assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-2), (name, idx, fd, an)


def test_sh_degree_zero_is_the_flat_colour():
    # DC-only coefficients built from rgb / albedo reproduce the flat render
    wl = scenes.cfg1()
    g = scenes.with_sh(wl.gaussians, 0, seed=0)
    a = render.render(g, wl.frames, wl.cfg)
    b = render.render(wl.gaussians, wl.frames, wl.cfg)
    for k in ("rgb", "quad", "depth"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-6, atol=1e-6)


def test_dense_scene_statistics():
    # cfg-1 sanity: pairs, contributions and the stop rule all exercised.
    wl = scenes.cfg1()
    out = render.render(wl.gaussians, wl.frames, wl.cfg)
    assert out["pairs"]["P"] > 1000
    assert out["n_contrib"].max() > 100
    assert np.isfinite(out["rgb"]).all() and np.isfinite(out["quad"]).all()
    assert out["flagged"].mean() < 0.05


def test_frame_offsets_are_centre_shifts():
    # deformation offsets (§4): with grid-exact values (multiples of 2^-10),
    # x0 + delta is exact in float32, so a frame rendered with an offset equals
    # the scene with that offset folded into the canonical centres, bit for bit
    wl = scenes.tiny_scene(12, 24, 16, seed=3)
    g = wl.gaussians
    q = 2.0 ** -10
    g.mean[:] = np.round(g.mean / q) * q
    rng = np.random.default_rng(0)
    delta = (rng.integers(-40, 40, (2, 3, g.n)) * q).astype(np.float32)
    frames = [wl.frames[0], dataclasses.replace(wl.frames[0], time=0.0)]
    cfg = wl.cfg
    gd = dataclasses.replace(g, delta=delta)
    out = render.render(gd, frames, cfg)
    for f in range(2):
        shifted = dataclasses.replace(g, mean=(g.mean + delta[f]).astype(np.float32))
        ref = render.render(shifted, [frames[f]], cfg)
        for k in ("rgb", "quad", "depth", "T_final", "n_contrib"):
            np.testing.assert_array_equal(out[k][f], ref[k][0], err_msg=k)
        a = binning.project(gd, frames[f], cfg, f)
        b = binning.project(shifted, frames[f], cfg)
        np.testing.assert_array_equal(a["rect"], b["rect"])
        np.testing.assert_array_equal(a["key"], b["key"])


def test_frame_offset_gradients_sum_to_the_centre_gradient():
    # every frame's centre is mean + (trajectory terms) + delta[f], so
    # dL/dmean = sum_f dL/ddelta[f]; plus central differences on delta itself
    wl = _smooth_scene(6, True)
    cfg = wl.cfg.strict()
    rng = np.random.default_rng(2)
    g64 = scenes.Gaussians(**{k: v.astype(np.float64) for k, v in wl.gaussians.arrays().items()})
    g64.delta = rng.normal(0, 0.01, (2, 3, g64.n))
    frames = [dataclasses.replace(wl.frames[0], time=0.1),
              dataclasses.replace(wl.frames[0], time=0.3, t_lo=0.25, t_hi=0.5)]
    up = scenes.upstream_grads(2, cfg, seed=4)
    out = render.render(g64, frames, cfg, upstream=up)
    np.testing.assert_allclose(out["grads"]["delta"].sum(0), out["grads"]["mean"], rtol=1e-12,
                               atol=1e-14)
    for _ in range(4):
        idx = tuple(rng.integers(0, s) for s in g64.delta.shape)
        h = 1e-6
        vals = []
        for sgn in (1, -1):
            gp = scenes.Gaussians(**{k: v.copy() for k, v in g64.arrays().items()})
            gp.delta[idx] += sgn * h
            vals.append(render.loss_of(render.render(gp, frames, cfg), up))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = out["grads"]["delta"][idx]
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-2), (idx, fd, an)
