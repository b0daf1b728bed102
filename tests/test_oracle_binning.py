"""Pins for oracle.binning (projection, tile rectangles, depth keys, order)."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import binning, render


def _single(mean, scale, quat=(1, 0, 0, 0), omega=(0, 0, 0), vel=(0, 0, 0), acc=(0, 0, 0)):
    f = lambda x, n: np.asarray(x, np.float32).reshape(n, 1)
    return scenes.Gaussians(mean=f(mean, 3), vel=f(vel, 3), acc=f(acc, 3), scale=f(scale, 3),
                            quat=f(quat, 4), omega=f(omega, 3),
                            opacity_logit=np.zeros(1, np.float32),
                            rgb=np.full((3, 1), 0.5, np.float32), albedo=np.ones(1, np.float32))


def test_axis_aligned_on_optical_axis_closed_form():
    # On the optical axis the Jacobian's third column vanishes, so
    # Sigma' = diag(fx^2 sx^2 / z^2, fy^2 sy^2 / z^2) + dilation I exactly.
    z, sx, sy, sz = 2.0, 0.05, 0.02, 0.3
    g = _single((0, 0, z), (sx, sy, sz))
    cfg = scenes.RenderConfig(width=64, height=48)
    fr = scenes.Frame(fx=60.0, fy=55.0, cx=32.0, cy=24.0)
    p = binning.project(g, fr, cfg)
    sx32, sy32 = float(np.float32(sx)), float(np.float32(sy))
    s00 = 60.0 ** 2 * sx32 ** 2 / z ** 2 + float(np.float32(0.3))
    s11 = 55.0 ** 2 * sy32 ** 2 / z ** 2 + float(np.float32(0.3))
    assert p["S00"][0] == pytest.approx(s00, rel=1e-14)
    assert p["S11"][0] == pytest.approx(s11, rel=1e-14)
    assert p["S01"][0] == 0.0
    assert (p["u"][0], p["v"][0]) == (32.0, 24.0)
    # the extent box: half-widths 3 sqrt(S00), 3 sqrt(S11); its tiles are those
    # whose pixel-centre range [16 t + 1/2, 16 t + 15.5] reaches into it
    hx, hy = 3.0 * math.sqrt(p["S00"][0]), 3.0 * math.sqrt(p["S11"][0])
    assert (p["half"][0][0], p["half"][1][0]) == (hx, hy)
    assert hx == pytest.approx(3.0 * math.sqrt(s00), rel=1e-14)
    tiles_x = [t for t in range(4) if 16 * t + 0.5 <= 32 + hx and 16 * t + 15.5 >= 32 - hx]
    tiles_y = [t for t in range(3) if 16 * t + 0.5 <= 24 + hy and 16 * t + 15.5 >= 24 - hy]
    assert list(p["rect"][:, 0]) == [tiles_x[0], tiles_x[-1], tiles_y[0], tiles_y[-1]]
    assert tiles_x != [0, 1, 2, 3] or tiles_y != [0, 1, 2]   # not the whole frame
    assert p["key"][0] == np.float32(z).view(np.uint32)


def test_extent_box_is_the_tight_box_of_the_ellipse():
    # The tile rectangle is the set of tiles whose pixel-centre ranges meet
    # the axis-aligned bounding box of the 3 sigma ellipse: for random
    # ellipses (covariances from random scales and rotations) the box's
    # half-widths equal the ellipse's extreme x and y (by dense sampling of
    # its boundary), and every tile of the rectangle has a pixel centre in
    # the box while its neighbours outside the rectangle have none
    rng = np.random.default_rng(3)
    cfg = scenes.RenderConfig(width=256, height=192)
    fr = scenes.Frame(fx=120.0, fy=120.0, cx=128.0, cy=96.0)
    n = 200
    g = scenes.draw_gaussians(n, 256, 192, 120.0, 120.0, seed=4, z_range=(1.0, 3.0),
                              log_scale_mean=float(np.log(0.08)), log_scale_std=0.6)
    p = binning.project(g, fr, cfg)
    th = np.linspace(0, 2 * np.pi, 20001)
    checked = 0
    for k in np.nonzero(p["valid"])[0]:
        S = np.array([[p["S00"][k], p["S01"][k]], [p["S01"][k], p["S11"][k]]])
        L = np.linalg.cholesky(S)
        pts = 3.0 * (L @ np.stack([np.cos(th), np.sin(th)]))
        hx, hy = p["half"][0][k], p["half"][1][k]
        assert np.abs(pts[0]).max() == pytest.approx(hx, rel=1e-6)
        assert np.abs(pts[1]).max() == pytest.approx(hy, rel=1e-6)
        xl, xh, yl, yh = p["rect"][:, k]
        u, v = p["u"][k], p["v"][k]
        meets_x = lambda t: 16 * t + 0.5 <= u + hx and 16 * t + 15.5 >= u - hx
        meets_y = lambda t: 16 * t + 0.5 <= v + hy and 16 * t + 15.5 >= v - hy
        assert all(meets_x(t) for t in range(xl, xh + 1)) and all(meets_y(t) for t in range(yl, yh + 1))
        assert (xl == 0 or not meets_x(xl - 1)) and (xh == cfg.tiles_x - 1 or not meets_x(xh + 1))
        assert (yl == 0 or not meets_y(yl - 1)) and (yh == cfg.tiles_y - 1 or not meets_y(yh + 1))
        checked += 1
    assert checked > 100


def test_rotation_about_z_closed_form():
    # q0 = identity, omega = (0, 0, w): q(t) = (1, 0, 0, w t / 2), a rotation by
    # theta = 2 atan(w t / 2) about z.  On the optical axis the 2D covariance is
    # then (f/z)^2 R2 diag(sx^2, sy^2) R2^T + dilation.
    w, t, z, sx, sy = 3.0, 0.25, 2.5, 0.06, 0.02
    g = _single((0, 0, z), (sx, sy, 0.01), omega=(0, 0, w))
    cfg = scenes.RenderConfig(width=64, height=48, dilation=0.0)
    fr = scenes.Frame(fx=60.0, fy=60.0, cx=32.0, cy=24.0, time=t)
    p = binning.project(g, fr, cfg)
    th = 2.0 * math.atan(w * t / 2.0)
    c, s = math.cos(th), math.sin(th)
    sx, sy = float(np.float32(sx)), float(np.float32(sy))
    k = (60.0 / z) ** 2
    assert p["S00"][0] == pytest.approx(k * (c * c * sx * sx + s * s * sy * sy), rel=1e-12)
    assert p["S11"][0] == pytest.approx(k * (s * s * sx * sx + c * c * sy * sy), rel=1e-12)
    assert p["S01"][0] == pytest.approx(k * c * s * (sx * sx - sy * sy), rel=1e-12)


def test_trajectory_closed_form():
    g = _single((0.1, -0.2, 2.0), (0.01, 0.01, 0.01), vel=(0.5, 0.25, -1.0), acc=(2.0, 0.0, 4.0))
    cfg = scenes.RenderConfig(width=64, height=48)
    t = np.float32(0.125)
    fr = scenes.Frame(time=float(t))
    p = binning.project(g, fr, cfg)
    t = float(t)
    x = float(np.float32(0.1)) + 0.5 * t + 1.0 * t * t
    z = 2.0 - 1.0 * t + 2.0 * t * t
    assert p["px"][0] == pytest.approx(x, rel=1e-15)
    assert p["pz"][0] == pytest.approx(z, rel=1e-15)


def test_eq7_unit_spacing_is_the_literal_formula():
    # Eq. 7 with integer timesteps i1, i2 = i1 + 1 and a fractional j between:
    # x_j = (i2 - j) x_i1 + (j - i1) x_i2, with x from the trajectory closed form.
    x0, v, a = (0.1, -0.2, 2.0), (0.5, 0.25, -1.0), (2.0, -3.0, 4.0)
    g = _single(x0, (0.01, 0.01, 0.01), vel=v, acc=a)
    cfg = scenes.RenderConfig(width=64, height=48)
    f32 = lambda z: float(np.float32(z))
    i1, j = 3.0, 3.25
    fr = scenes.Frame(time=j, t_lo=i1, t_hi=i1 + 1.0)
    p = binning.project(g, fr, cfg)
    traj = lambda t: np.array([f32(x0[c]) + f32(v[c]) * t + 0.5 * f32(a[c]) * t * t for c in range(3)])
    xj = (i1 + 1.0 - j) * traj(i1) + (j - i1) * traj(i1 + 1.0)
    np.testing.assert_allclose([p["px"][0], p["py"][0], p["pz"][0]], xj, rtol=1e-14)
    # ... which differs from the trajectory at j itself (the acceleration term)
    assert abs(p["pz"][0] - traj(j)[2]) > 0.1


def test_eq7_at_an_anchor_and_without_acceleration():
    wl = scenes.cfg3(n=500, n_frames=1, seed=4)
    g, cfg = wl.gaussians, wl.cfg
    base = wl.frames[0]
    # at t = t_lo the weights are exactly (1, 0): bit-identical to direct evaluation
    a = binning.project(g, dataclasses.replace(base, time=0.2, t_lo=0.2, t_hi=0.3), cfg)
    b = binning.project(g, dataclasses.replace(base, time=0.2), cfg)
    for k in ("px", "py", "pz", "u", "v", "key", "count"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(a["rect"], b["rect"])
    # without acceleration the trajectory is affine: interpolation = evaluation
    g0 = dataclasses.replace(g, acc=np.zeros_like(g.acc))
    a = binning.project(g0, dataclasses.replace(base, time=0.23, t_lo=0.2, t_hi=0.3), cfg)
    b = binning.project(g0, dataclasses.replace(base, time=0.23), cfg)
    np.testing.assert_allclose(a["pz"], b["pz"], rtol=1e-14)
    np.testing.assert_allclose(a["u"][a["valid"]], b["u"][a["valid"]], rtol=1e-12)


def test_eq7_differentiable_form_matches():
    wl = scenes.cfg3(n=800, n_frames=1, seed=6)
    for fr in scenes.async_quartet_frames(1, 0.1, wl.frames[0]):
        p = binning.project(wl.gaussians, fr, wl.cfg)
        q = render.gaussian_quantities(render.params_to_torch(wl.gaussians), fr, wl.cfg)
        v = p["valid"]
        np.testing.assert_allclose(p["u"][v], q["u"].numpy()[v], rtol=1e-10)
        np.testing.assert_allclose(p["v"][v], q["v"].numpy()[v], rtol=1e-10)


def test_culling():
    g = _single((0, 0, 0.1), (0.01, 0.01, 0.01))           # behind the near plane
    cfg = scenes.RenderConfig(width=64, height=48)
    assert not binning.project(g, scenes.Frame(), cfg)["valid"][0]
    g = _single((10.0, 0, 1.0), (0.01, 0.01, 0.01))         # far outside the image
    assert not binning.project(g, scenes.Frame(), cfg)["valid"][0]
    g = _single((0, 0, 1.0), (0.01, 0.01, 0.01))
    assert binning.project(g, scenes.Frame(), cfg)["valid"][0]


def test_matches_differentiable_projection():
    # Two independent formulations (pinned op order vs torch matrices).
    wl = scenes.cfg3(n=3000, n_frames=3)
    for fr in wl.frames:
        p = binning.project(wl.gaussians, fr, wl.cfg)
        q = render.gaussian_quantities(render.params_to_torch(wl.gaussians), fr, wl.cfg)
        v = p["valid"]
        det = p["S00"] * p["S11"] - p["S01"] ** 2
        np.testing.assert_allclose(p["u"][v], q["u"].numpy()[v], rtol=1e-10)
        np.testing.assert_allclose(p["v"][v], q["v"].numpy()[v], rtol=1e-10)
        np.testing.assert_allclose((p["S11"] / det)[v], q["A"].numpy()[v], rtol=1e-8)
        np.testing.assert_allclose((p["S00"] / det)[v], q["C"].numpy()[v], rtol=1e-8)


@pytest.mark.parametrize("maker", [lambda: scenes.cfg1(),
                                   lambda: scenes.cfg3(n=400, n_frames=3),
                                   lambda: scenes.tiny_scene(40, 20, 13, seed=3)])
def test_sorted_pairs_equal_python_sorted(maker):
    wl = maker()
    pairs = binning.sorted_pairs(wl.gaussians, wl.frames, wl.cfg)
    ref = []
    for f, fr in enumerate(wl.frames):
        p = binning.project(wl.gaussians, fr, wl.cfg)
        xl, xh, yl, yh = p["rect"]
        for k in range(wl.gaussians.n):
            if not p["valid"][k]:
                continue
            for ty in range(yl[k], yh[k] + 1):
                for tx in range(xl[k], xh[k] + 1):
                    ref.append((f, ty * wl.cfg.tiles_x + tx, int(p["key"][k]), k))
    ref.sort()
    got = list(zip(pairs["frame"].tolist(), pairs["tile"].tolist(), pairs["key"].tolist(),
                   pairs["index"].tolist()))
    assert got == ref
    assert pairs["P"] == len(ref) > 0


def test_scene_generation_deterministic():
    a = scenes.cfg3(seed=7, n=500).gaussians
    b = scenes.cfg3(seed=7, n=500).gaussians
    c = scenes.cfg3(seed=8, n=500).gaussians
    for k in scenes.Gaussians.FIELDS:
        assert getattr(a, k).tobytes() == getattr(b, k).tobytes()
        assert getattr(a, k).dtype == np.float32
    assert a.mean.tobytes() != c.mean.tobytes()


def test_lists_for_tiles_equal_full_binning():
    wl = scenes.cfg3(n=2000, n_frames=2)
    pairs = binning.sorted_pairs(wl.gaussians, wl.frames, wl.cfg)
    n_tiles = wl.cfg.tiles_x * wl.cfg.tiles_y
    for f, fr in enumerate(wl.frames):
        full = binning.tile_lists(pairs, f, n_tiles)
        some = binning.lists_for_tiles(binning.project(wl.gaussians, fr, wl.cfg), wl.cfg,
                                       [0, 7, n_tiles // 2, n_tiles - 1])
        for t, lst in some.items():
            np.testing.assert_array_equal(lst, full[t])
