"""Pins for oracle.tof (phasor, d_ToF and amplitude from raw quads)."""
import math

import numpy as np
import pytest

import scenes
from oracle import render, tof

C = 299_792_458.0


def test_single_gaussian_amplitude_and_range():
    # One Gaussian on the optical axis at range z, no background: the phasor
    # of the quads has length 2 (s r / z^2) alpha, so the amplitude is
    # s r / z^2 alpha (paper §2 with alpha = 1 for an opaque surface), and the
    # recovered range is z modulo c / 2f.
    for z, f in ((2.0, 30e6), (3.7, 60e6)):
        n = 1
        g = scenes.Gaussians(mean=np.array([[0.0], [0.0], [z]], np.float32),
                             vel=np.zeros((3, 1), np.float32), acc=np.zeros((3, 1), np.float32),
                             scale=np.full((3, 1), 0.1, np.float32),
                             quat=np.array([[1.0], [0], [0], [0]], np.float32),
                             omega=np.zeros((3, 1), np.float32),
                             opacity_logit=np.array([1.0], np.float32),
                             rgb=np.ones((3, 1), np.float32), albedo=np.array([0.6], np.float32))
        cfg = scenes.RenderConfig(width=16, height=16, tile_w=8, tile_h=8, freqs=(f,)).strict()
        out = render.render(g, [scenes.Frame(fx=16.0, fy=16.0, cx=8.0, cy=8.0)], cfg)
        t = tof.tof_epilogue(out["quad"], cfg)
        alpha = 1.0 - out["T_final"][0]
        zf = float(np.float32(z))
        amp = float(np.float32(0.6)) / zf ** 2 * alpha
        np.testing.assert_allclose(t["amplitude"][0, 0], amp, rtol=1e-6, atol=1e-7 * amp.max())
        ok = amp > 1e-3 * amp.max()   # the phase is only defined where light returns
        du = C / (2 * float(np.float32(f)))
        np.testing.assert_allclose(t["d_tof"][0, 0][ok], zf % du, rtol=1e-6)


def test_eq1_differences_for_standard_offsets():
    wl = scenes.tiny_scene(20, 16, 12, seed=2)
    out = render.render(wl.gaussians, wl.frames, wl.cfg)
    t = tof.tof_epilogue(out["quad"], wl.cfg)
    q = out["quad"][0]
    scale = np.abs(q).max()
    np.testing.assert_allclose(t["phasor"][0, 0, 1], q[0] - q[2], atol=1e-6 * scale)
    np.testing.assert_allclose(t["phasor"][0, 0, 0], q[1] - q[3], atol=1e-6 * scale)


@pytest.mark.parametrize("freq,d", [(30e6, 2.1), (60e6, 3.6)])
def test_shell_range_recovery(freq, d):
    # every Gaussian at range d: d_ToF = d modulo the unambiguous range c / 2f
    rng = np.random.default_rng(1)
    n = 40
    u, v = rng.uniform(2, 30, n), rng.uniform(2, 22, n)
    dirs = np.stack([(u - 16) / 30, (v - 12) / 30, np.ones(n)], 1)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    m = (dirs * d).T.astype(np.float32)
    g = scenes.Gaussians(mean=m, vel=np.zeros((3, n), np.float32), acc=np.zeros((3, n), np.float32),
                         scale=np.full((3, n), 0.1, np.float32),
                         quat=np.tile(np.array([[1.0], [0], [0], [0]], np.float32), (1, n)),
                         omega=np.zeros((3, n), np.float32),
                         opacity_logit=rng.normal(0, 1, n).astype(np.float32),
                         rgb=np.ones((3, n), np.float32),
                         albedo=rng.uniform(0.2, 1, n).astype(np.float32))
    cfg = scenes.RenderConfig(width=32, height=24, tile_w=8, tile_h=8, freqs=(freq,))
    out = render.render(g, [scenes.Frame(fx=30.0, fy=30.0, cx=16.0, cy=12.0)], cfg)
    t = tof.tof_epilogue(out["quad"], cfg)
    a = t["amplitude"][0, 0]
    ok = a > 1e-4 * a.max()
    du = C / (2 * freq)
    ranges = np.linalg.norm(m.astype(np.float64), axis=0)
    assert np.abs(t["d_tof"][0, 0][ok] - (d % du)).max() < 1e-5 * du + (ranges.max() - ranges.min())
