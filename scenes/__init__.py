"""Seeded synthetic inputs for the C-ToF Gaussian rasterizer.

This module only *draws* inputs; it holds none of the rendering arithmetic.
Both the FP64 oracle (``oracle/``) and the HIP path consume the plain-data
structures defined here, so that the two implementations see identical bytes.

Scene model (paper §3, Eqs. 2-4): each Gaussian k has a centre x_k, a
covariance from scale + rotation, an opacity o_k, a colour c_k and a
reflectivity (albedo) r_k.  The dynamic configurations replace the paper's
deformation MLP (§4) by an analytic trajectory per Gaussian:
position x0 + v t + a t^2 / 2 and a constant angular rate omega.

All parameter arrays are float32, structure-of-arrays ([3][N], [4][N], [N]).
Random draws use numpy ``Generator(PCG64(seed))`` in float64, in this fixed
order: (u, v, z) -> log-scale -> quaternion -> opacity logit -> rgb -> albedo
-> velocity -> acceleration -> omega; then they are cast to float32.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SPEED_OF_LIGHT = 299_792_458.0  # m/s, used by the phase psi = 4 pi f d / c (paper §3)

# Quad phase offsets of a four-tap C-ToF camera (paper §2): 0, pi/2, pi, 3 pi/2.
QUAD_PHASES = (0.0, 0.5 * np.pi, np.pi, 1.5 * np.pi)


@dataclass
class Gaussians:
    """Structure-of-arrays Gaussian parameters, all float32."""

    mean: np.ndarray           # [3, N] position at t = 0 (m)
    vel: np.ndarray            # [3, N] velocity (m/s)
    acc: np.ndarray            # [3, N] acceleration (m/s^2)
    scale: np.ndarray          # [3, N] linear standard deviations (m)
    quat: np.ndarray           # [4, N] rotation quaternion (w, x, y, z) at t = 0
    omega: np.ndarray          # [3, N] angular rate (rad/s)
    opacity_logit: np.ndarray  # [N] o = sigmoid(logit)
    rgb: np.ndarray            # [3, N] colour c_k
    albedo: np.ndarray         # [N] reflectivity r_k
    # optional view-dependent colour / reflectivity (paper §3): real spherical
    # harmonic coefficients, [K, 3, N] and [K, N] with K = (degree + 1)^2;
    # when present they replace rgb / albedo
    sh_rgb: Optional[np.ndarray] = None
    sh_albedo: Optional[np.ndarray] = None
    # optional per-frame centre offsets [F, 3, N] (paper §4: the deformation
    # network's delta x, evaluated at each rendered frame's time); frame f of
    # a batch adds delta[f] to its centres
    delta: Optional[np.ndarray] = None

    FIELDS = ("mean", "vel", "acc", "scale", "quat", "omega",
              "opacity_logit", "rgb", "albedo")
    SH_FIELDS = ("sh_rgb", "sh_albedo")
    OPTIONAL = SH_FIELDS + ("delta",)

    @property
    def n(self) -> int:
        return int(self.opacity_logit.shape[0])

    def arrays(self):
        out = {k: getattr(self, k) for k in self.FIELDS}
        out.update({k: getattr(self, k) for k in self.OPTIONAL if getattr(self, k) is not None})
        return out

    def copy(self) -> "Gaussians":
        return Gaussians(**{k: np.array(v, dtype=np.float32, copy=True)
                            for k, v in self.arrays().items()})

    def subset(self, idx) -> "Gaussians":
        return Gaussians(**{k: np.ascontiguousarray(v[..., idx])
                            for k, v in self.arrays().items()})


@dataclass
class Frame:
    """One rendered time frame: a pinhole camera with a co-located emitter.

    R, t map world to camera coordinates (p = R x + t), OpenCV convention:
    x right, y down, z forward.  Pixel (i, j) is sampled at (i + 0.5, j + 0.5).
    """

    R: np.ndarray = field(default_factory=lambda: np.eye(3, dtype=np.float32))
    t: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=np.float32))
    fx: float = 60.0
    fy: float = 60.0
    cx: float = 32.0
    cy: float = 24.0
    time: float = 0.0
    bg_rgb: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=np.float32))
    bg_quad: Optional[np.ndarray] = None  # [n_freq, n_phase] float32, None = 0
    # asynchronous raw quads: with t_hi > t_lo the Gaussian centres lie on the
    # line between their positions at t_lo and t_hi (paper Eq. 7)
    t_lo: float = 0.0
    t_hi: float = 0.0
    quad_mask: int = 0                    # rendered quad channels (bits), 0 = all


@dataclass
class RenderConfig:
    """Per-call constants.  Defaults follow common Gaussian-splatting practice;
    the paper leaves the rasterizer constants unstated."""

    width: int = 64
    height: int = 48
    freqs: Tuple[float, ...] = (30e6,)
    phases: Tuple[float, ...] = QUAD_PHASES
    tile_w: int = 16
    tile_h: int = 16
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    extent_sigma: float = 3.0   # <= 0 means unbounded support (every tile)
    dilation: float = 0.3       # px^2 added to the 2D covariance diagonal
    near_z: float = 0.2
    source_intensity: float = 1.0
    bg_T_power: int = 1         # background weight T_final^p

    @property
    def n_freq(self) -> int:
        return len(self.freqs)

    @property
    def n_phase(self) -> int:
        return len(self.phases)

    @property
    def n_quad(self) -> int:
        return self.n_freq * self.n_phase

    @property
    def tiles_x(self) -> int:
        return -(-self.width // self.tile_w)

    @property
    def tiles_y(self) -> int:
        return -(-self.height // self.tile_h)

    def strict(self) -> "RenderConfig":
        """No skip / stop thresholds and unbounded support: closed-form mode."""
        return dataclasses.replace(self, alpha_min=0.0, T_min=0.0, extent_sigma=0.0)


# ----------------------------------------------------------------------------
# Draws
# ----------------------------------------------------------------------------

def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def draw_gaussians(n: int, width: int, height: int, fx: float, fy: float,
                   seed: int, dynamic: bool = False, cx: float = None,
                   cy: float = None, z_range=(0.5, 4.5),
                   log_scale_mean=float(np.log(0.03)), log_scale_std=0.3,
                   vel_std=0.5, acc_std=1.0, omega_std=1.0) -> Gaussians:
    """Gaussians uniform in the frustum of an identity camera.

    u ~ U(0, W), v ~ U(0, H), z ~ U(z_range), back-projected through the
    pinhole; per-axis log-scales ~ N(log 0.03, 0.3); quaternion = normalised
    N(0, I4); opacity logit ~ N(0, 1); rgb, albedo ~ U(0, 1); for dynamic
    scenes v ~ N(0, 0.5 m/s), a ~ N(0, 1 m/s^2), omega ~ N(0, 1 rad/s).
    """
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(0.0, width, n)
    v = rng.uniform(0.0, height, n)
    z = rng.uniform(z_range[0], z_range[1], n)
    x = (u - cx) * z / fx
    y = (v - cy) * z / fy
    log_scale = rng.normal(log_scale_mean, log_scale_std, (3, n))
    q = rng.normal(0.0, 1.0, (4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    logit = rng.normal(0.0, 1.0, n)
    rgb = rng.uniform(0.0, 1.0, (3, n))
    albedo = rng.uniform(0.0, 1.0, n)
    if dynamic:
        vel = rng.normal(0.0, vel_std, (3, n))
        acc = rng.normal(0.0, acc_std, (3, n))
        omega = rng.normal(0.0, omega_std, (3, n))
    else:
        vel = np.zeros((3, n))
        acc = np.zeros((3, n))
        omega = np.zeros((3, n))
    return Gaussians(mean=_f32(np.stack([x, y, z])), vel=_f32(vel), acc=_f32(acc),
                     scale=_f32(np.exp(log_scale)), quat=_f32(q), omega=_f32(omega),
                     opacity_logit=_f32(logit), rgb=_f32(rgb), albedo=_f32(albedo))


def identity_frames(times: Sequence[float], width: int, height: int, fx: float,
                    fy: float, n_quad: int, bg_seed: Optional[int] = None,
                    n_freq: int = 1) -> List[Frame]:
    """Static identity camera at the origin, one frame per time.

    With ``bg_seed`` the backgrounds are drawn U(-1, 1) per frame (the paper's
    random background, §4); otherwise they are zero.
    """
    frames = []
    rng = None if bg_seed is None else np.random.Generator(np.random.PCG64(bg_seed))
    for tm in times:
        if rng is None:
            bg_rgb = np.zeros(3, np.float32)
            bg_quad = np.zeros((n_freq, n_quad // n_freq), np.float32)
        else:
            bg_rgb = _f32(rng.uniform(-1.0, 1.0, 3))
            bg_quad = _f32(rng.uniform(-1.0, 1.0, (n_freq, n_quad // n_freq)))
        frames.append(Frame(fx=float(np.float32(fx)), fy=float(np.float32(fy)),
                            cx=float(np.float32(width / 2.0)), cy=float(np.float32(height / 2.0)),
                            time=float(np.float32(tm)), bg_rgb=bg_rgb, bg_quad=bg_quad))
    return frames


def upstream_grads(n_frames: int, cfg: RenderConfig, seed: int):
    """N(0, 1) upstream gradient on every rendered element (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = cfg.height, cfg.width
    return {
        "rgb": _f32(rng.normal(0.0, 1.0, (n_frames, 3, H, W))),
        "quad": _f32(rng.normal(0.0, 1.0, (n_frames, cfg.n_quad, H, W))),
        "depth": _f32(rng.normal(0.0, 1.0, (n_frames, H, W))),
    }


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    gaussians: Gaussians
    frames: List[Frame]
    cfg: RenderConfig
    description: str = ""


def cfg1(seed: int = 0) -> Workload:
    """Static, 2,000 Gaussians, one 64x48 frame, fx = fy = 60, 30 MHz, 4 quads."""
    W, H, f = 64, 48, 60.0
    g = draw_gaussians(2000, W, H, f, f, seed)
    cfg = RenderConfig(width=W, height=H, freqs=(30e6,))
    return Workload("static-2k-64x48", g, identity_frames([0.0], W, H, f, f, 4), cfg,
                    "static scene, 2,000 Gaussians, 64x48, 1 frame")


def cfg2(seed: int = 0, n: int = 100_000) -> Workload:
    """Static, 100k Gaussians, one 640x480 frame, fx = fy = 525, 30 MHz."""
    W, H, f = 640, 480, 525.0
    g = draw_gaussians(n, W, H, f, f, seed)
    cfg = RenderConfig(width=W, height=H, freqs=(30e6,))
    return Workload(f"static-{n // 1000}k-640x480", g,
                    identity_frames([0.0], W, H, f, f, 4), cfg,
                    f"static scene, {n} Gaussians, 640x480, 1 frame")


def cfg2_320(seed: int = 0, n: int = 100_000) -> Workload:
    """cfg2's distributions at the paper's dataset resolution, 320x240
    (fx = fy = 262.5, the same field of view)."""
    W, H, f = 320, 240, 262.5
    g = draw_gaussians(n, W, H, f, f, seed)
    cfg = RenderConfig(width=W, height=H, freqs=(30e6,))
    return Workload(f"static-{n // 1000}k-320x240", g,
                    identity_frames([0.0], W, H, f, f, 4), cfg,
                    f"static scene, {n} Gaussians, 320x240, 1 frame")


def cfg3(seed: int = 0, n: int = 200_000, n_frames: int = 8) -> Workload:
    """Dynamic, 200k Gaussians, 8 frames at t in [0, 0.25 s], 640x480."""
    W, H, f = 640, 480, 525.0
    g = draw_gaussians(n, W, H, f, f, seed, dynamic=True)
    times = [0.25 * i / max(n_frames - 1, 1) for i in range(n_frames)]
    cfg = RenderConfig(width=W, height=H, freqs=(30e6,))
    return Workload(f"dynamic-{n // 1000}k-640x480-{n_frames}f", g,
                    identity_frames(times, W, H, f, f, 4), cfg,
                    f"dynamic scene, {n} Gaussians, {n_frames} frames, 640x480")


def cfg4(seed: int = 0, n: int = 1_000_000, n_frames: int = 16,
         tile: Tuple[int, int] = (16, 16)) -> Workload:
    """Dynamic, 1M Gaussians, 1024x768, 30 + 60 MHz, 16 frames; a seeded half
    of the Gaussians gets a lateral velocity that carries it out of the
    frustum at an exit time ~ U(0, 0.5 s)."""
    W, H, f = 1024, 768, 840.0
    g = draw_gaussians(n, W, H, f, f, seed, dynamic=True)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    leave = rng.permutation(n)[: n // 2]
    t_exit = rng.uniform(0.0, 0.5, leave.size)
    side = rng.choice([-1.0, 1.0], leave.size)
    z = g.mean[2, leave].astype(np.float64)
    half_width = (W / 2.0) * z / f
    dist = half_width * side - g.mean[0, leave].astype(np.float64)
    # travel the lateral distance to the frustum edge plus 1 m past it
    vx = (dist + side * 1.0) / np.maximum(t_exit, 1e-3)
    g.vel[0, leave] = _f32(vx)
    times = [i / 30.0 for i in range(n_frames)]
    cfg = RenderConfig(width=W, height=H, freqs=(30e6, 60e6), tile_w=tile[0], tile_h=tile[1])
    return Workload(f"dynamic-{n // 1000}k-1024x768-{n_frames}f-2freq", g,
                    identity_frames(times, W, H, f, f, 8, n_freq=2), cfg,
                    f"dynamic scene, {n} Gaussians, {n_frames} frames, 1024x768, 2 freqs")


def cfg5_scenes(n: int = 300_000, gt_seed: int = 1, train_seed: int = 0):
    """Ground-truth and trainable scenes for the optimisation-step loop.
    The trainable scene starts with albedo 0.1 (the paper's initial
    reflectivity, §4)."""
    W, H, f = 640, 480, 525.0
    gt = draw_gaussians(n, W, H, f, f, gt_seed, dynamic=True)
    tr = draw_gaussians(n, W, H, f, f, train_seed, dynamic=True)
    tr.albedo[:] = np.float32(0.1)
    cfg = RenderConfig(width=W, height=H, freqs=(30e6,))
    return gt, tr, cfg


def tiny_scene(n: int, width: int, height: int, seed: int, f: float = None,
               dynamic: bool = False, z_range=(1.0, 3.0), log_scale_mean=None) -> Workload:
    """Small seeded scene for brute-force and finite-difference checks."""
    f = f if f is not None else 1.2 * width
    lsm = float(np.log(0.15)) if log_scale_mean is None else log_scale_mean
    g = draw_gaussians(n, width, height, f, f, seed, dynamic=dynamic,
                       z_range=z_range, log_scale_mean=lsm)
    cfg = RenderConfig(width=width, height=height, freqs=(30e6,), tile_w=8, tile_h=8)
    return Workload(f"tiny-{n}-{width}x{height}", g,
                    identity_frames([0.0], width, height, f, f, 4), cfg)


def with_sh(g: Gaussians, degree: int = 3, seed: int = 0, scale: float = 0.3,
            rgb: bool = True, albedo: bool = True) -> Gaussians:
    """A copy of `g` with spherical-harmonic colour and reflectivity: the DC
    coefficient reproduces the flat colour / albedo (c = 1/2 + Y_00 k_0), the
    higher ones are N(0, scale^2 / (l + 1)) (seeded PCG64, drawn after
    everything else)."""
    K = (degree + 1) ** 2
    rng = np.random.Generator(np.random.PCG64(seed))
    y00 = 0.5 / np.sqrt(np.pi)
    lvl = np.concatenate([[l] * (2 * l + 1) for l in range(degree + 1)])
    out = dataclasses.replace(g)
    if rgb:
        k = rng.normal(0.0, 1.0, (K, 3, g.n)) * (scale / (lvl + 1.0))[:, None, None]
        k[0] = (g.rgb.astype(np.float64) - 0.5) / y00
        out.sh_rgb = _f32(k)
    if albedo:
        k = rng.normal(0.0, 1.0, (K, g.n)) * (scale / (lvl + 1.0))[:, None]
        k[0] = (g.albedo.astype(np.float64) - 0.5) / y00
        out.sh_albedo = _f32(k)
    return out


def async_quartet_frames(n_quartets: int, period: float, base: Frame, n_phase: int = 4,
                         n_freq: int = 1) -> List[Frame]:
    """Raw quads captured one at a time (paper §2, §4): raw frame k of quartet
    i = k // n_phase, offset j = k % n_phase, is taken at time
    (i + j / n_phase) * period and renders only its offset's channels (at
    every frequency); its Gaussian centres are interpolated between the
    integer timesteps i * period and (i + 1) * period (Eq. 7)."""
    frames = []
    for k in range(n_quartets * n_phase):
        i, j = divmod(k, n_phase)
        mask = sum(1 << (f * n_phase + j) for f in range(n_freq))
        frames.append(dataclasses.replace(
            base, time=float(np.float32((i + j / n_phase) * period)),
            t_lo=float(np.float32(i * period)), t_hi=float(np.float32((i + 1) * period)), quad_mask=mask))
    return frames


def frames_for_times(times, wl: Workload) -> List[Frame]:
    fr0 = wl.frames[0]
    return [dataclasses.replace(fr0, time=float(np.float32(t))) for t in times]


def mlp_params(seed: int = 0, n_in: int = 84, width: int = 256, depth: int = 8, n_out: int = 3,
               last_std: float = 1e-5, bias_std: float = 0.0, gain: float = 1.0) -> np.ndarray:
    """Flat float32 parameters of the deformation network (paper §4, "MLP"):
    for every linear layer in order, W [out][in] row-major then b [out].
    Weights are Xavier-normal, std = gain sqrt(2 / (fan_in + fan_out)), except
    the last layer's, N(0, last_std^2); biases are 0 (paper) or, for tests
    that need every term exercised, N(0, bias_std^2).  Seeded PCG64, layer by
    layer, weights before biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(width, n_in)] + [(width, width)] * (depth - 1) + [(n_out, width)]
    parts = []
    for l, (o, i) in enumerate(shapes):
        std = last_std if l == len(shapes) - 1 else gain * np.sqrt(2.0 / (i + o))
        parts.append(rng.normal(0.0, std, o * i))
        parts.append(rng.normal(0.0, bias_std, o) if bias_std > 0 else np.zeros(o))
    return _f32(np.concatenate(parts))


def mlp_rows(n: int, n_times: int, seed: int = 0, extent: float = 4.5, duration: float = 0.25):
    """Canonical centres [3][n] (float32, uniform in a box of the given extent
    in front of the camera, z in [0.5, extent]) and n_times time stamps spread
    over [0, duration] for the deformation network."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.stack([rng.uniform(-0.5 * extent, 0.5 * extent, n),
                   rng.uniform(-0.5 * extent, 0.5 * extent, n),
                   rng.uniform(0.5, extent, n)])
    times = np.linspace(0.0, duration, n_times) if n_times > 1 else np.zeros(1)
    return _f32(x0), _f32(times)
