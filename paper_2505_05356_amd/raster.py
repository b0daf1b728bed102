"""Python binding of the C-ToF Gaussian rasterizer (argument marshalling only).

PyTorch provides device memory and streams; every step of the forward and
backward pass runs in the HIP kernels of libgftorf.so.

    params  dict of float32 CUDA tensors: mean [3,N], vel [3,N] | None,
            acc [3,N] | None, scale [3,N], quat [4,N], omega [3,N] | None,
            opacity_logit [N], rgb [3,N], albedo [N]; optional sh_rgb [K,3,N],
            sh_albedo [K,N] (spherical harmonics) and delta [F,3,N] (per-frame
            centre offsets, e.g. deform.offsets)
    frames  list of frame descriptors (objects with R, t, fx, fy, cx, cy,
            time, bg_rgb, bg_quad, and optionally t_lo, t_hi, quad_mask) or a
            packed float32 CUDA tensor [F, 40]
    cfg     object with width, height, freqs, phases, tile_w, tile_h,
            alpha_min, alpha_max, T_min, extent_sigma, dilation, near_z,
            source_intensity, bg_T_power
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Dict, Optional

import numpy as np
import torch

from . import _lib
from ._lib import FIELDS, FRAME_FLOATS, MAX_QUAD, OFFSET_FIELDS, SH_FIELDS

ALL_FIELDS = FIELDS + SH_FIELDS + OFFSET_FIELDS
_SH_DEGREE = {1: 0, 4: 1, 9: 2, 16: 3}


@dataclasses.dataclass
class RasterConfig:
    """Per-call constants (same names as the C struct gftorf_config)."""
    width: int = 640
    height: int = 480
    freqs: tuple = (30e6,)
    phases: tuple = (0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi)
    tile_w: int = 16
    tile_h: int = 16
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    extent_sigma: float = 3.0
    dilation: float = 0.3
    near_z: float = 0.2
    source_intensity: float = 1.0
    bg_T_power: int = 1


def config_struct(cfg, max_pairs: int) -> _lib.ConfigC:
    c = _lib.ConfigC()
    c.width, c.height = int(cfg.width), int(cfg.height)
    c.n_freq, c.n_phase = len(cfg.freqs), len(cfg.phases)
    # counts beyond the struct's capacity are passed through for the library
    # to reject (GFTORF_EINVAL)
    for i, f in enumerate(list(cfg.freqs)[:_lib.MAX_FREQ]):
        c.freq_hz[i] = float(np.float32(f))
    for j, p in enumerate(list(cfg.phases)[:_lib.MAX_PHASE]):
        c.phase[j] = float(p)
    c.tile_w, c.tile_h = int(cfg.tile_w), int(cfg.tile_h)
    c.alpha_min, c.alpha_max, c.T_min = cfg.alpha_min, cfg.alpha_max, cfg.T_min
    c.extent_sigma, c.dilation, c.near_z = cfg.extent_sigma, cfg.dilation, cfg.near_z
    c.source_intensity, c.bg_T_power = cfg.source_intensity, int(cfg.bg_T_power)
    c.max_pairs = int(max_pairs)
    return c


def n_quad(cfg) -> int:
    return len(cfg.freqs) * len(cfg.phases)


def pack_frames(frames, cfg, device="cuda") -> torch.Tensor:
    """Frame descriptors -> float32 device tensor [F, 40] (struct gftorf_frame)."""
    if isinstance(frames, torch.Tensor):
        return frames
    F = len(frames)
    a = np.zeros((F, FRAME_FLOATS), np.float32)
    nq = n_quad(cfg)
    for i, fr in enumerate(frames):
        a[i, 0:9] = np.asarray(fr.R, np.float32).reshape(9)
        a[i, 9:12] = np.asarray(fr.t, np.float32).reshape(3)
        a[i, 12:16] = [fr.fx, fr.fy, fr.cx, fr.cy]
        a[i, 16] = fr.time
        a[i, 17:20] = np.asarray(fr.bg_rgb, np.float32).reshape(3)
        if fr.bg_quad is not None:
            a[i, 20:20 + nq] = np.asarray(fr.bg_quad, np.float32).reshape(-1)[:nq]
        a[i, 36] = getattr(fr, "t_lo", 0.0)
        a[i, 37] = getattr(fr, "t_hi", 0.0)
        a[i, 38:39].view(np.uint32)[0] = np.uint32(getattr(fr, "quad_mask", 0))
    return torch.from_numpy(a).to(device)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_offsets(params, n_frames):
    d = params.get("delta")
    if d is not None and d.shape[0] != n_frames:
        raise ValueError(f"delta has {d.shape[0]} frames, the call renders {n_frames}")


def gaussians_struct(params: Dict[str, torch.Tensor]) -> _lib.GaussiansC:
    g = _lib.GaussiansC()
    n = params["opacity_logit"].shape[0]
    g.n = n
    # spherical-harmonic colour [K, 3, n] / reflectivity [K, n] replace rgb / albedo
    degree = None
    for k in SH_FIELDS:
        t = params.get(k)
        if t is None:
            setattr(g, k, None)
            continue
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"parameter {k} must be a contiguous float32 CUDA tensor")
        K = t.shape[0]
        if K not in _SH_DEGREE or t.numel() != K * (3 if k == "sh_rgb" else 1) * n:
            raise ValueError(f"parameter {k} must be [K{', 3' if k == 'sh_rgb' else ''}, n] with K in 1, 4, 9, 16")
        if degree is not None and _SH_DEGREE[K] != degree:
            raise ValueError("sh_rgb and sh_albedo must have the same degree")
        degree = _SH_DEGREE[K]
        setattr(g, k, t.data_ptr())
    g.sh_degree = degree or 0
    d = params.get("delta")   # per-frame centre offsets [F, 3, n]
    if d is not None:
        if not (d.is_cuda and d.dtype == torch.float32 and d.is_contiguous()) or \
                d.dim() != 3 or d.shape[1:] != (3, n):
            raise ValueError("delta must be a contiguous float32 CUDA tensor [F, 3, n]")
        g.delta = d.data_ptr()
    for k in FIELDS:
        t = params.get(k)
        replaced = (k == "rgb" and params.get("sh_rgb") is not None) or \
                   (k == "albedo" and params.get("sh_albedo") is not None)
        if t is None:
            if k not in _lib.OPTIONAL and not replaced:
                raise ValueError(f"parameter {k} is required")
            setattr(g, k, None)
            continue
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"parameter {k} must be a contiguous float32 CUDA tensor")
        if t.numel() != _lib.ROWS[k] * n:
            raise ValueError(f"parameter {k} has {t.numel()} elements, expected {_lib.ROWS[k] * n}")
        setattr(g, k, t.data_ptr())
    return g


class Workspace:
    """Device workspace of a (N, F, cfg) problem; keeps the forward's sorted
    lists and records for the backward.  Grows when the pair capacity
    overflows.  `generation` counts the forwards enqueued on it and its
    reallocations, so a pending backward can tell that its forward's state
    was overwritten."""

    def __init__(self, n: int, n_frames: int, cfg, max_pairs: Optional[int] = None,
                 device="cuda"):
        self.n, self.n_frames, self.cfg, self.device = n, n_frames, cfg, device
        self.generation = 0
        if max_pairs is None:
            max_pairs = max(1 << 16, 48 * n * n_frames)
        self._alloc(max_pairs)

    def _alloc(self, max_pairs):
        lib = _lib.load()
        self.generation = getattr(self, "generation", 0) + 1
        self.max_pairs = int(min(max_pairs, 0xF0000000))
        self.cstruct = config_struct(self.cfg, self.max_pairs)
        size = lib.gftorf_workspace_size(self.n, self.n_frames, ctypes.byref(self.cstruct))
        if size == 0:
            raise _lib.GftorfError(_lib.EINVAL, lib.gftorf_last_error().decode())
        self.buf = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
        off = (-self.buf.data_ptr()) % 256
        self.ptr = self.buf.data_ptr() + off
        self.nbytes = size
        self.buf[off:off + 64].zero_()   # status header: no forward has run yet

    def grow(self, pairs: int):
        self._alloc(int(pairs * 1.25) + 4096)

    def status(self, stream=None) -> dict:
        lib = _lib.load()
        st = _lib.StatusC()
        rc = lib.gftorf_read_status(ctypes.c_void_p(self.ptr), ctypes.byref(st), _stream(stream))
        if rc not in (_lib.OK, _lib.EOVERFLOW):
            _lib.check(rc)
        return dict(n_pairs=st.n_pairs, max_pairs=st.max_pairs, overflow=bool(st.overflow),
                    nonfinite=st.nonfinite, n_evaluated=st.n_evaluated,
                    n_composited=st.n_composited, overflow_seen=bool(st.overflow_seen),
                    n_pairs_seen=st.n_pairs_seen, sort_fault=bool(st.sort_fault))

    def clear_status(self, stream=None):
        """Clears the status header, including the sticky overflow_seen and
        n_pairs_seen, with a kernel on the stream (capturable)."""
        _lib.check(_lib.load().gftorf_clear_status(ctypes.c_void_p(self.ptr), _stream(stream)))


def alloc_outputs(n_frames, cfg, device="cuda", channels=("rgb", "quad", "depth")):
    H, W = cfg.height, cfg.width
    out = dict(T_final=torch.empty((n_frames, H, W), device=device),
               n_contrib=torch.empty((n_frames, H, W), dtype=torch.int32, device=device))
    if "rgb" in channels:
        out["rgb"] = torch.empty((n_frames, 3, H, W), device=device)
    if "quad" in channels:
        out["quad"] = torch.empty((n_frames, n_quad(cfg), H, W), device=device)
    if "depth" in channels:
        out["depth"] = torch.empty((n_frames, H, W), device=device)
    nf = len(cfg.freqs)
    if "phasor" in channels:
        out["phasor"] = torch.empty((n_frames, nf, 2, H, W), device=device)
    if "d_tof" in channels:
        out["d_tof"] = torch.empty((n_frames, nf, H, W), device=device)
    if "amplitude" in channels:
        out["amplitude"] = torch.empty((n_frames, nf, H, W), device=device)
    return out


def outputs_struct(out) -> _lib.OutputsC:
    o = _lib.OutputsC()
    for k in ("rgb", "quad", "depth", "T_final", "n_contrib", "phasor", "d_tof", "amplitude"):
        setattr(o, k, out[k].data_ptr() if out.get(k) is not None else None)
    return o


def forward(params, frames_dev, cfg, ws: Workspace, out=None, stream=None, check=True):
    """Enqueues the forward on `stream` (torch's current stream by default).
    With check=True, reads the pair count back (one sync) and, on overflow,
    grows the workspace and renders again."""
    lib = _lib.load()
    F = frames_dev.shape[0]
    if out is None:
        out = alloc_outputs(F, cfg, frames_dev.device)
    g = gaussians_struct(params)
    _check_offsets(params, frames_dev.shape[0])
    o = outputs_struct(out)
    while True:
        ws.generation += 1
        _lib.check(lib.gftorf_render_fwd(ctypes.byref(g), _ptr(frames_dev), F,
                                         ctypes.byref(ws.cstruct), ctypes.byref(o),
                                         ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream)))
        if not check:
            return out
        st = ws.status(stream)
        if not st["overflow"]:
            return out
        ws.grow(st["n_pairs"])


def backward(params, frames_dev, cfg, ws: Workspace, saved, d_rgb=None, d_quad=None,
             d_depth=None, want_bg=False, stream=None, grads=None):
    """Enqueues the backward; returns dict of parameter gradients (and
    'bg' [F, 3 + NQ] if want_bg)."""
    lib = _lib.load()
    F = frames_dev.shape[0]
    if grads is None:
        grads = {k: (torch.empty_like(params[k]) if params.get(k) is not None else None)
                 for k in ALL_FIELDS}
    gg = _lib.GaussiansGradC()
    for k in ALL_FIELDS:
        setattr(gg, k, grads[k].data_ptr() if grads.get(k) is not None else None)
    d_bg = torch.empty((F, 3 + n_quad(cfg)), device=frames_dev.device) if want_bg else None
    g = gaussians_struct(params)
    _check_offsets(params, frames_dev.shape[0])
    o = outputs_struct(saved)
    for t in (d_rgb, d_quad, d_depth):
        if t is not None and not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("upstream gradients must be contiguous float32 CUDA tensors")
    _lib.check(lib.gftorf_render_bwd(ctypes.byref(g), _ptr(frames_dev), F, ctypes.byref(ws.cstruct),
                                     ctypes.byref(o), _ptr(d_rgb), _ptr(d_quad), _ptr(d_depth),
                                     ctypes.byref(gg), _ptr(d_bg), ctypes.c_void_p(ws.ptr),
                                     ws.nbytes, _stream(stream)))
    if want_bg:
        grads["bg"] = d_bg
    return grads


class RasterizeCToF(torch.autograd.Function):
    """Differentiable render of RGB, raw quads and depth for a batch of frames.

    forward(ctx, ws, frames_dev, cfg, *params) -> (rgb, quad, depth)

    The backward reads the tile lists and records that this forward left in
    `ws`; it raises if another forward has used `ws` since (or `ws` was
    regrown), and autograd's version check raises if a parameter or the
    frame descriptors were modified in place in between.
    """

    @staticmethod
    def forward(ctx, ws, frames_dev, cfg, *plist):
        params = {k: (p.contiguous() if p is not None else None) for k, p in zip(ALL_FIELDS, plist)}
        out = forward(params, frames_dev, cfg, ws)
        ctx.ws, ctx.cfg, ctx.generation = ws, cfg, ws.generation
        ctx.present = [p is not None for p in plist]
        ctx.save_for_backward(frames_dev, out["T_final"], out["n_contrib"],
                              *[p for p in params.values() if p is not None])
        ctx.mark_non_differentiable(out["T_final"], out["n_contrib"])
        return out["rgb"], out["quad"], out["depth"], out["T_final"], out["n_contrib"]

    @staticmethod
    def backward(ctx, g_rgb, g_quad, g_depth, _gT, _gn):
        if ctx.ws.generation != ctx.generation:
            raise RuntimeError("RasterizeCToF: the workspace was used by another forward (or regrown) "
                               "after this one, so its tile lists and records are not this forward's; "
                               "give every pending backward its own Workspace")
        frames, T_final, n_contrib, *plist = ctx.saved_tensors
        it = iter(plist)
        params = {k: (next(it) if present else None) for k, present in zip(ALL_FIELDS, ctx.present)}
        c = lambda t: None if t is None else t.contiguous()
        grads = backward(params, frames, ctx.cfg, ctx.ws, dict(T_final=T_final, n_contrib=n_contrib),
                         c(g_rgb), c(g_quad), c(g_depth))
        res = [grads[k] if present else None for k, present in zip(ALL_FIELDS, ctx.present)]
        return (None, None, None, *res)


def render(params, frames, cfg, ws: Optional[Workspace] = None):
    """Differentiable batched render.  Returns dict(rgb, quad, depth, T_final,
    n_contrib, workspace)."""
    frames_dev = pack_frames(frames, cfg)
    n = params["opacity_logit"].shape[0]
    if ws is None:
        ws = Workspace(n, frames_dev.shape[0], cfg)
    plist = [params.get(k) for k in ALL_FIELDS]
    rgb, quad, depth, Tf, nc = RasterizeCToF.apply(ws, frames_dev, cfg, *plist)
    return dict(rgb=rgb, quad=quad, depth=depth, T_final=Tf, n_contrib=nc, workspace=ws)


def to_device_params(g, device="cuda", static=None) -> Dict[str, torch.Tensor]:
    """Plain arrays (objects with the FIELDS attributes) -> float32 device tensors.
    With static=True (or auto when vel, acc, omega are all zero) the optional
    fields are passed as NULL."""
    arrs = {k: np.asarray(getattr(g, k), np.float32) for k in FIELDS}
    if static is None:
        static = all(not np.any(arrs[k]) for k in _lib.OPTIONAL)
    out = {}
    for k, a in arrs.items():
        if static and k in _lib.OPTIONAL:
            out[k] = None
        else:
            out[k] = torch.from_numpy(np.ascontiguousarray(a)).to(device)
    for k in SH_FIELDS + OFFSET_FIELDS:   # only when the Gaussians carry them
        a = getattr(g, k, None)
        if a is not None:
            out[k] = torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    return out
