"""Deformation network of paper §4 ("MLP"): argument marshalling for the
gftorf_mlp_* entry points of libgftorf.so.

The network maps the positional encoding of (s_x x0, s_t t) through 8 ReLU
layers of 256 units to a centre offset delta x for every (time, Gaussian)
row; every product runs in the library's gfx950 kernels (bfloat16 operands on
the matrix cores, float32 accumulation).  The offsets plug into the
rasterizer as the per-frame `delta` field of the Gaussians.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib

SPEED_OF_LIGHT = 299_792_458.0


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _f32dev(t: torch.Tensor, name: str, shape=None):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class DeformNet:
    """Workspace and configuration for n Gaussians at up to n_times times.

    pos_scale defaults to the inverse unambiguous range 2 f / c of the
    modulation frequency `freq_hz` (paper §4: network inputs rescaled to
    mostly [0, 1]); time_scale maps the sequence's times to [0, 1]."""

    def __init__(self, n: int, n_times: int, freq_hz: float = 30e6, time_scale: float = 1.0,
                 pos_scale: Optional[float] = None, lx: int = 10, lt: int = 10,
                 training: bool = True, device="cuda"):
        lib = _lib.load()
        sx = pos_scale if pos_scale is not None else 2.0 * freq_hz / SPEED_OF_LIGHT
        self.cfg = _lib.MlpConfigC(lx, lt, 256, 8, sx, time_scale)
        self.n, self.n_times, self.training = n, n_times, training
        self.n_params = int(lib.gftorf_mlp_param_count(ctypes.byref(self.cfg)))
        nbytes = int(lib.gftorf_mlp_workspace_size(ctypes.byref(self.cfg), n, n_times, int(training)))
        if self.n_params <= 0 or nbytes <= 0:
            raise ValueError("unsupported network configuration")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes
        self.generation = 0   # training forwards enqueued on ws (their saved state replaces the last)

    def _times(self, times: Sequence[float]):
        if not 1 <= len(times) <= self.n_times:
            raise ValueError(f"between 1 and {self.n_times} times")
        return (ctypes.c_float * len(times))(*[float(t) for t in times])

    def forward(self, params: torch.Tensor, x0: torch.Tensor, times: Sequence[float],
                save: bool = True, out: Optional[torch.Tensor] = None, stream=None):
        """delta [T, 3, n] for canonical centres x0 [3, n] at the T times."""
        lib = _lib.load()
        T = len(times)
        _f32dev(params, "params", (self.n_params,))
        _f32dev(x0, "x0", (3, self.n))
        if save and not self.training:
            raise ValueError("save needs a training workspace")
        if out is None:
            out = torch.empty((T, 3, self.n), device=x0.device)
        _f32dev(out, "out", (T, 3, self.n))
        if save:
            self.generation += 1
        _lib.check(lib.gftorf_mlp_fwd(ctypes.byref(self.cfg), _ptr(params), _ptr(x0), self.n,
                                      self._times(times), T, _ptr(out), int(save),
                                      _ptr(self.ws), self.nbytes, _stream(stream)))
        return out

    def backward(self, params: torch.Tensor, x0: torch.Tensor, times: Sequence[float],
                 d_delta: torch.Tensor, d_params: Optional[torch.Tensor] = None,
                 want_x0: bool = True, stream=None):
        """(d_params [P], d_x0 [3, n] or None) for the upstream d_delta [T, 3, n];
        needs the forward with save=True on the same arguments just before."""
        lib = _lib.load()
        T = len(times)
        _f32dev(d_delta, "d_delta", (T, 3, self.n))
        if d_params is None:
            d_params = torch.empty(self.n_params, device=x0.device)
        d_x0 = torch.empty((3, self.n), device=x0.device) if want_x0 else None
        _lib.check(lib.gftorf_mlp_bwd(ctypes.byref(self.cfg), _ptr(params), _ptr(x0), self.n,
                                      self._times(times), T, _ptr(d_delta), _ptr(d_params),
                                      _ptr(d_x0), _ptr(self.ws), self.nbytes, _stream(stream)))
        return d_params, d_x0


    def decisions(self, n_times: int, stream=None) -> torch.Tensor:
        """The ReLU decisions the last training forward over n_times times
        recorded: uint8 [n_times * n, 8, 256], row t * n + k, 1 = active."""
        lib = _lib.load()
        if not self.training:
            raise ValueError("decisions are kept by a training workspace only")
        dec = torch.empty((n_times * self.n, 8, 256), dtype=torch.uint8, device=self.ws.device)
        _lib.check(lib.gftorf_mlp_get_decisions(ctypes.byref(self.cfg), self.n, n_times, _ptr(dec),
                                                _ptr(self.ws), self.nbytes, _stream(stream)))
        return dec

    def set_decisions(self, dec: torch.Tensor, stream=None) -> None:
        """Replaces the recorded decisions (same layout as decisions()); the
        next backward gates its gradients with them."""
        lib = _lib.load()
        if not self.training:
            raise ValueError("decisions are kept by a training workspace only")
        if not (dec.is_cuda and dec.dtype == torch.uint8 and dec.is_contiguous() and dec.dim() == 3
                and tuple(dec.shape[1:]) == (8, 256) and dec.shape[0] % self.n == 0):
            raise ValueError("decisions must be a contiguous uint8 CUDA tensor [T * n, 8, 256]")
        n_times = dec.shape[0] // self.n
        _lib.check(lib.gftorf_mlp_set_decisions(ctypes.byref(self.cfg), self.n, n_times, _ptr(dec),
                                                _ptr(self.ws), self.nbytes, _stream(stream)))


class DeformOffsets(torch.autograd.Function):
    """delta [T, 3, n] = network(params, x0, times) as an autograd node: its
    backward is gftorf_mlp_bwd on the same workspace, so it composes with
    raster.RasterizeCToF (pass the result as the Gaussians' `delta`).  The
    backward raises if another training forward used the network's workspace
    in between (its saved activations would not be this forward's)."""

    @staticmethod
    def forward(ctx, net: DeformNet, times, params, x0):
        params, x0 = params.contiguous(), x0.contiguous()
        ctx.net, ctx.times = net, list(times)
        ctx.save_for_backward(params, x0)
        out = net.forward(params, x0, ctx.times, save=True)
        ctx.generation = net.generation
        return out

    @staticmethod
    def backward(ctx, d_delta):
        if ctx.net.generation != ctx.generation:
            raise RuntimeError("DeformOffsets: the network's workspace was used by another training "
                               "forward after this one; give every pending backward its own DeformNet")
        params, x0 = ctx.saved_tensors
        d_params, d_x0 = ctx.net.backward(params, x0, ctx.times, d_delta.contiguous(),
                                          want_x0=ctx.needs_input_grad[3])
        return None, None, d_params, d_x0


def offsets(net: DeformNet, params: torch.Tensor, x0: torch.Tensor, times: Sequence[float]):
    """Differentiable per-frame centre offsets for the rasterizer."""
    return DeformOffsets.apply(net, times, params, x0)


def _anchors(anchors, n_frames):
    flat = [int(v) for pair in anchors for v in pair]
    if len(flat) != 2 * n_frames:
        raise ValueError("one (lo, hi) anchor pair per frame")
    return (ctypes.c_int32 * len(flat))(*flat)


def blend(delta_steps: torch.Tensor, frames_dev: torch.Tensor, anchors, stream=None):
    """Eq. 7 with the network: per-frame offsets [F, 3, n] from the offsets at
    integer timesteps delta_steps [S, 3, n]; frame f blends steps anchors[f] =
    (lo, hi) with its Eq. 7 weights (frames_dev: packed frame descriptors)."""
    lib = _lib.load()
    _f32dev(delta_steps, "delta_steps")
    S, _, n = delta_steps.shape
    F = frames_dev.shape[0]
    out = torch.empty((F, 3, n), device=delta_steps.device)
    _lib.check(lib.gftorf_blend_offsets(_ptr(delta_steps), S, n, _ptr(frames_dev), F,
                                        _anchors(anchors, F), _ptr(out), _stream(stream)))
    return out


def blend_backward(d_frames: torch.Tensor, frames_dev: torch.Tensor, anchors, n_steps: int,
                   stream=None):
    """Transpose of blend: d delta_steps [S, 3, n] from d_frames [F, 3, n]."""
    lib = _lib.load()
    _f32dev(d_frames, "d_frames")
    F, _, n = d_frames.shape
    out = torch.empty((n_steps, 3, n), device=d_frames.device)
    _lib.check(lib.gftorf_blend_offsets_bwd(_ptr(d_frames), F, n, _ptr(frames_dev),
                                            _anchors(anchors, F), n_steps, _ptr(out), _stream(stream)))
    return out


class BlendOffsets(torch.autograd.Function):
    """blend as an autograd node (network at the timesteps -> raw frames)."""

    @staticmethod
    def forward(ctx, frames_dev, anchors, delta_steps):
        ctx.frames, ctx.anchors, ctx.S = frames_dev, list(anchors), delta_steps.shape[0]
        return blend(delta_steps.contiguous(), frames_dev, ctx.anchors)

    @staticmethod
    def backward(ctx, d_frames):
        return None, None, blend_backward(d_frames.contiguous(), ctx.frames, ctx.anchors, ctx.S)
