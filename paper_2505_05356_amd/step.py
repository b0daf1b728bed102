"""Optimisation step over a frame sequence, eager or replayed as one HIP graph.

One step: select the batch's frames and random backgrounds from the device
step counter -> forward render of the batch -> L2 losses on quads and RGB
(paper Eq. 9, L2 part) -> backward -> Adam on every parameter field
(paper §4: beta = (0.9, 0.999), eps = 1e-15, per-field learning rates).
All buffers are allocated up front; a captured step allocates nothing and
needs no host involvement, so it can be replayed with gftorf_graph_launch.

With a deformation network (paper §4, "MLP") the step also evaluates the
network at the selected frames' times (read on the device from the frame
descriptors), renders with its offsets as the per-frame `delta`, takes the
network's backward after the rasterizer's (the canonical centres are the
`mean` field, so their gradient adds to the mean's) and updates the network
weights with their own Adam group, whose rate decays exponentially from the
device step counter (§4: 8e-4 to 1.6e-6 over 60K iterations).
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional

import torch

from . import _lib, raster
from ._lib import FIELDS, SH_FIELDS

# Per-field learning rates.  The paper states the reflectivity (albedo) rate
# 1.6e-4 (heuristic H1, §4); the others are not stated and follow common
# Gaussian-splatting practice for these parameterisations.
DEFAULT_LR = {"mean": 1.6e-4, "vel": 1.6e-4, "acc": 1.6e-4, "scale": 5e-4, "quat": 1e-3,
              "omega": 1e-3, "opacity_logit": 5e-2, "rgb": 2.5e-3, "albedo": 1.6e-4,
              "sh_rgb": 2.5e-3, "sh_albedo": 1.6e-4}
# the network's rate and its exponential decay (paper §4)
NET_LR, NET_LR_FINAL, NET_DECAY_STEPS = 8e-4, 1.6e-6, 60_000


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class TrainStep:
    """params: trainable float32 device tensors (FIELDS and, if used, the
    spherical-harmonic SH_FIELDS; optional ones may be None)
    seq_frames: packed frame descriptors of the sequence [S, 40] (device)
    targets_rgb [S, 3, H, W], targets_quad [S, NQ, H, W] (device)
    bg_table: None or [n_bg, batch, 3 + NQ] backgrounds drawn per step (device)
    net, net_params: optional deform.DeformNet (training workspace for the
    Gaussians at `batch` times) and its flat float32 weights (device), updated
    in place like the other parameters
    """

    def __init__(self, params: Dict[str, torch.Tensor], seq_frames, targets_rgb, targets_quad,
                 cfg, batch: int = 4, lrs: Optional[Dict[str, float]] = None,
                 bg_table: Optional[torch.Tensor] = None, quad_weight: float = 1.0,
                 max_pairs: Optional[int] = None, stream: Optional[torch.cuda.Stream] = None,
                 net=None, net_params: Optional[torch.Tensor] = None,
                 net_lr: float = NET_LR, net_lr_final: float = NET_LR_FINAL,
                 net_decay_steps: int = NET_DECAY_STEPS):
        self.lib = _lib.load()
        dev = seq_frames.device
        self.params, self.cfg, self.batch = params, cfg, batch
        self.seq, self.tr, self.tq = seq_frames, targets_rgb, targets_quad
        self.bg_table = bg_table
        self.quad_weight = float(quad_weight)
        self.n = params["opacity_logit"].shape[0]
        self.stream = stream or torch.cuda.Stream(device=dev)
        self.frames = seq_frames[:batch].clone()
        self.frame_index = torch.zeros(batch, dtype=torch.int32, device=dev)
        self.step_counter = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.ws = raster.Workspace(self.n, batch, cfg, max_pairs=max_pairs, device=dev)
        self.out = raster.alloc_outputs(batch, cfg, dev, channels=("rgb", "quad"))
        self.d_rgb = torch.empty_like(self.out["rgb"])
        self.d_quad = torch.empty_like(self.out["quad"])
        self.grads = {k: (torch.empty_like(v) if v is not None else None) for k, v in params.items()}
        self.m = {k: (torch.zeros_like(v) if v is not None else None) for k, v in params.items()}
        self.v = {k: (torch.zeros_like(v) if v is not None else None) for k, v in params.items()}
        lrs = dict(DEFAULT_LR, **(lrs or {}))
        groups = [k for k in FIELDS + SH_FIELDS if params.get(k) is not None]
        self.net, self.net_params = net, net_params
        if net is not None:
            if net_params is None or tuple(net_params.shape) != (net.n_params,) or \
                    net_params.dtype != torch.float32 or not net_params.is_contiguous():
                raise ValueError("net_params must be the network's flat float32 weights")
            if net.n != self.n or net.n_times < batch or not net.training:
                raise ValueError("the network workspace must cover n Gaussians at `batch` times, training")
            self.delta = torch.zeros((batch, 3, self.n), device=dev)
            self.d_delta = torch.empty_like(self.delta)
            self.net_grad = torch.empty_like(net_params)
            self.net_m, self.net_v = torch.zeros_like(net_params), torch.zeros_like(net_params)
        self.groups = (_lib.AdamGroupC * (len(groups) + (net is not None)))()
        for i, k in enumerate(groups):
            g = self.groups[i]
            g.param, g.grad = params[k].data_ptr(), self.grads[k].data_ptr()
            g.m, g.v = self.m[k].data_ptr(), self.v[k].data_ptr()
            g.n, g.lr = params[k].numel(), lrs[k]
        if net is not None:
            g = self.groups[len(groups)]
            g.param, g.grad = net_params.data_ptr(), self.net_grad.data_ptr()
            g.m, g.v = self.net_m.data_ptr(), self.net_v.data_ptr()
            g.n, g.lr, g.lr_final, g.decay_steps = net.n_params, net_lr, net_lr_final, net_decay_steps
        self.graph = None
        self._gs = raster.gaussians_struct(params)
        self._gg = _lib.GaussiansGradC()
        for k in FIELDS + SH_FIELDS:
            setattr(self._gg, k, self.grads[k].data_ptr() if self.grads.get(k) is not None else None)
        if net is not None:
            self._gs.delta = self.delta.data_ptr()
            self._gg.delta = self.d_delta.data_ptr()
        self._o = raster.outputs_struct(self.out)

    def _enqueue(self, s):
        lib, chk = self.lib, _lib.check
        nq = raster.n_quad(self.cfg)
        n_bg = 0 if self.bg_table is None else self.bg_table.shape[0]
        chk(lib.gftorf_select_frames(_p(self.frames), self.batch, _p(self.seq), self.seq.shape[0],
                                     _p(self.bg_table), n_bg, nq, _p(self.step_counter),
                                     _p(self.frame_index), s))
        net = self.net
        if net is not None:
            chk(lib.gftorf_mlp_fwd_frames(ctypes.byref(net.cfg), _p(self.net_params), _p(self.params["mean"]),
                                          self.n, _p(self.frames), self.batch, _p(self.delta), 1,
                                          _p(net.ws), net.nbytes, s))
        chk(lib.gftorf_render_fwd(ctypes.byref(self._gs), _p(self.frames), self.batch,
                                  ctypes.byref(self.ws.cstruct), ctypes.byref(self._o),
                                  ctypes.c_void_p(self.ws.ptr), self.ws.nbytes, s))
        chk(lib.gftorf_fill_f32(_p(self.loss), 0.0, 1, s))
        H, W = self.cfg.height, self.cfg.width
        chk(lib.gftorf_l2_loss_grad(_p(self.out["quad"]), _p(self.tq), _p(self.frame_index),
                                    self.batch, nq * H * W, self.quad_weight, _p(self.d_quad),
                                    _p(self.loss), s))
        chk(lib.gftorf_l2_loss_grad(_p(self.out["rgb"]), _p(self.tr), _p(self.frame_index),
                                    self.batch, 3 * H * W, 1.0, _p(self.d_rgb), _p(self.loss), s))
        chk(lib.gftorf_render_bwd(ctypes.byref(self._gs), _p(self.frames), self.batch,
                                  ctypes.byref(self.ws.cstruct), ctypes.byref(self._o),
                                  _p(self.d_rgb), _p(self.d_quad), None, ctypes.byref(self._gg),
                                  None, ctypes.c_void_p(self.ws.ptr), self.ws.nbytes, s))
        if net is not None:
            # d x0 adds to the rasterizer's mean gradient (x0 is the mean)
            chk(lib.gftorf_mlp_bwd_frames(ctypes.byref(net.cfg), _p(self.net_params), _p(self.params["mean"]),
                                          self.n, _p(self.frames), self.batch, _p(self.d_delta),
                                          _p(self.net_grad), _p(self.grads["mean"]), 1,
                                          _p(net.ws), net.nbytes, s))
        chk(lib.gftorf_adam_step(self.groups, len(self.groups), _p(self.step_counter),
                                 0.9, 0.999, 1e-15, s))

    def size_workspace(self, steps: int = None):
        """Runs the forward of every batch of the sequence once (with pair
        count checks) so the workspace fits all of them; no state changes."""
        S = self.seq.shape[0]
        steps = steps if steps is not None else (S + self.batch - 1) // self.batch
        for st in range(steps):
            idx = [(self.batch * st + b) % S for b in range(self.batch)]
            fr = self.seq[idx].contiguous()
            params = self.params
            if self.net is not None:   # offsets move the centres, hence the tile lists
                times = fr[:, _lib.FRAME_TIME].cpu().tolist()
                params = dict(params, delta=self.net.forward(self.net_params, params["mean"], times,
                                                             save=False))
            raster.forward(params, fr, self.cfg, self.ws, check=True)
        self.ws.max_pairs = int(self.ws.max_pairs * 1.1)
        self.ws._alloc(self.ws.max_pairs)

    def step(self):
        """One eager step on this object's stream."""
        with torch.cuda.stream(self.stream):
            self._enqueue(ctypes.c_void_p(self.stream.cuda_stream))

    def capture(self):
        """Captures one step as a HIP graph (replaces a previous capture)."""
        lib = self.lib
        if self.graph is not None:
            lib.gftorf_graph_destroy(self.graph)
            self.graph = None
        torch.cuda.synchronize()
        s = ctypes.c_void_p(self.stream.cuda_stream)
        _lib.check(lib.gftorf_graph_begin(s))
        try:
            self._enqueue(s)
        finally:
            g = ctypes.c_void_p()
            rc = lib.gftorf_graph_end(s, ctypes.byref(g))
        _lib.check(rc)
        self.graph = g

    def replay(self):
        _lib.check(self.lib.gftorf_graph_launch(self.graph, ctypes.c_void_p(self.stream.cuda_stream)))

    def status(self):
        return self.ws.status(self.stream)

    def __del__(self):
        try:
            if self.graph is not None:
                self.lib.gftorf_graph_destroy(self.graph)
        except Exception:
            pass
