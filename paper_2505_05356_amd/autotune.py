"""Tile-shape autotuner: times forward + backward for each supported tile
shape (8x8, 16x16, 32x8) on the caller's problem and keeps the fastest.

Results are cached per problem signature (Gaussians, frames, image size,
frequencies, phases) and per build (a hash of the loaded libgftorf.so, its
version and the GPU architecture) in a JSON file, so a training loop tunes
once and a rebuilt library or another GPU tunes again.
"""
from __future__ import annotations

import dataclasses
import functools
import hashlib
import json
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import raster

CANDIDATES = ((8, 8), (16, 16), (32, 8))


@functools.lru_cache(maxsize=None)
def build_id(device_index: int = 0) -> str:
    """Library version, a hash of the loaded library file and the GPU
    architecture: a tile choice holds only for the kernels and GPU it was
    timed on."""
    lib = raster._lib.load()
    with open(lib._name, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()[:16]
    arch = torch.cuda.get_device_properties(device_index).gcnArchName.split(":")[0]
    return f"v{int(lib.gftorf_version())}-{digest}-{arch}"


def signature(n: int, n_frames: int, cfg, device_index: int = 0) -> str:
    return (f"n{n}-f{n_frames}-{cfg.width}x{cfg.height}-nf{len(cfg.freqs)}-np{len(cfg.phases)}-"
            + build_id(device_index))


def _time(params, frames_dev, cfg, upstream, reps: int, warmup: int) -> float:
    n = params["opacity_logit"].shape[0]
    F = frames_dev.shape[0]
    ws = raster.Workspace(n, F, cfg, device=frames_dev.device)
    out = raster.alloc_outputs(F, cfg, frames_dev.device)
    raster.forward(params, frames_dev, cfg, ws, out=out, check=True)   # sizes the pair capacity
    grads = {k: (torch.empty_like(v) if v is not None else None) for k, v in params.items()}

    def step():
        raster.forward(params, frames_dev, cfg, ws, out=out, check=False)
        if upstream is not None:
            raster.backward(params, frames_dev, cfg, ws, out, upstream["rgb"], upstream["quad"],
                            upstream.get("depth"), grads=grads)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        step()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def autotune(params: Dict[str, torch.Tensor], frames_dev: torch.Tensor, cfg,
             upstream: Optional[Dict[str, torch.Tensor]] = None,
             candidates: Sequence[Tuple[int, int]] = CANDIDATES, reps: int = 5, warmup: int = 2,
             cache_path: Optional[str] = None):
    """Returns (cfg with the fastest tile shape, {"WxH": ms per fwd(+bwd)})."""
    n = params["opacity_logit"].shape[0]
    dev = frames_dev.device
    key = signature(n, frames_dev.shape[0], cfg, dev.index if dev.index is not None else torch.cuda.current_device())
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            tw, th = cache[key]["best"]
            return dataclasses.replace(cfg, tile_w=tw, tile_h=th), cache[key]["ms"]
    times = {}
    for tw, th in candidates:
        c = dataclasses.replace(cfg, tile_w=tw, tile_h=th)
        try:
            times[f"{tw}x{th}"] = _time(params, frames_dev, c, upstream, reps, warmup)
        except raster._lib.GftorfError:
            continue   # e.g. too many tile groups per frame for this shape
    best = min(times, key=times.get)
    tw, th = (int(v) for v in best.split("x"))
    if cache_path:
        cache[key] = {"best": [tw, th], "ms": times}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return dataclasses.replace(cfg, tile_w=tw, tile_h=th), times
