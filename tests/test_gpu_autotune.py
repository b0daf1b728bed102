"""Tile-shape autotuner (needs an MI355X)."""
import os

import numpy as np
import pytest
import torch

import scenes
from paper_2505_05356_amd import autotune, raster

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_supported_shape_and_caches(tmp_path):
    wl = scenes.cfg3(n=20000, n_frames=2)
    params = raster.to_device_params(wl.gaussians, "cuda")
    fdev = raster.pack_frames(wl.frames, wl.cfg)
    up = {k: torch.from_numpy(v).cuda() for k, v in scenes.upstream_grads(2, wl.cfg, 0).items()}
    cache = str(tmp_path / "tiles.json")
    cfg, times = autotune.autotune(params, fdev, wl.cfg, upstream=up, reps=2, warmup=1, cache_path=cache)
    assert (cfg.tile_w, cfg.tile_h) in autotune.CANDIDATES
    assert set(times) == {"8x8", "16x16", "32x8"}
    assert times[f"{cfg.tile_w}x{cfg.tile_h}"] == min(times.values())
    assert os.path.exists(cache)
    cfg2, times2 = autotune.autotune(params, fdev, wl.cfg, upstream=up, cache_path=cache)
    assert (cfg2.tile_w, cfg2.tile_h) == (cfg.tile_w, cfg.tile_h) and times2 == times
    # the cache key names the build and the GPU: another library build tunes again
    key = autotune.signature(wl.gaussians.n, 2, wl.cfg)
    assert autotune.build_id() in key and "gfx950" in key
    import json
    with open(cache) as fh:
        stored = json.load(fh)
    assert list(stored) == [key]
    stale = {key.replace(autotune.build_id(), "v1-0000000000000000-gfx950"): stored[key]}
    with open(cache, "w") as fh:
        json.dump(stale, fh)
    cfg3, times3 = autotune.autotune(params, fdev, wl.cfg, upstream=up, reps=1, warmup=1, cache_path=cache)
    assert times3 != times and key in json.load(open(cache))
