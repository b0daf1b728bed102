"""Full-size workloads in the benchmark's launch configuration, checked on
sampled tiles against the FP64 oracle (needs an MI355X).

The GPU renders every frame of the batch; the oracle evaluates a seeded
sample of tiles of the first and last frame.  Gradients are compared for the
scalar sum(upstream * outputs) with the upstream gradient restricted to the
sampled, unflagged pixels, which the oracle differentiates exactly.  A frame
that renders only some quad channels (an asynchronous raw quad) is compared
on those, and the oracle is given zero upstream gradient on the others."""
import dataclasses

import numpy as np
import pytest
import torch

import scenes
from oracle import binning, render as oref
from tests.gpu_common import assert_grads_close, assert_images_close, gpu_lists, run_gpu

pytestmark = pytest.mark.gpu


def _cfg3_sh():
    wl = scenes.cfg3()
    return dataclasses.replace(wl, gaussians=scenes.with_sh(wl.gaussians, 3, seed=1))


def _cfg3_async():
    wl = scenes.cfg3()
    return dataclasses.replace(wl, frames=scenes.async_quartet_frames(2, 0.125, wl.frames[0]))


WORKLOADS = {
    "static-100k-640x480": lambda: scenes.cfg2(),
    "dynamic-200k-8f-640x480": lambda: scenes.cfg3(),
    "dynamic-200k-8f-640x480-sh3": _cfg3_sh,
    "dynamic-200k-8f-640x480-async-quartets": _cfg3_async,
    "dynamic-1M-16f-1024x768-2freq": lambda: scenes.cfg4(),
    "dynamic-1M-16f-1024x768-2freq-8x8": lambda: scenes.cfg4(tile=(8, 8)),
    "dynamic-1M-16f-1024x768-2freq-32x8": lambda: scenes.cfg4(tile=(32, 8)),
}


def _channels(frame, cfg):
    """Quad channels the frame renders (all when its quad_mask is 0)."""
    m = getattr(frame, "quad_mask", 0)
    return np.array([m == 0 or bool(m >> c & 1) for c in range(cfg.n_quad)])


def _sample(wl, k=3, seed=0):
    n_tiles = wl.cfg.tiles_x * wl.cfg.tiles_y
    rng = np.random.default_rng(seed)
    F = len(wl.frames)
    chosen = {0: sorted(rng.choice(n_tiles, k, replace=False).tolist())}
    chosen[F - 1] = sorted(set(chosen.get(F - 1, [])) | set(rng.choice(n_tiles, k, replace=False).tolist()))
    return chosen


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fullsize_sampled_tiles(name):
    wl = WORKLOADS[name]()
    F = len(wl.frames)
    chosen = _sample(wl)
    sel_frames = sorted(chosen)
    frames = [wl.frames[f] for f in sel_frames]
    tiles = [chosen[f] for f in sel_frames]
    ref = oref.render(wl.gaussians, frames, wl.cfg, tiles=tiles)
    ok = ref["computed"] & ~ref["flagged"]
    assert ok.sum() > 0.97 * ref["computed"].sum()

    # upstream restricted to the sampled, unflagged pixels of frames 0 and F-1
    up = scenes.upstream_grads(F, wl.cfg, seed=2)
    mask = np.zeros((F,) + ok.shape[1:], bool)
    for i, f in enumerate(sel_frames):
        mask[f] = ok[i]
    up = {k: (v * (mask[:, None] if v.ndim == 4 else mask)).astype(np.float32) for k, v in up.items()}
    res = run_gpu(wl.gaussians, wl.frames, wl.cfg, upstream=up)
    assert not res["status"]["overflow"]

    for i, f in enumerate(sel_frames):
        m = ok[i][None]
        for k in ("rgb", "depth", "T_final"):
            assert_images_close(res[k][f:f + 1], np.nan_to_num(ref[k][i:i + 1]), m, f"{name}/f{f}/{k}")
        ch = _channels(wl.frames[f], wl.cfg)
        assert_images_close(res["quad"][f:f + 1, ch], np.nan_to_num(ref["quad"][i:i + 1, ch]), m,
                            f"{name}/f{f}/quad")
        np.testing.assert_array_equal(res["n_contrib"][f][ok[i]], ref["n_contrib"][i][ok[i]])

    # tile lists of the sampled tiles, bit-exact
    lists = gpu_lists(res, wl.gaussians, wl.frames, wl.cfg, pairs_to_host=False)
    n_tiles = wl.cfg.tiles_x * wl.cfg.tiles_y
    assert int(lists["ranges"][-1, 1]) == res["status"]["n_pairs"]
    for i, f in enumerate(sel_frames):
        proj = binning.project(wl.gaussians, wl.frames[f], wl.cfg)
        exp = binning.lists_for_tiles(proj, wl.cfg, chosen[f])
        for t, lst in exp.items():
            a, b = lists["ranges"][f * n_tiles + t]
            got = lists["pair_item_dev"][int(a):int(b)].cpu().numpy().view(np.uint32)
            np.testing.assert_array_equal(got, (f * wl.gaussians.n + lst).astype(np.uint32))

    up_sel = {k: v[sel_frames].copy() for k, v in up.items()}
    for i, f in enumerate(sel_frames):
        up_sel["quad"][i, ~_channels(wl.frames[f], wl.cfg)] = 0.0
    gref = oref.render(wl.gaussians, frames, wl.cfg, tiles=tiles, upstream=up_sel)
    dynamic = np.any(wl.gaussians.vel)
    for k, r in gref["grads"].items():
        if not dynamic and k in ("vel", "acc", "omega"):
            continue
        assert_grads_close(res["grads"][k], r, f"{name}/{k}")


@pytest.mark.parametrize("max_pairs", [20_000_000, 200_000_000])
def test_large_batch_overflow_is_recovered(max_pairs):
    """1M Gaussians x 16 frames, whose level-A chunks of 1024 items are placed
    by (chunk, group row), with a pair capacity below the need: 20M cuts
    through the group lists, 200M only through the tile lists, so some lists
    take the capacity-checked stores and the others the unchecked ones.  The
    status reports the overflow, and the forward regrows the workspace and
    renders exactly what a sufficient capacity renders."""
    wl = scenes.cfg4()
    res = run_gpu(wl.gaussians, wl.frames, wl.cfg, max_pairs=max_pairs, channels=("rgb",))
    st = res["status"]
    assert st["n_pairs"] > max_pairs and res["_ws"].max_pairs >= st["n_pairs"]
    rgb = res["rgb"]
    del res
    ref = run_gpu(wl.gaussians, wl.frames, wl.cfg, channels=("rgb",))
    assert not ref["status"]["overflow"]
    np.testing.assert_array_equal(rgb, ref["rgb"])
