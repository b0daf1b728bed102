"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X)."""
import dataclasses

import numpy as np
import pytest
import torch

import scenes
from oracle import binning, render as oref
from tests.gpu_common import (assert_grads_close, assert_images_close, gpu_lists, mask_upstream,
                              run_gpu)

pytestmark = pytest.mark.gpu


def _cases():
    c = {}
    c["cfg1"] = scenes.cfg1()
    w = scenes.cfg1(seed=3)
    c["ragged-70x45"] = scenes.Workload("ragged", w.gaussians,
                                        scenes.identity_frames([0.0], 70, 45, 60.0, 60.0, 4),
                                        dataclasses.replace(w.cfg, width=70, height=45))
    d = scenes.cfg3(seed=2, n=3000, n_frames=3)
    fr = scenes.identity_frames([0.0, 0.1, 0.25], 96, 72, 80.0, 80.0, 4, bg_seed=5)
    g = scenes.draw_gaussians(3000, 96, 72, 80.0, 80.0, seed=2, dynamic=True)
    c["dynamic-3f-8x8-bg"] = scenes.Workload("dyn", g, fr, scenes.RenderConfig(
        width=96, height=72, tile_w=8, tile_h=8))
    c["dynamic-3f-32x8-p2"] = scenes.Workload("dyn2", g, fr, scenes.RenderConfig(
        width=96, height=72, tile_w=32, tile_h=8, bg_T_power=2))
    g2 = scenes.draw_gaussians(1500, 80, 60, 70.0, 70.0, seed=4, dynamic=True)
    fr2 = scenes.identity_frames([0.05, 0.2], 80, 60, 70.0, 70.0, 8, bg_seed=6, n_freq=2)
    c["two-freq"] = scenes.Workload("2f", g2, fr2, scenes.RenderConfig(
        width=80, height=60, freqs=(30e6, 60e6)))
    t = scenes.tiny_scene(40, 24, 20, seed=7, dynamic=True)
    c["strict"] = scenes.Workload("strict", t.gaussians, scenes.frames_for_times([0.0, 0.2], t),
                                  t.cfg.strict())
    return c


CASES = _cases()


@pytest.fixture(scope="module")
def oracle_cache():
    return {}


def _oracle(name, cache, upstream=False):
    key = (name, upstream)
    if key not in cache:
        wl = CASES[name]
        up = scenes.upstream_grads(len(wl.frames), wl.cfg, seed=1) if upstream else None
        if upstream:
            base = _oracle(name, cache, False)[0]
            up = mask_upstream(up, ~base["flagged"])
        cache[key] = (oref.render(wl.gaussians, wl.frames, wl.cfg, upstream=up), up)
    return cache[key]


@pytest.mark.parametrize("name", list(CASES))
def test_binning_bit_exact(name):
    wl = CASES[name]
    g, frames, cfg = wl.gaussians, wl.frames, wl.cfg
    res = run_gpu(g, frames, cfg)
    lists = gpu_lists(res, g, frames, cfg)
    ref = binning.sorted_pairs(g, frames, cfg)
    n_tiles = cfg.tiles_x * cfg.tiles_y
    assert res["status"]["n_pairs"] == ref["P"]
    assert not res["status"]["overflow"]
    np.testing.assert_array_equal(lists["pair_key"], (ref["frame"] * n_tiles + ref["tile"]).astype(np.uint32))
    np.testing.assert_array_equal(lists["pair_item"], (ref["frame"] * g.n + ref["index"]).astype(np.uint32))
    # per-item rectangles, counts and depth keys
    cnt_ref = np.concatenate([p["count"] for p in ref["projections"]]).astype(np.uint32)
    np.testing.assert_array_equal(lists["count"], cnt_ref)
    key_by_item = np.empty_like(lists["depth_key"])
    key_by_item[lists["depth_item"]] = lists["depth_key"]
    key_ref = np.concatenate([p["key"] for p in ref["projections"]])
    np.testing.assert_array_equal(key_by_item, key_ref)
    valid = cnt_ref > 0
    rect_ref = np.concatenate([p["rect"].T for p in ref["projections"]])
    got = lists["rect"]
    gx = np.stack([got[:, 0] & 0xFFFF, got[:, 0] >> 16, got[:, 1] & 0xFFFF, got[:, 1] >> 16], 1)
    np.testing.assert_array_equal(gx[valid], rect_ref[valid])
    # items are frame-major and depth-ordered inside each frame, ties by index
    frames_of = lists["depth_item"] // g.n
    assert np.all(np.diff(frames_of.astype(np.int64)) >= 0)
    for f in range(len(frames)):
        sel = frames_of == f
        k = lists["depth_key"][sel].astype(np.int64)
        i = lists["depth_item"][sel].astype(np.int64)
        assert np.all((np.diff(k) > 0) | ((np.diff(k) == 0) & (np.diff(i) > 0)))


@pytest.mark.parametrize("name", list(CASES))
def test_forward_matches_oracle(name, oracle_cache):
    wl = CASES[name]
    ref, _ = _oracle(name, oracle_cache)
    res = run_gpu(wl.gaussians, wl.frames, wl.cfg)
    ok = ~ref["flagged"]
    assert ok.mean() > 0.97, f"too many flagged pixels: {1 - ok.mean():.3%}"
    for k in ("rgb", "quad", "depth", "T_final"):
        assert_images_close(res[k], ref[k], ok, f"{name}/{k}")
    np.testing.assert_array_equal(res["n_contrib"][ok], ref["n_contrib"][ok])
    _check_workload_counts(res["status"], ref, wl)


def _check_workload_counts(status, ref, wl):
    # the evaluated / composited (pixel, entry) totals that the library reports
    # (the work measure of the roofline figures) against the oracle's per-pixel
    # counts: equal on unflagged pixels; a flagged pixel may count anything
    # from 0 to its tile's list length
    cfg, F = wl.cfg, len(wl.frames)
    ok = ~ref["flagged"] & ref["computed"]
    pairs = ref["pairs"]
    n_tiles = cfg.tiles_x * cfg.tiles_y
    L = np.bincount(np.asarray(pairs["frame"], np.int64) * n_tiles + np.asarray(pairs["tile"], np.int64),
                    minlength=F * n_tiles).reshape(F, cfg.tiles_y, cfg.tiles_x)
    Lpx = np.repeat(np.repeat(L, cfg.tile_h, axis=1), cfg.tile_w, axis=2)[:, :cfg.height, :cfg.width]
    slack = int(Lpx[ref["computed"] & ref["flagged"]].sum())
    for key, ref_key in (("n_evaluated", "n_evaluated"), ("n_composited", "n_composited")):
        base = int(ref[ref_key][ok].sum())
        got = int(status[key])
        assert base <= got <= base + slack, (key, got, base, slack)
        if slack == 0:
            assert got == base


@pytest.mark.parametrize("name", list(CASES))
def test_backward_matches_oracle(name, oracle_cache):
    wl = CASES[name]
    ref, up = _oracle(name, oracle_cache, upstream=True)
    res = run_gpu(wl.gaussians, wl.frames, wl.cfg, upstream=up, want_bg=True)
    dynamic = np.any(wl.gaussians.vel)
    for k, r in ref["grads"].items():
        if not dynamic and k in ("vel", "acc", "omega"):
            continue
        assert_grads_close(res["grads"][k], r, f"{name}/{k}")
    F = len(wl.frames)
    bg_ref = np.concatenate([ref["grad_bg_rgb"], ref["grad_bg_quad"]], 1)
    assert_grads_close(res["grad_bg"], bg_ref, f"{name}/bg")


def test_batched_equals_per_frame():
    wl = CASES["dynamic-3f-8x8-bg"]
    batched = run_gpu(wl.gaussians, wl.frames, wl.cfg)
    for f, fr in enumerate(wl.frames):
        single = run_gpu(wl.gaussians, [fr], wl.cfg)
        for k in ("rgb", "quad", "depth", "T_final", "n_contrib"):
            np.testing.assert_array_equal(batched[k][f], single[k][0], err_msg=f"frame {f} {k}")


def test_forward_deterministic():
    wl = CASES["cfg1"]
    a = run_gpu(wl.gaussians, wl.frames, wl.cfg)
    b = run_gpu(wl.gaussians, wl.frames, wl.cfg)
    for k in ("rgb", "quad", "depth", "T_final", "n_contrib"):
        np.testing.assert_array_equal(a[k], b[k])


def test_overflow_is_reported_and_recovered():
    wl = CASES["cfg1"]
    res = run_gpu(wl.gaussians, wl.frames, wl.cfg, max_pairs=100)
    # forward() regrows the workspace and renders again
    assert res["_ws"].max_pairs >= res["status"]["n_pairs"] > 100
    ref = run_gpu(wl.gaussians, wl.frames, wl.cfg)
    np.testing.assert_array_equal(res["rgb"], ref["rgb"])


def test_empty_scene_renders_background():
    wl = CASES["dynamic-3f-8x8-bg"]
    g = wl.gaussians.subset(np.arange(0))
    res = run_gpu(g, wl.frames, wl.cfg)
    for f, fr in enumerate(wl.frames):
        np.testing.assert_array_equal(res["rgb"][f], np.broadcast_to(fr.bg_rgb[:, None, None], res["rgb"][f].shape))
        np.testing.assert_array_equal(res["T_final"][f], 1.0)
        assert (res["n_contrib"] == 0).all()


def test_nonfinite_gaussians_are_culled_and_counted():
    wl = CASES["cfg1"]
    g = wl.gaussians.copy()
    g.mean[0, 5] = np.nan
    g.scale[1, 7] = np.inf
    res = run_gpu(g, wl.frames, wl.cfg)
    assert res["status"]["nonfinite"] == 2
    assert np.isfinite(res["rgb"]).all()


@pytest.mark.parametrize("name", ["cfg1", "two-freq", "dynamic-3f-32x8-p2"])
def test_tof_epilogue_matches_oracle(name, oracle_cache):
    # Phasor, d_ToF and amplitude written by the forward kernel against the
    # oracle's epilogue applied to the oracle's own quads.  The bound follows
    # from the quad tolerance: each projection is a sum of the n_phase quads
    # with weights of modulus <= 1, so its error is at most
    # e = FWD_RTOL * sum_j (|Q_j| + max |Q_j|); the amplitude then moves by at
    # most e / sqrt(2) and the phase by about sqrt(2) e / |phasor| where the
    # phasor is well away from zero.
    from oracle import tof
    from tests.gpu_common import FWD_RTOL
    wl = CASES[name]
    cfg = wl.cfg
    ref, _ = _oracle(name, oracle_cache)
    res = run_gpu(wl.gaussians, wl.frames, cfg,
                  channels=("quad", "phasor", "d_tof", "amplitude"))
    exp = tof.tof_epilogue(ref["quad"], cfg)
    ok = ~ref["flagged"]
    F, H, W = ok.shape
    nf, nphi = len(cfg.freqs), len(cfg.phases)
    q = ref["quad"].astype(np.float64).reshape(F, nf, nphi, H, W)
    qmax = np.abs(q).max(axis=(-2, -1), keepdims=True)
    e = FWD_RTOL * (np.abs(q) + qmax).sum(2) * 1.01 + 1e-6 * qmax.max()
    okf = np.broadcast_to(ok[:, None], e.shape)
    for c in range(2):
        err = np.abs(res["phasor"][:, :, c].astype(np.float64) - exp["phasor"][:, :, c])
        assert np.all(err[okf] <= e[okf]), f"{name}/phasor[{c}] max excess {np.max(err[okf] - e[okf]):.3g}"
    err = np.abs(res["amplitude"].astype(np.float64) - exp["amplitude"])
    assert np.all(err[okf] <= e[okf]), f"{name}/amplitude"
    # phase: only where the phasor is at least 10 error bounds long
    mag = 2 * exp["amplitude"]
    well = okf & (mag > 10 * np.sqrt(2) * e)
    assert well.mean() > 0.5, f"{name}: too few well-conditioned pixels ({well.mean():.2%})"
    lam = np.array([299_792_458.0 / (2 * f) for f in cfg.freqs])[None, :, None, None]
    dd = np.abs(res["d_tof"].astype(np.float64) - exp["d_tof"])
    dd = np.minimum(dd, lam - dd)            # distance modulo the ambiguity range c / 2f
    tol = lam / (2 * np.pi) * (1.5 * np.sqrt(2) * e / np.maximum(mag, 1e-30)) + 1e-6 * lam
    assert np.all(dd[well] <= tol[well]), f"{name}/d_tof max excess {np.max(dd[well] - tol[well]):.3g} m"
    assert np.all((res["d_tof"] >= 0) & (res["d_tof"] <= lam * (1 + 1e-6)))


def test_async_quartets_match_oracle():
    # Two asynchronous raw quartets (Eq. 7): eight frames, each at its own
    # time with interpolated centres, each rendering one phase offset.  Tile
    # lists bit-exact; RGB, depth, T_final, n_contrib and the rendered quad
    # channel against the oracle; the backward ignores the upstream gradient
    # of the channels a frame does not render (the oracle is given zeros there).
    g = scenes.draw_gaussians(2500, 80, 64, 70.0, 70.0, seed=11, dynamic=True)
    base = scenes.identity_frames([0.0], 80, 64, 70.0, 70.0, 4, bg_seed=8)[0]
    frames = scenes.async_quartet_frames(2, 0.1, base)
    cfg = scenes.RenderConfig(width=80, height=64, tile_w=16, tile_h=16)
    F = len(frames)
    res = run_gpu(g, frames, cfg)
    lists = gpu_lists(res, g, frames, cfg)
    ref_pairs = binning.sorted_pairs(g, frames, cfg)
    n_tiles = cfg.tiles_x * cfg.tiles_y
    np.testing.assert_array_equal(lists["pair_key"], (ref_pairs["frame"] * n_tiles + ref_pairs["tile"]).astype(np.uint32))
    np.testing.assert_array_equal(lists["pair_item"], (ref_pairs["frame"] * g.n + ref_pairs["index"]).astype(np.uint32))
    ref = oref.render(g, frames, cfg)
    ok = ~ref["flagged"]
    for k in ("rgb", "depth", "T_final"):
        assert_images_close(res[k], ref[k], ok, f"async/{k}")
    np.testing.assert_array_equal(res["n_contrib"][ok], ref["n_contrib"][ok])
    ch = np.array([fr.quad_mask.bit_length() - 1 for fr in frames])
    assert_images_close(res["quad"][np.arange(F), ch], ref["quad"][np.arange(F), ch], ok, "async/quad")
    # backward
    up = mask_upstream(scenes.upstream_grads(F, cfg, seed=3), ok)
    up_ref = dict(up)
    qmask = np.zeros_like(up["quad"])
    qmask[np.arange(F), ch] = 1.0
    up_ref["quad"] = up["quad"] * qmask
    ref_b = oref.render(g, frames, cfg, upstream=up_ref)
    res_b = run_gpu(g, frames, cfg, upstream=up, want_bg=True)
    for k, r in ref_b["grads"].items():
        assert_grads_close(res_b["grads"][k], r, f"async/{k}")
    bg_ref = np.concatenate([ref_b["grad_bg_rgb"], ref_b["grad_bg_quad"]], 1)
    assert_grads_close(res_b["grad_bg"], bg_ref, "async/bg")


@pytest.mark.parametrize("degree", [3, 1])
def test_spherical_harmonics_match_oracle(degree):
    # View-dependent colour (16 x 3 coefficients at degree 3) and reflectivity
    # (16): forward against the oracle, and the gradients of every field
    # including the coefficients (rgb and albedo are replaced: zero gradient).
    g = scenes.with_sh(scenes.draw_gaussians(2000, 80, 64, 70.0, 70.0, seed=13, dynamic=True), degree,
                       seed=5, scale=0.6)
    frames = scenes.identity_frames([0.0, 0.15], 80, 64, 70.0, 70.0, 4, bg_seed=9)
    cfg = scenes.RenderConfig(width=80, height=64)
    ref = oref.render(g, frames, cfg)
    ok = ~ref["flagged"]
    res = run_gpu(g, frames, cfg)
    for k in ("rgb", "quad", "depth", "T_final"):
        assert_images_close(res[k], ref[k], ok, f"sh{degree}/{k}")
    up = mask_upstream(scenes.upstream_grads(len(frames), cfg, seed=2), ok)
    ref_b = oref.render(g, frames, cfg, upstream=up)
    res_b = run_gpu(g, frames, cfg, upstream=up)
    assert set(ref_b["grads"]) >= {"sh_rgb", "sh_albedo"}
    for k, r in ref_b["grads"].items():
        if k in ("rgb", "albedo"):
            assert not np.any(res_b["grads"][k]), k
            continue
        assert_grads_close(res_b["grads"][k], r, f"sh{degree}/{k}")


def test_backward_twice_after_one_forward():
    # every backward starts from cleared gradient records, so a second
    # backward after one forward repeats the first
    wl = CASES["dynamic-3f-8x8-bg"]
    up = scenes.upstream_grads(len(wl.frames), wl.cfg, seed=4)
    res = run_gpu(wl.gaussians, wl.frames, wl.cfg, upstream=up)
    d = {k: torch.from_numpy(np.ascontiguousarray(up[k], dtype=np.float32)).cuda()
         for k in ("rgb", "quad", "depth")}
    from paper_2505_05356_amd import raster
    again = raster.backward(res["_params"], res["_frames"], wl.cfg, res["_ws"], res["_out"],
                            d["rgb"], d["quad"], d["depth"])
    torch.cuda.synchronize()
    for k, v in again.items():
        if v is None:
            continue
        # equal up to the float32 atomic summation order of the composite backward
        assert_grads_close(v.cpu().numpy(), res["grads"][k], f"twice/{k}", rtol=1e-4)


def test_depth_key_ties_bit_exact():
    # Many Gaussians share one camera-space depth, so their float32 depth keys
    # tie and the order inside a tile list falls to the Gaussian index (the
    # ascending-index tie-break): lists bit-exact against the oracle, ties
    # present in them, and the forward composited in that order.
    g = scenes.draw_gaussians(1500, 64, 48, 60.0, 60.0, seed=21)
    z_new = np.array([1.5, 2.0, 2.5], np.float32)[np.random.default_rng(22).integers(0, 3, g.n)]
    s = z_new.astype(np.float64) / g.mean[2].astype(np.float64)
    g.mean[0] = (g.mean[0] * s).astype(np.float32)
    g.mean[1] = (g.mean[1] * s).astype(np.float32)
    g.mean[2] = z_new
    frames = scenes.identity_frames([0.0], 64, 48, 60.0, 60.0, 4, bg_seed=1)
    cfg = scenes.RenderConfig(width=64, height=48)
    res = run_gpu(g, frames, cfg)
    lists = gpu_lists(res, g, frames, cfg)
    ref = binning.sorted_pairs(g, frames, cfg)
    n_tiles = cfg.tiles_x * cfg.tiles_y
    np.testing.assert_array_equal(lists["pair_key"], (ref["frame"] * n_tiles + ref["tile"]).astype(np.uint32))
    np.testing.assert_array_equal(lists["pair_item"], (ref["frame"] * g.n + ref["index"]).astype(np.uint32))
    # ties really occur inside tile lists, and the items of every tie ascend
    key = ref["key"]
    same = (np.diff(ref["tile"]) == 0) & (np.diff(key.astype(np.int64)) == 0)
    assert same.sum() > 1000
    assert np.all(np.diff(ref["index"].astype(np.int64))[same] > 0)
    ref_img = oref.render(g, frames, cfg)
    ok = ~ref_img["flagged"]
    for k in ("rgb", "quad", "depth", "T_final"):
        assert_images_close(res[k], ref_img[k], ok, f"ties/{k}")
    np.testing.assert_array_equal(res["n_contrib"][ok], ref_img["n_contrib"][ok])


@pytest.mark.parametrize("n,F", [(100_000, 1), (30_000, 3), (2048 * 128, 2), (2048 * 128 + 5, 2)])
def test_depth_sort_order(n, F):
    # Batches of at most 256 sort tiles (2048 items each) sort each pass in
    # one launch whose tiles add the digit counts of the frame's earlier tiles
    # by look-back; larger batches use three launches per pass.  Both sides of
    # that line: every frame's items in ascending (depth key, index) order,
    # keys equal to the oracle's, and a third of the Gaussians moved to one of
    # three depths, so that runs of equal keys span several sort tiles.
    W, H = 96, 72
    g = scenes.draw_gaussians(n, W, H, 80.0, 80.0, seed=31)
    rng = np.random.default_rng(32)
    tie = rng.random(n) < 0.33
    z_new = np.array([1.5, 2.5, 4.0], np.float32)[rng.integers(0, 3, n)]
    s = np.where(tie, z_new.astype(np.float64) / g.mean[2].astype(np.float64), 1.0)
    g.mean[0] = (g.mean[0] * s).astype(np.float32)
    g.mean[1] = (g.mean[1] * s).astype(np.float32)
    g.mean[2] = np.where(tie, z_new, g.mean[2]).astype(np.float32)
    frames = scenes.identity_frames([0.1 * f for f in range(F)], W, H, 80.0, 80.0, 4)
    cfg = scenes.RenderConfig(width=W, height=H)
    res = run_gpu(g, frames, cfg, channels=("rgb",))
    assert not res["status"]["sort_fault"] and not res["status"]["overflow"]
    lists = gpu_lists(res, g, frames, cfg, pairs_to_host=False)
    key = lists["depth_key"].astype(np.int64)
    item = lists["depth_item"].astype(np.int64)
    np.testing.assert_array_equal(np.sort(item), np.arange(n * F))
    key_ref = np.concatenate([binning.project(g, fr, cfg, f)["key"].astype(np.int64)
                              for f, fr in enumerate(frames)])
    np.testing.assert_array_equal(key, key_ref[item])
    frame_of = item // n
    assert np.all(np.diff(frame_of) >= 0)
    same_frame = np.diff(frame_of) == 0
    dk, di = np.diff(key), np.diff(item)
    assert np.all(((dk > 0) | ((dk == 0) & (di > 0)))[same_frame])
    # runs of equal keys longer than a sort tile
    starts = np.flatnonzero(np.concatenate([[True], (dk != 0) | ~same_frame, [True]]))
    assert np.max(np.diff(starts)) > 2048


@pytest.mark.parametrize("n_freq,phases", [
    (3, scenes.QUAD_PHASES), (4, scenes.QUAD_PHASES),
    (1, (0.3,)), (2, (0.0, 2 * np.pi / 3, 4 * np.pi / 3)), (4, (0.1, 2.0, 4.0))])
def test_frequencies_and_phase_offsets(n_freq, phases):
    # every frequency count up to the maximum of 4 and phase-offset counts
    # other than the four-tap camera: forward, backward and the background
    # gradients against the oracle (16 quad channels at 4 x 4)
    freqs = (20e6, 30e6, 45e6, 60e6)[:n_freq]
    g = scenes.draw_gaussians(1500, 72, 56, 65.0, 65.0, seed=23, dynamic=True)
    nq = n_freq * len(phases)
    frames = scenes.identity_frames([0.0, 0.12], 72, 56, 65.0, 65.0, nq, bg_seed=24, n_freq=n_freq)
    cfg = scenes.RenderConfig(width=72, height=56, freqs=freqs, phases=tuple(phases))
    ref = oref.render(g, frames, cfg)
    ok = ~ref["flagged"]
    res = run_gpu(g, frames, cfg)
    for k in ("rgb", "quad", "depth", "T_final"):
        assert_images_close(res[k], ref[k], ok, f"{n_freq}x{len(phases)}/{k}")
    up = mask_upstream(scenes.upstream_grads(len(frames), cfg, seed=25), ok)
    ref_b = oref.render(g, frames, cfg, upstream=up)
    res_b = run_gpu(g, frames, cfg, upstream=up, want_bg=True)
    for k, r in ref_b["grads"].items():
        assert_grads_close(res_b["grads"][k], r, f"{n_freq}x{len(phases)}/{k}")
    bg_ref = np.concatenate([ref_b["grad_bg_rgb"], ref_b["grad_bg_quad"]], 1)
    assert_grads_close(res_b["grad_bg"], bg_ref, f"{n_freq}x{len(phases)}/bg")


def _fd_scene():
    # strict mode (no skip or stop thresholds, every Gaussian in every tile),
    # opacities <= 0.82 (below alpha_max), depths 0.08 m apart and slow in z,
    # so that no discrete decision changes under the perturbations
    wl = scenes.tiny_scene(24, 32, 24, seed=26, dynamic=True)
    g = wl.gaussians
    z = 1.0 + 0.08 * np.random.default_rng(27).permutation(g.n)
    s = z / g.mean[2].astype(np.float64)
    g.mean[0] = (g.mean[0] * s).astype(np.float32)
    g.mean[1] = (g.mean[1] * s).astype(np.float32)
    g.mean[2] = z.astype(np.float32)
    g.vel[2] *= 0.1
    g.acc[2] *= 0.1
    g.opacity_logit[:] = np.clip(g.opacity_logit, -2.0, 1.5)
    frames = scenes.identity_frames([0.0, 0.1], 32, 24, 38.4, 38.4, 4, bg_seed=28)
    cfg = dataclasses.replace(wl.cfg, tile_w=16, tile_h=16).strict()
    return g, frames, cfg


def test_backward_directional_finite_differences():
    # The HIP backward against central differences of the HIP forward
    # (supplement C, Eqs. S1-S3 plus the background term): for random
    # directions d per parameter field, L(theta + d) - L(theta - d) of
    # L = sum(upstream * outputs) equals <grad, 2 d> to first order with a
    # third-order remainder.  The steps move each field by about 1e-3 of its
    # scale or of its effect on the centre; the float32 rounding of the two
    # renders' outputs, independent between them, moves L by far less than
    # 1e-6 sqrt(sum (upstream * out)^2) (16 units in the last place per
    # element).
    from paper_2505_05356_amd import raster
    g, frames, cfg = _fd_scene()
    up = scenes.upstream_grads(len(frames), cfg, seed=29)
    res = run_gpu(g, frames, cfg, upstream=up)
    step = dict(mean=1e-3, vel=1e-2, acc=1e-1, scale=1e-4, quat=1e-3, omega=1e-2,
                opacity_logit=1e-2, rgb=1e-3, albedo=1e-2)

    def loss(gg):
        params = raster.to_device_params(gg, "cuda")
        fdev = raster.pack_frames(frames, cfg, "cuda")
        ws = raster.Workspace(gg.n, len(frames), cfg, device="cuda")
        out = raster.forward(params, fdev, cfg, ws)
        o = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        terms = [up[k].astype(np.float64) * o[k] for k in ("rgb", "quad", "depth")]
        return sum(t.sum() for t in terms), sum((t * t).sum() for t in terms)

    rng = np.random.default_rng(30)
    checked = 0
    for field, h in step.items():
        for _ in range(2):
            base = getattr(g, field).astype(np.float64)
            d = rng.normal(size=base.shape) * h
            gp, gm = g.copy(), g.copy()
            setattr(gp, field, (base + d).astype(np.float32))
            setattr(gm, field, (base - d).astype(np.float32))
            dtheta = getattr(gp, field).astype(np.float64) - getattr(gm, field).astype(np.float64)
            lp, sp = loss(gp)
            lm, sm = loss(gm)
            pred = float((res["grads"][field].astype(np.float64) * dtheta).sum())
            noise = 1e-6 * np.sqrt(sp + sm)
            assert abs(pred) > 20 * noise, f"{field}: step too small for float32 ({pred:.3g} vs {noise:.3g})"
            assert abs((lp - lm) - pred) <= 1e-2 * abs(pred) + noise, \
                f"{field}: finite difference {lp - lm:.6g} vs gradient {pred:.6g}"
            checked += 1
    assert checked == 18


def test_status_keeps_overflow_across_forwards():
    # the sticky status fields: an overflowing forward, then one that fits
    # the same workspace; the second clears `overflow` but `overflow_seen` and
    # `n_pairs_seen` remember the first until the header is cleared
    from paper_2505_05356_amd import raster
    wl = CASES["cfg1"]
    params = raster.to_device_params(wl.gaussians, "cuda")
    fdev = raster.pack_frames(wl.frames, wl.cfg, "cuda")
    ws = raster.Workspace(wl.gaussians.n, len(wl.frames), wl.cfg, max_pairs=100, device="cuda")
    raster.forward(params, fdev, wl.cfg, ws, check=False)
    first = ws.status()
    assert first["overflow"] and first["overflow_seen"] and first["n_pairs_seen"] == first["n_pairs"] > 100
    behind = wl.gaussians.copy()
    behind.mean[2] = -1.0                                   # every Gaussian behind the camera
    raster.forward(raster.to_device_params(behind, "cuda"), fdev, wl.cfg, ws, check=False)
    second = ws.status()
    assert not second["overflow"] and second["n_pairs"] <= 100
    assert second["overflow_seen"] and second["n_pairs_seen"] == first["n_pairs"]
    ws.clear_status()
    cleared = ws.status()
    assert not cleared["overflow_seen"] and cleared["n_pairs_seen"] == 0


def test_autograd_backward_refuses_a_reused_workspace():
    # a second forward on the same workspace replaces the tile lists the first
    # forward's backward needs: that backward raises instead of using them
    from paper_2505_05356_amd import raster
    wl = CASES["cfg1"]
    params = {k: (v.requires_grad_(True) if v is not None else None)
              for k, v in raster.to_device_params(wl.gaussians, "cuda").items()}
    ws = raster.Workspace(wl.gaussians.n, len(wl.frames), wl.cfg, device="cuda")
    a = raster.render(params, wl.frames, wl.cfg, ws=ws)
    b = raster.render(params, wl.frames, wl.cfg, ws=ws)
    with pytest.raises(RuntimeError, match="another forward"):
        a["rgb"].sum().backward(retain_graph=True)
    b["rgb"].sum().backward()
    assert params["mean"].grad is not None and torch.isfinite(params["mean"].grad).all()
