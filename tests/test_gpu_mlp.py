"""Deformation network (paper §4, "MLP") on the GPU against the FP64 oracle,
and the rasterizer with per-frame centre offsets (needs an MI355X).

Tolerance.  The network's products take bfloat16 operands (8 significant
bits, unit roundoff u = 2^-8) with float32 accumulation.  Each of the 9
layers rounds its weights and its input activations once, a relative
perturbation of at most 2u per product with random signs, so a layer adds
about sqrt(2) u / sqrt(3) ~ 3e-3 relative RMS error and the 9 layers about
sqrt(9) times that, ~1e-2 relative RMS, forward and backward alike.  The
check is the gradient criterion used for the rasterizer: per tensor,
relative L2 <= 2e-2 and elementwise |gpu - ref| <= 2e-2 (|ref| + max |ref|).
The oracle takes the ReLU decisions in the products' precision
(decide="bf16").  Decisions are integers decided by floating point, so two
correct evaluations may take a unit within rounding of its kink either way,
and then its whole gradient term differs.  The tests therefore check the two
parts separately, with no allowance anywhere:
* the decisions the kernel recorded (gftorf_mlp_get_decisions) equal the
  oracle's at every unit, except units whose |z| lies within
  oracle.mlp.DECISION_MARGIN of their scale, where either is correct (the
  count of such differences is reported);
* the backward, gated with the oracle's decisions (gftorf_mlp_set_decisions),
  matches the oracle's gradients element by element.
The backward with the kernel's own decisions is also checked per tensor
(relative L2).
"""
import dataclasses

import numpy as np
import pytest
import torch

import scenes
from oracle import binning, mlp as omlp, render as oref
from paper_2505_05356_amd import deform
from tests.gpu_common import assert_grads_close, assert_images_close, gpu_lists, mask_upstream, run_gpu

pytestmark = pytest.mark.gpu

MLP_RTOL = 2e-2
SX, ST = 2 * 30e6 / 299_792_458.0, 4.0


def _net_inputs(n, times, seed, last_std=0.05, bias_std=0.1):
    theta = scenes.mlp_params(seed=seed, last_std=last_std, bias_std=bias_std)
    x0, _ = scenes.mlp_rows(n, 1, seed=seed + 100)
    return theta, x0, np.asarray(times, np.float32)


def _close(got, ref, name, elementwise=True):
    # relative L2 <= 2e-2 and elementwise |gpu - ref| <= 2e-2 (|ref| + max |ref|)
    g = np.asarray(got, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    rel = np.linalg.norm(g - r) / np.linalg.norm(r)
    assert rel <= MLP_RTOL, f"{name}: relative L2 error {rel:.3e}"
    if elementwise:
        bad = np.abs(g - r) > MLP_RTOL * (np.abs(r) + np.abs(r).max())
        assert not bad.any(), f"{name}: {int(bad.sum())} of {bad.size} elements beyond tolerance"


def _per_layer(flat, name, ref, elementwise=True):
    W, b = omlp.unpack(flat, omlp.layer_shapes())
    Wr, br = omlp.unpack(ref, omlp.layer_shapes())
    for l in range(len(W)):
        _close(W[l], Wr[l], f"{name}/W{l}", elementwise)
        _close(b[l], br[l], f"{name}/b{l}", elementwise)


def _use_oracle_decisions(net, masks, ratio, rows=None, n_times=None):
    # the kernel's recorded decisions (of the given rows, or all) must equal
    # the oracle's except within the decision margin; then the oracle's
    # replace them for the next backward
    dec = net.decisions(n_times)
    got = (dec[torch.from_numpy(rows).cuda()] if rows is not None else dec).cpu().numpy() != 0
    differ = got != masks
    assert np.all(ratio[differ] <= omlp.DECISION_MARGIN), \
        f"decisions differ at |z|/scale up to {ratio[differ].max():.3e}"
    print(f"decisions: {int(differ.sum())} of {differ.size} differ, all within the margin "
          f"({int((ratio <= omlp.DECISION_MARGIN).sum())} units inside it)")
    want = torch.from_numpy(masks.astype(np.uint8)).cuda()
    if rows is not None:
        dec[torch.from_numpy(rows).cuda()] = want
    else:
        dec = want.contiguous()
    net.set_decisions(dec)
    return int(differ.sum())


@pytest.mark.parametrize("n,times", [(300, [0.0, 0.1, 0.25]), (1, [0.05]), (128, [0.0, 0.2])])
def test_mlp_forward_backward_match_oracle(n, times):
    # 900 rows (7 full blocks and a ragged tail), a single row, and exactly one block
    theta, x0, times = _net_inputs(n, times, seed=1)
    net = deform.DeformNet(n, len(times), pos_scale=SX, time_scale=ST)
    p, x = torch.from_numpy(theta).cuda(), torch.from_numpy(x0).cuda()
    delta = net.forward(p, x, times)
    ref = omlp.offsets(theta, x0, times, SX, ST, decide="bf16")
    torch.cuda.synchronize()
    assert_grads_close(delta.cpu().numpy(), ref, "delta", rtol=MLP_RTOL)
    rng = np.random.default_rng(2)
    up = rng.normal(size=ref.shape).astype(np.float32)
    g_ref, gx_ref, gx_terms = omlp.offsets_backward(theta, x0, times, SX, ST, up, decide="bf16",
                                                    terms=True)
    # with the kernel's own decisions: per tensor
    d_params, d_x0 = net.backward(p, x, times, torch.from_numpy(up).cuda())
    _per_layer(d_params.cpu().numpy(), "d_params (own decisions)", g_ref, elementwise=False)
    _close(d_x0.cpu().numpy(), gx_ref, "d_x0 (own decisions)", elementwise=False)
    # with the oracle's decisions: element by element
    _use_oracle_decisions(net, *omlp.offsets_decision_table(theta, x0, times, SX, ST), n_times=len(times))
    d_params, d_x0 = net.backward(p, x, times, torch.from_numpy(up).cuda())
    torch.cuda.synchronize()
    _per_layer(d_params.cpu().numpy(), "d_params", g_ref)
    _centre_close(d_x0.cpu().numpy(), gx_ref, gx_terms, "d_x0")


def _centre_close(got, ref, terms, name):
    # d x0 = s_x sum_t sum_f enc'_f sum_j g_j W_0[j, f] sums terms as large
    # as 2^9 pi times the first layer's products, which mostly cancel, and the
    # bfloat16 roundings enter in those products, so each element's rounding
    # error scales with the sum of the terms' magnitudes
    # sum_t sum_f |enc'_f| sum_j |g_j W_0[j, f]|: relative L2 <= 2e-2 and
    # elementwise |gpu - ref| <= 2e-2 (|ref| + sum |terms|).
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= MLP_RTOL, f"{name}: relative L2 error {rel:.3e}"
    bad = np.abs(got - ref) > MLP_RTOL * (np.abs(ref) + terms)
    assert not bad.any(), f"{name}: {int(bad.sum())} of {bad.size} elements beyond tolerance"


def test_mlp_paper_initialisation():
    # Xavier-normal layers, last layer N(0, 1e-5^2), zero biases (§4): tiny offsets
    theta, x0, times = _net_inputs(500, [0.0, 0.125], seed=3, last_std=1e-5, bias_std=0.0)
    net = deform.DeformNet(500, 2, pos_scale=SX, time_scale=ST)
    delta = net.forward(torch.from_numpy(theta).cuda(), torch.from_numpy(x0).cuda(), times, save=False)
    ref = omlp.offsets(theta, x0, times, SX, ST, decide="bf16")
    torch.cuda.synchronize()
    assert np.abs(ref).max() < 1e-3
    assert_grads_close(delta.cpu().numpy(), ref, "delta@init", rtol=MLP_RTOL)


def test_mlp_backward_deterministic_and_repeatable():
    theta, x0, times = _net_inputs(700, [0.0, 0.1], seed=4)
    net = deform.DeformNet(700, 2, pos_scale=SX, time_scale=ST)
    p, x = torch.from_numpy(theta).cuda(), torch.from_numpy(x0).cuda()
    up = torch.randn((2, 3, 700), device="cuda")
    outs = []
    for _ in range(2):
        net.forward(p, x, times)
        outs.append([t.cpu().numpy() for t in net.backward(p, x, times, up)])
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)


def test_mlp_full_size_sampled_rows():
    # The benchmark's launch shape: 200k Gaussians at 8 times (1.6M rows).
    # Forward: 64 sampled rows against the oracle, row by row.  Backward: the
    # gradient is linear in d_delta, so an upstream gradient that is non-zero
    # on the sampled rows only has the oracle's gradient of those rows alone.
    n, T = 200_000, 8
    theta = scenes.mlp_params(seed=5, last_std=0.05, bias_std=0.1)
    x0, times = scenes.mlp_rows(n, T, seed=6)
    net = deform.DeformNet(n, T, pos_scale=SX, time_scale=ST)
    p, x = torch.from_numpy(theta).cuda(), torch.from_numpy(x0).cuda()
    delta = net.forward(p, x, times)
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(n * T, 64, replace=False))
    rows[-1] = n * T - 1                                   # the last row of the last block
    t_idx, k_idx = rows // n, rows % n
    got = delta.cpu().numpy()[t_idx, :, k_idx]
    sx32 = float(np.float32(SX))                          # the scale as the device receives it
    x_in = (sx32 * x0[:, k_idx].astype(np.float64)).T
    t_in = ST * times[t_idx].astype(np.float64)
    ref, cache = omlp.forward(theta, x_in, t_in, decide="bf16")
    assert_grads_close(got, ref, "delta@sampled rows", rtol=MLP_RTOL)
    up = np.zeros((T, 3, n), np.float32)
    up_rows = rng.normal(size=(64, 3)).astype(np.float32)
    up[t_idx, :, k_idx] = up_rows
    # only the sampled rows carry gradient, so only their decisions matter
    _use_oracle_decisions(net, *omlp.decision_table(theta, x_in, t_in), rows=rows, n_times=T)
    d_params, d_x0 = net.backward(p, x, times, torch.from_numpy(up).cuda())
    g_ref, g_x, _ = omlp.backward(theta, cache, up_rows)
    _per_layer(d_params.cpu().numpy(), "d_params@sampled rows", g_ref)
    gx, gt = np.zeros((3, n)), np.zeros((3, n))
    np.add.at(gx.T, k_idx, sx32 * g_x)
    np.add.at(gt.T, k_idx, sx32 * cache["d_x_terms"])
    _centre_close(d_x0.cpu().numpy()[:, k_idx], gx[:, k_idx], gt[:, k_idx], "d_x0@sampled rows")
    assert not np.abs(d_x0.cpu().numpy()[:, np.setdiff1d(np.arange(n), k_idx)]).any()


def test_render_with_network_offsets_matches_oracle():
    # network offsets as per-frame centre offsets of the rasterizer: tile lists
    # bit-exact, images and gradients (including d delta) vs the oracle.  The
    # offsets are the oracle network's (float32), the same input for both sides.
    g = scenes.draw_gaussians(1500, 64, 48, 60.0, 60.0, seed=12, dynamic=True)
    frames = scenes.identity_frames([0.0, 0.1, 0.2], 64, 48, 60.0, 60.0, 4, bg_seed=2)
    cfg = scenes.RenderConfig(width=64, height=48, tile_w=16, tile_h=16)
    theta = scenes.mlp_params(seed=8, last_std=0.02, bias_std=0.05)
    delta = omlp.offsets(theta, g.mean, [fr.time for fr in frames], SX, ST).astype(np.float32)
    gd = dataclasses.replace(g, delta=np.ascontiguousarray(delta))
    assert np.abs(gd.delta).max() > 1e-3
    res = run_gpu(gd, frames, cfg)
    lists = gpu_lists(res, gd, frames, cfg)
    ref_pairs = binning.sorted_pairs(gd, frames, cfg)
    n_tiles = cfg.tiles_x * cfg.tiles_y
    np.testing.assert_array_equal(lists["pair_key"], (ref_pairs["frame"] * n_tiles + ref_pairs["tile"]).astype(np.uint32))
    np.testing.assert_array_equal(lists["pair_item"], (ref_pairs["frame"] * g.n + ref_pairs["index"]).astype(np.uint32))
    ref = oref.render(gd, frames, cfg)
    ok = ~ref["flagged"]
    for k in ("rgb", "quad", "depth", "T_final"):
        assert_images_close(res[k], ref[k], ok, f"offsets/{k}")
    up = mask_upstream(scenes.upstream_grads(len(frames), cfg, seed=5), ok)
    ref_b = oref.render(gd, frames, cfg, upstream=up)
    res_b = run_gpu(gd, frames, cfg, upstream=up)
    for k, r in ref_b["grads"].items():
        assert_grads_close(res_b["grads"][k], r, f"offsets/{k}")


def test_network_offsets_compose_with_the_rasterizer_under_autograd():
    # a loss on the rendered images back-propagates through the rasterizer's
    # per-frame offsets into the network (one torch graph), and the result
    # equals the two library backwards called by hand
    from paper_2505_05356_amd import raster
    g = scenes.draw_gaussians(800, 48, 32, 45.0, 45.0, seed=21)
    frames = scenes.identity_frames([0.0, 0.1], 48, 32, 45.0, 45.0, 4, bg_seed=3)
    cfg = scenes.RenderConfig(width=48, height=32, tile_w=16, tile_h=16)
    theta = torch.from_numpy(scenes.mlp_params(seed=9, last_std=0.02, bias_std=0.05)).cuda()
    net = deform.DeformNet(g.n, 2, pos_scale=SX, time_scale=ST)
    params = raster.to_device_params(g, "cuda")
    times = [fr.time for fr in frames]
    theta.requires_grad_(True)
    params["mean"].requires_grad_(True)
    delta = deform.offsets(net, theta, params["mean"], times)
    out = raster.render(dict(params, delta=delta), frames, cfg)
    up = {k: torch.from_numpy(v).cuda() for k, v in scenes.upstream_grads(2, cfg, seed=4).items()}
    loss = (out["rgb"] * up["rgb"]).sum() + (out["quad"] * up["quad"]).sum() + (out["depth"] * up["depth"]).sum()
    loss.backward()
    g_theta, g_mean = theta.grad.clone(), params["mean"].grad.clone()
    # by hand: rasterizer backward -> d delta -> network backward
    fdev = raster.pack_frames(frames, cfg)
    p2 = {k: (v.detach() if v is not None else None) for k, v in params.items()}
    d_fixed = net.forward(theta.detach(), p2["mean"], times)
    p2["delta"] = d_fixed
    ws = raster.Workspace(g.n, 2, cfg)
    o2 = raster.forward(p2, fdev, cfg, ws)
    gr = raster.backward(p2, fdev, cfg, ws, o2, up["rgb"], up["quad"], up["depth"])
    net.forward(theta.detach(), p2["mean"], times)
    d_params, d_x0 = net.backward(theta.detach(), p2["mean"], times, gr["delta"])
    torch.cuda.synchronize()
    assert_grads_close(g_theta.cpu().numpy(), d_params.cpu().numpy(), "autograd/params", rtol=1e-4)
    assert_grads_close(g_mean.cpu().numpy(), (gr["mean"] + d_x0).cpu().numpy(), "autograd/mean", rtol=1e-4)


def test_eq7_blend_of_network_offsets_matches_oracle():
    # two asynchronous quartets (8 raw frames) between three integer
    # timesteps: per-frame offsets and their transpose against the oracle
    from paper_2505_05356_amd import raster
    n = 1000
    rng = np.random.default_rng(11)
    steps = rng.normal(0, 0.02, (3, 3, n)).astype(np.float32)
    base = scenes.identity_frames([0.0], 32, 32, 30.0, 30.0, 4)[0]
    frames = scenes.async_quartet_frames(2, 0.1, base)
    anchors = [(k // 4, k // 4 + 1) for k in range(8)]
    cfg = scenes.RenderConfig(width=32, height=32)
    fdev = raster.pack_frames(frames, cfg)
    out = deform.blend(torch.from_numpy(steps).cuda(), fdev, anchors)
    ref = omlp.blend_offsets(steps, frames, anchors)
    up = rng.normal(size=ref.shape).astype(np.float32)
    back = deform.blend_backward(torch.from_numpy(up).cuda(), fdev, anchors, 3)
    ref_b = omlp.blend_offsets_backward(up, frames, anchors, 3)
    torch.cuda.synchronize()
    # float32 error of w1 a + w2 b is relative to |w1 a| + |w2 b| (the weights
    # are in [0, 1]), not to the possibly cancelled result
    scale = omlp.blend_offsets(np.abs(steps), frames, anchors)
    assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-6 * scale + 1e-12)
    scale_b = omlp.blend_offsets_backward(np.abs(up), frames, anchors, 3)
    assert np.all(np.abs(back.cpu().numpy() - ref_b) <= 1e-6 * scale_b + 1e-12)
    # out-of-range anchors are refused on the host
    with pytest.raises(Exception):
        deform.blend(torch.from_numpy(steps).cuda(), fdev, [(0, 3)] * 8)


def test_mlp_maximum_times_ragged_rows():
    # 64 times (the maximum) x 33 Gaussians = 2112 rows: 16 full blocks and a
    # 64-row tail; offsets and gradients against the oracle
    n, T = 33, 64
    theta = scenes.mlp_params(seed=13, last_std=0.05, bias_std=0.1)
    x0, times = scenes.mlp_rows(n, T, seed=14)
    net = deform.DeformNet(n, T, pos_scale=SX, time_scale=ST)
    p, x = torch.from_numpy(theta).cuda(), torch.from_numpy(x0).cuda()
    delta = net.forward(p, x, times)
    ref = omlp.offsets(theta, x0, times, SX, ST, decide="bf16")
    up = np.random.default_rng(15).normal(size=ref.shape).astype(np.float32)
    _use_oracle_decisions(net, *omlp.offsets_decision_table(theta, x0, times, SX, ST), n_times=T)
    d_params, d_x0 = net.backward(p, x, times, torch.from_numpy(up).cuda())
    g_ref, gx_ref, gx_terms = omlp.offsets_backward(theta, x0, times, SX, ST, up, decide="bf16",
                                                    terms=True)
    torch.cuda.synchronize()
    assert_grads_close(delta.cpu().numpy(), ref, "delta@64 times", rtol=MLP_RTOL)
    _per_layer(d_params.cpu().numpy(), "d_params@64 times", g_ref)
    _centre_close(d_x0.cpu().numpy(), gx_ref, gx_terms, "d_x0@64 times")
    with pytest.raises(ValueError):
        net.forward(p, x, np.zeros(65, np.float32))


def test_eq7_blend_maximum_frames():
    # 256 frames (the maximum) between 65 timesteps, every frame its own
    # fraction of the step; the transpose sums up to 8 frames per step
    from paper_2505_05356_amd import raster
    n, S, F = 70, 65, 256
    rng = np.random.default_rng(16)
    steps = rng.normal(0, 0.02, (S, 3, n)).astype(np.float32)
    base = scenes.identity_frames([0.0], 16, 16, 15.0, 15.0, 4)[0]
    frames, anchors = [], []
    for f in range(F):
        i, j = divmod(f, 4)
        frames.append(dataclasses.replace(base, time=float(np.float32(0.1 * (i + j / 4))),
                                          t_lo=float(np.float32(0.1 * i)),
                                          t_hi=float(np.float32(0.1 * (i + 1)))))
        anchors.append((i, i + 1))
    cfg = scenes.RenderConfig(width=16, height=16)
    fdev = raster.pack_frames(frames, cfg)
    out = deform.blend(torch.from_numpy(steps).cuda(), fdev, anchors)
    up = rng.normal(size=(F, 3, n)).astype(np.float32)
    back = deform.blend_backward(torch.from_numpy(up).cuda(), fdev, anchors, S)
    ref = omlp.blend_offsets(steps, frames, anchors)
    ref_b = omlp.blend_offsets_backward(up, frames, anchors, S)
    torch.cuda.synchronize()
    assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-6 * omlp.blend_offsets(np.abs(steps), frames, anchors) + 1e-12)
    assert np.all(np.abs(back.cpu().numpy() - ref_b)
                  <= 1e-6 * omlp.blend_offsets_backward(np.abs(up), frames, anchors, S) + 1e-12)
    with pytest.raises(Exception):
        deform.blend(torch.from_numpy(steps).cuda(), raster.pack_frames(frames + frames[:1], cfg),
                     anchors + anchors[:1])


def test_render_offsets_with_quartets_and_spherical_harmonics():
    # the optional paths together: per-frame offsets blended between integer
    # timesteps (Eq. 7), asynchronous quartets and degree-2 harmonics; tile
    # lists bit-exact, images and every gradient against the oracle
    g = scenes.draw_gaussians(1200, 48, 40, 45.0, 45.0, seed=17, dynamic=True)
    g = scenes.with_sh(g, 2, seed=17)
    base = scenes.identity_frames([0.0], 48, 40, 45.0, 45.0, 4, bg_seed=5)[0]
    frames = scenes.async_quartet_frames(1, 0.1, base)
    cfg = scenes.RenderConfig(width=48, height=40, tile_w=16, tile_h=16)
    theta = scenes.mlp_params(seed=18, last_std=0.02, bias_std=0.05)
    steps = omlp.offsets(theta, g.mean, [0.0, 0.1], SX, ST)
    delta = omlp.blend_offsets(steps, frames, [(0, 1)] * 4).astype(np.float32)
    gd = dataclasses.replace(g, delta=np.ascontiguousarray(delta))
    res = run_gpu(gd, frames, cfg)
    lists = gpu_lists(res, gd, frames, cfg)
    ref_pairs = binning.sorted_pairs(gd, frames, cfg)
    n_tiles = cfg.tiles_x * cfg.tiles_y
    np.testing.assert_array_equal(lists["pair_key"], (ref_pairs["frame"] * n_tiles + ref_pairs["tile"]).astype(np.uint32))
    np.testing.assert_array_equal(lists["pair_item"], (ref_pairs["frame"] * g.n + ref_pairs["index"]).astype(np.uint32))
    ref = oref.render(gd, frames, cfg)
    ok = ~ref["flagged"]
    for k in ("rgb", "depth", "T_final"):
        assert_images_close(res[k], ref[k], ok, f"combined/{k}")
    ch = np.array([fr.quad_mask.bit_length() - 1 for fr in frames])
    assert_images_close(res["quad"][np.arange(4), ch], ref["quad"][np.arange(4), ch], ok, "combined/quad")
    up = mask_upstream(scenes.upstream_grads(4, cfg, seed=6), ok)
    up_ref = dict(up)
    qmask = np.zeros_like(up["quad"])
    qmask[np.arange(4), ch] = 1.0
    up_ref["quad"] = up["quad"] * qmask
    ref_b = oref.render(gd, frames, cfg, upstream=up_ref)
    res_b = run_gpu(gd, frames, cfg, upstream=up)
    for k, r in ref_b["grads"].items():
        assert_grads_close(res_b["grads"][k], r, f"combined/{k}")


def _net_step(seed=3, decay_steps=4):
    # the optimisation step's scene with a deformation network: frames 0 and 1
    # of a 6-frame sequence, step-0 backgrounds, network weights of moderate size
    from paper_2505_05356_amd import raster, step as gstep
    from tests.test_gpu_optim import _train_setup
    g, cfg, seq, tr, tq, bg = _train_setup(seed=seed)
    theta = scenes.mlp_params(seed=seed + 20, last_std=0.02, bias_std=0.05)
    net = deform.DeformNet(g.n, 2, pos_scale=SX, time_scale=ST)
    params = raster.to_device_params(g, "cuda", static=False)
    ts = gstep.TrainStep(params, raster.pack_frames(seq, cfg), torch.from_numpy(tr).cuda(),
                         torch.from_numpy(tq).cuda(), cfg, batch=2, bg_table=torch.from_numpy(bg).cuda(),
                         net=net, net_params=torch.from_numpy(theta).cuda(), net_decay_steps=decay_steps)
    return ts, g, cfg, seq, tr, tq, bg, theta


def test_train_step_with_network():
    # one optimisation step with the network in the loop: the offsets at the
    # frames' device times and the loss against the oracle; the gradients
    # against the same chain called by hand through the separately checked
    # entry points (network at host times, rasterizer forward/backward); the
    # network's Adam update against the oracle's Adam
    from oracle import optim as ooptim
    from paper_2505_05356_amd import raster
    ts, g, cfg, seq, tr, tq, bg, theta = _net_step()
    p0 = {k: v.clone() for k, v in ts.params.items() if v is not None}
    th0 = ts.net_params.clone()
    ts.step()
    torch.cuda.synchronize()
    assert ts.step_counter.item() == 1
    times = [seq[0].time, seq[1].time]
    ref_delta = omlp.offsets(theta, g.mean, times, SX, ST, decide="bf16")
    assert np.abs(ref_delta).max() > 1e-3
    _close(ts.delta.cpu().numpy(), ref_delta, "step/delta")
    # loss: the oracle renders with its own offsets; the GPU's offsets differ
    # by the network's bfloat16 error, which moves the loss by at most
    # sum |d loss / d delta| |delta_gpu - delta_ref| to first order
    frames = [dataclasses.replace(seq[b], bg_rgb=bg[0, b, :3], bg_quad=bg[0, b, 3:].reshape(1, 4))
              for b in range(2)]
    gd = dataclasses.replace(g, delta=np.ascontiguousarray(ref_delta.astype(np.float32)))
    out = oref.render(gd, frames, cfg)
    loss_ref, d_rgb, d_quad = ooptim.l2_loss_grad(out["rgb"], out["quad"], tr[:2], tq[:2], 1.0)
    ref_b = oref.render(gd, frames, cfg, upstream={"rgb": d_rgb, "quad": d_quad, "depth": np.zeros((2, 32, 40))})
    first = np.sum(np.abs(ref_b["grads"]["delta"]) * np.abs(ts.delta.cpu().numpy() - ref_delta))
    assert abs(ts.loss.item() - loss_ref) <= 2.0 * first + 1e-4 * loss_ref
    # the chain by hand on the step's own frames and loss gradients
    fdev = ts.frames
    d_fixed = ts.net.forward(th0, p0["mean"], times)
    np.testing.assert_array_equal(d_fixed.cpu().numpy(), ts.delta.cpu().numpy())
    p_in = dict(p0, delta=d_fixed)
    ws = raster.Workspace(g.n, 2, cfg)
    o2 = raster.forward(p_in, fdev, cfg, ws)
    for k in ("rgb", "quad"):
        np.testing.assert_allclose(o2[k].cpu().numpy(), ts.out[k].cpu().numpy(), rtol=1e-6, atol=1e-7)
    gr = raster.backward(p_in, fdev, cfg, ws, o2, ts.d_rgb, ts.d_quad, None)
    ts.net.forward(th0, p0["mean"], times)
    d_params, d_x0 = ts.net.backward(th0, p0["mean"], times, gr["delta"])
    torch.cuda.synchronize()
    assert_grads_close(ts.net_grad.cpu().numpy(), d_params.cpu().numpy(), "step/net grad", rtol=1e-4)
    assert_grads_close(ts.grads["mean"].cpu().numpy(), (gr["mean"] + d_x0).cpu().numpy(), "step/mean", rtol=1e-4)
    for k in ("vel", "scale", "opacity_logit", "rgb", "albedo"):
        assert_grads_close(ts.grads[k].cpu().numpy(), gr[k].cpu().numpy(), f"step/{k}", rtol=1e-4)
    # the network's Adam group: first step at the undecayed rate
    gk = ts.net_grad.cpu().numpy().astype(np.float64)
    exp, _, _ = ooptim.adam_step(theta, gk, np.zeros_like(gk), np.zeros_like(gk), 1,
                                 ooptim.decayed_lr(8e-4, 1.6e-6, 4, 1))
    np.testing.assert_allclose(ts.net_params.cpu().numpy(), exp, rtol=1e-6, atol=8e-4 * 1e-4)


def test_train_step_with_network_graph_replay():
    # the step with the network captured as one graph and replayed: equal to
    # eager steps (up to the rasterizer's atomic summation order), the
    # network's rate decaying from the device step counter
    eager = _net_step(seed=5)[0]
    graph = _net_step(seed=5)[0]
    graph.capture()
    from oracle import optim as ooptim
    for it in range(4):
        eager.step()
        graph.replay()
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()
        assert graph.step_counter.item() == eager.step_counter.item() == it + 1
        assert graph.loss.item() == pytest.approx(eager.loss.item(), rel=1e-5)
        assert_grads_close(graph.net_grad.cpu().numpy(), eager.net_grad.cpu().numpy(),
                           f"replay {it} net grad", rtol=1e-4)
        assert_grads_close(graph.grads["mean"].cpu().numpy(), eager.grads["mean"].cpu().numpy(),
                           f"replay {it} mean grad", rtol=1e-4)
        # an entry whose gradient sits at rounding level may move by up to 2 lr
        a, b = eager.net_params.cpu().numpy(), graph.net_params.cpu().numpy()
        bound = sum(2.01 * ooptim.decayed_lr(8e-4, 1.6e-6, 4, s) for s in range(1, it + 2))
        assert np.abs(a - b).max() <= bound
        close = np.abs(a - b) <= 1e-5 * np.abs(a) + 1e-7
        assert close.mean() >= 0.999, close.mean()
        np.testing.assert_array_equal(graph.frames.cpu().numpy(), eager.frames.cpu().numpy())
    assert not graph.status()["overflow"]


def test_mlp_decisions_round_trip():
    # decisions written with gftorf_mlp_set_decisions read back unchanged
    # (900 rows: a ragged last block), and the forward's own decisions are
    # the oracle's within the margin
    n, times = 300, [0.0, 0.1, 0.25]
    theta, x0, times = _net_inputs(n, times, seed=16)
    net = deform.DeformNet(n, len(times), pos_scale=SX, time_scale=ST)
    net.forward(torch.from_numpy(theta).cuda(), torch.from_numpy(x0).cuda(), times)
    masks, ratio = omlp.offsets_decision_table(theta, x0, times, SX, ST)
    got = net.decisions(len(times)).cpu().numpy() != 0
    assert np.all(ratio[got != masks] <= omlp.DECISION_MARGIN)
    rnd = np.random.default_rng(17).integers(0, 2, masks.shape).astype(np.uint8)
    net.set_decisions(torch.from_numpy(rnd).cuda())
    np.testing.assert_array_equal(net.decisions(len(times)).cpu().numpy(), rnd)
