"""Optimisation-step kernels (loss, Adam, frame selection) and the graph-captured
step, against the FP64 oracle (needs an MI355X)."""
import ctypes
import dataclasses

import numpy as np
import pytest
import torch

import scenes
from oracle import optim as ooptim, render as oref
from paper_2505_05356_amd import _lib, raster, step as gstep

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# 16-byte path; one-float path; 16-byte path over several unrolled rounds and a ragged tail
@pytest.mark.parametrize("E", [4 * 33 * 29, 3 * 33 * 29 + 1, 4 * 300_007])
def test_l2_loss_matches_oracle(E):
    lib = _lib.load()
    rng = np.random.default_rng(0)
    F, S = 3, 7
    pred = rng.normal(size=(F, E)).astype(np.float32)
    tgt = rng.normal(size=(S, E)).astype(np.float32)
    idx = np.array([5, 0, 3], np.int32)
    d_pred, d_tgt, d_idx = (torch.from_numpy(a).cuda() for a in (pred, tgt, idx))
    grad = torch.empty_like(d_pred)
    loss = torch.zeros(1, device="cuda")
    _lib.check(lib.gftorf_l2_loss_grad(_p(d_pred), _p(d_tgt), _p(d_idx), F, E, 2.5, _p(grad),
                                       _p(loss), _s()))
    torch.cuda.synchronize()
    # the quad term of the oracle loss alone (zero-size RGB term contributes 0)
    ref_loss, _, ref_grad = ooptim.l2_loss_grad(np.zeros((1,)), pred, np.zeros((1,)), tgt[idx],
                                                quad_weight=2.5)
    assert loss.item() == pytest.approx(ref_loss, rel=1e-5)
    np.testing.assert_allclose(grad.cpu().numpy(), ref_grad, rtol=1e-5, atol=1e-12)


def _offset(n, misalign):
    """A zeroed device vector of n floats, 4 bytes past a 16-byte boundary
    when misalign is set (the kernel then takes its one-float path)."""
    return torch.zeros(n + 1, device="cuda")[1:] if misalign else torch.zeros(n, device="cuda")


def test_adam_matches_oracle():
    # Adam isolated from gradient noise: the GPU update equals FP64 Adam
    # applied to the same gradients (two steps, three groups: whole 4096-element
    # chunks with a ragged tail, a group shorter than a chunk, and a group of
    # several chunks whose arrays are not 16-byte aligned)
    lib = _lib.load()
    rng = np.random.default_rng(1)
    sizes, lrs, misalign = (10003, 37, 9000), (1e-3, 1.6e-4, 5e-4), (False, False, True)
    G = len(sizes)
    p = [rng.normal(size=n).astype(np.float32) for n in sizes]
    gs = [[rng.normal(size=n).astype(np.float32) * 1e-2 for n in sizes] for _ in range(2)]
    dp = [_offset(n, ma) for n, ma in zip(sizes, misalign)]
    for i in range(G):
        dp[i].copy_(torch.from_numpy(p[i]))
    dm = [_offset(n, ma) for n, ma in zip(sizes, misalign)]
    dv = [_offset(n, ma) for n, ma in zip(sizes, misalign)]
    dg = [_offset(n, ma) for n, ma in zip(sizes, misalign)]
    assert dp[2].data_ptr() % 16 != 0 and dp[0].data_ptr() % 16 == 0
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    groups = (_lib.AdamGroupC * G)()
    for i in range(G):
        groups[i].param, groups[i].grad = dp[i].data_ptr(), dg[i].data_ptr()
        groups[i].m, groups[i].v = dm[i].data_ptr(), dv[i].data_ptr()
        groups[i].n, groups[i].lr = sizes[i], lrs[i]
    ref = [(a.astype(np.float64), np.zeros(len(a)), np.zeros(len(a))) for a in p]
    for t in range(2):
        for i in range(G):
            dg[i].copy_(torch.from_numpy(gs[t][i]))
        _lib.check(lib.gftorf_adam_step(groups, G, _p(step), 0.9, 0.999, 1e-15, _s()))
        ref = [ooptim.adam_step(r[0], gs[t][i], r[1], r[2], t + 1, lrs[i]) for i, r in enumerate(ref)]
        torch.cuda.synchronize()
        for i in range(G):
            # the parameters live in float32, so every step rounds them by up
            # to half a unit in the last place: the measured update carries
            # (t + 1) / 2 ulp(p) beyond the float32 arithmetic of the update
            got = dp[i].cpu().numpy()
            upd = got.astype(np.float64) - p[i]
            exp = ref[i][0] - p[i]
            ulp = np.spacing(np.maximum(np.abs(got), np.abs(p[i]))).astype(np.float64)
            bound = 2e-4 * np.abs(exp) + 0.5 * (t + 1) * ulp
            assert np.all(np.abs(upd - exp) <= bound), np.max(np.abs(upd - exp) - bound)
    assert step.item() == 2


def test_select_frames_from_step_counter():
    lib = _lib.load()
    cfg = scenes.RenderConfig(width=16, height=16)
    seq = scenes.identity_frames([0.1 * i for i in range(10)], 16, 16, 20.0, 20.0, 4)
    seq_dev = raster.pack_frames(seq, cfg)
    B, n_bg = 4, 3
    table = torch.arange(n_bg * B * 7, dtype=torch.float32, device="cuda").reshape(n_bg, B, 7)
    frames = torch.empty((B, _lib.FRAME_FLOATS), device="cuda")
    idx = torch.empty(B, dtype=torch.int32, device="cuda")
    for s in (0, 1, 2, 7):
        step = torch.full((1,), s, dtype=torch.int32, device="cuda")
        _lib.check(lib.gftorf_select_frames(_p(frames), B, _p(seq_dev), 10, _p(table), n_bg, 4,
                                            _p(step), _p(idx), _s()))
        torch.cuda.synchronize()
        exp = [(B * s + b) % 10 for b in range(B)]
        assert idx.cpu().tolist() == exp
        f = frames.cpu().numpy()
        for b in range(B):
            np.testing.assert_array_equal(f[b, :17], seq_dev[exp[b]].cpu().numpy()[:17])
            np.testing.assert_array_equal(f[b, 17:24], table[s % n_bg, b].cpu().numpy())


def _train_setup(seed=3, sh_degree=None, n=30):
    wl = scenes.tiny_scene(n, 40, 32, seed=seed, dynamic=True)
    g = wl.gaussians
    g.opacity_logit[:] = np.clip(g.opacity_logit, -2.0, 1.5)
    if sh_degree is not None:
        g = scenes.with_sh(g, sh_degree, seed=seed)
    cfg = dataclasses.replace(wl.cfg, tile_w=8, tile_h=8).strict()
    seq = scenes.frames_for_times([0.05 * i for i in range(6)], wl)
    rng = np.random.default_rng(seed)
    tr = rng.uniform(0, 1, (6, 3, 32, 40)).astype(np.float32)
    tq = rng.normal(0, 0.05, (6, 4, 32, 40)).astype(np.float32)
    bg = rng.uniform(-1, 1, (3, 2, 7)).astype(np.float32)
    return g, cfg, seq, tr, tq, bg


def _make_step(g, cfg, seq, tr, tq, bg):
    params = raster.to_device_params(g, "cuda", static=False)
    return gstep.TrainStep(params, raster.pack_frames(seq, cfg), torch.from_numpy(tr).cuda(),
                           torch.from_numpy(tq).cuda(), cfg, batch=2,
                           bg_table=torch.from_numpy(bg).cuda(), quad_weight=1.0)


@pytest.mark.parametrize("sh_degree", [None, 2])
def test_train_step_matches_oracle(sh_degree):
    g, cfg, seq, tr, tq, bg = _train_setup(sh_degree=sh_degree)
    ts = _make_step(g, cfg, seq, tr, tq, bg)
    p0 = {k: v.cpu().numpy().copy() for k, v in ts.params.items()}
    ts.step()
    torch.cuda.synchronize()
    assert ts.step_counter.item() == 1
    # the oracle: frames 0, 1 with the step-0 backgrounds, L2 loss gradients
    frames = [dataclasses.replace(seq[b], bg_rgb=bg[0, b, :3], bg_quad=bg[0, b, 3:].reshape(1, 4))
              for b in range(2)]
    out = oref.render(g, frames, cfg)
    loss_ref, d_rgb, d_quad = ooptim.l2_loss_grad(out["rgb"], out["quad"], tr[:2], tq[:2], 1.0)
    up = {"rgb": d_rgb, "quad": d_quad, "depth": np.zeros((2, 32, 40))}
    ref = oref.render(g, frames, cfg, upstream=up)
    assert ts.loss.item() == pytest.approx(loss_ref, rel=1e-4)
    from tests.gpu_common import assert_grads_close
    for k, r in ref["grads"].items():
        assert_grads_close(ts.grads[k].cpu().numpy(), r, f"step/{k}")
    # Adam applied to the GPU's own gradients (first step: -lr g / (|g| + eps))
    for k, lr in gstep.DEFAULT_LR.items():
        if ts.grads.get(k) is None:
            continue
        gk = ts.grads[k].cpu().numpy().astype(np.float64)
        exp, _, _ = ooptim.adam_step(p0[k], gk, np.zeros_like(gk), np.zeros_like(gk), 1, lr)
        np.testing.assert_allclose(ts.params[k].cpu().numpy(), exp, rtol=1e-6, atol=lr * 1e-4)


@pytest.mark.parametrize("n", [30, 5000])
def test_graph_replay_equals_eager(n):
    # n = 5000: three sort tiles per frame, so the replayed one-launch sort
    # passes wait on earlier tiles (their counters cleared inside the graph)
    g, cfg, seq, tr, tq, bg = _train_setup(seed=5, n=n)
    eager = _make_step(g, cfg, seq, tr, tq, bg)
    graph = _make_step(g, cfg, seq, tr, tq, bg)
    graph.capture()
    for it in range(3):
        eager.step()
        graph.replay()
        torch.cuda.synchronize()
        # eager work between replays
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()
        assert graph.step_counter.item() == eager.step_counter.item() == it + 1
        assert graph.loss.item() == pytest.approx(eager.loss.item(), rel=1e-5)
        from tests.gpu_common import assert_grads_close
        for k in scenes.Gaussians.FIELDS:
            assert_grads_close(graph.grads[k].cpu().numpy(), eager.grads[k].cpu().numpy(),
                               f"replay {it} grad {k}", rtol=1e-4)
            # the gradients differ only in float32 summation order (atomics);
            # Adam normalises, so an entry whose gradient is at rounding level
            # may move by up to 2 lr per step
            a, b = eager.params[k].cpu().numpy(), graph.params[k].cpu().numpy()
            lr = gstep.DEFAULT_LR[k]
            assert np.abs(a - b).max() <= 2.01 * lr * (it + 1), k
            close = np.abs(a - b) <= 1e-5 * np.abs(a) + 1e-7
            assert close.mean() >= 0.999, (k, close.mean())
    assert not graph.status()["overflow"]


def test_adam_with_learning_rate_decay():
    # §4's exponential decay computed on the device from the step counter: a
    # decaying group and a constant one, at steps inside and past the horizon
    lib = _lib.load()
    rng = np.random.default_rng(4)
    n = 500
    for t_new, S in ((3, 4), (9, 4)):
        p0 = rng.normal(size=(2, n)).astype(np.float32)
        g = rng.normal(size=(2, n)).astype(np.float32) * 1e-2
        dp = [torch.from_numpy(p0[i].copy()).cuda() for i in range(2)]
        dg = [torch.from_numpy(g[i]).cuda() for i in range(2)]
        dm = [torch.zeros(n, device="cuda") for _ in range(2)]
        dv = [torch.zeros(n, device="cuda") for _ in range(2)]
        groups = (_lib.AdamGroupC * 2)()
        for i in range(2):
            groups[i].param, groups[i].grad = dp[i].data_ptr(), dg[i].data_ptr()
            groups[i].m, groups[i].v = dm[i].data_ptr(), dv[i].data_ptr()
            groups[i].n, groups[i].lr = n, 8e-4
        groups[0].lr_final, groups[0].decay_steps = 8e-6, S
        step = torch.full((1,), t_new - 1, dtype=torch.int32, device="cuda")
        _lib.check(lib.gftorf_adam_step(groups, 2, _p(step), 0.9, 0.999, 1e-15, _s()))
        torch.cuda.synchronize()
        assert step.item() == t_new
        for i in range(2):
            lr = ooptim.decayed_lr(8e-4, 8e-6, S, t_new) if i == 0 else 8e-4
            exp, _, _ = ooptim.adam_step(p0[i], g[i], np.zeros(n), np.zeros(n), t_new, lr)
            got = dp[i].cpu().numpy().astype(np.float64)
            ulp = np.spacing(np.abs(p0[i])).astype(np.float64)
            assert np.all(np.abs((got - p0[i]) - (exp - p0[i])) <= 1e-4 * np.abs(exp - p0[i]) + ulp), (t_new, i)
    bad = (_lib.AdamGroupC * 1)()
    bad[0].n, bad[0].lr, bad[0].decay_steps = 0, 0.0, 5
    assert lib.gftorf_adam_step(bad, 1, _p(torch.zeros(1, dtype=torch.int32, device="cuda")),
                                0.9, 0.999, 1e-15, _s()) == _lib.EINVAL
