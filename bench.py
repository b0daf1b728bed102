#!/usr/bin/env python3
"""Forward + backward frames/s of the C-ToF Gaussian rasterizer on one GPU.

Workload (default): dynamic scene of 200,000 Gaussians (linear + quadratic
trajectories, constant rotation rate), 8 time frames at t in [0, 0.25 s],
640x480, fx = fy = 525, 30 MHz, RGB + 4 raw quads + depth, upstream gradient
N(0, 1) on every output element.  A step is one forward + backward of all 8
frames.  Two paths are timed on the same inputs, already resident in HBM:
  batched   -- one gftorf_render_fwd / gftorf_render_bwd call for all frames;
  per-frame -- the same library called with n_frames = 1 for each frame, with
               the per-frame parameter gradients summed.
`value` is the batched frames/s.  A second timed region of the same steps
records HIP events around every kernel (gftorf_profile_*) for the roofline of
the dominant kernel; the FP64 CPU oracle is timed on a bounded tile sample.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed-FP32 instructions (the kernels are built with
# them disabled): 256 CUs x 64 lanes x 2 FLOP (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12

# Algorithmic work per unit, NF = 1 (the FLOP that the method's arithmetic
# needs per evaluated and per composited (pixel, Gaussian) pair):
#   alpha evaluation: dx, dy (4 sub), quadratic form (3 mul + 2 fma), exp2, o*G  -> 12
#   forward composite: 1 - a, T(1 - a), w1, w2 (4) + 6 FMA (rgb 3, depth 1, S, C) -> 16
#   backward composite: T / (1 - a), S2 terms for rgb and depth (16), S3 terms (11),
#     background term (3), weights (2), per-Gaussian colour / depth / phasor grads (6),
#     accumulator updates (20), chain to o, conic, centre (17), field sums (12)    -> 87
FLOP_PER_EVAL = 12
FWD_FLOP_PER_COMP = 16
BWD_FLOP_PER_COMP = 87
SORT_BYTES_PER_KEY_PASS = 16  # read key + value, write key + value (4 B each)

# HBM traffic per launch from rocprofv3 counter runs of this script
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same
# counter reads for a plain device copy of known size (--calibration-copy-mib).
# A figure holds only for the workload and the kernel source it was measured
# on: it is keyed by the workload name of the JSON line and the kernel, and
# the sha256 of the kernel's source files must match; otherwise traffic is null.
FETCH_SCALE, WRITE_SCALE = 1048576 / 524318, 1048576 / 1048576   # 1 GiB copy: FETCH 524318 KiB, WRITE 1048576 KiB
COMPOSITE_FILES = ("paper_2505_05356_amd/csrc/composite.hip", "paper_2505_05356_amd/csrc/common.h")
BIN_FILES = ("paper_2505_05356_amd/csrc/bin.hip", "paper_2505_05356_amd/csrc/common.h")
MLP_FILES = ("paper_2505_05356_amd/csrc/mlp.hip", "paper_2505_05356_amd/csrc/mlp.h")
_COMPOSITE_SHA = "cd6b927c33cc7ddfef92101e8b2c3ebed96655616a2d324514a6c5f5a1bcdb0f"
_BIN_SHA = "30381ced515e4468a2d60342f3df0e581007aa0fb0ac54ed325fcfd08fc4f716"
# {workload: {kernel: (source files, sha256, (FETCH KiB, WRITE KiB) per launch)}};
# k_mlp_dw counts its three launches together
TRAFFIC = {
    "dynamic-200k-gaussians-8f-640x480": {
        "k_composite_bwd": (COMPOSITE_FILES, _COMPOSITE_SHA, (52202, 50919)),
        "k_composite_fwd": (COMPOSITE_FILES, _COMPOSITE_SHA, (5290, 96157)),
        "k_tile_place": (BIN_FILES, _BIN_SHA, (9291, 154473)),
        "k_group_place": (BIN_FILES, _BIN_SHA, (12834, 18412))},
    "dynamic-1000k-1024x768-16f-2freq": {
        "k_composite_bwd": (COMPOSITE_FILES, _COMPOSITE_SHA, (361242, 247936)),
        "k_composite_fwd": (COMPOSITE_FILES, _COMPOSITE_SHA, (19686, 691885)),
        "k_tile_place": (BIN_FILES, _BIN_SHA, (85160, 2046582)),
        "k_group_place": (BIN_FILES, _BIN_SHA, (126590, 198364))},
    "deform-mlp-200k-x8-8x256-pe10": {
        k: (MLP_FILES, "38e594eb67121042452a36773f57beafc9891fcba0d2e72955acb9977e09c681", kib)
        for k, kib in (("k_mlp_fwd", (214120, 7156260)), ("k_mlp_bwd", (368285, 6468750)),
                       ("k_mlp_dw", (6575120, 275395)))},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--tile", default="16x16", help="WxH (8x8, 16x16, 32x8) or auto")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle tile work in the CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-frame", action="store_true")
    ap.add_argument("--workload", default="cfg3",
                    choices=("cfg2", "cfg3", "cfg4", "cfg5", "cfg5net", "mlp", "fwd320", "cfg3sh", "cfg3async"),
                    help="cfg3 (default): the headline batched vs per-frame line; cfg2 / cfg4: the "
                         "same measurement on the static 100k / 1M-Gaussian 16-frame workloads; "
                         "cfg5: the graph-replayed optimisation step; cfg5net: the same step "
                         "with the deformation network's offsets in the loop; mlp: the deformation "
                         "network's forward + backward over (Gaussian, time) rows; fwd320: "
                         "forward-only rendering at 320x240 (cfg2's distributions), the "
                         "resolution of the paper's rendering-rate statement; cfg3sh / cfg3async: "
                         "cfg3's batched fwd+bwd with degree-3 spherical-harmonic colour and "
                         "reflectivity / with the 8 frames as two asynchronous raw quartets (Eq. 7)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after timing, one device-to-device copy of this many MiB (for counter runs)")
    return ap.parse_args()


def bench_train_step(args):
    """Optimisation-step loop: 300k trainable Gaussians fitted to a 60-frame
    sequence rendered by the forward from a seeded ground-truth scene, batch of
    4 frames per step, RGB + quad L2 loss, Adam on every field, one captured
    HIP graph replayed per step.  With --workload cfg5net the deformation
    network (8 x 256, paper initialisation: last layer N(0, 1e-10), zero
    biases) adds its offsets at the batch's times, and the step also runs its
    backward and its Adam group.  Prints one JSON line (steps/s)."""
    import torch

    import scenes
    from paper_2505_05356_amd import deform, raster, step as gstep

    dev = "cuda:0"
    gt, tr, cfg = scenes.cfg5_scenes()
    S = 60
    W, H, f = cfg.width, cfg.height, 525.0
    seq = scenes.identity_frames([i / 30.0 for i in range(S)], W, H, f, f, cfg.n_quad)
    seq_dev = raster.pack_frames(seq, cfg, dev)
    # targets: the ground-truth scene rendered by the forward, 8 frames at a time
    gt_params = raster.to_device_params(gt, dev)
    tgt_rgb = torch.empty((S, 3, H, W), device=dev)
    tgt_quad = torch.empty((S, cfg.n_quad, H, W), device=dev)
    ws = raster.Workspace(gt.n, 8, cfg, device=dev)
    for c0 in range(0, S, 8):
        fr = seq_dev[c0:c0 + 8].contiguous()
        out = raster.forward(gt_params, fr, cfg, ws, check=True)
        tgt_rgb[c0:c0 + fr.shape[0]] = out["rgb"]
        tgt_quad[c0:c0 + fr.shape[0]] = out["quad"]
    del ws, gt_params
    rng = np.random.default_rng(7)
    bg = torch.from_numpy(rng.uniform(-1, 1, (64, 4, 3 + cfg.n_quad)).astype(np.float32)).to(dev)
    params = raster.to_device_params(tr, dev, static=False)
    with_net = args.workload == "cfg5net"
    net_kw = {}
    if with_net:
        # network inputs: centres scaled by 2 f / c, the sequence's times (0 .. 2 s) by 1/2
        net = deform.DeformNet(tr.n, 4, freq_hz=cfg.freqs[0], time_scale=0.5, device=dev)
        theta = torch.from_numpy(scenes.mlp_params(seed=11)).to(dev)
        net_kw = dict(net=net, net_params=theta)
    ts = gstep.TrainStep(params, seq_dev, tgt_rgb, tgt_quad, cfg, batch=4, bg_table=bg, **net_kw)
    ts.size_workspace()
    ts.capture()
    for _ in range(args.warmup):
        ts.replay()
    torch.cuda.synchronize()
    l0 = ts.loss.item()
    t0 = time.perf_counter()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record(ts.stream)
    for _ in range(args.steps):
        ts.replay()
    e_ev.record(ts.stream)
    torch.cuda.synchronize()
    ms = s_ev.elapsed_time(e_ev)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_train(tr, seq, cfg, theta.cpu().numpy() if with_net else None, args.cpu_budget)
    # every replayed forward (capture, warm-up and timed) must have rendered
    # complete tile lists: the status keeps the OR of their overflow flags
    st = ts.status()
    if st["overflow_seen"]:
        raise SystemExit(f"pair capacity overflowed in a replayed step (largest pair count "
                         f"{st['n_pairs_seen']} > capacity {st['max_pairs']}): the timing is invalid")
    line = {
        "metric": ("optimisation steps/s (4-frame batch: deformation network fwd + render fwd + L2 loss + "
                   "render bwd + network bwd + Adam, one HIP graph)" if with_net else
                   "optimisation steps/s (4-frame batch: fwd + L2 loss + bwd + Adam, one HIP graph)"),
        "value": round(args.steps / (ms / 1e3), 2), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded ground-truth scene rendered as targets; no dataset)",
        "config": {"workload": f"train-{tr.n // 1000}k-{S}f-{W}x{H}-batch4" + ("-deform-mlp" if with_net else ""),
                   "n_gaussians": tr.n, "network_rows": 4 * tr.n if with_net else 0,
                   "sequence_frames": S, "batch": 4, "wall_s": round(time.perf_counter() - t0, 3),
                   "loss_after_warmup": l0, "loss_last": ts.loss.item(),
                   "pairs_max": st["n_pairs_seen"], "pair_capacity": st["max_pairs"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)




def source_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(workload, name):
    """Counter-measured HBM bytes per launch of kernel `name` on `workload`,
    or None when there is no measurement of that workload with the kernel
    source as it is now."""
    entry = TRAFFIC.get(workload, {}).get(name)
    if entry is None:
        return None
    files, sha, (fetch, write) = entry
    if source_sha256(files) != sha:
        return None
    return int(round((fetch * FETCH_SCALE + write * WRITE_SCALE) * 1024))


def host_info():
    """CPUs this process may run on (nproc) and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def oracle_threads():
    """Threads the FP64 oracle's numpy / torch-CPU arithmetic may use."""
    import torch
    return max(torch.get_num_threads(), int(os.environ.get("OMP_NUM_THREADS", "1") or 1))


MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bf16 matrix peak


def mlp_flop_per_row(n_in=84, width=256, depth=8, n_out=3):
    """Multiply-adds x 2 of one row through every linear layer (unpadded)."""
    return 2 * (n_in * width + (depth - 1) * width * width + width * n_out)


def mlp_bytes_per_row(width=256, depth=8, k0=96, head_pad=16):
    """HBM bytes per row that each network kernel must move in training mode
    (bfloat16 saved activations h_0 .. h_7 and gradients gz_0 .. gz_8, ReLU
    bits at 2 bytes per row and hidden layer, float32 offsets and centres)."""
    h = 2 * (k0 + (depth - 1) * width) + 2 * width   # h_0 .. h_8 as stored (h_8 feeds the head's dW)
    gz = 2 * (depth * width + head_pad)
    bits = depth * width // 8                         # one ReLU bit per hidden unit and row
    return {"k_mlp_fwd": h + bits + 12 + 12, "k_mlp_bwd": gz + bits + 12 + 12, "k_mlp_dw": gz + h}


def bench_mlp(args):
    """Deformation network (paper §4): forward with saved activations, then the
    backward to every parameter and to the canonical centres, for args.n
    Gaussians at args.frames times.  Prints one JSON line (rows/s)."""
    import torch

    import scenes
    from paper_2505_05356_amd import deform, profile

    n, T = args.n, args.frames
    theta = torch.from_numpy(scenes.mlp_params(seed=0)).cuda()
    x0_np, times = scenes.mlp_rows(n, T, seed=1)
    x0 = torch.from_numpy(x0_np).cuda()
    times = [float(t) for t in times]
    net = deform.DeformNet(n, T, time_scale=4.0)
    delta = torch.empty((T, 3, n), device="cuda")
    up = torch.randn((T, 3, n), device="cuda")
    d_params = torch.empty(net.n_params, device="cuda")

    def step():
        net.forward(theta, x0, times, out=delta)
        net.backward(theta, x0, times, up, d_params=d_params)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(args.steps):
        step()
    e_ev.record()
    torch.cuda.synchronize()
    ms = s_ev.elapsed_time(e_ev) / args.steps
    with profile.KernelTimer(max_launches=16 * args.steps + 16) as kt:
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
    kern = {k: v[1] / max(v[0], 1) for k, v in kt.totals.items()}
    rows = n * T
    flop = rows * mlp_flop_per_row()
    per_kernel = {}
    bpr = mlp_bytes_per_row()
    for k in ("k_mlp_fwd", "k_mlp_bwd", "k_mlp_dw"):
        if k in kern:
            tf = flop / (kern[k] / 1e3) / 1e12
            nbytes = rows * bpr[k]
            gbs = nbytes / (kern[k] / 1e3) / 1e9
            # the binding roofline: the larger of the two ideal times
            bound = "hbm" if nbytes / (HBM_PEAK_GBS * 1e9) > flop / (MFMA_BF16_PEAK_TFLOPS * 1e12) else "mfma"
            per_kernel[k] = dict(avg_ms=round(kern[k], 4), tflops=round(tf, 1),
                                 frac=round(tf / MFMA_BF16_PEAK_TFLOPS, 4), hbm_gbs=round(gbs, 1),
                                 hbm_frac=round(gbs / HBM_PEAK_GBS, 4), bound=bound)
    dominant = max(per_kernel, key=lambda k: per_kernel[k]["avg_ms"])
    pk = per_kernel[dominant]
    traffic = traffic_bytes(f"deform-mlp-{n // 1000}k-x{T}-8x256-pe10", dominant)
    if pk["bound"] == "hbm":
        roof = dict(bound="hbm", achieved=pk["hbm_gbs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=pk["hbm_frac"],
                    traffic=traffic, kernel=dominant, avg_ms=pk["avg_ms"],
                    work=f"{rows * bpr[dominant]:.4g} B per launch = {rows} rows x {bpr[dominant]} B "
                         f"(matrix cores: {pk['tflops']} TFLOP/s, {pk['frac']} of the bf16 peak)")
    else:
        roof = dict(bound="mfma", achieved=pk["tflops"], peak=MFMA_BF16_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=pk["frac"], traffic=traffic, kernel=dominant, avg_ms=pk["avg_ms"],
                    work=f"{flop:.4g} FLOP per launch = {rows} rows x {mlp_flop_per_row()} (bf16 products)")
    print("# kernels: " + ", ".join(f"{k} {v * 1e3:.1f}us" for k, v in sorted(kern.items(), key=lambda kv: -kv[1])),
          file=sys.stderr, flush=True)
    if args.calibration_copy_mib > 0:   # a plain copy of known size for counter scaling
        src = torch.ones(args.calibration_copy_mib * 262144, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import mlp as omlp
        R = 512
        rng = np.random.default_rng(0)
        xs, ts = rng.uniform(-0.5, 0.5, (R, 3)), rng.uniform(0, 1, R)
        th = theta.cpu().numpy()
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < min(args.cpu_budget, 10.0) or reps == 0:
            _, cache = omlp.forward(th, xs, ts)
            omlp.backward(th, cache, rng.normal(size=(R, 3)))
            reps += 1
        dt = time.perf_counter() - t0
        cpu = {"value": round(reps * R / dt, 1), "unit": "rows/s", "cores": oracle_threads(),
               "kind": "oracle", "sample": f"{reps} x {R} rows forward + backward (FP64 numpy)",
               **host_info()}
    line = {
        "metric": "deformation MLP fwd+bwd rows/s (200k Gaussians x 8 times)",
        "value": round(rows / (ms / 1e3), 1), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded centres, paper initialisation; no dataset)",
        "config": {"workload": f"deform-mlp-{n // 1000}k-x{T}-8x256-pe10", "rows": rows,
                   "flop_per_step": 3 * flop, "step_tflops": round(3 * flop / (ms / 1e3) / 1e12, 1)},
        "roofline": roof, "kernels": per_kernel,
        "kernels_ms": {k: round(v, 4) for k, v in kern.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_forward_320(args):
    """Forward-only rendering of RGB + 4 quads + depth, one frame per call, at
    320x240 with cfg2's scene distributions: the setting of the paper's
    rendering-rate statement (§5.1).  Prints one JSON line (frames/s)."""
    import torch

    import scenes
    from paper_2505_05356_amd import raster

    wl = scenes.cfg2_320()
    cfg = wl.cfg
    params = raster.to_device_params(wl.gaussians, "cuda")
    fdev = raster.pack_frames(wl.frames, cfg, "cuda")
    ws = raster.Workspace(wl.gaussians.n, 1, cfg, device="cuda")
    out = raster.alloc_outputs(1, cfg, "cuda")
    raster.forward(params, fdev, cfg, ws, out=out, check=True)
    for _ in range(args.warmup):
        raster.forward(params, fdev, cfg, ws, out=out, check=False)
    torch.cuda.synchronize()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(args.steps):
        raster.forward(params, fdev, cfg, ws, out=out, check=False)
    e_ev.record()
    torch.cuda.synchronize()
    ms = s_ev.elapsed_time(e_ev) / args.steps
    st = ws.status()
    line = {
        "metric": "forward-only frames/s at 320x240 (RGB + 4 quads + depth)",
        "value": round(1e3 / ms, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded static scene; no dataset)",
        "config": {"workload": wl.name, "n_gaussians": wl.gaussians.n, "pairs": st["n_pairs"],
                   "paper": "real time at 100+ Hz on an RTX 3090 at 320x240, Gaussian count not stated"},
    }
    print(json.dumps(line), flush=True)


def bench_cfg3_variant(args):
    """cfg3's scene and batched forward + backward of 8 frames, with (cfg3sh)
    spherical-harmonic colour and reflectivity of degree 3 (paper §3), or
    (cfg3async) the 8 frames as two quartets of raw quads taken one offset at
    a time, each rendering only its offset's channel at its own time with the
    centres interpolated between the quartets' timesteps (Eq. 7).  Prints
    one JSON line (frames/s, eager, HIP events)."""
    import torch

    import scenes
    from paper_2505_05356_amd import raster

    wl = scenes.cfg3()
    g, frames, cfg = wl.gaussians, wl.frames, wl.cfg
    if args.workload == "cfg3sh":
        g = scenes.with_sh(g, 3, seed=1)
        desc = "cfg3 with degree-3 spherical harmonics (48 colour + 16 reflectivity coefficients per Gaussian)"
    else:
        frames = scenes.async_quartet_frames(2, 0.125, frames[0])
        desc = "cfg3 as two asynchronous quartets: 8 raw frames at t = (i + j/4) 0.125 s, one quad channel each"
    F = len(frames)
    params = raster.to_device_params(g, "cuda")
    fdev = raster.pack_frames(frames, cfg, "cuda")
    up = scenes.upstream_grads(F, cfg, seed=1)
    d = {k: torch.from_numpy(v).cuda() for k, v in up.items()}
    ws = raster.Workspace(g.n, F, cfg, device="cuda")
    out = raster.alloc_outputs(F, cfg, "cuda")
    raster.forward(params, fdev, cfg, ws, out=out, check=True)
    grads = raster.backward(params, fdev, cfg, ws, out, d["rgb"], d["quad"], d["depth"])

    def step():
        raster.forward(params, fdev, cfg, ws, out=out, check=False)
        raster.backward(params, fdev, cfg, ws, out, d["rgb"], d["quad"], d["depth"], grads=grads)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(args.steps):
        step()
    e_ev.record()
    torch.cuda.synchronize()
    ms = s_ev.elapsed_time(e_ev) / args.steps
    st = ws.status()
    line = {
        "metric": "fwd+bwd frames/s at 640x480, 200k Gaussians (batched, " + args.workload + ")",
        "value": round(F * 1e3 / ms, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded dynamic Gaussian scene; no dataset)",
        "config": {"workload": args.workload, "description": desc, "n_gaussians": g.n, "frames": F,
                   "pairs": st["n_pairs"], "evals_fwd": st["n_evaluated"], "composited": st["n_composited"]},
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import scenes
    from paper_2505_05356_amd import profile, raster

    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.workload in ("cfg5", "cfg5net"):
        return bench_train_step(args)
    if args.workload == "mlp":
        return bench_mlp(args)
    if args.workload == "fwd320":
        return bench_forward_320(args)
    if args.workload in ("cfg3sh", "cfg3async"):
        return bench_cfg3_variant(args)
    if args.workload == "cfg2":
        wl = scenes.cfg2()
    elif args.workload == "cfg4":
        wl = scenes.cfg4()
    else:
        wl = scenes.cfg3(n=args.n, n_frames=args.frames)
    F = len(wl.frames)
    g = wl.gaussians
    params = raster.to_device_params(g, dev)
    up = scenes.upstream_grads(F, wl.cfg, seed=1)
    d = {k: torch.from_numpy(v).to(dev) for k, v in up.items()}
    tile_times = None
    if args.tile == "auto":
        from paper_2505_05356_amd import autotune
        cfg, tile_times = autotune.autotune(params, raster.pack_frames(wl.frames, wl.cfg, dev),
                                            wl.cfg, upstream=d, reps=5, warmup=2)
        args.tile = f"{cfg.tile_w}x{cfg.tile_h}"
        print(f"# autotuned tile {args.tile}: {tile_times}", file=sys.stderr, flush=True)
    else:
        tw, th = (int(x) for x in args.tile.split("x"))
        cfg = dataclasses.replace(wl.cfg, tile_w=tw, tile_h=th)
    fdev = raster.pack_frames(wl.frames, cfg, dev)
    fdev1 = [fdev[f:f + 1].contiguous() for f in range(F)]
    d1 = [{k: v[f:f + 1].contiguous() for k, v in d.items()} for f in range(F)]

    # batched path: size the pair capacity once (one checked forward), then
    # every timed call runs without host synchronisation
    ws = raster.Workspace(g.n, F, cfg, device=dev)
    out = raster.alloc_outputs(F, cfg, dev)
    raster.forward(params, fdev, cfg, ws, out=out, check=True)
    P = ws.status()["n_pairs"]
    flat = torch.zeros(24 * g.n, device=dev)
    sizes = {k: raster._lib.ROWS[k] * g.n for k in raster.FIELDS}
    grads, o = {}, 0
    for k in raster.FIELDS:
        grads[k] = flat[o:o + sizes[k]].view(raster._lib.ROWS[k], g.n) if params[k] is not None else None
        o += sizes[k]

    def step_batched():
        raster.forward(params, fdev, cfg, ws, out=out, check=False)
        raster.backward(params, fdev, cfg, ws, out, d["rgb"], d["quad"], d["depth"], grads=grads)

    # per-frame path: the same entry points with n_frames = 1 (set up only
    # when it is timed, so that a profile of the batched path holds only its calls)
    ws1 = raster.Workspace(g.n, 1, cfg, device=dev)
    out1 = raster.alloc_outputs(1, cfg, dev)
    if not args.no_per_frame:
        for f in range(F):
            raster.forward(params, fdev1[f], cfg, ws1, out=out1, check=True)
    flat1 = torch.zeros_like(flat)
    flat_acc = torch.zeros_like(flat)
    grads1, o = {}, 0
    for k in raster.FIELDS:
        grads1[k] = flat1[o:o + sizes[k]].view(raster._lib.ROWS[k], g.n) if params[k] is not None else None
        o += sizes[k]

    def step_per_frame():
        flat_acc.zero_()
        for f in range(F):
            raster.forward(params, fdev1[f], cfg, ws1, out=out1, check=False)
            raster.backward(params, fdev1[f], cfg, ws1, out1, d1[f]["rgb"], d1[f]["quad"],
                            d1[f]["depth"], grads=grads1)
            flat_acc.add_(flat1)

    def timed(step, k):
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        s.record()
        for _ in range(k):
            step()
        e.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return s.elapsed_time(e), wall

    def median_step(step, k):
        """Median of k single-step times (an event after every step)."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for i in range(k):
            step()
            ev[i + 1].record()
        torch.cuda.synchronize()
        return float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(k)]))

    for _ in range(args.warmup):
        step_batched()
    ms_b, wall_b = timed(step_batched, args.steps)
    st = ws.status()
    assert not st["overflow"], st
    ms_step = ms_b / args.steps
    value = F * args.steps / (ms_b / 1e3)
    print(f"# batched: {ms_step:.3f} ms/step, {value:.1f} frames/s, P={P}", file=sys.stderr, flush=True)

    # the same batched step captured once as a HIP graph and replayed
    import ctypes
    lib = raster._lib.load()
    gstream = torch.cuda.Stream(device=dev)
    gsp = ctypes.c_void_p(gstream.cuda_stream)
    torch.cuda.synchronize()
    gexec = ctypes.c_void_p()
    raster._lib.check(lib.gftorf_graph_begin(gsp))
    try:
        raster.forward(params, fdev, cfg, ws, out=out, check=False, stream=gstream)
        raster.backward(params, fdev, cfg, ws, out, d["rgb"], d["quad"], d["depth"], grads=grads,
                        stream=gstream)
    finally:
        rc = lib.gftorf_graph_end(gsp, ctypes.byref(gexec))
    raster._lib.check(rc)
    for _ in range(args.warmup):
        raster._lib.check(lib.gftorf_graph_launch(gexec, gsp))
    torch.cuda.synchronize()
    gs_ev, ge_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gs_ev.record(gstream)
    for _ in range(args.steps):
        raster._lib.check(lib.gftorf_graph_launch(gexec, gsp))
    ge_ev.record(gstream)
    torch.cuda.synchronize()
    ms_g = gs_ev.elapsed_time(ge_ev) / args.steps
    raster._lib.check(lib.gftorf_graph_destroy(gexec))
    graph_value = F / (ms_g / 1e3)
    print(f"# batched, graph-replayed: {ms_g:.3f} ms/step, {graph_value:.1f} frames/s",
          file=sys.stderr, flush=True)

    med_b = median_step(step_batched, args.steps)
    print(f"# batched, median of {args.steps} steps: {med_b:.3f} ms/step", file=sys.stderr, flush=True)

    per_frame = med_p = None
    if not args.no_per_frame:
        for _ in range(args.warmup):
            step_per_frame()
        ms_p, _ = timed(step_per_frame, args.steps)
        per_frame = F * args.steps / (ms_p / 1e3)
        med_p = median_step(step_per_frame, args.steps)
        print(f"# per-frame: {ms_p / args.steps:.3f} ms/step, {per_frame:.1f} frames/s",
              file=sys.stderr, flush=True)

    # second timed region: per-kernel HIP events around every launch
    with profile.KernelTimer(max_launches=64 * args.steps + 64) as kt:
        for _ in range(args.steps):
            step_batched()
        torch.cuda.synchronize()
    kern = {k: dict(launches=v[0], avg_ms=v[1] / max(v[0], 1), total_ms=v[1])
            for k, v in kt.totals.items()}
    dominant = max(kern, key=lambda k: kern[k]["total_ms"])
    st = ws.status()
    work = dict(P=P, E_fwd=st["n_evaluated"], C=st["n_composited"],
                E_bwd=int(out["n_contrib"].sum().item()))   # backward walks up to n_contrib
    roof = roofline(dominant, kern[dominant]["avg_ms"], **work)
    workload = (wl.name if args.workload != "cfg3" else
                f"dynamic-{g.n // 1000}k-gaussians-{F}f-{cfg.width}x{cfg.height}")
    if args.tile != "16x16":
        workload += f"-{args.tile}"
    roof["traffic"] = traffic_bytes(workload, dominant)
    print("# kernels: " + ", ".join(f"{k} {v['avg_ms']:.3f}ms x{v['launches'] // args.steps}"
                                    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["total_ms"])),
          file=sys.stderr, flush=True)

    if args.calibration_copy_mib > 0:   # a plain copy of known size for counter scaling
        src = torch.ones(args.calibration_copy_mib * 262144, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, cfg, up, args.cpu_budget)

    line = {
        "metric": f"fwd+bwd frames/s at {cfg.width}x{cfg.height}, {g.n // 1000}k Gaussians; "
                  "batched vs per-frame launch",
        "value": round(value, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded dynamic Gaussian scene; no dataset)",
        "config": {"workload": workload, "n_gaussians": g.n, "frames": F, "width": cfg.width, "height": cfg.height,
                   "tile": args.tile, "freqs_hz": list(cfg.freqs), "quads": cfg.n_quad,
                   "outputs": "rgb+quad+depth", "pairs": P, "evals_fwd": work["E_fwd"],
                   "evals_bwd": work["E_bwd"], "composited": work["C"],
                   "tile_times_ms": tile_times},
        "graph_value": round(graph_value, 2),
        "graph_ms_per_step": round(ms_g, 4),
        "per_frame_value": None if per_frame is None else round(per_frame, 2),
        "batched_over_per_frame": None if per_frame is None else round(value / per_frame, 3),
        "median_ms_per_step": round(med_b, 4),
        "median_value": round(F / (med_b / 1e3), 2),
        "per_frame_median_value": None if med_p is None else round(F / (med_p / 1e3), 2),
        "roofline": roof,
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in kern.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_train(g, seq, cfg, theta, budget_s):
    """The FP64 oracle as it stands for one optimisation step of the 4-frame
    batch: forward + backward of one frame on a bounded tile sample
    (cpu_baseline), times 4; the L2 loss and its gradient over the batch and
    Adam over every parameter, timed in full; with the network, its forward +
    backward on a 512-row sample extrapolated to the batch's rows."""
    import scenes
    from oracle import optim as oopt
    wl = scenes.Workload("train", g, list(seq[:1]), cfg)
    frame = cpu_baseline(wl, cfg, scenes.upstream_grads(1, cfg, seed=1), budget_s)
    t_frame = 1.0 / frame["value"]
    rng = np.random.default_rng(0)
    H, W, B = cfg.height, cfg.width, 4
    pr, tr_ = rng.normal(size=(B, 3, H, W)), rng.normal(size=(B, 3, H, W))
    pq, tq = rng.normal(size=(B, cfg.n_quad, H, W)), rng.normal(size=(B, cfg.n_quad, H, W))
    t0 = time.perf_counter()
    oopt.l2_loss_grad(pr, pq, tr_, tq)
    t_loss = time.perf_counter() - t0
    P = 24 * g.n
    p, gr = rng.normal(size=P), rng.normal(size=P)
    t0 = time.perf_counter()
    oopt.adam_step(p, gr, np.zeros(P), np.zeros(P), 1, 1e-3)
    t_adam = time.perf_counter() - t0
    t_net, net_note = 0.0, ""
    if theta is not None:
        from oracle import mlp as omlp
        R = 512
        xs, ts = rng.uniform(-0.5, 0.5, (R, 3)), rng.uniform(0, 1, R)
        t0, reps = time.perf_counter(), 0
        while time.perf_counter() - t0 < min(budget_s, 10.0) or reps == 0:
            _, cache = omlp.forward(theta, xs, ts)
            omlp.backward(theta, cache, rng.normal(size=(R, 3)))
            reps += 1
        t_row = (time.perf_counter() - t0) / (reps * R)
        t0 = time.perf_counter()
        oopt.adam_step(theta, theta, np.zeros_like(theta), np.zeros_like(theta), 1, 1e-3)
        t_net = B * g.n * t_row + time.perf_counter() - t0
        net_note = f" + network fwd+bwd {B * g.n} rows at {t_row * 1e6:.1f} us/row ({reps} x {R}-row sample)"
    per_step = B * t_frame + t_loss + t_adam + t_net
    return {"value": round(1.0 / per_step, 6), "unit": "steps/s", "cores": oracle_threads(),
            **host_info(), "kind": "oracle",
            "sample": f"{B} frames x ({frame['sample']}) + L2 loss {t_loss:.2f} s + Adam over {P} "
                      f"parameters {t_adam:.2f} s{net_note}, extrapolated"}


def roofline(name, avg_ms, P, E_fwd, E_bwd, C):
    """Roofline object of the dominant kernel from its algorithmic work."""
    t = avg_ms / 1e3
    alu = lambda flops, how: dict(
        bound="alu", achieved=round(flops / t / 1e12, 3), peak=round(ALU_PEAK_TFLOPS, 1),
        unit="TFLOP/s", frac=round(flops / t / 1e12 / ALU_PEAK_TFLOPS, 4), traffic=None,
        kernel=name, avg_ms=round(avg_ms, 4), work=f"{flops:.4g} FLOP per launch = {how}")
    if name == "k_composite_fwd":
        return alu(E_fwd * FLOP_PER_EVAL + C * FWD_FLOP_PER_COMP,
                   f"{E_fwd} evals x {FLOP_PER_EVAL} + {C} composited x {FWD_FLOP_PER_COMP}")
    if name == "k_composite_bwd":
        return alu(E_bwd * FLOP_PER_EVAL + C * BWD_FLOP_PER_COMP,
                   f"{E_bwd} evals x {FLOP_PER_EVAL} + {C} composited x {BWD_FLOP_PER_COMP}")
    if name == "k_tile_place":
        b = P * 4   # every (tile, Gaussian) entry written once, 4 B; its group-list reads are extra
        a = b / t / 1e9
        return dict(bound="hbm", achieved=round(a, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(a / HBM_PEAK_GBS, 4), traffic=None, kernel=name,
                    avg_ms=round(avg_ms, 4), work=f"{b:.4g} B per launch = {P} pairs x 4 B written")
    if name == "k_sort_downsweep<pairs>":
        b = P * SORT_BYTES_PER_KEY_PASS
        a = b / t / 1e9
        return dict(bound="hbm", achieved=round(a, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(a / HBM_PEAK_GBS, 4), traffic=None, kernel=name,
                    avg_ms=round(avg_ms, 4),
                    work=f"{b:.4g} B per launch = {P} pairs x {SORT_BYTES_PER_KEY_PASS}")
    return dict(bound="hbm", achieved=None, peak=HBM_PEAK_GBS, unit="GB/s", frac=None,
                traffic=None, kernel=name, work=f"no algorithmic model for {name}")


def cpu_baseline(wl, cfg, up, budget_s):
    """The FP64 oracle as it stands, on a bounded sample of the workload:
    frame 0, forward + backward, on seeded tiles added in groups of 8 until
    about `budget_s` seconds of tile work; extrapolated to frames/s."""
    import torch

    import scenes
    from oracle import render as oref
    fr = [wl.frames[0]]
    n_tiles = cfg.tiles_x * cfg.tiles_y
    order = np.random.default_rng(0).permutation(n_tiles).tolist()
    up0 = {k: v[:1] for k, v in up.items()}
    # first-call costs (imports, allocator, thread pools) are paid on a tiny scene
    tiny = scenes.tiny_scene(20, 16, 16, seed=0)
    oref.render(tiny.gaussians, tiny.frames, tiny.cfg,
                upstream=scenes.upstream_grads(1, tiny.cfg, seed=0))
    t_fixed = float("inf")
    for _ in range(2):
        t0 = time.perf_counter()
        oref.render(wl.gaussians, fr, cfg, tiles=[[]], upstream=up0)
        t_fixed = min(t_fixed, time.perf_counter() - t0)
    done, t_tiles, step = 0, 0.0, 8
    wall0 = time.perf_counter()
    while done < n_tiles and t_tiles < budget_s and time.perf_counter() - wall0 < 2.5 * budget_s:
        chunk = order[done:done + step]
        t0 = time.perf_counter()
        oref.render(wl.gaussians, fr, cfg, tiles=[chunk], upstream=up0)
        t_tiles += max(time.perf_counter() - t0 - t_fixed, 0.0)
        done += len(chunk)
        step *= 2
    per_tile = t_tiles / max(done, 1)
    per_frame = t_fixed + per_tile * n_tiles
    return {"value": round(1.0 / per_frame, 6), "unit": "frames/s", "cores": oracle_threads(), **host_info(),
            "kind": "oracle",
            "sample": f"frame 0 fwd+bwd on {done} of {n_tiles} tiles (seeded order); per frame = "
                      f"{t_fixed:.2f} s fixed (binning + per-Gaussian chain) + {per_tile:.4f} s/tile "
                      f"x {n_tiles} tiles, extrapolated",
            "measured_s": round(time.perf_counter() - wall0 + 3 * t_fixed, 1)}


if __name__ == "__main__":
    main()
