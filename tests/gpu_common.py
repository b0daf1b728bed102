"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare with the FP64 oracle under the stated tolerances."""
import ctypes

import numpy as np
import torch

from paper_2505_05356_amd import _lib, raster

FWD_RTOL = 1e-4     # per channel image: |gpu - ref| <= 1e-4 (|ref| + max |ref|)
GRAD_RTOL = 2e-2    # per parameter tensor: relative L2 and elementwise (|ref| + max |ref|)


def run_gpu(g, frames, cfg, upstream=None, max_pairs=None, want_bg=False, device="cuda",
            channels=("rgb", "quad", "depth")):
    params = raster.to_device_params(g, device)
    fdev = raster.pack_frames(frames, cfg, device)
    ws = raster.Workspace(g.n, len(frames), cfg, max_pairs=max_pairs, device=device)
    out = raster.forward(params, fdev, cfg, ws,
                         out=raster.alloc_outputs(len(frames), cfg, device, channels))
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["status"] = ws.status()
    res["_ws"], res["_params"], res["_frames"], res["_out"] = ws, params, fdev, out
    if upstream is not None:
        d = {k: torch.from_numpy(np.ascontiguousarray(upstream[k], dtype=np.float32)).to(device)
             for k in ("rgb", "quad", "depth")}
        grads = raster.backward(params, fdev, cfg, ws, out, d["rgb"], d["quad"], d["depth"],
                                want_bg=want_bg)
        torch.cuda.synchronize()
        res["grads"] = {k: (v.cpu().numpy() if v is not None else None) for k, v in grads.items()
                        if k != "bg"}
        if want_bg:
            res["grad_bg"] = grads["bg"].cpu().numpy()
    return res


def gpu_lists(res, g, frames, cfg, pairs_to_host=True):
    """Tile lists and per-item binning copied out of the workspace.  With
    pairs_to_host=False the pair arrays stay on the device (large batches)."""
    lib = _lib.load()
    ws = res["_ws"]
    n, F = g.n, len(frames)
    M = n * F
    K = F * cfg.tiles_x * cfg.tiles_y
    P = min(res["status"]["n_pairs"], ws.max_pairs)
    dev = "cuda"
    pk = torch.empty(max(P, 1), dtype=torch.int32, device=dev) if pairs_to_host else None
    pi = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    dk = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
    di = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
    cnt = torch.empty(max(M, 1), dtype=torch.int32, device=dev)
    rect = torch.empty(max(2 * M, 1), dtype=torch.int32, device=dev)
    rng = torch.empty(2 * K, dtype=torch.int32, device=dev)
    v = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    _lib.check(lib.gftorf_copy_lists(ctypes.c_void_p(ws.ptr), n, F, ctypes.byref(ws.cstruct),
                                     v(pk), v(pi), P, v(dk), v(di), v(cnt), v(rect), v(rng),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    u = lambda t, k: t.cpu().numpy().view(np.uint32)[:k]
    out = dict(depth_key=u(dk, M), depth_item=u(di, M), count=u(cnt, M),
               rect=u(rect, 2 * M).reshape(M, 2), ranges=u(rng, 2 * K).reshape(K, 2), P=P)
    if pairs_to_host:
        out["pair_key"], out["pair_item"] = u(pk, P), u(pi, P)
    else:
        out["pair_item_dev"] = pi
    return out


def assert_images_close(got, ref, ok, name, rtol=FWD_RTOL):
    """got, ref [F, C, H, W] or [F, H, W]; ok [F, H, W] pixels to check."""
    if got.ndim == 3:
        got, ref = got[:, None], ref[:, None]
    ref = ref.astype(np.float64)
    scale = np.abs(ref).max(axis=(-2, -1), keepdims=True)
    bound = rtol * (np.abs(ref) + scale)
    err = np.abs(got.astype(np.float64) - ref)
    bad = (err > bound) & ok[:, None]
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{name}: {int(bad.sum())} elements beyond tolerance, e.g. "
                             + ", ".join(f"{tuple(i)} gpu={got[tuple(i)]:.7g} ref={ref[tuple(i)]:.7g}"
                                         for i in idx))


def assert_grads_close(got, ref, name, rtol=GRAD_RTOL):
    g = np.asarray(got, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    nr = np.linalg.norm(r)
    if nr == 0:
        assert np.abs(g).max() <= 1e-6, name
        return
    rel = np.linalg.norm(g - r) / nr
    assert rel <= rtol, f"{name}: relative L2 error {rel:.3e}"
    bound = rtol * (np.abs(r) + np.abs(r).max())
    bad = np.abs(g - r) > bound
    assert not bad.any(), f"{name}: {int(bad.sum())} elements beyond tolerance (rel L2 {rel:.2e})"
    return rel


def mask_upstream(up, ok):
    """Zero the upstream gradient on pixels excluded from the comparison."""
    out = {}
    for k, v in up.items():
        out[k] = (v * (ok[:, None] if v.ndim == 4 else ok)).astype(np.float32)
    return out
