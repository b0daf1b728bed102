"""The allocation-free inference forward of the deformation network
(gftorf_mlp_fwd_noalloc, needs an MI355X): through the C ABI, against the
workspace entry point gftorf_mlp_fwd with save = 0 on the same inputs.  Both
run the same kernels, so the offsets must agree bit for bit.  Two calls in a
row share the library's static scratch; the second is smaller, so it must
not depend on what the first left there."""
import ctypes

import numpy as np
import pytest
import torch

import scenes
from paper_2505_05356_amd import _lib, deform

pytestmark = pytest.mark.gpu

SX, ST = 2 * 30e6 / 299_792_458.0, 4.0


def _workspace_forward(theta, x0, times):
    net = deform.DeformNet(x0.shape[1], len(times), pos_scale=SX, time_scale=ST, training=False)
    out = net.forward(theta, x0, times, save=False)
    torch.cuda.synchronize()
    return out.cpu().numpy(), net.cfg


def _noalloc_forward(cfg, theta, x0, times):
    lib = _lib.load()
    n, T = x0.shape[1], len(times)
    out = torch.full((T, 3, n), float("nan"), device="cuda")
    ct = (ctypes.c_float * T)(*[float(t) for t in times])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.gftorf_mlp_fwd_noalloc(ctypes.byref(cfg), ctypes.c_void_p(theta.data_ptr()),
                                          ctypes.c_void_p(x0.data_ptr()), n, ct, T,
                                          ctypes.c_void_p(out.data_ptr()), stream))
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("first,second", [((900, [0.0, 0.1, 0.25]), (300, [0.05, 0.2]))])
def test_noalloc_forward_equals_workspace_forward(first, second):
    for i, (n, times) in enumerate((first, second)):
        # different parameters for the two calls, so stale weight copies would show
        theta = torch.from_numpy(scenes.mlp_params(seed=20 + i, last_std=0.05, bias_std=0.1)).cuda()
        x0 = torch.from_numpy(scenes.mlp_rows(n, 1, seed=30 + i)[0]).cuda()
        ref, cfg = _workspace_forward(theta, x0, times)
        got = _noalloc_forward(cfg, theta, x0, times)
        assert np.isfinite(got).all(), f"call {i}: offsets not all written"
        np.testing.assert_array_equal(got, ref, err_msg=f"call {i} (n={n}, {len(times)} times)")
