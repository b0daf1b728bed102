"""MI355X-native differentiable C-ToF Gaussian rasterizer.

The hot path (projection, depth sort, tile binning, front-to-back compositing
of RGB, mean depth and raw continuous-wave ToF quads, and its backward) runs
in hand-written gfx950 HIP kernels behind the C ABI of include/gftorf.h
(libgftorf.so, built by ``paper_2505_05356_amd.build``).  This package is the
thin Python binding: ctypes marshalling, a torch.autograd.Function, a
graph-captured optimisation step and the tile-shape autotuner.
"""
from ._lib import FIELDS, GftorfError, load  # noqa: F401
from .raster import (RasterConfig, RasterizeCToF, Workspace, alloc_outputs, backward,  # noqa: F401
                     forward, pack_frames, render, to_device_params)
