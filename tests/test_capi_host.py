"""Host-side checks of libgftorf.so that need no GPU: every symbol the header
declares is exported, and argument validation returns the documented codes
before anything touches the device."""
import ctypes
import os
import re

import pytest

import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gftorf.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2505_05356_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gftorf_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gftorf_render_fwd", "gftorf_render_bwd", "gftorf_workspace_size",
                     "gftorf_read_status", "gftorf_adam_step", "gftorf_l2_loss_grad",
                     "gftorf_graph_begin", "gftorf_graph_end", "gftorf_graph_launch",
                     "gftorf_strerror"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(lib._name)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_struct_sizes_match_header(lib):
    from paper_2505_05356_amd import _lib
    assert ctypes.sizeof(_lib.ConfigC) == 112
    assert ctypes.sizeof(_lib.GaussiansC) == 8 * 14
    assert ctypes.sizeof(_lib.GaussiansGradC) == 8 * 12
    assert ctypes.sizeof(_lib.MlpConfigC) == 24
    assert ctypes.sizeof(_lib.AdamGroupC) == 56
    assert _lib.FRAME_FLOATS * 4 == 160


def _cfg(**kw):
    from paper_2505_05356_amd import raster
    c = raster.RasterConfig(width=64, height=48)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_workspace_size_and_validation(lib):
    from paper_2505_05356_amd import _lib, raster
    good = raster.config_struct(_cfg(), 100000)
    assert lib.gftorf_workspace_size(2000, 1, ctypes.byref(good)) > 100000 * 4
    # grows with the pair capacity and the frame count
    big = raster.config_struct(_cfg(), 200000)
    assert lib.gftorf_workspace_size(2000, 1, ctypes.byref(big)) > \
        lib.gftorf_workspace_size(2000, 1, ctypes.byref(good))
    assert lib.gftorf_workspace_size(2000, 4, ctypes.byref(good)) > \
        lib.gftorf_workspace_size(2000, 1, ctypes.byref(good))
    for bad in (dict(tile_w=12), dict(alpha_max=1.0), dict(bg_T_power=3), dict(freqs=()),
                dict(phases=(0.0,) * 5), dict(T_min=-1.0), dict(width=0)):
        c = raster.config_struct(_cfg(**bad), 1000)
        assert lib.gftorf_workspace_size(2000, 1, ctypes.byref(c)) == 0, bad
    assert lib.gftorf_workspace_size(2000, 0, ctypes.byref(good)) == 0
    assert lib.gftorf_workspace_size(-1, 1, ctypes.byref(good)) == 0


def test_error_codes_before_device_work(lib):
    from paper_2505_05356_amd import _lib, raster
    cfg = raster.config_struct(_cfg(), 1000)
    g = _lib.GaussiansC()
    g.n = 10                      # required arrays missing
    out = _lib.OutputsC()
    rc = lib.gftorf_render_fwd(ctypes.byref(g), None, 1, ctypes.byref(cfg), ctypes.byref(out),
                               None, 0, None)
    assert rc == _lib.EINVAL
    assert b"required" in lib.gftorf_last_error()
    g.n = 0
    rc = lib.gftorf_render_fwd(ctypes.byref(g), ctypes.c_void_p(256), 1, ctypes.byref(cfg),
                               ctypes.byref(out), None, 0, None)
    assert rc == _lib.EINVAL     # outputs missing
    out.T_final = 256
    out.n_contrib = 512
    rc = lib.gftorf_render_fwd(ctypes.byref(g), ctypes.c_void_p(256), 1, ctypes.byref(cfg),
                               ctypes.byref(out), ctypes.c_void_p(4096), 16, None)
    assert rc == _lib.ENOWS
    assert lib.gftorf_strerror(_lib.ENOWS) == b"workspace too small"
    g.sh_rgb = 1024               # spherical harmonics of an unsupported degree
    g.sh_degree = 4
    rc = lib.gftorf_render_fwd(ctypes.byref(g), ctypes.c_void_p(256), 1, ctypes.byref(cfg),
                               ctypes.byref(out), ctypes.c_void_p(4096), 16, None)
    assert rc == _lib.EINVAL and b"sh_degree" in lib.gftorf_last_error()
    assert lib.gftorf_version() == 1


def test_mlp_sizes_and_argument_checks(lib):
    # the deformation network's parameter count (paper §4: 8 x 256, L_x = L_t = 10)
    # and workspace sizing; invalid shapes are refused without touching a GPU
    from paper_2505_05356_amd import _lib
    good = _lib.MlpConfigC(10, 10, 256, 8, 0.2, 4.0)
    assert lib.gftorf_mlp_param_count(ctypes.byref(good)) == 483_075
    small = lib.gftorf_mlp_workspace_size(ctypes.byref(good), 1000, 2, 0)
    train = lib.gftorf_mlp_workspace_size(ctypes.byref(good), 1000, 2, 1)
    assert 0 < small < train
    # 9.2 KB of saved activations and gradients per row when training
    assert train - small >= 2000 * (96 + 8 * 256 + 8 * 256 + 16) * 2
    for bad in (_lib.MlpConfigC(10, 10, 128, 8, 0.2, 4.0), _lib.MlpConfigC(10, 10, 256, 6, 0.2, 4.0),
                _lib.MlpConfigC(14, 10, 256, 8, 0.2, 4.0), _lib.MlpConfigC(-1, 10, 256, 8, 0.2, 4.0)):
        assert lib.gftorf_mlp_param_count(ctypes.byref(bad)) == 0
        assert lib.gftorf_mlp_workspace_size(ctypes.byref(bad), 1000, 2, 1) == 0
    assert lib.gftorf_mlp_workspace_size(ctypes.byref(good), 1000, 65, 1) == 0
    assert lib.gftorf_mlp_workspace_size(ctypes.byref(good), 0, 2, 1) == 0
    times = (ctypes.c_float * 2)(0.0, 0.1)
    rc = lib.gftorf_mlp_fwd(ctypes.byref(good), None, None, 1000, times, 2, None, 1,
                            None, 0, None)
    assert rc == _lib.EINVAL
    rc = lib.gftorf_mlp_fwd(ctypes.byref(good), ctypes.c_void_p(256), ctypes.c_void_p(256), 1000,
                            times, 2, ctypes.c_void_p(256), 1, ctypes.c_void_p(256), small, None)
    assert rc == _lib.ENOWS


def test_mlp_device_time_entry_points_check_arguments(lib):
    # the entry points that read the times from device frame descriptors refuse
    # missing pointers, too many frames and a short workspace before any launch
    from paper_2505_05356_amd import _lib
    cfg = _lib.MlpConfigC(10, 10, 256, 8, 0.2, 4.0)
    need = lib.gftorf_mlp_workspace_size(ctypes.byref(cfg), 1000, 2, 1)
    dev = ctypes.c_void_p(256)
    assert lib.gftorf_mlp_fwd_frames(ctypes.byref(cfg), dev, dev, 1000, None, 2, dev, 1,
                                     dev, need, None) == _lib.EINVAL
    assert lib.gftorf_mlp_fwd_frames(ctypes.byref(cfg), dev, dev, 1000, dev, 65, dev, 1,
                                     dev, need, None) == _lib.EINVAL
    assert lib.gftorf_mlp_fwd_frames(ctypes.byref(cfg), dev, dev, 1000, dev, 2, dev, 1,
                                     dev, need - 256, None) == _lib.ENOWS
    assert lib.gftorf_mlp_bwd_frames(ctypes.byref(cfg), dev, dev, 1000, None, 2, dev, dev, dev, 1,
                                     dev, need, None) == _lib.EINVAL
    assert lib.gftorf_mlp_bwd_frames(ctypes.byref(cfg), dev, dev, 1000, dev, 2, None, dev, dev, 1,
                                     dev, need, None) == _lib.EINVAL


def test_mlp_decisions_check_arguments(lib):
    # reading or replacing the recorded ReLU decisions needs a training
    # workspace of the forward's size and both pointers
    from paper_2505_05356_amd import _lib
    cfg = _lib.MlpConfigC(10, 10, 256, 8, 0.2, 4.0)
    need = lib.gftorf_mlp_workspace_size(ctypes.byref(cfg), 1000, 2, 1)
    infer = lib.gftorf_mlp_workspace_size(ctypes.byref(cfg), 1000, 2, 0)
    assert 0 < infer < need
    dev = ctypes.c_void_p(256)
    for fn in (lib.gftorf_mlp_get_decisions, lib.gftorf_mlp_set_decisions):
        assert fn(ctypes.byref(cfg), 1000, 2, None, dev, need, None) == _lib.EINVAL
        assert fn(ctypes.byref(cfg), 1000, 2, dev, None, need, None) == _lib.EINVAL
        assert fn(ctypes.byref(cfg), 1000, 2, dev, dev, infer, None) == _lib.ENOWS
        assert fn(ctypes.byref(cfg), 1000, 65, dev, dev, need, None) == _lib.EINVAL
        assert fn(ctypes.byref(cfg), 1000, 2, dev, ctypes.c_void_p(512 + 16), need, None) == _lib.EINVAL
        assert fn(None, 1000, 2, dev, dev, need, None) == _lib.EINVAL


def test_mlp_noalloc_checks_arguments(lib):
    # the allocation-free inference forward refuses bad shapes and missing
    # pointers before it resolves its static scratch or launches anything,
    # and the supported network's weight copies fit that scratch
    from paper_2505_05356_amd import _lib
    cfg = _lib.MlpConfigC(10, 10, 256, 8, 0.2, 4.0)
    need = lib.gftorf_mlp_workspace_size(ctypes.byref(cfg), 1000, 2, 0)
    assert 0 < need <= 4 << 20
    times = (ctypes.c_float * 2)(0.0, 0.1)
    dev = ctypes.c_void_p(256)
    assert lib.gftorf_mlp_fwd_noalloc(ctypes.byref(cfg), None, dev, 1000, times, 2, dev, None) == _lib.EINVAL
    assert lib.gftorf_mlp_fwd_noalloc(ctypes.byref(cfg), dev, dev, 1000, None, 2, dev, None) == _lib.EINVAL
    assert lib.gftorf_mlp_fwd_noalloc(ctypes.byref(cfg), dev, dev, 1000, times, 2, None, None) == _lib.EINVAL
    assert lib.gftorf_mlp_fwd_noalloc(ctypes.byref(cfg), dev, dev, 1000, times, 65, dev, None) == _lib.EINVAL
    assert lib.gftorf_mlp_fwd_noalloc(ctypes.byref(cfg), dev, dev, 0, times, 2, dev, None) == _lib.EINVAL
    bad = _lib.MlpConfigC(10, 10, 128, 8, 0.2, 4.0)
    assert lib.gftorf_mlp_fwd_noalloc(ctypes.byref(bad), dev, dev, 1000, times, 2, dev, None) == _lib.EINVAL
