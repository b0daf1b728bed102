"""ctypes view of libgftorf.so (include/gftorf.h): struct layouts and symbols.

Argument marshalling only: every step of the rendering path runs in the HIP
kernels behind these symbols.  Loading fails loudly when the library has not
been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgftorf.so")

FIELDS = ("mean", "vel", "acc", "scale", "quat", "omega", "opacity_logit", "rgb", "albedo")
ROWS = {"mean": 3, "vel": 3, "acc": 3, "scale": 3, "quat": 4, "omega": 3,
        "opacity_logit": 1, "rgb": 3, "albedo": 1}
OPTIONAL = ("vel", "acc", "omega")

MAX_FREQ = 4
MAX_PHASE = 4
MAX_QUAD = 16
FRAME_FLOATS = 9 + 3 + 4 + 1 + 3 + MAX_QUAD + 4   # 40: ... t_lo, t_hi, quad_mask, reserved
FRAME_TIME = 9 + 3 + 4                            # column of .time

OK, EINVAL, ENOWS, EHIP, EOVERFLOW = 0, -1, -2, -3, -4


SH_FIELDS = ("sh_rgb", "sh_albedo")


# per-frame centre offsets [F][3][n] (the deformation network's output)
OFFSET_FIELDS = ("delta",)


class GaussiansC(ctypes.Structure):
    _fields_ = ([("n", c_int64)] + [(k, c_void_p) for k in FIELDS] +
                [("sh_degree", c_int32), ("reserved", c_int32)] +
                [(k, c_void_p) for k in SH_FIELDS + OFFSET_FIELDS])


class GaussiansGradC(ctypes.Structure):
    _fields_ = [(k, c_void_p) for k in FIELDS + SH_FIELDS + OFFSET_FIELDS]


class MlpConfigC(ctypes.Structure):
    _fields_ = [("n_freq_x", c_int32), ("n_freq_t", c_int32), ("width", c_int32),
                ("depth", c_int32), ("pos_scale", c_float), ("time_scale", c_float)]


class ConfigC(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("n_freq", c_int32), ("n_phase", c_int32),
                ("freq_hz", c_double * MAX_FREQ), ("phase", c_float * MAX_PHASE),
                ("tile_w", c_int32), ("tile_h", c_int32),
                ("alpha_min", c_float), ("alpha_max", c_float), ("T_min", c_float),
                ("extent_sigma", c_float), ("dilation", c_float), ("near_z", c_float),
                ("source_intensity", c_float), ("bg_T_power", c_int32), ("max_pairs", c_int64)]


class OutputsC(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("quad", c_void_p), ("depth", c_void_p),
                ("T_final", c_void_p), ("n_contrib", c_void_p), ("phasor", c_void_p),
                ("d_tof", c_void_p), ("amplitude", c_void_p)]


class StatusC(ctypes.Structure):
    _fields_ = [("n_pairs", c_int64), ("max_pairs", c_int64), ("overflow", c_int32),
                ("nonfinite", c_int32), ("n_evaluated", c_int64), ("n_composited", c_int64),
                ("overflow_seen", c_int32), ("sort_fault", c_int32), ("n_pairs_seen", c_int64)]


class AdamGroupC(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("grad", c_void_p), ("m", c_void_p), ("v", c_void_p),
                ("n", c_int64), ("lr", c_float), ("lr_final", c_float), ("decay_steps", c_int32),
                ("reserved", c_int32)]


class ProfileEntryC(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", c_int64), ("total_ms", c_double)]


_SIGS = {
    "gftorf_workspace_size": (c_size_t, [c_int64, c_int32, POINTER(ConfigC)]),
    "gftorf_render_fwd": (c_int32, [POINTER(GaussiansC), c_void_p, c_int32, POINTER(ConfigC),
                                    POINTER(OutputsC), c_void_p, c_size_t, c_void_p]),
    "gftorf_render_bwd": (c_int32, [POINTER(GaussiansC), c_void_p, c_int32, POINTER(ConfigC),
                                    POINTER(OutputsC), c_void_p, c_void_p, c_void_p,
                                    POINTER(GaussiansGradC), c_void_p, c_void_p, c_size_t, c_void_p]),
    "gftorf_read_status": (c_int32, [c_void_p, POINTER(StatusC), c_void_p]),
    "gftorf_clear_status": (c_int32, [c_void_p, c_void_p]),
    "gftorf_copy_lists": (c_int32, [c_void_p, c_int64, c_int32, POINTER(ConfigC), c_void_p,
                                    c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p]),
    "gftorf_l2_loss_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int64, c_float,
                                      c_void_p, c_void_p, c_void_p]),
    "gftorf_adam_step": (c_int32, [POINTER(AdamGroupC), c_int32, c_void_p, c_float, c_float,
                                   c_float, c_void_p]),
    "gftorf_select_frames": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_int32,
                                       c_int32, c_void_p, c_void_p, c_void_p]),
    "gftorf_fill_f32": (c_int32, [c_void_p, c_float, c_int64, c_void_p]),
    "gftorf_graph_begin": (c_int32, [c_void_p]),
    "gftorf_graph_end": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "gftorf_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "gftorf_graph_destroy": (c_int32, [c_void_p]),
    "gftorf_profile_begin": (c_int32, [c_int32]),
    "gftorf_profile_collect": (c_int32, []),
    "gftorf_profile_end": (c_int32, [POINTER(ProfileEntryC), c_int32, POINTER(c_int32)]),
    "gftorf_mlp_param_count": (c_int64, [POINTER(MlpConfigC)]),
    "gftorf_mlp_workspace_size": (c_size_t, [POINTER(MlpConfigC), c_int64, c_int32, c_int32]),
    "gftorf_mlp_fwd": (c_int32, [POINTER(MlpConfigC), c_void_p, c_void_p, c_int64, POINTER(c_float),
                                 c_int32, c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "gftorf_mlp_bwd": (c_int32, [POINTER(MlpConfigC), c_void_p, c_void_p, c_int64, POINTER(c_float),
                                 c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gftorf_mlp_get_decisions": (c_int32, [POINTER(MlpConfigC), c_int64, c_int32, c_void_p, c_void_p,
                                           c_size_t, c_void_p]),
    "gftorf_mlp_set_decisions": (c_int32, [POINTER(MlpConfigC), c_int64, c_int32, c_void_p, c_void_p,
                                           c_size_t, c_void_p]),
    "gftorf_mlp_fwd_noalloc": (c_int32, [POINTER(MlpConfigC), c_void_p, c_void_p, c_int64, POINTER(c_float),
                                         c_int32, c_void_p, c_void_p]),
    "gftorf_mlp_fwd_frames": (c_int32, [POINTER(MlpConfigC), c_void_p, c_void_p, c_int64, c_void_p, c_int32,
                                        c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "gftorf_mlp_bwd_frames": (c_int32, [POINTER(MlpConfigC), c_void_p, c_void_p, c_int64, c_void_p, c_int32,
                                        c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "gftorf_blend_offsets": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_int32, POINTER(c_int32),
                                       c_void_p, c_void_p]),
    "gftorf_blend_offsets_bwd": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, POINTER(c_int32), c_int32,
                                           c_void_p, c_void_p]),
    "gftorf_strerror": (c_char_p, [c_int32]),
    "gftorf_last_error": (c_char_p, []),
    "gftorf_version": (c_int32, []),
}

_lib = None


class GftorfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gftorf error {code}: {msg}")
        self.code = code


def load(path: str = None):
    """Loads the library once (dlopen); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_2505_05356_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != OK:
        lib = load()
        msg = lib.gftorf_last_error().decode(errors="replace")
        raise GftorfError(rc, msg or lib.gftorf_strerror(rc).decode())
    return rc
