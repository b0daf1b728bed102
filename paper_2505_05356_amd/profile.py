"""Per-kernel HIP-event timing of everything libgftorf.so launches."""
from __future__ import annotations

import ctypes

from . import _lib


class KernelTimer:
    """with KernelTimer() as kt: ...;  kt.totals -> {name: (launches, total_ms)}"""

    def __init__(self, max_launches: int = 4096):
        self.max_launches = max_launches
        self.totals = {}

    def __enter__(self):
        _lib.check(_lib.load().gftorf_profile_begin(self.max_launches))
        return self

    def collect(self):
        _lib.check(_lib.load().gftorf_profile_collect())

    def __exit__(self, *exc):
        lib = _lib.load()
        buf = (_lib.ProfileEntryC * 256)()
        n = ctypes.c_int32(0)
        _lib.check(lib.gftorf_profile_end(buf, 256, ctypes.byref(n)))
        self.totals = {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
                       for i in range(min(n.value, 256))}
        return False

    def average_ms(self, name):
        launches, total = self.totals[name]
        return total / max(launches, 1)
