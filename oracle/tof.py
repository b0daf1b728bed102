"""Time-of-flight quantities derived from rendered raw quads (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper §2: with the four offsets 0, pi/2, pi, 3pi/2 a camera recovers the
phase from Q0 - Qpi and Qpi/2 - Q3pi/2 (Eq. 1), the phasor is
(Q0 - Qpi) + i (Qpi/2 - Q3pi/2) up to the sign convention of the angle, the
amplitude is half its length, and d_ToF = c / (4 pi f) psi.  For general
offsets the two differences are the projections S^ = sum_j cos(phi_j) Q_j and
C^ = sum_j sin(phi_j) Q_j (for the standard offsets exactly the differences
above); the phase is atan2(S^, C^) taken in [0, 2 pi) (Eq. 1 with the
quadrant resolved), which for a surface at range d is 4 pi f d / c modulo
2 pi, consistent with Eq. 3's phasor 2 (C + i S) of the Gaussian sums.

Pins: tests/test_oracle_tof.py (single-Gaussian amplitude s r / d^2 alpha,
range recovery modulo c / 2f on equal-range shells, Eq. 1 differences).
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299_792_458.0


def _f32(x):
    return float(np.float32(x))


def tof_epilogue(quad, cfg):
    """quad [F, n_freq * n_phase, H, W] -> dict(phasor [F, n_freq, 2, H, W],
    d_tof [F, n_freq, H, W], amplitude [F, n_freq, H, W]), float64."""
    q = np.asarray(quad, np.float64)
    F, _, H, W = q.shape
    nf, nphi = cfg.n_freq, cfg.n_phase
    q = q.reshape(F, nf, nphi, H, W)
    cphi = np.array([math.cos(_f32(p)) for p in cfg.phases])
    sphi = np.array([math.sin(_f32(p)) for p in cfg.phases])
    sh = np.einsum("j,fnjhw->fnhw", cphi, q)
    ch = np.einsum("j,fnjhw->fnhw", sphi, q)
    psi = np.mod(np.arctan2(sh, ch), 2 * np.pi)
    freqs = np.array([_f32(f) for f in cfg.freqs])
    d_tof = C_LIGHT / (4 * np.pi * freqs)[None, :, None, None] * psi
    return dict(phasor=np.stack([ch, sh], 2), d_tof=d_tof, amplitude=0.5 * np.hypot(sh, ch))
