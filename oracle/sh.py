"""Real spherical harmonics up to degree 3 (FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Paper §3: the colour c_k is view dependent, parameterised by 16 x 3
spherical-harmonic coefficients, and the reflectivity r_k by 16
coefficients.  The paper defers the details to the Gaussian-splatting prior
art, so the readings here are that art's conventions:

* the basis is the real spherical harmonics Y_{l,m}, l <= 3, in the order
  (l, m) = (0,0), (1,-1), (1,0), (1,1), (2,-2), ..., (3,3), evaluated at the
  unit direction from the optical centre to the Gaussian centre;
* Y_{l,m} = sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0), Y_l^0
  (m = 0), with Y_l^m the complex harmonics including the Condon-Shortley
  phase;
* colour channel c = max(0, 1/2 + sum_i Y_i(dir) k_{i,c}), reflectivity
  r = max(0, 1/2 + sum_i Y_i(dir) k_i) (the 1/2 offset and the clamp at 0 of
  the prior art).

The polynomial forms below follow from those definitions with x, y, z the
components of the unit direction; the constants are the normalisations
written as their closed forms.

Pins: tests/test_oracle_sh.py (equal to scipy's complex harmonics through the
definition above; orthonormal on the sphere by quadrature).
"""
from __future__ import annotations

import math

import torch

N_COEFFS = {0: 1, 1: 4, 2: 9, 3: 16}

_K0 = 0.5 / math.sqrt(math.pi)                  # Y_00
_K1 = math.sqrt(3.0 / (4.0 * math.pi))          # l = 1
_K2a = 0.5 * math.sqrt(15.0 / math.pi)          # l = 2, |m| = 1, 2 (xy, yz, xz)
_K2b = 0.25 * math.sqrt(5.0 / math.pi)          # l = 2, m = 0
_K2c = 0.25 * math.sqrt(15.0 / math.pi)         # l = 2, m = 2 (x^2 - y^2)
_K3a = 0.25 * math.sqrt(35.0 / (2.0 * math.pi))  # l = 3, |m| = 3
_K3b = 0.5 * math.sqrt(105.0 / math.pi)         # l = 3, m = -2 (xyz)
_K3c = 0.25 * math.sqrt(21.0 / (2.0 * math.pi))  # l = 3, |m| = 1
_K3d = 0.25 * math.sqrt(7.0 / math.pi)          # l = 3, m = 0
_K3e = 0.25 * math.sqrt(105.0 / math.pi)        # l = 3, m = 2


def basis(d, degree: int = 3):
    """d: [3, N] unit directions (torch, any float dtype) -> [K, N] basis values."""
    x, y, z = d[0], d[1], d[2]
    out = [torch.full_like(x, _K0)]
    if degree >= 1:
        out += [-_K1 * y, _K1 * z, -_K1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [_K2a * x * y, -_K2a * y * z, _K2b * (2.0 * zz - xx - yy), -_K2a * x * z,
                _K2c * (xx - yy)]
    if degree >= 3:
        out += [-_K3a * y * (3.0 * xx - yy), _K3b * x * y * z, -_K3c * y * (4.0 * zz - xx - yy),
                _K3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy), -_K3c * x * (4.0 * zz - xx - yy),
                _K3e * z * (xx - yy), -_K3a * x * (xx - 3.0 * yy)]
    return torch.stack(out)


def colour(coeffs, d, degree: int):
    """coeffs [K, C, N], d [3, N] unit directions -> [C, N] = max(0, 1/2 + sum Y k)."""
    Y = basis(d, degree)
    return torch.clamp(0.5 + (Y[:, None, :] * coeffs).sum(0), min=0.0)
