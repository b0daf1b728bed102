"""Pins for oracle.sh (real spherical harmonics, degree <= 3)."""
import math

import numpy as np
import pytest
import scipy.special as sp

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")
import torch

from oracle import sh


def _scipy_real(l, m, polar, azim):
    # real harmonics from scipy's complex ones (Condon-Shortley phase included)
    if m == 0:
        return sp.sph_harm(0, l, azim, polar).real
    Y = sp.sph_harm(abs(m), l, azim, polar)
    return math.sqrt(2.0) * (Y.real if m > 0 else Y.imag)


def test_matches_scipy_definition():
    rng = np.random.default_rng(0)
    v = rng.normal(size=(3, 200))
    v /= np.linalg.norm(v, axis=0)
    polar = np.arccos(np.clip(v[2], -1, 1))
    azim = np.arctan2(v[1], v[0])
    Y = sh.basis(torch.tensor(v), 3).numpy()
    i = 0
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[i], _scipy_real(l, m, polar, azim), atol=1e-12,
                                       err_msg=f"l={l} m={m}")
            i += 1
    assert i == 16


def test_orthonormal_on_the_sphere():
    # Gauss-Legendre in cos(polar) x uniform azimuth integrates these
    # polynomials (degree <= 6) exactly
    xg, wg = np.polynomial.legendre.leggauss(12)
    az = np.arange(24) * (2 * np.pi / 24)
    ct, a = np.meshgrid(xg, az, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(a), st * np.sin(a), ct]).reshape(3, -1)
    w = (wg[:, None] * np.full(az.shape, 2 * np.pi / 24)[None, :]).reshape(-1)
    Y = sh.basis(torch.tensor(d), 3).numpy()
    G = (Y * w) @ Y.T
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


@pytest.mark.parametrize("degree", [0, 1, 2])
def test_lower_degree_is_a_prefix(degree):
    d = torch.tensor([[0.3], [-0.4], [math.sqrt(1 - 0.25)]], dtype=torch.float64)
    np.testing.assert_array_equal(sh.basis(d, degree).numpy(), sh.basis(d, 3).numpy()[:sh.N_COEFFS[degree]])


def test_colour_offset_and_clamp():
    d = torch.tensor([[0.0], [0.0], [1.0]], dtype=torch.float64)
    k = torch.zeros((16, 3, 1), dtype=torch.float64)
    np.testing.assert_allclose(sh.colour(k, d, 3).numpy(), 0.5)          # zero coefficients: grey
    k[0, 0, 0] = 1.0 / sh.basis(d, 0)[0, 0]                              # DC term: +1 on red
    k[0, 1, 0] = -2.0 / sh.basis(d, 0)[0, 0]                             # -2 on green: clamped
    c = sh.colour(k, d, 3).numpy()[:, 0]
    np.testing.assert_allclose(c, [1.5, 0.0, 0.5])
