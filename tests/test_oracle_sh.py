"""Pins of the real SH basis used for view-dependent colour."""
import math

import numpy as np
import torch
from scipy import special

from oracle.sh import sh_basis


def _dirs(n, seed):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_orthonormal_under_exact_quadrature():
    # Gauss-Legendre in cos(theta) (exact to degree 19) x 16 uniform azimuths
    # (exact for trigonometric degree < 16) integrates products of degree <= 6.
    zs, wz = np.polynomial.legendre.leggauss(10)
    phis = np.arange(16) * 2 * math.pi / 16
    Z, PHI = np.meshgrid(zs, phis, indexing="ij")
    Wt = (wz[:, None] * np.full_like(PHI, 2 * math.pi / 16)).ravel()
    r = np.sqrt(1 - Z ** 2)
    d = np.stack([r * np.cos(PHI), r * np.sin(PHI), Z], -1).reshape(-1, 3)
    Y = sh_basis(torch.tensor(d), 3).numpy()
    G = (Y * Wt[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_matches_scipy_complex_harmonics():
    d = _dirs(500, 1)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))       # polar, from +z
    phi = np.arctan2(d[:, 1], d[:, 0])               # azimuth, from +x
    Y = sh_basis(torch.tensor(d), 3).numpy()
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            c = special.sph_harm_y(l, abs(m), theta, phi)   # includes the Condon-Shortley phase
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * c.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * c.imag
            else:
                ref = c.real
            assert np.abs(Y[:, k] - ref).max() < 1e-12, (l, m)


def test_addition_theorem_and_hand_values():
    d = _dirs(200, 2)
    Y = sh_basis(torch.tensor(d), 3).numpy()
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(1)
        assert np.abs(s - (2 * l + 1) / (4 * math.pi)).max() < 1e-12
    e = sh_basis(torch.tensor([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]), 1).numpy()
    assert abs(e[0, 0] - 1 / (2 * math.sqrt(math.pi))) < 1e-15
    assert abs(e[0, 3] - math.sqrt(3 / (4 * math.pi))) < 1e-15 and abs(e[0, 2]) < 1e-15
    assert abs(e[1, 2] - math.sqrt(3 / (4 * math.pi))) < 1e-15
