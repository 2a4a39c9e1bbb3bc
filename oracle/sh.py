"""Oracle: real spherical-harmonic basis up to degree 3 (float64, torch).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper keeps third-degree SH colour per Gaussian (Sec. II, "full
representation fidelity") but does not fix the basis.  Reading used here:
the orthonormal real basis with index k = l*l + l + m, polar angle from
world +z, azimuth from world +x, and no Condon-Shortley phase, so that
Y_{1,-1}, Y_{1,0}, Y_{1,1} are proportional to y, z, x.

Pinned (tests/test_oracle_sh.py) by: orthonormality under exact quadrature
(Gauss-Legendre in cos(theta) x uniform azimuth), agreement with SciPy's
complex spherical harmonics converted to the real basis, and the addition
theorem sum_m Y_lm(d)^2 = (2l+1)/(4 pi).
"""
from __future__ import annotations

import math

import torch


def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """d: [n, 3] unit directions (float64).  Returns [n, (degree+1)^2]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [c1 * y, c1 * z, c1 * x]
    if degree >= 2:
        c2a = 0.5 * math.sqrt(15.0 / pi)
        c20 = 0.25 * math.sqrt(5.0 / pi)
        c22 = 0.25 * math.sqrt(15.0 / pi)
        out += [c2a * x * y, c2a * y * z, c20 * (3.0 * z * z - 1.0), c2a * x * z, c22 * (x * x - y * y)]
    if degree >= 3:
        c33 = 0.25 * math.sqrt(35.0 / (2.0 * pi))
        c32 = 0.5 * math.sqrt(105.0 / pi)
        c31 = 0.25 * math.sqrt(21.0 / (2.0 * pi))
        c30 = 0.25 * math.sqrt(7.0 / pi)
        c32b = 0.25 * math.sqrt(105.0 / pi)
        out += [c33 * y * (3.0 * x * x - y * y), c32 * x * y * z, c31 * y * (5.0 * z * z - 1.0),
                c30 * z * (5.0 * z * z - 3.0), c31 * x * (5.0 * z * z - 1.0), c32b * z * (x * x - y * y),
                c33 * x * (x * x - 3.0 * y * y)]
    return torch.stack(out, dim=1)
