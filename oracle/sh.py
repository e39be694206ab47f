"""Real spherical harmonics up to degree 3 (view-dependent colour of 3D-GS).

The paper takes colour from the cited 3D-GS model (Sec. II, Sec. III) without
formulas.  Reading used: real SH with the Condon-Shortley phase, ordered
l = 0..3 and m = -l..l, evaluated at the unit view direction d = (x, y, z):

    l=0: k0
    l=1: -k1 y, k1 z, -k1 x
    l=2: k2 xy, -k2 yz, k3 (2z^2 - x^2 - y^2), -k2 xz, k2/2 (x^2 - y^2)
    l=3: -a y(3x^2 - y^2), b xyz, -c y(4z^2 - x^2 - y^2), e z(2z^2 - 3x^2 - 3y^2),
         -c x(4z^2 - x^2 - y^2), b/2 z(x^2 - y^2), -a x(x^2 - 3y^2)

with k0 = 1/(2 sqrt(pi)), k1 = sqrt(3/(4 pi)), k2 = sqrt(15/pi)/2,
k3 = sqrt(5/pi)/4, a = sqrt(35/(2 pi))/4, b = sqrt(105/pi)/2,
c = sqrt(21/(2 pi))/4, e = sqrt(7/pi)/4 (the usual normalisation constants,
written from their definitions rather than as decimals).
"""
from __future__ import annotations

import math

import numpy as np

K0 = 1.0 / (2.0 * math.sqrt(math.pi))
K1 = math.sqrt(3.0 / (4.0 * math.pi))
K2 = math.sqrt(15.0 / math.pi) / 2.0
K3 = math.sqrt(5.0 / math.pi) / 4.0
A3 = math.sqrt(35.0 / (2.0 * math.pi)) / 4.0
B3 = math.sqrt(105.0 / math.pi) / 2.0
C3 = math.sqrt(21.0 / (2.0 * math.pi)) / 4.0
E3 = math.sqrt(7.0 / math.pi) / 4.0


def basis(d, degree):
    """Y_j(d) for j < (degree+1)^2; d is (3, N); returns ((degree+1)^2, N)."""
    x, y, z = d
    out = [np.full_like(x, K0)]
    if degree >= 1:
        out += [-K1 * y, K1 * z, -K1 * x]
    if degree >= 2:
        out += [K2 * x * y, -K2 * y * z, K3 * (2 * z * z - x * x - y * y),
                -K2 * x * z, 0.5 * K2 * (x * x - y * y)]
    if degree >= 3:
        out += [-A3 * y * (3 * x * x - y * y), B3 * x * y * z,
                -C3 * y * (4 * z * z - x * x - y * y),
                E3 * z * (2 * z * z - 3 * x * x - 3 * y * y),
                -C3 * x * (4 * z * z - x * x - y * y),
                0.5 * B3 * z * (x * x - y * y), -A3 * x * (x * x - 3 * y * y)]
    return np.stack(out, 0)


def basis_grad(d, degree):
    """dY_j/d(x, y, z) of the polynomials above; returns ((degree+1)^2, 3, N)."""
    x, y, z = d
    zero = np.zeros_like(x)
    rows = [(zero, zero, zero)]
    if degree >= 1:
        rows += [(zero, -K1 + zero, zero), (zero, zero, K1 + zero), (-K1 + zero, zero, zero)]
    if degree >= 2:
        rows += [(K2 * y, K2 * x, zero),
                 (zero, -K2 * z, -K2 * y),
                 (-2 * K3 * x, -2 * K3 * y, 4 * K3 * z),
                 (-K2 * z, zero, -K2 * x),
                 (K2 * x, -K2 * y, zero)]
    if degree >= 3:
        rows += [(-A3 * 6 * x * y, -A3 * (3 * x * x - 3 * y * y), zero),
                 (B3 * y * z, B3 * x * z, B3 * x * y),
                 (C3 * 2 * x * y, -C3 * (4 * z * z - x * x - 3 * y * y), -C3 * 8 * y * z),
                 (-E3 * 6 * x * z, -E3 * 6 * y * z, E3 * (6 * z * z - 3 * x * x - 3 * y * y)),
                 (-C3 * (4 * z * z - 3 * x * x - y * y), C3 * 2 * x * y, -C3 * 8 * x * z),
                 (B3 * x * z, -B3 * y * z, 0.5 * B3 * (x * x - y * y)),
                 (-A3 * (3 * x * x - 3 * y * y), A3 * 6 * x * y, zero)]
    return np.stack([np.stack(r, 0) for r in rows], 0)
