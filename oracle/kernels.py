"""Yukawa layer kernels and their target gradients (oracle step O3).

G(x, y) = K0(kappa |x - y|) / (2 pi)             (eq. Gfunc, kappa = 1/rho)
dG/dnu_y = (kappa / 2 pi) K1(kappa r) (x - y).nu_y / r,      r = |x - y|
grad_x dG/dnu_y = (kappa / 2 pi) [ K1(kappa r) nu_y / r
                  - ((x - y).nu_y) (x - y) (kappa r K0(kappa r) + 2 K1(kappa r)) / r^3 ]
grad_x G = -(kappa / 2 pi) K1(kappa r) (x - y) / r
The second line follows from grad_y K0(kappa|x-y|) = kappa K1 (x-y)/r, the
third from K1'(z) = -K0(z) - K1(z)/z, the last from K0' = -K1.  G is the kernel
of the single layer potential (eq. single-layer-def), dG/dnu_y that of the
double layer (eq. double-layer-def).
"""
from __future__ import annotations

import numpy as np
from scipy import special


def dl_kernel(x, y, ny, kappa):
    """dG/dnu_y for targets x (..., 2), sources y (..., 2), normals ny (..., 2)."""
    d = x - y
    r = np.hypot(d[..., 0], d[..., 1])
    dn = d[..., 0] * ny[..., 0] + d[..., 1] * ny[..., 1]
    return kappa / (2.0 * np.pi) * special.k1(kappa * r) * dn / r


def dl_grad_kernel(x, y, ny, kappa):
    """grad_x dG/dnu_y, returned as (gx, gy)."""
    d = x - y
    r = np.hypot(d[..., 0], d[..., 1])
    dn = d[..., 0] * ny[..., 0] + d[..., 1] * ny[..., 1]
    k0 = special.k0(kappa * r)
    k1 = special.k1(kappa * r)
    a = k1 / r
    b = dn * (kappa * r * k0 + 2.0 * k1) / r**3
    c = kappa / (2.0 * np.pi)
    return c * (a * ny[..., 0] - b * d[..., 0]), c * (a * ny[..., 1] - b * d[..., 1])


def sl_kernel(x, y, kappa):
    """G(x, y) for targets x (..., 2) and sources y (..., 2)."""
    d = x - y
    r = np.hypot(d[..., 0], d[..., 1])
    return special.k0(kappa * r) / (2.0 * np.pi)


def sl_grad_kernel(x, y, kappa):
    """grad_x G, returned as (gx, gy)."""
    d = x - y
    r = np.hypot(d[..., 0], d[..., 1])
    a = -kappa / (2.0 * np.pi) * special.k1(kappa * r) / r
    return a * d[..., 0], a * d[..., 1]
