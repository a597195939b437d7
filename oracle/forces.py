"""Surface gradient, hydrophobic traction, forces, torques and energy (oracle step O6).

Eq. stress:  T = gamma rho^-1 u^2 I + 2 rho gamma (1/2 |grad u|^2 I - grad u (x) grad u).
With rho = 1/kappa and nu the unit normal out of the particle (nu_i of eq.
force_torque, the same direction as the double-layer normal):

    T.nu = gamma [kappa u^2 + kappa^-1 |grad u|^2] nu - 2 gamma kappa^-1 (grad u . nu) grad u.

Eq. force_torque: F_i = int T.nu_i dS,  tau0_i = int r0 x (T.nu_i) dS;
eq. scalar-torque: tau_i = tau0_i - a_i x F_i = int (x - a_i) x (T.nu_i) dS.

Energy (eq. main, main2): Phi = gamma I[u].  Green's first identity with
Lap u = kappa^2 u gives int_Omega |grad u|^2 + kappa^2 u^2 = -int_Sigma u du/dnu
(nu points into Omega here), so Phi = -gamma kappa^-1 int_Sigma f du/dnu dS.

On the boundary u = f exactly (eq. SL); grad u is the exterior limit from the
same QBX expansions as the operator (QBX rows differentiated at the target).
"""
from __future__ import annotations

import numpy as np


def surface_fields(Gx, Gy, sigma):
    """grad u at the nodes, (N, 2), from the gradient matrices."""
    return np.stack([Gx @ sigma, Gy @ sigma], axis=1)


def traction(disc, f, grad, gamma=1.0):
    """T.nu at every node, (N, 2)."""
    kap = disc.kappa
    un = (grad * disc.normal).sum(axis=1)
    g2 = (grad**2).sum(axis=1)
    iso = gamma * (kap * f**2 + g2 / kap)
    return iso[:, None] * disc.normal - (2.0 * gamma / kap) * un[:, None] * grad


def forces_torques(disc, f, grad, gamma=1.0):
    """Per-particle force (n, 2), torque about a_i (n,), torque about the origin (n,), energy."""
    tn = traction(disc, f, grad, gamma)
    n = disc.n
    F = np.zeros((n, 2))
    tau = np.zeros(n)
    tau0 = np.zeros(n)
    for i in range(n):
        m = disc.particle == i
        w = disc.w[m]
        F[i] = (w[:, None] * tn[m]).sum(axis=0)
        rel = disc.x[m] - disc.center[i]
        tau[i] = (w * (rel[:, 0] * tn[m][:, 1] - rel[:, 1] * tn[m][:, 0])).sum()
        xo = disc.x[m]
        tau0[i] = (w * (xo[:, 0] * tn[m][:, 1] - xo[:, 1] * tn[m][:, 0])).sum()
    un = (grad * disc.normal).sum(axis=1)
    energy = -gamma / disc.kappa * (disc.w * f * un).sum()
    return F, tau, tau0, energy
