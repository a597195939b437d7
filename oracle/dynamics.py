"""Excluded-volume repulsion and the constant-drag time step (oracle step O8).

Repulsion of two circles (eq. repul): with centres a_i, a_j, radii b_i, b_j and
order q,

    F_ij = c0 q (|a_i - a_j| - (b_i + b_j))^-(q+1) (a_i - a_j) / |a_i - a_j|,

the negative gradient in a_i of the pair potential c0 (|a_i - a_j| - (b_i + b_j))^-q.

Ellipses (supplementary section S1): particle i is represented by three circles
of radius B_i (its semi-minor axis) centred at a_i + k h_i d_i, k in {-1, 0, +1},
h_i = A_i - B_i, d_i = (cos theta_i, sin theta_i).  Each of the nine circle
pairs of two particles interacts through eq. repul with c0 / 3:

    f_ij^kl   = (c0/3) q (|a_i^k - a_j^l| - (B_i + B_j))^-(q+1) e_ij^kl,
    F_i^rep   = sum_{j != i} sum_{k,l} f_ij^kl,
    tau_i^rep = sum_{j != i} sum_l h_i (f_ij^{-1,l} - f_ij^{+1,l}) x d_i,
    Phi_rep   = 1/2 sum_i sum_{j != i} sum_{k,l} (c0/3) (|a_i^k - a_j^l| - (B_i + B_j))^-q,

with e_ij^kl the unit vector from a_j^l to a_i^k and u x v = u_x v_y - u_y v_x.
tau_i^rep is the torque about a_i of the forces on the two end circles.

Readings (the supplement's formulas are partly garbled):
  * the printed potential sums over k alone while its summand depends on l: it
    is read as the sum over k and l, the potential whose negative gradient is
    the printed force;
  * the printed closing remark says the ellipse force equals eq. repul for
    circles.  With A = B the three circles coincide and the nine pairs give three
    times eq. repul; the printed formulas are followed and c0 is the caller's;
  * circles that touch or overlap (|a_i^k - a_j^l| <= B_i + B_j) have no finite
    repulsion: an error.

Time step (eq. euler, the constant-drag law of the supplement's numerical
validations; Algorithm 1 without the Stokes mobility solve):

    a_i     <- a_i     + dt / xi_x     (F_i   + F_i^rep),
    theta_i <- theta_i + dt / xi_theta (tau_i + tau_i^rep).

Reading: the torque of eq. euler holds the repulsion torque too (Algorithm 1
computes both kinds of force before the update).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def circle_centres(center, angle, axes):
    """Centres (n, 3, 2) of the circles k = -1, 0, +1, their radius (n,) and h (n,)."""
    center = np.asarray(center, dtype=np.float64)
    angle = np.asarray(angle, dtype=np.float64)
    axes = np.asarray(axes, dtype=np.float64)
    d = np.stack([np.cos(angle), np.sin(angle)], axis=1)
    h = axes[:, 0] - axes[:, 1]
    ks = np.array([-1.0, 0.0, 1.0])
    cc = center[:, None, :] + ks[None, :, None] * h[:, None, None] * d[:, None, :]
    return cc, axes[:, 1].copy(), h


def repulsion(center, angle, axes, c0, q=3):
    """Excluded-volume force (n, 2), torque about a_i (n,) and potential Phi_rep.

    Plain loops over particle pairs and over the nine circle pairs of each.
    """
    cc, rad, h = circle_centres(center, angle, axes)
    n = cc.shape[0]
    F = np.zeros((n, 2))
    tau = np.zeros(n)
    phi = 0.0
    c = c0 / 3.0
    for i in range(n):
        di = np.array([np.cos(angle[i]), np.sin(angle[i])])
        for j in range(n):
            if j == i:
                continue
            for k in range(3):
                fk = np.zeros(2)
                for l in range(3):
                    r = cc[i, k] - cc[j, l]
                    dist = float(np.hypot(r[0], r[1]))
                    gap = dist - (rad[i] + rad[j])
                    if not gap > 0.0:
                        raise ValueError(f"circles {i}:{k} and {j}:{l} touch or overlap")
                    f = c * q / gap ** (q + 1) * r / dist
                    fk += f
                    phi += 0.5 * c / gap ** q
                F[i] += fk
                # k - 1 in {-1, 0, +1}: the end circles carry the torque
                sgn = k - 1
                if sgn != 0:
                    tau[i] += -sgn * h[i] * (fk[0] * di[1] - fk[1] * di[0])
    return F, tau, phi


def euler_update(center, angle, force, torque, dt, xi_x, xi_theta):
    """One forward Euler step of eq. euler: new centres (n, 2) and angles (n,)."""
    return (np.asarray(center) + dt / xi_x * np.asarray(force),
            np.asarray(angle) + dt / xi_theta * np.asarray(torque))


@dataclasses.dataclass
class StepResult:
    sigma: np.ndarray        # density at the configuration the step started from
    force: np.ndarray        # hydrophobic force F_i (n, 2)
    torque: np.ndarray       # hydrophobic torque about a_i (n,)
    energy: float            # hydrophobic energy Phi
    force_rep: np.ndarray    # F_i^rep (n, 2)
    torque_rep: np.ndarray   # tau_i^rep (n,)
    energy_rep: float        # Phi_rep
    particles: object        # the configuration after the step


def time_step(particles, params, label, gamma, c0, q, dt, xi_x, xi_theta):
    """Solve eq. bie at the current configuration (dense LU), hydrophobic forces
    (eqs. stress, force_torque), repulsion, then the Euler update of eq. euler.

    label(disc) gives the boundary data f at the nodes.
    """
    from . import forces as _forces
    from . import geometry as _geometry
    from . import operator as _operator
    from . import solve as _solve

    d = _geometry.discretize(particles, params)
    A, Gx, Gy = _operator.build_matrices(d, gradient=True)
    f = label(d)
    sigma = _solve.lu_solve(A, f)
    F, tau, _, E = _forces.forces_torques(d, f, _forces.surface_fields(Gx, Gy, sigma), gamma)
    Fr, tr, Er = repulsion(particles.center, particles.angle, particles.axes, c0, q)
    c, a = euler_update(particles.center, particles.angle, F + Fr, tau + tr, dt, xi_x, xi_theta)
    new = particles.copy()
    new.center = c
    new.angle = a
    return StepResult(sigma, F, tau, E, Fr, tr, Er, new)
