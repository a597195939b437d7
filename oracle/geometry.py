"""Panel discretisation of ellipse boundaries (oracle step O1).

Section 2.1 gives the particles: centre a_i, director d_i = (cos th_i, sin th_i)
parallel to the major axis, semi-axes a_i >= b_i.  Section 5 (Theorem
qbx-accuracy) discretises the boundary with q-point composite Gauss-Legendre
panels.

Reading used here: the ellipse is parametrised counter-clockwise,
    gamma(t) = a + R(th) (A cos t, B sin t),   t in [0, 2 pi),
split into P equal-parameter panels [2 pi k / P, 2 pi (k+1) / P]; each panel
carries the q Gauss-Legendre nodes of that interval.  The unit normal points
out of the particle (into the water): nu = (gamma'_y, -gamma'_x) / |gamma'|.
The quadrature weight of a node is w = (pi / P) omega_m |gamma'(t_m)|.
Node order: particle, then panel (increasing t), then node (increasing t).

Adaptive refinement near contact (section 5 states QBX's preconditions after
Theorem qbx-accuracy: the expansion disks must be free of other geometry and the
panels next to a target adequately resolved; the paper refines at most 3-5
levels per time step).  Reading used: a panel is the parameter interval
2 pi / P (k + [idx, idx + 1] 2^-lev) of base panel k at level lev; refinement
passes split (at the parameter midpoint) every panel whose arclength h exceeds
refine_ratio times its distance to the nearest node of another particle, at
most refine_levels times; then the panels of a particle are balanced so that the
qbx_window panels on either side of any panel are at most one level coarser
than it (coarser ones are split).  With refine_ratio 2 the
expansion disk (radius qbx_radius h = h/4, centre h/4 off the boundary) stays at
least its own radius away from every other particle.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Params:
    """Discretisation parameters.

    panels: panels per particle;  q: Gauss-Legendre nodes per panel;
    qbx_order: p, the local expansion keeps orders -p..p (section 5);
    qbx_window: panels on each side of the target's own panel whose
        contribution goes through the expansion;
    qbx_nsub: sub-panels per window panel for the coefficient quadrature;
    qbx_radius: expansion radius as a fraction of the target's panel length;
    near_beta: a non-QBX panel J is near a target when the smallest distance
        from the target to one of J's nodes is below near_beta * h_J;
    near_nsub: sub-panels for the oversampled direct rule of such panels;
    pot_nsub: sub-panels for off-surface targets closer than pot_beta * h_J;
    refine_levels, refine_ratio: adaptive refinement near contact (module
        docstring); 0 levels keeps the P equal-parameter panels;
    eta: coupling of the combined representation u = D[sigma] + eta S[sigma]
        (the Brakhage-Werner form of eq. bwform written for the screened
        equation: with k = i kappa the coupling is real; reading used: eta >= 0,
        eta = 0 is the double layer of eq. intrep).  The second-kind equation
        becomes 1/2 sigma + D sigma + eta S sigma = f.
    """

    panels: int = 16
    q: int = 16
    qbx_order: int = 8
    qbx_nsub: int = 4
    qbx_radius: float = 0.25
    qbx_window: int = 2
    near_beta: float = 0.5
    near_nsub: int = 4
    pot_nsub: int = 8
    pot_beta: float = 0.5
    eta: float = 0.0
    refine_levels: int = 0
    refine_ratio: float = 2.0


def gauss_legendre(q: int):
    """Nodes (ascending) and weights of the q-point Gauss-Legendre rule on [-1, 1]."""
    x, w = np.polynomial.legendre.leggauss(q)
    return x, w


def ellipse_eval(center, angle, axes, t):
    """Position and derivative of gamma(t) for one ellipse; t an array."""
    t = np.asarray(t, dtype=np.float64)
    c, s = np.cos(angle), np.sin(angle)
    ex, ey = axes[0] * np.cos(t), axes[1] * np.sin(t)
    dx, dy = -axes[0] * np.sin(t), axes[1] * np.cos(t)
    pos = np.stack([center[0] + c * ex - s * ey, center[1] + s * ex + c * ey], axis=-1)
    der = np.stack([c * dx - s * dy, s * dx + c * dy], axis=-1)
    return pos, der


def normal_and_speed(der):
    speed = np.hypot(der[..., 0], der[..., 1])
    nrm = np.stack([der[..., 1], -der[..., 0]], axis=-1) / speed[..., None]
    return nrm, speed


@dataclasses.dataclass
class Discretization:
    x: np.ndarray        # (N, 2) node positions
    normal: np.ndarray   # (N, 2) unit normals into the water
    w: np.ndarray        # (N,)   quadrature weights (arclength)
    t: np.ndarray        # (N,)   parameter values
    particle: np.ndarray  # (N,) particle index
    panel: np.ndarray    # (N,)   global panel index (node i is node i % q of panel i // q)
    panel_h: np.ndarray  # (npan,) panel arclengths (sum of the panel's weights)
    params: Params
    center: np.ndarray
    angle: np.ndarray
    axes: np.ndarray
    kappa: float
    desc: np.ndarray = None       # (npan, 3) base panel k, level, index at that level
    panel_pid: np.ndarray = None  # (npan,) particle of each panel
    poff: np.ndarray = None       # (n + 1,) first panel of each particle

    @property
    def N(self):
        return self.x.shape[0]

    @property
    def n(self):
        return self.center.shape[0]


def panel_params(desc, P, xi):
    """Parameter t at coordinates xi in [-1, 1] of panel desc = (k, lev, idx), and the
    factor dt/dxi = (pi / P) 2^-lev."""
    k, lev, idx = (int(desc), 0, 0) if np.ndim(desc) == 0 else (int(desc[0]), int(desc[1]),
                                                                   int(desc[2]))
    t = 2.0 * np.pi / P * (k + np.ldexp(idx + (xi + 1.0) / 2.0, -lev))
    return t, np.ldexp(np.pi / P, -lev)


def panel_nodes(center, angle, axes, k, P, q, nsub=1):
    """Nodes of panel k of one ellipse (a base panel index, or (k, lev, idx) of a
    refined panel), optionally split into nsub equal sub-panels.

    Returns positions (nsub*q, 2), normals, weights and the local coordinate of
    every node in the coarse panel's [-1, 1] (used for interpolation).
    """
    xg, wg = gauss_legendre(q)
    pos_l, nrm_l, w_l, xi_l = [], [], [], []
    for s in range(nsub):
        xi = -1.0 + (2.0 * s + (xg + 1.0)) / nsub          # coordinate in the coarse panel
        t, dt = panel_params(k, P, xi)
        pos, der = ellipse_eval(center, angle, axes, t)
        nrm, speed = normal_and_speed(der)
        pos_l.append(pos)
        nrm_l.append(nrm)
        w_l.append((dt / nsub) * wg * speed)
        xi_l.append(xi)
    return (np.concatenate(pos_l), np.concatenate(nrm_l), np.concatenate(w_l),
            np.concatenate(xi_l))


def refine_panels(particles, params: Params):
    """Panels of every particle after adaptive refinement near contact (module
    docstring): a list per particle of (k, lev, idx) in increasing t."""
    P, q = params.panels, params.q
    n = particles.center.shape[0]
    pans = [[(k, 0, 0) for k in range(P)] for _ in range(n)]
    if params.refine_levels <= 0 or n < 2:
        return pans

    def nodes_of(i):
        out, hs = [], []
        for d in pans[i]:
            pos, _, w, _ = panel_nodes(particles.center[i], particles.angle[i], particles.axes[i],
                                       d, P, q)
            out.append(pos)
            hs.append(w.sum())
        return out, np.array(hs)

    for _ in range(params.refine_levels):
        cur = [nodes_of(i) for i in range(n)]
        allpts = [np.concatenate(c[0]) for c in cur]
        split_any = False
        new = []
        for i in range(n):
            other = np.concatenate([allpts[j] for j in range(n) if j != i])
            keep = []
            for d, pos, h in zip(pans[i], cur[i][0], cur[i][1]):
                d2 = ((pos[:, None, :] - other[None, :, :]) ** 2).sum(-1).min()
                if d[1] < params.refine_levels and h > params.refine_ratio * np.sqrt(d2):
                    keep += [(d[0], d[1] + 1, 2 * d[2]), (d[0], d[1] + 1, 2 * d[2] + 1)]
                    split_any = True
                else:
                    keep.append(d)
            new.append(keep)
        pans = new
        if not split_any:
            break
    # balance: along each particle's ring, the panels within qbx_window of a panel
    # (those its QBX expansion takes) are at most one level coarser than it
    w = max(params.qbx_window, 1)
    for i in range(n):
        while True:
            ring = pans[i]
            m = len(ring)
            bad = [a for a in range(m)
                   if ring[a][1] + 1 < max(ring[(a + o) % m][1] for o in range(-w, w + 1))]
            if not bad:
                break
            out = []
            for a, d in enumerate(ring):
                if a in bad:
                    out += [(d[0], d[1] + 1, 2 * d[2]), (d[0], d[1] + 1, 2 * d[2] + 1)]
                else:
                    out.append(d)
            pans[i] = out
    return pans


def discretize(particles, params: Params) -> Discretization:
    """Discretise every ellipse of `particles` (any object with center/angle/axes/kappa)."""
    P, q = params.panels, params.q
    if P < 2 * params.qbx_window + 1:
        raise ValueError("need at least 2*qbx_window+1 panels per particle")
    xs, ns, ws, ts, pid, pan, hs = [], [], [], [], [], [], []
    desc, ppid, poff = [], [], [0]
    xg, wg = gauss_legendre(q)
    for i, pans in enumerate(refine_panels(particles, params)):
        for d in pans:
            t, dt = panel_params(d, P, xg)
            pos, der = ellipse_eval(particles.center[i], particles.angle[i], particles.axes[i], t)
            nrm, speed = normal_and_speed(der)
            w = dt * wg * speed
            xs.append(pos)
            ns.append(nrm)
            ws.append(w)
            ts.append(t)
            pid.append(np.full(q, i))
            pan.append(np.full(q, len(desc)))
            hs.append(w.sum())
            desc.append(d)
            ppid.append(i)
        poff.append(len(desc))
    return Discretization(np.concatenate(xs), np.concatenate(ns), np.concatenate(ws),
                          np.concatenate(ts), np.concatenate(pid), np.concatenate(pan),
                          np.asarray(hs), params, np.asarray(particles.center, dtype=np.float64),
                          np.asarray(particles.angle, dtype=np.float64),
                          np.asarray(particles.axes, dtype=np.float64), float(particles.kappa),
                          np.asarray(desc, dtype=np.int64), np.asarray(ppid), np.asarray(poff))
