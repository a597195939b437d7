"""Near lists, QBX rows and oversampled rows (oracle step O4).

QBX (section 5, eqs. local-exp, graf-coefficient, graf-addition).  The paper
states the scheme for the Helmholtz kernel with wavenumber k; the Yukawa
kernel is the case k = i kappa.  With K0(z) = (i pi/2) H0(iz), J_l(iz) =
i^l I_l(z) and H_l(iz) = (2/pi) i^(-l-1) K_l(z), Graf's addition theorem becomes

    K0(kappa |x - y|) = sum_l K_l(kappa |y - c|) I_l(kappa |x - c|) e^{i l (th_y - th_x)},
    |x - c| < |y - c|,

so the double layer of density sigma has, about a centre c, the local expansion

    u(x) = sum_{l=-p..p} alpha_l I_l(kappa r_x) e^{-i l th_x},
    alpha_l = (1/2pi) int d/dnu_y [K_l(kappa r_y) e^{i l th_y}] sigma(y) ds_y,
    d/dnu [K_l(kappa r) e^{i l th}] = e^{i l th} [kappa K_l'(kappa r) (rhat.nu) + (i l / r) K_l(kappa r) (thhat.nu)],

and the single layer (eq. single-layer-def) the same expansion with
alpha_l = (1/2pi) int K_l(kappa r_y) e^{i l th_y} sigma(y) ds_y; the combined
representation D + eta S (eq. bwform, params.eta) adds eta times those.  The single
layer is continuous across the boundary, so both one-sided expansions carry it,
and their mean below keeps it.

with (r, th) polar coordinates about c.  Readings used (the paper defers the
details to the GIGAQBX references):

* centres c_i = x_i +/- r_i nu_i with r_i = qbx_radius * h_k, h_k the
  arclength of the target's panel.  The centre on the water side (side=+1)
  gives the exterior limit 1/2 sigma + D sigma at x_i (eq. djump), the centre
  inside the particle (side=-1) the interior limit -1/2 sigma + D sigma.
* the operator row (operator_qbx_row) takes the principal value D sigma as
  the mean of the two one-sided limits and adds 1/2 sigma explicitly.  A
  truncated expansion cannot follow node-scale oscillations of sigma, so a
  one-sided operator maps them to almost zero instead of 1/2 sigma: with the
  exterior limit alone the discrete matrix of three ellipses (12 panels,
  p = 10) has a cluster of singular values near 7e-5 (condition 1e4, 167
  GMRES iterations on random data); with the mean it has condition 16 and
  needs 20 iterations.  The surface gradient used for the stress stays the
  exterior one-sided limit.
* the expansion takes the contribution of the target's own panel and the
  qbx_window panels on either side of it on the same particle (a window of
  2*qbx_window + 1 panels).  The truncated series of a partial arc converges
  at the rate set by the distance from the centre to the arc's end points, so
  the window must reach well beyond the expansion disk: with a 3-panel window
  and r = h/2 the truncation error on the unit disk is about 1e-6 for p = 10,
  with a 5-panel window and r = h/4 it is about 5e-12 (32 panels).  The
  coefficient integrals use qbx_nsub
  equal sub-panels of q Gauss-Legendre nodes each, with sigma carried to the
  sub-panel nodes by the degree q-1 Lagrange interpolant of the coarse values.
* orders l = -p..p (2p + 1 terms).
* every other panel J whose nearest node lies closer than near_beta * h_J to
  the target is summed with near_nsub sub-panels (oversampled direct rule);
  all remaining panels use the plain q-point rule.
"""
from __future__ import annotations

import functools

import numpy as np
from scipy import special

from .geometry import gauss_legendre, panel_nodes
from .kernels import dl_kernel, dl_grad_kernel, sl_kernel, sl_grad_kernel


def interp_matrix(src, dst):
    """Lagrange interpolation matrix L[f, m] = prod_{j != m} (dst_f - src_j) / (src_m - src_j)."""
    src = np.asarray(src, dtype=np.float64)
    dst = np.asarray(dst, dtype=np.float64)
    L = np.ones((dst.size, src.size))
    for m in range(src.size):
        for j in range(src.size):
            if j != m:
                L[:, m] *= (dst - src[j]) / (src[m] - src[j])
    return L


@functools.lru_cache(maxsize=None)
def _sub_interp(q, nsub):
    """Interpolation matrix from the q coarse nodes to the nodes of nsub sub-panels."""
    xg, _ = gauss_legendre(q)
    xi = np.concatenate([-1.0 + (2.0 * s + (xg + 1.0)) / nsub for s in range(nsub)])
    return interp_matrix(xg, xi)


def qbx_panels(disc, i):
    """The panels whose contribution at target i goes through its expansion: the
    target's own panel and the qbx_window panels on either side of it along its
    particle's ring of panels."""
    win = disc.params.qbx_window
    p = disc.particle[i]
    first, m = int(disc.poff[p]), int(disc.poff[p + 1] - disc.poff[p])
    k = int(disc.panel[i]) - first
    return [first + (k + o) % m for o in range(-win, win + 1)]


def near_panels(disc, i):
    """(qbx panel list, extra near panel list) of target i."""
    P, q = disc.params.panels, disc.params.q
    qp = qbx_panels(disc, i)
    d2 = ((disc.x - disc.x[i]) ** 2).sum(axis=1).reshape(-1, q).min(axis=1)
    near = np.nonzero(d2 < (disc.params.near_beta * disc.panel_h) ** 2)[0]
    extra = [int(J) for J in near if J not in qp]
    return qp, extra


def qbx_row(disc, i, side=1, gradient=False):
    """Row of the discrete operator for target i restricted to its QBX panels.

    Returns (panels, vals) with vals[j, m] the weight of sigma at node m of
    panels[j]; with gradient=True also grads[j, m, :] for grad u at x_i.
    """
    prm = disc.params
    P, q, p = prm.panels, prm.q, prm.qbx_order
    kap = disc.kappa
    h = disc.panel_h[disc.panel[i]]
    r_c = prm.qbx_radius * h
    c = disc.x[i] + side * r_c * disc.normal[i]
    tx = disc.x[i] - c
    rx = np.hypot(tx[0], tx[1])
    thx = np.arctan2(tx[1], tx[0])
    rhat_x = np.array([np.cos(thx), np.sin(thx)])
    thhat_x = np.array([-np.sin(thx), np.cos(thx)])
    ls = np.arange(-p, p + 1)
    Il = special.iv(ls, kap * rx)
    Ilp = special.ivp(ls, kap * rx)
    e_x = np.exp(-1j * ls * thx)
    val_fac = Il * e_x                                                   # (2p+1,)
    grad_fac = e_x[:, None] * (kap * Ilp[:, None] * rhat_x[None, :]
                               - (1j * ls / rx * Il)[:, None] * thhat_x[None, :])  # (2p+1, 2)
    pid = disc.particle[i]
    panels = qbx_panels(disc, i)
    vals = np.zeros((len(panels), q))
    grads = np.zeros((len(panels), q, 2))
    for j, J in enumerate(panels):
        y, ny, wy, xi = panel_nodes(disc.center[pid], disc.angle[pid], disc.axes[pid],
                                    disc.desc[J], P, q, prm.qbx_nsub)
        L = _sub_interp(q, prm.qbx_nsub)
        d = y - c
        ry = np.hypot(d[:, 0], d[:, 1])
        thy = np.arctan2(d[:, 1], d[:, 0])
        rn = (d[:, 0] * ny[:, 0] + d[:, 1] * ny[:, 1]) / ry               # rhat . nu
        tn = (-np.sin(thy) * ny[:, 0] + np.cos(thy) * ny[:, 1])          # thhat . nu
        Kl = special.kv(ls[:, None], kap * ry[None, :])
        Klp = special.kvp(ls[:, None], kap * ry[None, :])
        dK = np.exp(1j * ls[:, None] * thy[None, :]) * (
            kap * Klp * rn[None, :] + (1j * ls[:, None] / ry[None, :]) * Kl * tn[None, :])
        if prm.eta != 0.0:
            dK = dK + prm.eta * np.exp(1j * ls[:, None] * thy[None, :]) * Kl
        coef = dK * (wy / (2.0 * np.pi))[None, :]                         # (2p+1, F)
        cf = np.real((val_fac[:, None] * coef).sum(axis=0))
        vals[j] = cf @ L
        if gradient:
            g = np.real((grad_fac[:, None, :] * coef[:, :, None]).sum(axis=0))  # (F, 2)
            grads[j] = L.T @ g
    if gradient:
        return panels, vals, grads
    return panels, vals


def operator_qbx_row(disc, i):
    """Row of 1/2 I + D for target i on its QBX window: the mean of the exterior and
    interior one-sided expansions, plus 1/2 at the target's own node."""
    pe, ve = qbx_row(disc, i, side=1)
    _, vi = qbx_row(disc, i, side=-1)
    vals = 0.5 * (ve + vi)
    q = disc.params.q
    own = pe.index(int(disc.panel[i]))
    vals[own, i - disc.panel[i] * q] += 0.5
    return pe, vals


def oversampled_row(disc, x, J, nsub, gradient=False):
    """Weights of sigma on panel J for the double layer (plus eta times the single
    layer) at point x, by an nsub-fold oversampled Gauss-Legendre rule with
    interpolated sigma."""
    prm = disc.params
    P, q = prm.panels, prm.q
    pid = int(disc.panel_pid[J])
    y, ny, wy, xi = panel_nodes(disc.center[pid], disc.angle[pid], disc.axes[pid], disc.desc[J], P,
                                q, nsub)
    L = _sub_interp(q, nsub)
    xx = np.broadcast_to(x, y.shape)
    k = dl_kernel(xx, y, ny, disc.kappa)
    if prm.eta != 0.0:
        k = k + prm.eta * sl_kernel(xx, y, disc.kappa)
    vals = (wy * k) @ L
    if not gradient:
        return vals
    gx, gy = dl_grad_kernel(xx, y, ny, disc.kappa)
    if prm.eta != 0.0:
        sx, sy = sl_grad_kernel(xx, y, disc.kappa)
        gx, gy = gx + prm.eta * sx, gy + prm.eta * sy
    return vals, np.stack([(wy * gx) @ L, (wy * gy) @ L], axis=-1)
