"""The discrete operator 1/2 I + D (oracle steps O3-O4) and its gradient twin.

Row i of the Nystrom matrix: the q-point rule w_j dG/dnu_y(x_i, y_j) for every
source node j that is neither on one of the target's QBX window panels nor on
an extra near panel; the QBX row on the window panels (the mean of the two
one-sided expansions plus 1/2 at the self node, which together give
1/2 sigma + D sigma, eq. djump and eq. bie); the oversampled row on extra
near panels.  The gradient matrices hold the same construction for grad u,
with the exterior one-sided expansion on the window (the exterior limit the
stress needs, eq. stress).
"""
from __future__ import annotations

import numpy as np

from .kernels import dl_kernel, dl_grad_kernel, sl_kernel, sl_grad_kernel
from .qbx import near_panels, qbx_row, operator_qbx_row, oversampled_row


def layer_kernel(disc, x, y, ny):
    """The kernel of the representation: dG/dnu_y, plus eta G for the combined
    form D + eta S (eq. bwform; eta = params.eta, 0 for eq. intrep)."""
    k = dl_kernel(x, y, ny, disc.kappa)
    if disc.params.eta != 0.0:
        k = k + disc.params.eta * sl_kernel(x, y, disc.kappa)
    return k


def layer_grad_kernel(disc, x, y, ny):
    gx, gy = dl_grad_kernel(x, y, ny, disc.kappa)
    if disc.params.eta != 0.0:
        sx, sy = sl_grad_kernel(x, y, disc.kappa)
        gx, gy = gx + disc.params.eta * sx, gy + disc.params.eta * sy
    return gx, gy


def _panel_cols(disc, J):
    q = disc.params.q
    return np.arange(J * q, (J + 1) * q)


def build_matrices(disc, gradient=False, chunk=512):
    """Dense A (N x N), and (Gx, Gy) when gradient=True."""
    N = disc.N
    A = np.empty((N, N))
    Gx = np.empty((N, N)) if gradient else None
    Gy = np.empty((N, N)) if gradient else None
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        xi = disc.x[s:e, None, :]
        A[s:e] = disc.w[None, :] * layer_kernel(disc, xi, disc.x[None, :, :], disc.normal[None, :, :])
        if gradient:
            gx, gy = layer_grad_kernel(disc, xi, disc.x[None, :, :], disc.normal[None, :, :])
            Gx[s:e] = disc.w[None, :] * gx
            Gy[s:e] = disc.w[None, :] * gy
    for i in range(N):
        qp, extra = near_panels(disc, i)
        _, vals = operator_qbx_row(disc, i)
        if gradient:
            _, _, grads = qbx_row(disc, i, side=1, gradient=True)
        for j, J in enumerate(qp):
            cols = _panel_cols(disc, J)
            A[i, cols] = vals[j]
            if gradient:
                Gx[i, cols] = grads[j][:, 0]
                Gy[i, cols] = grads[j][:, 1]
        for J in extra:
            cols = _panel_cols(disc, J)
            o = oversampled_row(disc, disc.x[i], J, disc.params.near_nsub, gradient=gradient)
            if gradient:
                A[i, cols] = o[0]
                Gx[i, cols] = o[1][:, 0]
                Gy[i, cols] = o[1][:, 1]
            else:
                A[i, cols] = o
    if gradient:
        return A, Gx, Gy
    return A


def far_rows(disc, rows, sigma):
    """Plain q-point direct sum over every source j != i (the far-field sum before
    near corrections): out_i = sum_{j != i} w_j dG/dnu_y(x_i, y_j) sigma_j."""
    out = np.empty(len(rows))
    for a, i in enumerate(rows):
        k = disc.w * layer_kernel(disc, disc.x[i][None, :], disc.x, disc.normal)
        k[i] = 0.0
        out[a] = k @ sigma
    return out


def far_grad_rows(disc, rows, sigma):
    out = np.empty((len(rows), 2))
    for a, i in enumerate(rows):
        gx, gy = layer_grad_kernel(disc, disc.x[i][None, :], disc.x, disc.normal)
        gx = disc.w * gx
        gy = disc.w * gy
        gx[i] = 0.0
        gy[i] = 0.0
        out[a] = [gx @ sigma, gy @ sigma]
    return out


def apply_rows(disc, rows, sigma, gradient=False):
    """(A sigma)_i for the listed rows, computed one row at a time (any N).

    With gradient=True returns (values, grads (len(rows), 2))."""
    vals = np.empty(len(rows))
    grads = np.empty((len(rows), 2))
    for a, i in enumerate(rows):
        qp, extra = near_panels(disc, i)
        k = disc.w * layer_kernel(disc, disc.x[i][None, :], disc.x, disc.normal)
        if gradient:
            gx, gy = layer_grad_kernel(disc, disc.x[i][None, :], disc.x, disc.normal)
            gx = disc.w * gx
            gy = disc.w * gy
        mask = np.ones(disc.N, dtype=bool)
        for J in qp + extra:
            mask[_panel_cols(disc, J)] = False
        v = k[mask] @ sigma[mask]
        if gradient:
            g = np.array([gx[mask] @ sigma[mask], gy[mask] @ sigma[mask]])
        _, qv = operator_qbx_row(disc, i)
        if gradient:
            _, _, qg = qbx_row(disc, i, side=1, gradient=True)
        for j, J in enumerate(qp):
            cols = _panel_cols(disc, J)
            v += qv[j] @ sigma[cols]
            if gradient:
                g += qg[j].T @ sigma[cols]
        for J in extra:
            cols = _panel_cols(disc, J)
            o = oversampled_row(disc, disc.x[i], J, disc.params.near_nsub, gradient=gradient)
            if gradient:
                v += o[0] @ sigma[cols]
                g += o[1].T @ sigma[cols]
            else:
                v += o @ sigma[cols]
        vals[a] = v
        if gradient:
            grads[a] = g
    if gradient:
        return vals, grads
    return vals
