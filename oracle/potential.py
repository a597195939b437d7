"""Off-surface potential u = D[sigma] (eq. intrep; oracle step O7), or
u = D[sigma] + eta S[sigma] for the combined form (eq. bwform, params.eta).

Reading used: at a target z every panel J is summed with the plain q-point
rule when the nearest node of J is at least pot_beta * h_J away, and with
pot_nsub sub-panels (sigma interpolated) otherwise.  Targets must lie in the
water; inside a particle the same sum gives the interior field of D[sigma].
"""
from __future__ import annotations

import numpy as np

from .operator import layer_kernel
from .qbx import oversampled_row


def eval_potential(disc, sigma, targets):
    targets = np.asarray(targets, dtype=np.float64).reshape(-1, 2)
    q = disc.params.q
    out = np.empty(targets.shape[0])
    for a, z in enumerate(targets):
        k = disc.w * layer_kernel(disc, z[None, :], disc.x, disc.normal)
        d2 = ((disc.x - z) ** 2).sum(axis=1).reshape(-1, q).min(axis=1)
        near = np.nonzero(d2 < (disc.params.pot_beta * disc.panel_h) ** 2)[0]
        mask = np.ones(disc.N, dtype=bool)
        v = 0.0
        for J in near:
            cols = np.arange(J * q, (J + 1) * q)
            mask[cols] = False
            v += oversampled_row(disc, z, int(J), disc.params.pot_nsub) @ sigma[cols]
        out[a] = v + k[mask] @ sigma[mask]
    return out
