"""Writes the full-size expected values of the GPU parity tests, from the oracle only.

Run from the repository root:  python tests/golden/make_goldens.py [c2] [c3] [member]

Every value here comes from `oracle/` (FP64, numpy/scipy) on inputs drawn by
`workloads/` (seeded): nothing is read back from the HIP library.

* c2: the 50-ellipse workload (N = 25,600, kappa = 1, 32 panels x 16 nodes, QBX
  order 10): the dense operator and its gradient twins, the density by dense LU
  for the smoothed 90-degree arc label, the exterior-limit surface gradient, the
  forces, torques and energy (eqs. bie, stress, force_torque, scalar-torque,
  main), and the off-surface potential (eq. intrep) at a grid of water points and
  at points 0.02-0.1 off the boundary.  -> c2_kappa1.npz
* c3: 1,024 sampled rows of the operator 1/2 I + D of the 500-ellipse workload
  (N = 256,000, kappa = 1) applied to a seeded random density.  -> c3_rows.npz
* member: a 200-ellipse configuration drawn like the batched workload's
  largest members (box 30 sqrt(200/50), kappa 1.7) at 8 panels per particle
  (N = 25,600, so that dense LU stays within reach): density by LU, forces,
  torques and energy.  -> member200_p8.npz
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle.geometry import Params  # noqa: E402


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def water_targets(parts, disc, grid_box, ngrid, min_dist):
    """Grid points outside every particle and at least min_dist from every node,
    plus points at distances 0.02, 0.05 and 0.1 off the boundary along the normal
    at every 800th node."""
    g = np.linspace(0.5, grid_box - 0.5, ngrid)
    gx, gy = np.meshgrid(g, g)
    pts = np.stack([gx.ravel(), gy.ravel()], 1)
    keep = np.ones(len(pts), dtype=bool)
    for c, a, (A, B) in zip(parts.center, parts.angle, parts.axes):
        d = pts - c
        u = np.cos(a) * d[:, 0] + np.sin(a) * d[:, 1]
        v = -np.sin(a) * d[:, 0] + np.cos(a) * d[:, 1]
        keep &= (u / A) ** 2 + (v / B) ** 2 > 1.0
    for s in range(0, len(pts), 256):
        d2 = ((pts[s:s + 256, None, :] - disc.x[None, :, :]) ** 2).sum(-1).min(1)
        keep[s:s + 256] &= d2 >= min_dist ** 2
    near = []
    for i in range(0, disc.N, 800):
        for dist in (0.02, 0.05, 0.1):
            near.append(disc.x[i] + dist * disc.normal[i])
    return np.concatenate([pts[keep], np.array(near)])


def solve_and_forces(disc):
    t = time.time()
    A, Gx, Gy = oracle.build_matrices(disc, gradient=True)
    log(f"  dense operator and gradient twins: {time.time() - t:.0f} s")
    f = oracle.arc_label(disc)
    t = time.time()
    sigma = oracle.lu_solve(A, f)
    log(f"  LU: {time.time() - t:.0f} s, residual {np.linalg.norm(A @ sigma - f) / np.linalg.norm(f):.2e}")
    del A
    grad = oracle.surface_fields(Gx, Gy, sigma)
    del Gx, Gy
    F, tau, _, energy = oracle.forces_torques(disc, f, grad)
    return f, sigma, grad, F, tau, energy


def make_c2():
    cfg = workloads.config_medium(kappa=1.0, seed=0)
    parts = cfg["particles"]
    disc = oracle.discretize(parts, Params(panels=cfg["panels"], qbx_order=cfg["qbx_order"]))
    log(f"c2: N = {disc.N}")
    f, sigma, grad, F, tau, energy = solve_and_forces(disc)
    targets = water_targets(parts, disc, 30.0, 32, 0.1)
    t = time.time()
    u = oracle.eval_potential(disc, sigma, targets)
    log(f"  potential at {len(targets)} targets: {time.time() - t:.0f} s")
    np.savez_compressed(os.path.join(HERE, "c2_kappa1.npz"), sigma=sigma, grad=grad, force=F,
                        torque=tau, energy=energy, targets=targets, potential=u, f=f)


def make_c3():
    cfg = workloads.config_large(seed=0)
    disc = oracle.discretize(cfg["particles"], Params(panels=cfg["panels"],
                                                      qbx_order=cfg["qbx_order"]))
    sigma = workloads.random_density(disc.N, 3)
    rows = np.sort(np.random.default_rng(5).choice(disc.N, 1024, replace=False))
    log(f"c3: N = {disc.N}, {len(rows)} rows")
    t = time.time()
    vals = oracle.apply_rows(disc, rows.tolist(), sigma)
    log(f"  rows: {time.time() - t:.0f} s")
    np.savez_compressed(os.path.join(HERE, "c3_rows.npz"), rows=rows, values=vals,
                        density_seed=np.array(3))


def make_member():
    parts = workloads.batch_member_200()
    disc = oracle.discretize(parts, Params(panels=8, qbx_order=10))
    log(f"member: N = {disc.N}")
    f, sigma, grad, F, tau, energy = solve_and_forces(disc)
    np.savez_compressed(os.path.join(HERE, "member200_p8.npz"), sigma=sigma, force=F, torque=tau,
                        energy=energy, f=f)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c3", "c2", "member"]
    for w in which:
        {"c2": make_c2, "c3": make_c3, "member": make_member}[w]()
    log("done")
