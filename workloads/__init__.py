"""Seeded synthetic particle ensembles.

This module only draws inputs: ellipse centres, orientations, semi-axes,
screening constants and random densities.  It holds none of the integral
equation arithmetic, so both the HIP path and the CPU oracle can be fed from
it without sharing any of the method.

The ensembles follow the paper's large-collection experiments (random,
non-overlapping particles in an Lx x Ly box, section S2.5, Table 2) with the
ellipse shapes of section 2.1 (centre a_i, director angle theta_i along the
major axis, semi-axes a_i >= b_i).

Placement recipe (rejection sampling, numpy ``default_rng(seed)``):
  * centre uniform in [A_max + margin, L - A_max - margin]^2, angle U[0, 2pi),
  * accept when the sampled boundary-to-boundary distance to every placed
    ellipse, minus the sampling resolution, is at least ``gap``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Particles",
    "two_ellipses",
    "random_ellipses",
    "config_small",
    "config_medium",
    "config_large",
    "batched_configs",
    "batched_plan",
    "batched_layout",
    "batch_member_200",
    "serving_trace",
    "single_disk",
    "grid_ellipses",
    "config_dynamics",
    "random_density",
]

_NSAMPLE = 128  # boundary samples per ellipse for the overlap test


@dataclasses.dataclass
class Particles:
    """A set of rigid ellipses.

    center: (n, 2) centres a_i;  angle: (n,) director angles theta_i (the
    director d_i = (cos, sin) is parallel to the major axis);  axes: (n, 2)
    semi-axes (A_i, B_i) with A_i along d_i.  kappa = 1/rho is the inverse
    screening length.
    """

    center: np.ndarray
    angle: np.ndarray
    axes: np.ndarray
    kappa: float
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.center.shape[0])

    def copy(self) -> "Particles":
        return Particles(self.center.copy(), self.angle.copy(), self.axes.copy(),
                         float(self.kappa), self.name)


def _boundary_samples(center, angle, axes, m=_NSAMPLE):
    t = np.linspace(0.0, 2.0 * np.pi, m, endpoint=False)
    c, s = math.cos(angle), math.sin(angle)
    ex = axes[0] * np.cos(t)
    ey = axes[1] * np.sin(t)
    return np.stack([center[0] + c * ex - s * ey, center[1] + s * ex + c * ey], axis=1)


def _sample_spacing(axes, m=_NSAMPLE):
    # the largest chord between consecutive samples is at most A * 2pi/m
    return float(axes[0]) * 2.0 * np.pi / m


def _place(rng, n, box, axes_fn, gap, amax, max_tries=200000):
    """Rejection sampling; placed ellipses are looked up through a grid of cells of
    side >= 2 amax + gap, so only the 3 x 3 cells around a candidate are checked."""
    centers: List[np.ndarray] = []
    angles: List[float] = []
    axes: List[np.ndarray] = []
    samples: List[np.ndarray] = []
    cell = 2.0 * amax + gap + 1e-6
    grid: dict = {}
    tries = 0
    while len(centers) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"could not place {n} ellipses in box {box} (placed {len(centers)})")
        ax = np.asarray(axes_fn(rng), dtype=np.float64)
        lo = ax[0] + 0.5 * gap
        c = rng.uniform(lo, box - lo, size=2)
        th = rng.uniform(0.0, 2.0 * np.pi)
        gx, gy = int(c[0] // cell), int(c[1] // cell)
        near = sorted(j for ix in (gx - 1, gx, gx + 1) for iy in (gy - 1, gy, gy + 1)
                      for j in grid.get((ix, iy), ()))
        ok = True
        sel = []
        cx, cy, a0, b0 = float(c[0]), float(c[1]), float(ax[0]), float(ax[1])
        for j in near:
            d = math.hypot(centers[j][0] - cx, centers[j][1] - cy)
            if d < axes[j][0] + a0 + gap + 1e-6:
                if d < axes[j][1] + b0 + gap:
                    ok = False  # the inscribed circles alone are closer than the gap
                    break
                sel.append(j)
        if ok and sel:
            sp = _boundary_samples(c, th, ax)
            for j in sel:
                dd = np.sqrt(((sp[:, None, :] - samples[j][None, :, :]) ** 2).sum(-1)).min()
                slack = 0.5 * (_sample_spacing(ax) + _sample_spacing(axes[j]))
                # the sampled minimum can only overestimate the true one
                if dd - slack < gap + 1e-3:
                    ok = False
                    break
        if ok:
            grid.setdefault((gx, gy), []).append(len(centers))
            centers.append(c)
            angles.append(th)
            axes.append(ax)
            samples.append(_boundary_samples(c, th, ax))
    return np.asarray(centers), np.asarray(angles), np.asarray(axes)


def random_ellipses(n: int, box: float, kappa: float, seed: int, gap: float = 0.2,
                    axes=(1.0, 0.5), axes_range=None, name: str = "") -> Particles:
    """n ellipses at random non-overlapping positions in a box x box square.

    axes: fixed semi-axes (A, B); or axes_range=((Alo, Ahi), (Blo, Bhi)) draws
    A and B uniformly per particle.
    """
    rng = np.random.default_rng(seed)
    if axes_range is None:
        fixed = np.asarray(axes, dtype=np.float64)
        axes_fn = lambda r: fixed
        amax = float(fixed[0])
    else:
        (alo, ahi), (blo, bhi) = axes_range
        axes_fn = lambda r: np.array([r.uniform(alo, ahi), r.uniform(blo, bhi)])
        amax = float(ahi)
    c, th, ax = _place(rng, n, box, axes_fn, gap, amax)
    return Particles(c, th, ax, float(kappa), name or f"{n} ellipses, box {box}, seed {seed}")


def two_ellipses(seed: int = 0, kappa: float = 1.0) -> Particles:
    """Two 1.0 x 0.5 ellipses with centres 2.5 apart and random orientations."""
    rng = np.random.default_rng(seed)
    center = np.array([[-1.25, 0.0], [1.25, 0.0]])
    angle = rng.uniform(0.0, 2.0 * np.pi, size=2)
    axes = np.array([[1.0, 0.5], [1.0, 0.5]])
    return Particles(center, angle, axes, float(kappa), f"2 ellipses, seed {seed}")


def single_disk(radius: float = 1.0, kappa: float = 0.25, angle: float = 0.0,
                center=(0.0, 0.0)) -> Particles:
    """One disk of the given radius (the single-particle validation, section S2.2)."""
    return Particles(np.array([list(center)], dtype=np.float64), np.array([angle]),
                     np.array([[radius, radius]]), float(kappa), "disk")


def grid_ellipses(nx: int = 10, ny: int = 10, spacing: float = 2.5, kappa: float = 1.0,
                  seed: int = 0, axes=(1.0, 0.5)) -> Particles:
    """nx x ny ellipses on a square grid with uniformly random orientations (the
    constant-drag movie of the supplement: 100 particles on a 10 x 10 grid).

    With spacing > 2 A no two ellipses, and no two circles of the three-circle
    repulsion model (each reaches at most A from its centre), can touch."""
    rng = np.random.default_rng(seed)
    gx, gy = np.meshgrid(np.arange(nx) * spacing, np.arange(ny) * spacing, indexing="xy")
    center = np.stack([gx.ravel(), gy.ravel()], axis=1).astype(np.float64)
    angle = rng.uniform(0.0, 2.0 * np.pi, size=nx * ny)
    ax = np.tile(np.asarray(axes, dtype=np.float64), (nx * ny, 1))
    return Particles(center, angle, ax, float(kappa), f"{nx}x{ny} grid, spacing {spacing}, seed {seed}")


# --- the named workloads -------------------------------------------------------------------

def config_small(seed: int = 0) -> dict:
    """2 ellipses 1.0x0.5, 16 panels x 16 nodes (N=512), kappa=1, QBX order 8."""
    return dict(particles=two_ellipses(seed, 1.0), panels=16, qbx_order=8, tol=1e-10,
                name="2 ellipses N=512")


def config_medium(kappa: float = 1.0, seed: int = 0) -> dict:
    """50 ellipses 1.0x0.5 in a 30x30 box, gap 0.2, 32 panels x 16 nodes (N=25,600), QBX order 10."""
    p = random_ellipses(50, 30.0, kappa, seed, gap=0.2)
    return dict(particles=p, panels=32, qbx_order=10, tol=1e-8,
                name=f"50 ellipses N=25600 kappa={kappa:g}")


def config_large(seed: int = 0) -> dict:
    """500 ellipses, A~U[0.8,1.2], B~U[0.4,0.6], 100x100 box, N=256,000, QBX order 10."""
    p = random_ellipses(500, 100.0, 1.0, seed, gap=0.2, axes_range=((0.8, 1.2), (0.4, 0.6)))
    return dict(particles=p, panels=32, qbx_order=10, tol=1e-8, fmm_order=20, fmm_leaf=64,
                name="500 ellipses N=256000")


def config_dynamics(seed: int = 0) -> dict:
    """100 ellipses 1.0x0.5 on a 10x10 grid of spacing 2.5 with random orientations,
    32 panels x 16 nodes (N=51,200), kappa=1, QBX order 10, FMM far field (far mode
    AUTO), linear extrapolation of the density as GMRES's guess; constant-drag time
    stepping with the supplement's movie drags xi_x = 1.5, xi_theta = 2.0, gamma = 1,
    repulsion c0 = 0.02, q = 3 and dt = 0.02.  Forward Euler is stable while
    2 k dt / xi_x < 2 for the relative motion of the closest pair, k = 4 c0 / g^5 the
    stiffness of one circle pair; the trajectory settles at gaps near 0.3, where
    dt = 0.02 keeps 2 k dt / xi_x near 1 (dt = 0.05 oscillates there)."""
    p = grid_ellipses(10, 10, 2.5, 1.0, seed)
    return dict(particles=p, panels=32, qbx_order=10, tol=1e-8, dt=0.02, xi_x=1.5, xi_theta=2.0,
                gamma=1.0, c0=0.02, q=3, name="100 ellipses on a 10x10 grid, N=51200")


def batched_plan(count: int, seed: int = 0, nmin: int = 10, nmax: int = 200,
                 kappa_range=(0.5, 2.0)) -> List[dict]:
    """The draws of `batched_configs` (particle count, kappa, layout seed per
    configuration) without the layouts, which `batched_layout` makes one by one."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        kappa = float(rng.uniform(*kappa_range))
        out.append(dict(id=c, n=n, kappa=kappa, seed=int(rng.integers(2**31))))
    return out


def batched_layout(item: dict) -> Particles:
    n = item["n"]
    return random_ellipses(n, 30.0 * math.sqrt(n / 50.0), item["kappa"], seed=item["seed"],
                           gap=0.2, name=f"batch {item['id']}: {n} ellipses")


def batched_configs(count: int, seed: int = 0, nmin: int = 10, nmax: int = 200,
                    kappa_range=(0.5, 2.0)) -> List[Particles]:
    """`count` independent configurations with log-uniform particle counts in [nmin, nmax].

    Box side L = 30 sqrt(n/50) keeps the 50-in-30x30 density; kappa ~ U(kappa_range).
    """
    return [batched_layout(it) for it in batched_plan(count, seed, nmin, nmax, kappa_range)]


def batch_member_200() -> Particles:
    """A 200-ellipse configuration drawn like the batched workload's largest members
    (box 30 sqrt(200/50) = 60, gap 0.2, axes 1.0 x 0.5, kappa 1.7, seed 11)."""
    n = 200
    return random_ellipses(n, 30.0 * math.sqrt(n / 50.0), 1.7, seed=11, gap=0.2,
                           name="200-ellipse batch member")


def serving_trace(count: int, rate: float = 200.0, seed: int = 0, nmin: int = 10,
                  nmax: int = 2000, kappa_range=(0.5, 2.0)) -> List[dict]:
    """A Poisson arrival trace of solve requests.

    Each request: arrival time (s), particle count log-uniform in [nmin, nmax],
    kappa ~ U(kappa_range), and the seed of its layout (drawn lazily with
    `trace_particles`).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        out.append(dict(id=k, arrival=t, n=n, kappa=float(rng.uniform(*kappa_range)),
                        seed=int(rng.integers(2**31))))
    return out


def trace_particles(req: dict) -> Particles:
    n = req["n"]
    return random_ellipses(n, 30.0 * math.sqrt(n / 50.0), req["kappa"], req["seed"], gap=0.2,
                           name=f"request {req['id']}: {n} ellipses")


def random_density(N: int, seed: int) -> np.ndarray:
    """A seeded random density vector (for operator tests)."""
    return np.random.default_rng(seed).standard_normal(N)
