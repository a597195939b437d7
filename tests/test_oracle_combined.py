"""Pins of the combined representation u = D[sigma] + eta S[sigma] (eq. bwform read
for the screened equation, k = i kappa, with a real coupling eta) in the oracle.

Each test compares the oracle with something other than its own formula:
closed forms on a disk (the single layer of e^{i n th} on a circle of radius a is
a I_n(kappa a) K_n(kappa a) e^{i n th}, so the combined operator has the
eigenvalues kappa a I_n'(kappa a) K_n(kappa a) + eta a I_n(kappa a) K_n(kappa a)),
the single layer of a constant density off the disk, a point-source manufactured
solution, the isolated-disk zero force, and the conditioning claim the paper
makes for large rho (small kappa).
"""
import math

import numpy as np
import pytest
from scipy import special

import oracle
import workloads
from oracle.geometry import Params


@pytest.mark.parametrize("kap,eta", [(0.25, 1.0), (1.0, 0.5), (2.0, 3.0)])
def test_combined_disk_eigenvalues(kap, eta):
    a = 1.0
    d = oracle.discretize(workloads.single_disk(a, kap), Params(panels=32, qbx_order=10, eta=eta))
    A = oracle.build_matrices(d)
    th = np.arctan2(d.x[:, 1], d.x[:, 0])
    for n in (0, 1, 2, 5):
        lam = kap * a * special.ivp(n, kap * a) * special.kv(n, kap * a) \
            + eta * a * special.iv(n, kap * a) * special.kv(n, kap * a)
        v = np.cos(n * th)
        assert np.abs(A @ v - lam * v).max() < 5e-11, (kap, eta, n)


def test_single_layer_of_one_on_a_disk_off_surface():
    # u = D[1] + eta S[1] outside a disk of radius a: (kappa a I_1(kappa a) +
    # eta a I_0(kappa a)) K_0(kappa R); D[1] alone is the eta = 0 case
    a, kap, eta = 1.3, 0.7, 2.0
    d = oracle.discretize(workloads.single_disk(a, kap), Params(panels=32, eta=eta))
    one = np.ones(d.N)
    for R in (1.6, 2.1, 4.0):
        x = np.array([R * math.cos(0.3), R * math.sin(0.3)])
        ref = (kap * a * special.i1(kap * a) + eta * a * special.i0(kap * a)) * special.k0(kap * R)
        u = oracle.eval_potential(d, one, np.array([x]))[0]
        assert abs(u - ref) < 1e-10, R


@pytest.fixture(scope="module")
def combined_point_sources():
    parts = workloads.Particles(np.array([[-1.3, 0.1], [1.25, -0.2], [0.1, 1.6]]),
                                np.array([0.3, 2.0, -0.9]), np.array([[1.0, 0.5]] * 3), 0.8)
    d = oracle.discretize(parts, Params(panels=12, qbx_order=10, eta=1.5))
    src = parts.center + 0.2 * np.array([[1, 0], [0, 1], [-1, 0]])
    qs = np.array([1.0, -0.6, 0.8])

    def u_exact(x):
        r = np.hypot(x[:, None, 0] - src[None, :, 0], x[:, None, 1] - src[None, :, 1])
        return (special.k0(parts.kappa * r) / (2 * np.pi)) @ qs

    def grad_exact(x):
        dx = x[:, None, :] - src[None, :, :]
        r = np.hypot(dx[..., 0], dx[..., 1])
        c = -parts.kappa * special.k1(parts.kappa * r) / r / (2 * np.pi) * qs[None, :]
        return (c[..., None] * dx).sum(1)

    A, Gx, Gy = oracle.build_matrices(d, gradient=True)
    sigma = oracle.lu_solve(A, u_exact(d.x))
    return dict(d=d, sigma=sigma, u=u_exact, g=grad_exact, Gx=Gx, Gy=Gy)


def test_combined_manufactured_solution_potential_and_gradient(combined_point_sources):
    P = combined_point_sources
    d = P["d"]
    rng = np.random.default_rng(4)
    pts = []
    while len(pts) < 30:
        z = rng.uniform(-3, 3, 2)
        if np.min(np.hypot(*(d.x - z).T)) < 0.15:
            continue
        inside = False
        for c, th, ax in zip(d.center, d.angle, d.axes):
            rel = z - c
            u = math.cos(th) * rel[0] + math.sin(th) * rel[1]
            v = -math.sin(th) * rel[0] + math.cos(th) * rel[1]
            inside |= (u / ax[0]) ** 2 + (v / ax[1]) ** 2 < 1
        if not inside:
            pts.append(z)
    pts = np.array(pts)
    u = oracle.eval_potential(d, P["sigma"], pts)
    assert np.abs(u - P["u"](pts)).max() < 1e-8
    g = oracle.surface_fields(P["Gx"], P["Gy"], P["sigma"])
    ge = P["g"](d.x)
    assert np.abs(g - ge).max() < 5e-6 * np.abs(ge).max()


def test_combined_isolated_disk_feels_no_force():
    a, kap = 1.0, 0.25
    d = oracle.discretize(workloads.single_disk(a, kap), Params(panels=16, qbx_order=8, eta=1.0))
    f = oracle.janus_label(d, 2)
    A, Gx, Gy = oracle.build_matrices(d, gradient=True)
    sigma = oracle.lu_solve(A, f)
    F, tau, _, E = oracle.forces_torques(d, f, oracle.surface_fields(Gx, Gy, sigma))
    assert np.abs(F).max() < 5e-8 and abs(tau[0]) < 5e-8
    # the energy depends on u only, not on the representation
    z = kap * a
    Eref = -(a * math.pi / 2) * (special.kvp(0, z) / special.k0(z) + 0.5 * special.kvp(1, z) / special.k1(z))
    assert abs(E - Eref) < 1e-7 * abs(Eref)


def test_combined_form_conditions_large_rho():
    # For large rho (small kappa) 1/2 I + D approaches the Laplace double layer, whose
    # exterior operator loses one dimension per particle (constants): its condition
    # number grows like 1/kappa^2.  Adding eta S keeps the system well conditioned.
    parts = workloads.Particles(np.array([[-1.3, 0.1], [1.25, -0.2], [0.1, 1.6]]),
                                np.array([0.3, 2.0, -0.9]), np.array([[1.0, 0.5]] * 3), 0.02)
    conds = {}
    for eta in (0.0, 1.0):
        d = oracle.discretize(parts, Params(panels=8, qbx_order=8, eta=eta))
        conds[eta] = np.linalg.cond(oracle.build_matrices(d))
    assert conds[0.0] > 1e3 and conds[1.0] < 1e2, conds
