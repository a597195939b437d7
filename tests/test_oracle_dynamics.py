"""Pins of the repulsion and time-step oracle (eq. repul, supplementary section S1, eq. euler).

Each test checks the oracle against something other than its own formula: the
gradient of the potential by centred differences, Newton's third law, closed
forms for circles and for collinear ellipses worked out by hand, invariance of
the boundary label under rigid motion, and the first-order energy decrease of
a gradient-flow step.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle.geometry import Params


def _four_ellipses():
    # gaps between every pair of circles stay above 0.3
    return workloads.Particles(
        np.array([[0.0, 0.0], [2.7, 0.6], [-0.4, 2.4], [2.9, 2.9]]),
        np.array([0.3, 2.1, -0.7, 1.2]),
        np.array([[1.0, 0.5], [1.2, 0.45], [0.9, 0.6], [0.8, 0.8]]), 1.0)


@pytest.mark.parametrize("q", [3, 4])
def test_repulsion_is_negative_gradient_of_its_potential(q):
    p = _four_ellipses()
    c0 = 0.02
    F, tau, _ = oracle.repulsion(p.center, p.angle, p.axes, c0, q)

    def phi(center, angle):
        return oracle.repulsion(center, angle, p.axes, c0, q)[2]

    def rich(g):
        e = 1e-3
        d1 = (g(e) - g(-e)) / (2 * e)
        d2 = (g(e / 2) - g(-e / 2)) / e
        return (4 * d2 - d1) / 3

    scale = np.abs(F).max()
    for i in range(p.n):
        for c in range(2):
            def g(e, i=i, c=c):
                cc = p.center.copy()
                cc[i, c] += e
                return phi(cc, p.angle)
            assert abs(-rich(g) - F[i, c]) < 1e-8 * scale, (i, c)

        def ga(e, i=i):
            aa = p.angle.copy()
            aa[i] += e
            return phi(p.center, aa)
        assert abs(-rich(ga) - tau[i]) < 1e-8 * max(scale, abs(tau).max()), i
    # the circle (A = B) carries no torque
    assert tau[3] == 0.0


def test_repulsion_newton_third_law_and_angular_momentum():
    p = _four_ellipses()
    F, tau, _ = oracle.repulsion(p.center, p.angle, p.axes, 0.05, 3)
    assert np.abs(F.sum(axis=0)).max() < 1e-13 * np.abs(F).max()
    # central pair forces: the total torque about the origin vanishes
    tot = tau + p.center[:, 0] * F[:, 1] - p.center[:, 1] * F[:, 0]
    assert abs(tot.sum()) < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("q", [3, 4])
def test_repulsion_of_two_circles_is_three_times_eq_repul(q):
    # A = B: the three circles of each particle coincide, so the nine pairs with
    # c0/3 give 3 c0 q / (d - 2b)^(q+1) along the line of centres.
    b, d, c0 = 0.7, 2.3, 0.1
    center = np.array([[0.0, 0.0], [d * 0.6, d * 0.8]])
    F, tau, phi = oracle.repulsion(center, np.array([0.4, -1.1]), np.array([[b, b], [b, b]]), c0, q)
    mag = 3 * c0 * q / (d - 2 * b) ** (q + 1)
    np.testing.assert_allclose(F[0], -mag * np.array([0.6, 0.8]), rtol=1e-14)
    np.testing.assert_allclose(F[1], mag * np.array([0.6, 0.8]), rtol=1e-14)
    assert np.all(tau == 0.0)
    assert abs(phi - 3 * c0 / (d - 2 * b) ** q) < 1e-14 * phi


def test_repulsion_of_collinear_ellipses_by_hand():
    # Two 1.0 x 0.5 ellipses on the x axis with directors along x, centres 3 apart:
    # h = 0.5, circles of radius 0.5 at x = -0.5, 0, 0.5 and 2.5, 3, 3.5 (the second
    # director points along -x, which changes nothing).  All forces lie on the x
    # axis, each circle pair's gap is its centre distance minus 1, no torque.
    xs1 = [-0.5, 0.0, 0.5]
    xs2 = [2.5, 3.0, 3.5]
    dists = [b - a for a in xs1 for b in xs2]
    assert sorted(dists) == [2.0, 2.5, 2.5, 3.0, 3.0, 3.0, 3.5, 3.5, 4.0]
    c0, q = 0.3, 3
    fx = -sum(c0 / 3 * q / (r - 1.0) ** (q + 1) for r in dists)
    ph = sum(c0 / 3 / (r - 1.0) ** q for r in dists)
    F, tau, phi = oracle.repulsion(np.array([[0.0, 0.0], [3.0, 0.0]]), np.array([0.0, math.pi]),
                                   np.array([[1.0, 0.5], [1.0, 0.5]]), c0, q)
    np.testing.assert_allclose(F, [[fx, 0.0], [-fx, 0.0]], rtol=1e-14, atol=1e-16)
    assert np.abs(tau).max() < 1e-15
    assert abs(phi - ph) < 1e-14 * ph


def test_repulsion_torque_sign_offset_pair():
    # Particle 2 sits above and to the right of particle 1 (director along x):
    # the right end circle of particle 1 is pushed down harder than the left one,
    # a clockwise (negative) torque.
    F, tau, _ = oracle.repulsion(np.array([[0.0, 0.0], [2.6, 1.2]]), np.array([0.0, 0.0]),
                                 np.array([[1.0, 0.5], [1.0, 0.5]]), 0.1, 3)
    assert F[0, 0] < 0 and F[0, 1] < 0 and tau[0] < 0


def test_repulsion_rejects_overlapping_circles():
    with pytest.raises(ValueError):
        oracle.repulsion(np.array([[0.0, 0.0], [0.9, 0.0]]), np.zeros(2),
                         np.array([[0.5, 0.5], [0.5, 0.5]]), 0.1, 3)


def test_label_moves_with_the_particle():
    # The nodes are fixed in each particle's frame, so the label at node k is the
    # same before and after a rigid motion (the time step keeps f per node).
    p = workloads.two_ellipses(3)
    prm = Params(panels=8, qbx_order=6)
    f0 = oracle.arc_label(oracle.discretize(p, prm))
    m = p.copy()
    m.center = m.center + np.array([[0.31, -0.2], [-0.05, 0.4]])
    m.angle = m.angle + np.array([0.7, -2.2])
    f1 = oracle.arc_label(oracle.discretize(m, prm))
    assert np.abs(f1 - f0).max() < 1e-12


def test_time_step_decreases_total_energy_at_first_order():
    # eq. euler is a gradient flow of Phi + Phi_rep: F_i = -dPhi_total/da_i and
    # tau_i = -dPhi_total/dtheta_i, so one step changes the total energy by
    # -dt sum (|F_i|^2 / xi_x + tau_i^2 / xi_theta) + O(dt^2).
    base = workloads.Particles(np.array([[-1.2, 0.0], [1.3, 0.4]]), np.array([0.3, 2.5]),
                               np.array([[1.0, 0.5]] * 2), 1.0)
    prm = Params(panels=10, qbx_order=8)
    lab = lambda d: oracle.janus_label(d, 4)
    c0, q, xi_x, xi_t, gamma = 0.02, 3, 1.5, 2.0, 1.0

    def step(parts, dt):
        return oracle.time_step(parts, prm, lab, gamma, c0, q, dt, xi_x, xi_t)

    r0 = step(base, 0.01)
    Ft = r0.force + r0.force_rep
    tt = r0.torque + r0.torque_rep
    rate = (Ft**2).sum() / xi_x + (tt**2).sum() / xi_t
    e0 = r0.energy + r0.energy_rep
    errs = []
    for dt in (0.01, 0.005):
        c, a = oracle.euler_update(base.center, base.angle, Ft, tt, dt, xi_x, xi_t)
        moved = base.copy()
        moved.center, moved.angle = c, a
        if dt == 0.01:
            assert np.array_equal(c, r0.particles.center) and np.array_equal(a, r0.particles.angle)
        r1 = step(moved, 0.0)
        assert np.array_equal(r1.particles.center, moved.center)   # dt = 0 moves nothing
        de = r1.energy + r1.energy_rep - e0
        assert de < 0
        errs.append(abs(de + dt * rate) / (dt * rate))
    assert errs[0] < 0.1
    assert 0.35 < errs[1] / errs[0] < 0.65, errs
