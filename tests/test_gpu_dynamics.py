"""Time stepping on the GPU (yq_repulsion, yq_step) against the oracle.

Tolerances: the repulsion is a direct FP64 sum of O(n^2) positive-gap terms, so
it agrees with the oracle to 1e-12 of the largest magnitude.  A step's density
and forces carry the FP64 solve's 1e-10 bound (GMRES to 1e-13); the new
centres and angles are the old ones plus dt/xi times those forces, so they agree
to 1e-10 * dt/xi * max|F| plus rounding of the positions.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle.geometry import Params

pytestmark = pytest.mark.gpu

yq = pytest.importorskip("paper_1810_04131_amd")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problem(parts, P, p, **kw):
    _torch()
    pb = yq.Problem(yq.default_params(panels_per_particle=P, qbx_order=p, **kw))
    pb.set_workload(parts)
    return pb


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n,q", [(1, 3), (2, 3), (37, 3), (150, 3), (150, 4)])
def test_repulsion_parity(n, q):
    # n = 150 spans three lane strides of the 64-lane loop and a ragged last block
    if n == 1:
        parts = workloads.single_disk(1.0, 1.0)
        parts.axes = np.array([[1.3, 0.6]])
    elif n == 2:
        parts = workloads.two_ellipses(5)
    else:
        parts = workloads.random_ellipses(n, 4.0 * math.sqrt(n) + 4.0, 1.0, seed=n, gap=0.3,
                                          axes_range=((0.8, 1.2), (0.4, 0.6)))
    pb = _problem(parts, 8, 6)
    c0 = 0.05
    F, T, E = pb.repulsion(c0, q)
    Fo, To, Eo = oracle.repulsion(parts.center, parts.angle, parts.axes, c0, q)
    if n == 1:
        assert np.all(_np(F) == 0.0) and np.all(_np(T) == 0.0) and E == 0.0
        return
    assert _rel(_np(F), Fo) < 1e-12
    assert np.abs(_np(T) - To).max() < 1e-12 * max(np.abs(Fo).max(), np.abs(To).max())
    assert abs(E - Eo) < 1e-12 * Eo


def test_repulsion_rejects_overlapping_circles():
    # Two thin parallel ellipses, offset along and across their axes: the ellipses
    # are 0.1 apart, but the end circles (radius 0.2 at +-0.8 along the axis)
    # reach outside the ellipses near the tips and overlap.
    parts = workloads.Particles(np.array([[0.0, 0.0], [1.8, 0.3]]), np.zeros(2),
                                np.array([[1.0, 0.2], [1.0, 0.2]]), 1.0)
    with pytest.raises(ValueError):
        oracle.repulsion(parts.center, parts.angle, parts.axes, 0.05, 3)
    pb = _problem(parts, 16, 6)
    with pytest.raises(yq.YQError) as ei:
        pb.repulsion(0.05, 3)
    assert ei.value.status == -2
    # the problem stays usable
    pb.set_boundary_data(pb.boundary_label())
    pb.solve()


def _two():
    return workloads.Particles(np.array([[-1.2, 0.0], [1.3, 0.4]]), np.array([0.3, 2.5]),
                               np.array([[1.0, 0.5]] * 2), 1.0)


@pytest.mark.parametrize("extrapolate", [False, True])
def test_step_parity_with_the_oracle_over_three_steps(extrapolate):
    P, p = 10, 8
    dyn = dict(dt=0.2, xi_x=1.5, xi_theta=2.0, c0=0.02, q=3, gamma=1.0)
    parts = _two()
    pb = _problem(parts, P, p, tol=1e-13)
    pb.set_boundary_data(pb.boundary_label())
    sigma = pb.torch.zeros(pb.N, dtype=pb.torch.float64, device=pb.device)
    prev = sigma.clone() if extrapolate else None
    cur = parts.copy()
    for k in range(3):
        c0_, a0_ = pb.particles()
        info, F, T, (E, Er) = pb.step(sigma, sigma_prev=prev, **dyn)
        r = oracle.time_step(cur, Params(panels=P, qbx_order=p), oracle.arc_label, dyn["gamma"],
                             dyn["c0"], dyn["q"], dyn["dt"], dyn["xi_x"], dyn["xi_theta"])
        Ft, Tt = r.force + r.force_rep, r.torque + r.torque_rep
        assert _rel(_np(sigma), r.sigma) < 1e-10, k
        assert _rel(_np(F), Ft) < 1e-9, k
        assert np.abs(_np(T) - Tt).max() < 1e-9 * max(np.abs(Ft).max(), np.abs(Tt).max()), k
        assert abs(E - r.energy) < 1e-9 * abs(r.energy), k
        assert abs(Er - r.energy_rep) < 1e-12 * r.energy_rep, k
        c, a = pb.particles()
        scale = dyn["dt"] / min(dyn["xi_x"], dyn["xi_theta"]) * max(np.abs(Ft).max(), 1.0)
        assert np.abs(c - r.particles.center).max() < 1e-9 * scale + 1e-14, k
        assert np.abs(a - r.particles.angle).max() < 1e-9 * scale + 1e-14, k
        # the update is exactly eq. euler of the returned totals
        np.testing.assert_allclose(c, c0_ + dyn["dt"] / dyn["xi_x"] * _np(F), rtol=0, atol=1e-15)
        np.testing.assert_allclose(a, a0_ + dyn["dt"] / dyn["xi_theta"] * _np(T), rtol=0,
                                   atol=1e-15)
        assert info["iterations"] > 0 and info["residual"] < 1e-13
        cur = r.particles


def test_step_with_zero_dt_keeps_the_configuration_and_solves():
    parts = _two()
    pb = _problem(parts, 10, 8, tol=1e-12)
    pb.set_boundary_data(pb.boundary_label())
    ref, _ = pb.solve()
    sigma = pb.torch.zeros(pb.N, dtype=pb.torch.float64, device=pb.device)
    pb.step(sigma, dt=0.0, xi_x=1.0, xi_theta=1.0, c0=0.02)
    c, a = pb.particles()
    assert np.array_equal(c, parts.center) and np.array_equal(a, parts.angle)
    assert _rel(_np(sigma), _np(ref)) < 1e-11
    # the rebuilt set-up kept the boundary data: a warm-started second step converges at once
    info, *_ = pb.step(sigma, dt=0.0, xi_x=1.0, xi_theta=1.0, c0=0.02)
    assert info["iterations"] <= 2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_warm_start_reduces_iterations(precision):
    parts = workloads.random_ellipses(20, 16.0, 1.0, seed=4, gap=0.4)
    kw = dict(tol=1e-10) if precision == "fp64" else dict(tol=1e-8, precision=yq.YQ_MIXED)
    pb = _problem(parts, 16, 8, **kw)
    pb.set_boundary_data(pb.boundary_label())
    sigma = pb.torch.zeros(pb.N, dtype=pb.torch.float64, device=pb.device)
    dyn = dict(dt=0.05, xi_x=1.5, xi_theta=2.0, c0=0.02)
    pb.step(sigma, **dyn)
    # a cold solve at the new configuration, then the warm-started step there
    _, cold = pb.solve()
    info, *_ = pb.step(sigma, **dyn)
    print(f"{precision}: cold {cold['iterations']} iterations, warm {info['iterations']}")
    assert info["residual"] <= kw["tol"]
    assert info["iterations"] < cold["iterations"], (info, cold)


def test_extrapolated_guess_is_two_sigma_minus_prev():
    # Two identical problems stopped after three iterations: passing (sigma, prev)
    # gives bit for bit the step from the guess 2 sigma - prev, and prev returns
    # holding sigma's value on entry.
    torch = _torch()
    out = []
    for use_prev in (True, False):
        pb = _problem(_two(), 10, 8, tol=1e-15, maxiter=3, restart=3)
        pb.set_boundary_data(pb.boundary_label())
        a = torch.randn(pb.N, dtype=torch.float64, generator=torch.Generator().manual_seed(1))
        b = torch.randn(pb.N, dtype=torch.float64, generator=torch.Generator().manual_seed(2))
        if use_prev:
            sigma, prev = a.to(pb.device), b.to(pb.device)
        else:
            sigma, prev = (2 * a - b).to(pb.device), None
        pb.step(sigma, dt=0.1, xi_x=1.0, xi_theta=1.0, c0=0.02, sigma_prev=prev,
                allow_noconv=True)
        if use_prev:
            assert torch.equal(prev.cpu(), a)
        out.append((_np(sigma), pb.particles()))
    assert np.array_equal(out[0][0], out[1][0])
    with pytest.raises(yq.YQError):
        pb.step(sigma, dt=0.1, xi_x=1.0, xi_theta=1.0, c0=0.02, sigma_prev=sigma)


def test_step_turns_the_window_correction_with_the_particles():
    # A step replaces the QBX build by turning the gradient rows of the window
    # correction with each particle; the operator and the surface gradient then
    # agree with a fresh set-up at the new configuration to rounding.  Both sides
    # build from absolute node coordinates (|x| ~ 14 here), whose 1e-16 relative
    # rounding becomes ~1e-13 in the differences of adjacent nodes, so the bounds are
    # the FP64 parity's: 1e-12 for the operator, 1e-11 for the gradient (its
    # near-singular rows cancel more).  A missing turn would be off by ~1e-1.
    torch = _torch()
    parts = workloads.random_ellipses(8, 14.0, 1.0, seed=6, gap=0.4)
    pb = _problem(parts, 16, 8, tol=1e-12)
    pb.set_boundary_data(pb.boundary_label())
    sigma = torch.zeros(pb.N, dtype=torch.float64, device=pb.device)
    for _ in range(2):
        pb.step(sigma, dt=0.3, xi_x=1.0, xi_theta=0.5, c0=0.02)
    c, a = pb.particles()
    assert np.abs(a - parts.angle).max() > 1e-3
    moved = parts.copy()
    moved.center, moved.angle = c, a
    fresh = _problem(moved, 16, 8, tol=1e-12)
    v = workloads.random_density(pb.N, 9)
    assert _rel(_np(pb.apply_operator(v)), _np(fresh.apply_operator(v))) < 1e-12
    g1, g2 = pb.surface_gradient(v), fresh.surface_gradient(v)
    scale = max(np.abs(_np(g2[0])).max(), np.abs(_np(g2[1])).max())
    for u, w in zip(g1, g2):
        assert np.abs(_np(u) - _np(w)).max() < 1e-11 * scale


def test_rejected_configuration_leaves_particles_in_place():
    # Hydrophobic heads facing each other 0.3 apart attract along the line of
    # centres; a dt that moves each particle by 1.5 gaps overlaps them.
    parts = workloads.Particles(np.array([[-1.15, 0.0], [1.15, 0.0]]), np.array([0.0, math.pi]),
                                np.array([[1.0, 0.5]] * 2), 1.0)
    pb = _problem(parts, 16, 8, tol=1e-12)
    pb.set_boundary_data(pb.boundary_label())
    sigma = pb.torch.zeros(pb.N, dtype=pb.torch.float64, device=pb.device)
    _, F, _, _ = pb.step(sigma, dt=0.0, xi_x=1.0, xi_theta=1.0, c0=0.0)
    F = _np(F)
    assert F[0, 0] > 0 and F[1, 0] < 0   # attraction
    ref = _np(sigma).copy()
    dt = 1.5 * 0.3 / abs(F[0, 0])
    with pytest.raises(yq.YQError) as ei:
        pb.step(sigma, dt=dt, xi_x=1.0, xi_theta=1.0, c0=0.0)
    assert ei.value.status == -2
    c, a = pb.particles()
    assert np.array_equal(c, parts.center) and np.array_equal(a, parts.angle)
    assert _rel(_np(sigma), ref) < 1e-11
    # the start configuration was rebuilt with its boundary data
    s2, info = pb.solve()
    assert _rel(_np(s2), ref) < 1e-11


def test_not_converged_step_does_not_move():
    parts = _two()
    pb = _problem(parts, 10, 8, tol=1e-15, maxiter=3, restart=3)
    pb.set_boundary_data(pb.boundary_label())
    sigma = pb.torch.zeros(pb.N, dtype=pb.torch.float64, device=pb.device)
    info, F, T, _ = pb.step(sigma, dt=0.1, xi_x=1.0, xi_theta=1.0, c0=0.02, allow_noconv=True)
    assert info["residual"] > 1e-15
    c, a = pb.particles()
    assert np.array_equal(c, parts.center) and np.array_equal(a, parts.angle)
    assert np.all(np.isfinite(_np(F))) and np.all(np.isfinite(_np(T)))


def test_step_rejects_bad_parameters():
    pb = _problem(_two(), 10, 8)
    pb.set_boundary_data(pb.boundary_label())
    sigma = pb.torch.zeros(pb.N, dtype=pb.torch.float64, device=pb.device)
    for bad in (dict(dt=-1.0), dict(xi_x=0.0), dict(xi_theta=-2.0), dict(c0=-1.0), dict(q=0),
                dict(dt=float("nan"))):
        kw = dict(dt=0.1, xi_x=1.0, xi_theta=1.0, c0=0.02, q=3)
        kw.update(bad)
        with pytest.raises(yq.YQError) as ei:
            pb.step(sigma, **kw)
        assert ei.value.status == -1, bad
    c, a = pb.particles()
    assert np.array_equal(c, _two().center)


def test_dynamics_workload_at_full_size():
    # the benchmark's configuration (100 ellipses, N = 51,200, mixed, direct far
    # field): the repulsion element by element against the oracle, the update
    # against eq. euler of the returned totals, the warm-started second step
    # within the tolerance, and the FMM path's step agreeing with the direct one.
    cfg = workloads.config_dynamics()
    parts = cfg["particles"]
    pb = _problem(parts, cfg["panels"], cfg["qbx_order"], tol=cfg["tol"], precision=yq.YQ_MIXED)
    F, T, E = pb.repulsion(cfg["c0"], cfg["q"])
    Fo, To, Eo = oracle.repulsion(parts.center, parts.angle, parts.axes, cfg["c0"], cfg["q"])
    assert _rel(_np(F), Fo) < 1e-12 and abs(E - Eo) < 1e-12 * Eo
    pb.set_boundary_data(pb.boundary_label())
    sigma = pb.torch.zeros(pb.N, dtype=pb.torch.float64, device=pb.device)
    dyn = dict(dt=cfg["dt"], xi_x=cfg["xi_x"], xi_theta=cfg["xi_theta"], c0=cfg["c0"], q=cfg["q"],
               gamma=cfg["gamma"])
    info1, F1, T1, _ = pb.step(sigma, **dyn)
    c1, a1 = pb.particles()
    np.testing.assert_allclose(c1, parts.center + dyn["dt"] / dyn["xi_x"] * _np(F1), rtol=0,
                               atol=1e-13)
    np.testing.assert_allclose(a1, parts.angle + dyn["dt"] / dyn["xi_theta"] * _np(T1), rtol=0,
                               atol=1e-13)
    info2, F2, T2, _ = pb.step(sigma, **dyn)
    print(f"steps: {info1['iterations']} then {info2['iterations']} iterations")
    assert info1["residual"] <= cfg["tol"] and info2["residual"] <= cfg["tol"]
    assert info2["iterations"] < info1["iterations"]

    fm = _problem(parts, cfg["panels"], cfg["qbx_order"], tol=cfg["tol"], precision=yq.YQ_MIXED,
                  far_mode=yq.YQ_FAR_FMM)
    fm.set_boundary_data(fm.boundary_label())
    s2 = fm.torch.zeros(fm.N, dtype=fm.torch.float64, device=fm.device)
    _, Fm, Tm, _ = fm.step(s2, **dyn)
    cm, am = fm.particles()
    assert _rel(_np(Fm), _np(F1)) < 1e-6
    assert np.abs(cm - c1).max() < 1e-6 * dyn["dt"] / dyn["xi_x"] * np.abs(_np(F1)).max() + 1e-14
