"""Cutoff far field (far_mode YQ_FAR_CUTOFF) against the exact sums.

The kernel decays like exp(-kappa r) (eq. exp_decay), and the paper suggests a
cut-off radius in the layer potential evaluations.  The cutoff mode skips every
(target group, source tile) pair whose bounding circles are at least z_c / kappa
apart.  z_c is chosen so that the skipped part of every far-field value is at
most cutoff_tol * ||sigma||_inf, and that of every gradient at most
cutoff_tol * kappa * ||sigma||_inf.  These tests check that bound against the
oracle's exact sums; that nothing changes when nothing is skipped; and the
solve and forces against the oracle.
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


def _np(t):
    return t.detach().cpu().numpy()


def _problem(parts, P, p, **kw):
    _torch()
    pb = yq.Problem(yq.default_params(panels_per_particle=P, qbx_order=p, **kw))
    pb.set_workload(parts)
    return pb


_CACHE = {}


def _case(kappa):
    # 24 ellipses in a 40 x 40 box, 12 panels (N = 4,608): at kappa 1 and 2 the
    # cutoff radius is a fraction of the box, so many tiles are skipped
    if kappa not in _CACHE:
        parts = workloads.random_ellipses(24, 40.0, kappa, seed=11, gap=0.3)
        d = oracle.discretize(parts, Params(panels=12, qbx_order=6))
        sig = workloads.random_density(d.N, 23)
        rows = list(range(d.N))
        from oracle.operator import far_grad_rows
        _CACHE[kappa] = (parts, d, sig, oracle.far_rows(d, rows, sig), far_grad_rows(d, rows, sig))
    return _CACHE[kappa]


@pytest.mark.parametrize("kappa,eps", [(1.0, 1e-6), (2.0, 1e-6), (2.0, 1e-10)])
def test_cutoff_far_field_within_its_bound(kappa, eps):
    parts, d, sig, ref, gref = _case(kappa)
    pb = _problem(parts, 12, 6, far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=eps)
    direct = _problem(parts, 12, 6)
    smax = np.abs(sig).max()
    got = _np(pb.apply_far(sig))
    err = np.abs(got - ref).max()
    assert err <= eps * smax + 1e-12 * np.abs(ref).max(), (err, eps * smax)
    # tiles were skipped: the result differs from the exact sum beyond rounding
    assert err > 1e-12 * np.abs(ref).max()
    eps32 = max(eps, 1e-7)   # the FP32 operator uses max(cutoff_tol, inner_tol / 10)
    got32 = _np(pb.apply_far(sig, precision=yq.YQ_MIXED))
    assert np.abs(got32 - ref).max() <= eps32 * smax + 5e-6 * np.abs(ref).max()
    # gradient: the direct mode's gradient of the same density as the reference
    gx, gy = pb.surface_gradient(sig)
    hx, hy = direct.surface_gradient(sig)
    gerr = max(np.abs(_np(gx) - _np(hx)).max(), np.abs(_np(gy) - _np(hy)).max())
    gscale = max(np.abs(_np(hx)).max(), np.abs(_np(hy)).max())
    assert gerr <= eps * kappa * smax + 1e-12 * gscale, (gerr, eps * kappa * smax)


def test_cutoff_that_skips_nothing_is_the_direct_sum_bitwise():
    parts, d, sig, ref, _ = _case(1.0)
    # the FP32 operator's bound is max(cutoff_tol, inner_tol / 10): both tiny
    pb = _problem(parts, 12, 6, far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=1e-300, inner_tol=1e-299)
    direct = _problem(parts, 12, 6)
    for prec in (yq.YQ_FP64, yq.YQ_MIXED):
        assert np.array_equal(_np(pb.apply_far(sig, precision=prec)),
                              _np(direct.apply_far(sig, precision=prec)))
    a = pb.surface_gradient(sig)
    b = direct.surface_gradient(sig)
    assert all(np.array_equal(_np(u), _np(v)) for u, v in zip(a, b))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cutoff_solve_and_forces_match_the_oracle(precision):
    # 6 ellipses in a 30 x 30 box at kappa 2: the cutoff radius (about 15 at
    # cutoff_tol 1e-12) drops the pairs of the farthest particles
    parts = workloads.random_ellipses(6, 30.0, 2.0, seed=8, gap=0.3)
    P, p = 10, 8
    kw = dict(tol=1e-11) if precision == "fp64" else dict(tol=1e-10, precision=yq.YQ_MIXED)
    pb = _problem(parts, P, p, far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=1e-12, **kw)
    pb.set_boundary_data(pb.boundary_label())
    sigma, info, F, T, E = pb.solve_forces()
    d = oracle.discretize(parts, Params(panels=P, qbx_order=p))
    A, Gx, Gy = oracle.build_matrices(d, gradient=True)
    f = oracle.arc_label(d)
    so = oracle.lu_solve(A, f)
    Fo, To, _, Eo = oracle.forces_torques(d, f, oracle.surface_fields(Gx, Gy, so))
    assert np.abs(_np(sigma) - so).max() / np.abs(so).max() < 1e-9
    assert np.abs(_np(F) - Fo).max() / np.abs(Fo).max() < 1e-8
    assert abs(E - Eo) < 1e-9 * abs(Eo)


def test_cutoff_at_the_large_workload_size():
    # The 500-ellipse workload (N = 256,000) at kappa 4, where the cutoff skips
    # all but a few percent of the tile pairs: 48 sampled rows against the
    # oracle's exact sums, within the bound.
    parts = workloads.config_large(seed=0)["particles"].copy()
    parts.kappa = 4.0
    pb = _problem(parts, 32, 10, far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=1e-12)
    d = oracle.discretize(parts, Params(panels=32, qbx_order=10))
    assert pb.N == d.N == 256000
    sig = workloads.random_density(d.N, 31)
    rows = np.linspace(0, d.N - 1, 48).astype(int)
    ref = oracle.far_rows(d, list(rows), sig)
    smax = np.abs(sig).max()
    got = _np(pb.apply_far(sig))[rows]
    assert np.abs(got - ref).max() <= 1e-12 * smax + 1e-12 * np.abs(ref).max()
    got32 = _np(pb.apply_far(sig, precision=yq.YQ_MIXED))[rows]
    assert np.abs(got32 - ref).max() <= 1e-7 * smax + 5e-6 * np.abs(ref).max()


def test_time_steps_with_the_cutoff_match_the_direct_sum():
    # Two constant-drag steps of 12 ellipses at kappa 2: with the cutoff the
    # forces and the new positions agree with the exact direct sums to the solve
    # tolerance.
    torch = _torch()
    parts = workloads.random_ellipses(12, 24.0, 2.0, seed=5, gap=0.4)
    dyn = dict(dt=0.05, xi_x=1.5, xi_theta=2.0, c0=0.02)
    out = []
    for mode in (yq.YQ_FAR_DIRECT, yq.YQ_FAR_CUTOFF):
        pb = _problem(parts, 16, 8, tol=1e-10, precision=yq.YQ_MIXED, far_mode=mode,
                      cutoff_tol=1e-12)
        pb.set_boundary_data(pb.boundary_label())
        sigma = torch.zeros(pb.N, dtype=torch.float64, device=pb.device)
        for _ in range(2):
            info, F, T, E = pb.step(sigma, **dyn)
        out.append((pb.particles(), _np(F), _np(T)))
    (c0, a0), F0, T0 = out[0]
    (c1, a1), F1, T1 = out[1]
    assert np.abs(F1 - F0).max() < 1e-8 * np.abs(F0).max()
    assert np.abs(T1 - T0).max() < 1e-8 * max(np.abs(F0).max(), np.abs(T0).max())
    assert np.abs(c1 - c0).max() < 1e-10 and np.abs(a1 - a0).max() < 1e-10


def test_cutoff_parameters_and_batches():
    _torch()
    with pytest.raises(yq.YQError):
        yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=0.0))
    with pytest.raises(yq.YQError):
        yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=1.0))
    with pytest.raises(yq.YQError):
        yq.Batch(yq.default_params(far_mode=yq.YQ_FAR_CUTOFF))
