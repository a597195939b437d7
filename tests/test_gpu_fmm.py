"""Quadtree Yukawa FMM (inner far field) against the direct sum and the oracle."""
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


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def medium():
    return workloads.config_medium(kappa=0.5, seed=1)


def test_fmm_converges_to_direct_far_field(medium):
    _torch()
    parts = medium["particles"]
    sig = workloads.random_density(25600, 3)
    errs = {}
    for p in (8, 14, 20, 26):
        pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=p, fmm_leaf_max=64))
        pb.set_workload(parts)
        direct = _np(pb.apply_far(sig, yq.YQ_FP64))
        errs[p] = _rel(_np(pb.apply_far(sig, yq.YQ_FMM64)), direct)
        e32 = _rel(_np(pb.apply_far(sig, yq.YQ_MIXED)), direct)
        assert e32 < max(errs[p], 0) + 5e-6
    # geometric convergence in the expansion order (error bound ~ 0.55^p per translation)
    assert errs[8] > errs[14] > errs[20] > errs[26]
    assert errs[20] < 1e-5 and errs[26] < 1e-6, errs


@pytest.mark.parametrize("order", [5, 20, 48])
def test_fmm_m2l_matrix_cores_match_vector_alu(medium, order):
    # the M2L on FP64 MFMA tiles and the per-coefficient VALU kernel compute the
    # same sums in a different order: they agree to rounding at every tile count
    _torch()
    parts = medium["particles"]
    sig = workloads.random_density(25600, 6)
    out = {}
    for m2l in (yq.YQ_M2L_MFMA, yq.YQ_M2L_VALU):
        pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=order, fmm_leaf_max=64,
                                          fmm_m2l=m2l))
        pb.set_workload(parts)
        out[m2l] = _np(pb.apply_far(sig, yq.YQ_FMM64))
    assert _rel(out[yq.YQ_M2L_MFMA], out[yq.YQ_M2L_VALU]) < 1e-12


def test_fmm_gradient_and_forces_match_direct(medium):
    # surface gradient and forces with the FP64 FMM far part (order 40) against
    # the direct FP64 sum on the same density
    torch = _torch()
    parts = medium["particles"]
    out = {}
    for mode in (yq.YQ_FAR_DIRECT, yq.YQ_FAR_FMM):
        pb = yq.Problem(yq.default_params(far_mode=mode, fmm_order=20, fmm_resid_order=40))
        pb.set_workload(parts)
        f = pb.boundary_label()
        pb.set_boundary_data(f)
        sig = torch.tensor(workloads.random_density(pb.N, 8), device="cuda", dtype=torch.float64)
        gx, gy = pb.surface_gradient(sig)
        F, T, E = pb.forces(sig)
        out[mode] = (_np(gx), _np(gy), _np(F), _np(T), E)
    d, m = out[yq.YQ_FAR_DIRECT], out[yq.YQ_FAR_FMM]
    g_ref = np.hypot(d[0], d[1]).max()
    assert np.abs(m[0] - d[0]).max() < 1e-9 * g_ref and np.abs(m[1] - d[1]).max() < 1e-9 * g_ref
    sc = max(np.abs(d[2]).max(), np.abs(d[3]).max())
    assert np.abs(m[2] - d[2]).max() < 1e-9 * sc and np.abs(m[3] - d[3]).max() < 1e-9 * sc
    assert abs(m[4] - d[4]) < 1e-9 * abs(d[4])


def test_fmm_far_field_against_oracle_rows(medium):
    _torch()
    parts = medium["particles"]
    d = oracle.discretize(parts, Params(panels=32, qbx_order=10))
    sig = workloads.random_density(d.N, 4)
    pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=26))
    pb.set_workload(parts)
    rows = sorted(set(np.random.default_rng(5).integers(0, d.N, 16).tolist()))
    ref = oracle.far_rows(d, rows, sig)
    got = _np(pb.apply_far(sig, yq.YQ_FMM64))[rows]
    assert np.abs(got - ref).max() < 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("resid_order", [0, 40])
def test_fmm_inner_solve_reaches_direct_tolerance(resid_order):
    _torch()
    parts = workloads.random_ellipses(6, 12.0, 1.1, seed=7)
    P, p = 16, 8
    d = oracle.discretize(parts, Params(panels=P, qbx_order=p))
    A = oracle.build_matrices(d)
    f = oracle.arc_label(d)
    so = oracle.lu_solve(A, f)
    pb = yq.Problem(yq.default_params(panels_per_particle=P, qbx_order=p, far_mode=yq.YQ_FAR_FMM,
                                      fmm_order=16, fmm_leaf_max=32, precision=yq.YQ_MIXED,
                                      tol=1e-10, fmm_resid_order=resid_order))
    pb.set_workload(parts)
    pb.set_boundary_data(f)
    sig, info = pb.solve()
    # the FMM only steers the inner solve; refinement residuals use the exact
    # operator (order 0) or the order-40 FP64 FMM, whose operator error is far
    # below the tolerance, so the exact residual also meets it
    assert info["residual"] <= 1e-10 and info["matvecs_fp32"] > 0
    exact = _np(pb.apply_operator(sig, yq.YQ_FP64)) - f
    assert np.linalg.norm(exact) <= 2e-10 * np.linalg.norm(f)
    assert _rel(_np(sig), so) < 1e-8


@pytest.mark.parametrize("resid_order", [0, 40])
def test_fmm_solve_forces_matches_solve_then_forces(resid_order):
    """With the FMM the solve's residuals are not fused with the gradient: the
    forces come from the FMM (or direct) gradient pass, as after a separate solve."""
    torch = _torch()
    parts = workloads.random_ellipses(6, 12.0, 1.1, seed=7)
    prm = dict(panels_per_particle=16, qbx_order=8, far_mode=yq.YQ_FAR_FMM, fmm_order=16,
               fmm_leaf_max=32, precision=yq.YQ_MIXED, tol=1e-9, fmm_resid_order=resid_order)
    pa = yq.Problem(yq.default_params(**prm))
    pa.set_workload(parts)
    pa.set_boundary_data(pa.boundary_label())
    sa, ia = pa.solve()
    Fa, Ta, Ea = pa.forces(sa, gamma=0.7)
    pf = yq.Problem(yq.default_params(**prm))
    pf.set_workload(parts)
    pf.set_boundary_data(pf.boundary_label())
    sf, inf_, Ff, Tf, Ef = pf.solve_forces(gamma=0.7)
    assert inf_["iterations"] == ia["iterations"] and inf_["residual"] <= 1e-9
    assert _rel(_np(sf), _np(sa)) < 1e-13
    assert _rel(_np(Ff), _np(Fa)) < 1e-12 and _rel(_np(Tf), _np(Ta)) < 1e-12
    assert abs(Ef - Ea) <= 1e-12 * abs(Ea)


def test_solve_forces_at_the_iteration_limit():
    """ENOCONV from yq_solve_forces: sigma is the last iterate and the forces are
    those of it (the direct path, where the last residual may be fused)."""
    torch = _torch()
    parts = workloads.random_ellipses(6, 12.0, 1.1, seed=7)
    prm = dict(panels_per_particle=16, qbx_order=8, precision=yq.YQ_MIXED, tol=1e-12, maxiter=5)
    pf = yq.Problem(yq.default_params(**prm))
    pf.set_workload(parts)
    pf.set_boundary_data(pf.boundary_label())
    sf, inf_, Ff, Tf, Ef = pf.solve_forces(gamma=1.0, allow_noconv=True)
    assert inf_["iterations"] == 5 and inf_["residual"] > 1e-12
    pa = yq.Problem(yq.default_params(**prm))
    pa.set_workload(parts)
    pa.set_boundary_data(pa.boundary_label())
    Fa, Ta, Ea = pa.forces(sf, gamma=1.0)
    assert _rel(_np(Ff), _np(Fa)) < 1e-12 and _rel(_np(Tf), _np(Ta)) < 1e-12
    assert abs(Ef - Ea) <= 1e-12 * abs(Ea)
    with pytest.raises(yq.YQError):
        pf.solve_forces()


def test_fmm_large_workload_residual_property():
    _torch()
    cfg = workloads.config_large(seed=0)
    parts = cfg["particles"]
    pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=20, fmm_leaf_max=64,
                                      precision=yq.YQ_MIXED, tol=1e-8, maxiter=400))
    pb.set_workload(parts)
    assert pb.N == 256000
    f = pb.boundary_label()
    pb.set_boundary_data(f)
    sig, info = pb.solve()
    assert info["residual"] <= 1e-8
    exact = pb.apply_operator(sig, yq.YQ_FP64) - f
    assert (exact.norm() / f.norm()).item() <= 2e-8
    d = oracle.discretize(parts, Params(panels=32, qbx_order=10))
    rows = sorted(set(np.random.default_rng(2).integers(0, d.N, 8).tolist()))
    r = oracle.apply_rows(d, rows, _np(sig)) - oracle.arc_label(d)[rows]
    assert np.abs(r).max() < 1e-6


@pytest.mark.parametrize("order,kappa", [(8, 1.0), (20, 0.5), (20, 2.0), (30, 1.0)])
def test_fmm_fp32_m2l_matches_fp64_m2l(order, kappa):
    # the inner operator's M2L in FP32 on scaled expansions against the same
    # operator with FP64 translations: the FP32 products change it by a relative
    # amount at the FP32 level, well below the order-20 truncation error
    _torch()
    parts = workloads.config_medium(kappa=kappa, seed=2)["particles"]
    sig = workloads.random_density(25600, 9)
    out = {}
    for m2l in (yq.YQ_M2L_MFMA, yq.YQ_M2L_MFMA64):
        pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=order, fmm_leaf_max=64,
                                          fmm_m2l=m2l))
        pb.set_workload(parts)
        out[m2l] = _np(pb.apply_far(sig, yq.YQ_MIXED))
    assert _rel(out[yq.YQ_M2L_MFMA], out[yq.YQ_M2L_MFMA64]) < 2e-6
