"""Full-size parity against values the oracle wrote (tests/golden/make_goldens.py).

* The 50-ellipse workload (N = 25,600, kappa = 1): density, surface gradient,
  forces, torques, energy and off-surface potential of the mixed path (tolerance
  1e-9) and of the FP64 path (1e-12) against the oracle's dense-LU solution,
  element by element.  Errors are max |x - x*| / max |x*| (reading R15 of the
  design notes: normwise, since per-particle relative errors are ill-posed for
  small forces).
* The 500-ellipse workload (N = 256,000): 1,024 sampled rows of the operator
  applied to a seeded density, with the order-20 FMM (FP32 leaf interactions and
  M2L, the inner operator of the mixed solves) and the order-40 FP64 FMM (the
  refinement residual's far field), against the oracle's rows.
* A 200-ellipse configuration (the batched workload's largest member size, 8
  panels per particle) solved inside a batch, with the fused direct far field and
  as a tree of the FMM forest: density, forces and torques against the oracle's LU.
"""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

yq = pytest.importorskip("paper_1810_04131_amd")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _load(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_goldens.py)")
    return np.load(path)


@pytest.mark.parametrize("precision,tol,bound", [(1, 1e-9, 1e-8), (0, 1e-12, 1e-10)])
def test_c2_solution_forces_potential_against_oracle_lu(precision, tol, bound):
    _torch()
    g = _load("c2_kappa1.npz")
    cfg = workloads.config_medium(kappa=1.0, seed=0)
    pb = yq.Problem(yq.default_params(panels_per_particle=32, qbx_order=10, tol=tol,
                                      precision=precision, maxiter=400))
    pb.set_workload(cfg["particles"])
    f = pb.boundary_label()
    assert _rel(_np(f), g["f"]) < 1e-13
    pb.set_boundary_data(f)
    sig, info, F, T, E = pb.solve_forces()
    errs = {"density": _rel(_np(sig), g["sigma"]),
            "force": _rel(_np(F).reshape(-1, 2), g["force"]),
            "torque": _rel(_np(T), g["torque"]),
            "energy": abs(E - float(g["energy"])) / abs(float(g["energy"]))}
    gx, gy = pb.surface_gradient(sig)
    errs["gradient"] = _rel(np.stack([_np(gx), _np(gy)], 1), g["grad"])
    u = pb.eval_potential(sig, g["targets"])
    errs["potential"] = _rel(_np(u), g["potential"])
    print(precision, info, errs)
    for k, v in errs.items():
        assert v <= bound, (k, v)


@pytest.fixture(scope="module")
def c3():
    g = _load("c3_rows.npz")
    parts = workloads.config_large(seed=0)["particles"]
    sigma = workloads.random_density(256000, int(g["density_seed"]))
    return parts, sigma, g["rows"], g["values"]


def test_c3_fmm_order20_operator_rows_against_oracle(c3):
    _torch()
    parts, sigma, rows, ref = c3
    pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=20, fmm_leaf_max=64))
    pb.set_workload(parts)
    st = pb.fmm_stats()
    assert st["max_leaf"] <= 64
    out = _np(pb.apply_operator(sigma, yq.YQ_MIXED))[rows]
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(st, err)
    assert err < 2e-6
    # the exact direct sum on the same rows (FP64 operator)
    ex = _np(pb.apply_operator(sigma, yq.YQ_FP64))[rows]
    assert np.abs(ex - ref).max() / np.abs(ref).max() < 1e-12


def test_c3_fmm_order40_fp64_operator_rows_against_oracle(c3):
    _torch()
    parts, sigma, rows, ref = c3
    pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=40, fmm_leaf_max=64))
    pb.set_workload(parts)
    # the order-40 FP64 FMM far field plus the exact near correction
    # (operator - far field of the direct FP64 path)
    far_fmm = _np(pb.apply_far(sigma, yq.YQ_FMM64))
    corr = _np(pb.apply_operator(sigma, yq.YQ_FP64)) - _np(pb.apply_far(sigma, yq.YQ_FP64))
    out = (far_fmm + corr)[rows]
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(err)
    assert err < 5e-10


@pytest.mark.parametrize("mode", ["fused", "forest"])
def test_batch_with_a_200_ellipse_member_against_oracle_lu(mode):
    # fused: the member's far field is the fused direct sum of the engine's work
    # list; forest: at 25,600 nodes it takes the FMM, as a tree of the engine's forest
    _torch()
    g = _load("member200_p8.npz")
    member = workloads.batch_member_200()
    small = [workloads.random_ellipses(n, 30.0 * np.sqrt(n / 50.0), k, seed=s, gap=0.2)
             for n, k, s in [(12, 0.6, 21), (40, 1.9, 22), (25, 1.1, 23)]]
    cfgs = [small[0], member, small[1], small[2]]
    b = yq.Batch(yq.default_params(panels_per_particle=8, qbx_order=10, tol=1e-9,
                                   precision=yq.YQ_MIXED, restart=60, maxiter=300))
    b.set_fmm(10 ** 9 if mode == "fused" else 20000)
    b.set_configs(cfgs)
    assert int(b.offsets[2] - b.offsets[1]) == 25600
    f = b.boundary_label()
    b.set_boundary_data(f)
    sig, infos = b.solve()
    F, T, E = b.forces(sig)
    s = _np(b.segment(sig, 1))
    p0 = int(b.nparticles[0])
    Fm = _np(F)[p0:p0 + 200]
    Tm = _np(T)[p0:p0 + 200]
    errs = {"density": _rel(s, g["sigma"]), "force": _rel(Fm, g["force"]),
            "torque": _rel(Tm, g["torque"]),
            "energy": abs(E[1] - float(g["energy"])) / abs(float(g["energy"]))}
    print(infos[1], errs)
    assert _rel(_np(b.segment(f, 1)), g["f"]) < 1e-13
    for k, v in errs.items():
        assert v <= 1e-8, (k, v)
