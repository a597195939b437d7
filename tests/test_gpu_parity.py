"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Tolerances (relative to the largest magnitude of the compared quantity):
  FP64 geometry 1e-14; FP64 operator / far field / gradient 1e-12 (rounding order
  of ~N terms, FP64 special functions within 1e-15);  FP32 far field 5e-6 (FP32
  unit roundoff 6e-8 in each term, special functions within 3e-7, summed over up
  to N terms of mixed sign);
  FP64 solve 1e-10 (the FP64 path's target bound; GMRES run to 1e-13 so the discrete
  solution's rounding dominates);  mixed solve 1e-8.
"""
import dataclasses
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
    prm = yq.default_params(panels_per_particle=P, qbx_order=p, **kw)
    pb = yq.Problem(prm)
    pb.set_workload(parts)
    return pb


def _oprm(P, p):
    return Params(panels=P, qbx_order=p)


def _np(t):
    return t.detach().cpu().numpy()


def _phase(pb, phase):
    """(launches, total ms) of a profiled phase since the last read."""
    import ctypes
    n, ms = ctypes.c_int64(), ctypes.c_double()
    pb._check(pb.lib.yq_profile_read(pb.h, phase, ctypes.byref(n), ctypes.byref(ms), 1))
    return n.value, ms.value


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ---- small cases against the full dense oracle ------------------------------------------

CASES = {
    "two_ellipses_N512": lambda: (workloads.two_ellipses(0, 1.0), 16, 8),
    # ragged: 3 particles x 7 panels x 16 = 336 nodes (not a multiple of 256), near contact
    "ragged_near_N336": lambda: (workloads.Particles(
        np.array([[0.0, 0.0], [2.06, 0.1], [0.2, 1.58]]), np.array([0.0, 0.05, 1.5]),
        np.array([[1.0, 0.5], [1.0, 0.5], [1.0, 0.6]]), 0.7), 7, 6),
    "single_disk_N160": lambda: (workloads.single_disk(1.0, 0.25), 10, 8),
}


@pytest.fixture(scope="module", params=list(CASES))
def small(request):
    parts, P, p = CASES[request.param]()
    d = oracle.discretize(parts, _oprm(P, p))
    A, Gx, Gy = oracle.build_matrices(d, gradient=True)
    f = oracle.arc_label(d)
    sig_lu = oracle.lu_solve(A, f)
    return dict(name=request.param, parts=parts, P=P, p=p, d=d, A=A, Gx=Gx, Gy=Gy, f=f,
                sigma=sig_lu)


def test_bessel_device_fp64_fp32():
    torch = _torch()
    from scipy import special
    z = np.concatenate([np.geomspace(1e-4, 1.999, 300), np.linspace(1.999, 2.001, 21),
                        np.geomspace(2.001, 600, 300)])
    for kind, ref in [(0, special.k0), (1, special.k1)]:
        got = _np(yq.bessel(kind, 0, z))
        assert np.abs(got / ref(z) - 1).max() < 4e-15, kind
        # FP32: the argument itself is rounded to float, and e^-z turns a relative
        # argument error eps into z*eps, so the bound grows with z
        zf = z[z < 80]
        got32 = _np(yq.bessel(kind, 0, zf, yq.YQ_MIXED))
        assert np.all(np.abs(got32 / ref(zf) - 1) < 2e-6 + 1.2e-7 * zf), kind
    zz = np.geomspace(1e-2, 50, 200)
    for l in [2, 5, 11]:
        assert np.abs(_np(yq.bessel(2, l, zz)) / special.kv(l, zz) - 1).max() < 1e-13
    zs = np.geomspace(1e-3, 5, 100)
    for l in [0, 1, 4, 12]:
        assert np.abs(_np(yq.bessel(3, l, zs)) / special.iv(l, zs) - 1).max() < 1e-14


def test_nodes_parity(small):
    pb = _problem(small["parts"], small["P"], small["p"])
    nd = pb.nodes()
    d = small["d"]
    assert pb.N == d.N
    assert _rel(_np(nd["x"]), d.x[:, 0]) < 1e-14 and _rel(_np(nd["y"]), d.x[:, 1]) < 1e-14
    assert _rel(_np(nd["nx"]), d.normal[:, 0]) < 1e-14 and _rel(_np(nd["ny"]), d.normal[:, 1]) < 1e-14
    assert _rel(_np(nd["w"]), d.w) < 1e-14


def test_near_lists_parity(small):
    pb = _problem(small["parts"], small["P"], small["p"])
    rp, pn = pb.near()
    rp, pn = _np(rp), _np(pn)
    d = small["d"]
    for i in range(d.N):
        _, extra = oracle.near_panels(d, i)
        assert list(pn[rp[i]:rp[i + 1]]) == sorted(extra), i
    if small["name"] == "ragged_near_N336":
        assert rp[-1] > 0, "the near-contact case must exercise extra near panels"


def test_far_field_parity(small):
    pb = _problem(small["parts"], small["P"], small["p"])
    d = small["d"]
    sig = workloads.random_density(d.N, 5)
    ref = oracle.far_rows(d, list(range(d.N)), sig)
    got = _np(pb.apply_far(sig))
    assert _rel(got, ref) < 1e-12
    got32 = _np(pb.apply_far(sig, precision=yq.YQ_MIXED))
    assert _rel(got32, ref) < 5e-6


@pytest.mark.parametrize("kappa", [0.1, 0.5, 1.0, 2.0, 8.0])
def test_far32_tile_paths_parity(kappa):
    """FP32 and FP64 far fields across the pair classes: at kappa 0.1 almost every
    (target group, source tile) pair is close (panel classes and the general path),
    at kappa 8 almost every one is z >= 8; in between a mix.  N = 4368 is ragged in
    both the 64-node groups and the 256-node tiles."""
    parts = workloads.random_ellipses(13, 16.0, kappa, seed=3)
    pb = _problem(parts, 21, 6)
    d = oracle.discretize(parts, _oprm(21, 6))
    assert pb.N == d.N == 4368
    sig = workloads.random_density(d.N, 17)
    ref = oracle.far_rows(d, list(range(d.N)), sig)
    got32 = _np(pb.apply_far(sig, precision=yq.YQ_MIXED))
    assert np.all(np.isfinite(got32))
    assert _rel(got32, ref) < 5e-6
    got64 = _np(pb.apply_far(sig, precision=yq.YQ_FP64))
    # Against the oracle's own nodes the FP64 sum agrees to a few 1e-12: the two
    # sides compute node positions independently, and their 1e-16-level
    # differences grow through the 1/r pairs of adjacent nodes.  The oracle's sum
    # at the GPU's nodes isolates the pair kernel and its summation.
    assert _rel(got64, ref) < 1e-11
    nd = pb.nodes()
    dg = dataclasses.replace(d, x=np.stack([_np(nd["x"]), _np(nd["y"])], 1),
                             normal=np.stack([_np(nd["nx"]), _np(nd["ny"])], 1), w=_np(nd["w"]))
    assert _rel(got64, oracle.far_rows(dg, list(range(d.N)), sig)) < 1e-13


def test_operator_parity(small):
    pb = _problem(small["parts"], small["P"], small["p"])
    d = small["d"]
    for seed in [1, 2]:
        sig = workloads.random_density(d.N, seed)
        ref = small["A"] @ sig
        assert _rel(_np(pb.apply_operator(sig)), ref) < 1e-12
        assert _rel(_np(pb.apply_operator(sig, precision=yq.YQ_MIXED)), ref) < 5e-6


def test_solve_parity_fp64_and_mixed(small):
    torch = _torch()
    pb = _problem(small["parts"], small["P"], small["p"], tol=1e-13)
    d = small["d"]
    pb.set_boundary_data(small["f"])
    sig, info = pb.solve()
    assert info["residual"] <= 1e-13
    assert _rel(_np(sig), small["sigma"]) < 1e-10
    assert info["iterations"] < 60
    pm = _problem(small["parts"], small["P"], small["p"], tol=1e-9, precision=yq.YQ_MIXED)
    pm.set_boundary_data(small["f"])
    sm, im = pm.solve()
    assert im["residual"] <= 1e-9 and im["matvecs_fp32"] > 0
    assert _rel(_np(sm), small["sigma"]) < 1e-8


def test_gradient_forces_parity(small):
    pb = _problem(small["parts"], small["P"], small["p"])
    d = small["d"]
    sig = small["sigma"]
    gx, gy = pb.surface_gradient(sig)
    rgx, rgy = small["Gx"] @ sig, small["Gy"] @ sig
    scale = max(np.abs(rgx).max(), np.abs(rgy).max())
    assert np.abs(_np(gx) - rgx).max() < 1e-11 * scale
    assert np.abs(_np(gy) - rgy).max() < 1e-11 * scale
    pb.set_boundary_data(small["f"])
    F, T, E = pb.forces(sig, gamma=1.3)
    g = np.stack([rgx, rgy], 1)
    Fr, Tr, _, Er = oracle.forces_torques(d, small["f"], g, gamma=1.3)
    # scale: the traction integrals themselves (an isolated disk has F = 0)
    sc = max(np.abs(Fr).max(), np.abs(Tr).max(), abs(Er))
    assert np.abs(_np(F) - Fr).max() < 1e-11 * sc
    assert np.abs(_np(T) - Tr).max() < 1e-11 * sc
    assert abs(E - Er) < 1e-11 * abs(Er)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_restarted_gmres_and_iteration_limit(small, precision):
    """Short restart cycles (several cycles, a stop inside a cycle) and an iteration
    limit that ends a cycle early: the device-side Arnoldi steps count exactly."""
    prec = yq.YQ_FP64 if precision == "fp64" else yq.YQ_MIXED
    tol = 1e-11 if precision == "fp64" else 1e-9
    pb = _problem(small["parts"], small["P"], small["p"], tol=tol, precision=prec, restart=4,
                  maxiter=400)
    pb.set_boundary_data(small["f"])
    sig, info = pb.solve()
    assert info["residual"] <= tol
    assert info["outer_steps"] >= 1
    assert _rel(_np(sig), small["sigma"]) < 50 * tol
    # the same problem with one long cycle takes no more iterations than restarted
    pl = _problem(small["parts"], small["P"], small["p"], tol=tol, precision=prec, restart=100)
    pl.set_boundary_data(small["f"])
    sl, il = pl.solve()
    if precision == "fp64":   # full GMRES minimises over the larger space
        assert il["iterations"] <= info["iterations"]
    assert _rel(_np(sl), small["sigma"]) < 50 * tol
    # an iteration limit of 6 with cycles of 4: exactly 6 Arnoldi steps, not converged
    pm = _problem(small["parts"], small["P"], small["p"], tol=1e-14, precision=yq.YQ_FP64,
                  restart=4, maxiter=6)
    pm.set_boundary_data(small["f"])
    _, im = pm.solve(allow_noconv=True)
    assert im["iterations"] == 6
    assert im["matvecs_fp64"] >= 6


def test_solve_forces_matches_solve_then_forces(small):
    """The fused final residual + gradient pass gives the separate calls' results."""
    kw = dict(tol=1e-9, precision=yq.YQ_MIXED)
    pa = _problem(small["parts"], small["P"], small["p"], **kw)
    pa.set_boundary_data(small["f"])
    sa, ia = pa.solve()
    Fa, Ta, Ea = pa.forces(sa, gamma=1.3)
    pf = _problem(small["parts"], small["P"], small["p"], **kw)
    pf.set_boundary_data(small["f"])
    pf.lib.yq_profile_enable(pf.h, -1)
    sf, inf_, Ff, Tf, Ef = pf.solve_forces(gamma=1.3)
    nfu, _ = _phase(pf, 6)
    assert nfu >= 1                       # the fused pass ran
    # one timed FP32 far-field launch per counted matvec: the look-ahead launches
    # that the stop flag turned into no-ops are not in the timing
    n32, ms32 = _phase(pf, 1)
    assert n32 == inf_["matvecs_fp32"] and ms32 > 0.0
    assert inf_["iterations"] == ia["iterations"]
    assert inf_["residual"] <= 1e-9
    assert _rel(_np(sf), _np(sa)) < 1e-13
    sc = max(np.abs(_np(Fa)).max(), np.abs(_np(Ta)).max(), abs(Ea))
    assert np.abs(_np(Ff) - _np(Fa)).max() < 1e-12 * sc
    assert np.abs(_np(Tf) - _np(Ta)).max() < 1e-12 * sc
    assert abs(Ef - Ea) < 1e-12 * abs(Ea)
    # against the oracle's forces of the oracle's sigma
    g = np.stack([small["Gx"] @ small["sigma"], small["Gy"] @ small["sigma"]], 1)
    Fr, Tr, _, Er = oracle.forces_torques(small["d"], small["f"], g, gamma=1.3)
    scr = max(np.abs(Fr).max(), np.abs(Tr).max(), abs(Er))
    assert np.abs(_np(Ff) - Fr).max() < 1e-7 * scr
    # FP64 solves take the unfused path and still agree
    p64 = _problem(small["parts"], small["P"], small["p"], tol=1e-12)
    p64.set_boundary_data(small["f"])
    s64, i64, F64, T64, E64 = p64.solve_forces(gamma=1.3)
    assert i64["residual"] <= 1e-12
    assert np.abs(_np(F64) - Fr).max() < 1e-9 * scr


def test_potential_parity(small):
    pb = _problem(small["parts"], small["P"], small["p"])
    d = small["d"]
    sig = small["sigma"]
    rng = np.random.default_rng(3)
    # points near the boundary (within pot_beta*h of a panel) and far away
    i = rng.integers(0, d.N, 40)
    off = rng.uniform(0.01, 0.4, 40)
    near = d.x[i] + off[:, None] * d.normal[i]
    far = rng.uniform(-4, 4, (40, 2))
    far = far[np.min(np.hypot(*(d.x[None] - far[:, None]).transpose(2, 0, 1)), axis=1) > 1e-3]
    pts = np.concatenate([near, far])
    ref = oracle.eval_potential(d, sig, pts)
    assert _rel(_np(pb.eval_potential(sig, pts)), ref) < 1e-12
    assert pb.eval_potential(sig, np.zeros((0, 2))).numel() == 0


# ---- full-size medium workload: sampled rows and properties ---------------------------------

@pytest.fixture(scope="module")
def medium():
    cfg = workloads.config_medium(kappa=1.0, seed=0)
    parts = cfg["particles"]
    d = oracle.discretize(parts, _oprm(cfg["panels"], cfg["qbx_order"]))
    return dict(cfg=cfg, parts=parts, d=d)


def test_medium_operator_sampled_rows(medium):
    d = medium["d"]
    pb = _problem(medium["parts"], medium["cfg"]["panels"], medium["cfg"]["qbx_order"])
    assert pb.N == 25600
    sig = workloads.random_density(d.N, 11)
    rows = sorted(set(np.random.default_rng(0).integers(0, d.N, 24).tolist()) | {0, d.N - 1})
    ref = oracle.apply_rows(d, rows, sig)
    got = _np(pb.apply_operator(sig))[rows]
    assert _rel(got, ref) < 1e-12
    got32 = _np(pb.apply_operator(sig, precision=yq.YQ_MIXED))[rows]
    assert _rel(got32, ref) < 5e-6


def test_medium_solve_residual_property(medium):
    d = medium["d"]
    cfg = medium["cfg"]
    pm = _problem(medium["parts"], cfg["panels"], cfg["qbx_order"], tol=1e-8,
                  precision=yq.YQ_MIXED)
    f = pm.boundary_label()
    fo = oracle.arc_label(d)
    assert _rel(_np(f), fo) < 1e-13
    pm.set_boundary_data(f)
    sig, info = pm.solve()
    assert info["residual"] <= 1e-8
    sig = _np(sig)
    rows = sorted(set(np.random.default_rng(1).integers(0, d.N, 16).tolist()))
    r = oracle.apply_rows(d, rows, sig) - fo[rows]
    assert np.abs(r).max() < 1e-7
    F, T, E = pm.forces(sig)
    F = _np(F)
    assert np.abs(F.sum(0)).max() < 1e-2 * np.abs(F).max()   # tanh arc edges: see oracle pins
    assert E > 0
    # the fused final residual + gradient at full size gives the same forces
    pm.lib.yq_profile_enable(pm.h, -1)
    sf, inf_, Ff, Tf, Ef = pm.solve_forces()
    assert _phase(pm, 6)[0] >= 1
    assert inf_["residual"] <= 1e-8
    assert _rel(_np(sf), sig) < 1e-12
    assert _rel(_np(Ff), F) < 1e-11 and abs(Ef - E) < 1e-11 * abs(E)


# ---- edge cases and error paths -----------------------------------------------------------------

def test_errors_and_edges():
    torch = _torch()
    import ctypes
    from paper_1810_04131_amd import _lib
    pb = yq.Problem(yq.default_params(panels_per_particle=8, qbx_order=6))
    with pytest.raises(yq.YQError) as e:
        pb.apply_operator(torch.zeros(16, dtype=torch.float64, device="cuda"))
    assert e.value.status == _lib.YQ_ESTATE
    # overlapping particles
    with pytest.raises(yq.YQError) as e:
        pb.set_particles([[0, 0], [0.5, 0]], [0, 0], [[1, 0.5], [1, 0.5]], 1.0)
    assert e.value.status == _lib.YQ_EGEOM
    with pytest.raises(yq.YQError) as e:
        pb.set_particles([[0, 0]], [0], [[0.5, 1.0]], 1.0)      # A < B
    assert e.value.status == _lib.YQ_EINVAL
    with pytest.raises(yq.YQError) as e:
        pb.set_particles([[0, 0]], [0], [[1.0, 0.5]], float("nan"))
    assert e.value.status == _lib.YQ_EINVAL
    # one particle, minimum panel count, non-convergence reported
    pb = yq.Problem(yq.default_params(panels_per_particle=5, qbx_order=4, maxiter=1, tol=1e-14))
    pb.set_particles([[0.3, 0.1]], [0.2], [[1.0, 0.7]], 2.0)
    assert pb.N == 80
    pb.set_boundary_data(pb.boundary_label(yq.YQ_LABEL_JANUS, 2.0, 0.0))
    sig, info = pb.solve(allow_noconv=True)
    assert info["iterations"] == 1 and info["residual"] > 1e-14
    with pytest.raises(yq.YQError) as e:
        pb.solve()
    assert e.value.status == _lib.YQ_ENOCONV


# ---- the paper's printed single-disk table (golden fixture) ----------------------------------

@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 1e-10)])
def test_table1_single_disk_meets_paper_error(precision, tol):
    """Table 1 (tests/golden/table1_single_disk.json): the HIP path on the paper's
    single-disk problem, evaluated on the paper's full 200 x 200 grid of the 5 x 5
    domain against eq. true_soln, is more accurate than every entry of the table."""
    from test_oracle_pins import _table1, _true_soln, table1_targets
    t = _table1()
    best = min(min(t[k]["linf"]) for k in ("p4", "p6", "p8"))
    pb = _problem(workloads.single_disk(1.0, 0.25), 20, 8, tol=tol, precision=precision)
    pb.set_boundary_data(pb.boundary_label(yq.YQ_LABEL_JANUS, 2.0, 0.0))
    sig, info = pb.solve()
    assert info["residual"] <= tol and info["iterations"] <= 30
    pts = table1_targets(1, 20)
    u = _np(pb.eval_potential(sig, pts))
    err = np.abs(u - _true_soln(pts, 0.25)).max()
    assert err < best, (err, best)
