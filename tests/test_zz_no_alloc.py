"""yq_eval_potential_noalloc (scratch in the library's device array, no
allocation) against yq_eval_potential, through the C ABI: two calls in a row,
the second with a smaller input, then the size limit."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

yq = pytest.importorskip("paper_1810_04131_amd")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _targets(parts, m, seed, box):
    # water points around the particles, some close to a boundary
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < m:
        z = rng.uniform(-1.0, box + 1.0, 2)
        inside = False
        for c, a, (A, B) in zip(parts.center, parts.angle, parts.axes):
            d = z - c
            u = np.cos(a) * d[0] + np.sin(a) * d[1]
            v = -np.sin(a) * d[0] + np.cos(a) * d[1]
            inside |= (u / A) ** 2 + (v / B) ** 2 <= 1.05
        if not inside:
            pts.append(z)
    return np.array(pts)


def _both(torch, pb, sigma, pts):
    lib = yq._lib.load()
    tx = torch.as_tensor(np.ascontiguousarray(pts[:, 0]), device="cuda")
    ty = torch.as_tensor(np.ascontiguousarray(pts[:, 1]), device="cuda")
    u_ref = torch.empty(len(pts), dtype=torch.float64, device="cuda")
    u_new = torch.full((len(pts),), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert lib.yq_eval_potential(pb.h, p(sigma), len(pts), p(tx), p(ty), p(u_ref)) == 0
    assert lib.yq_eval_potential_noalloc(pb.h, p(sigma), len(pts), p(tx), p(ty), p(u_new)) == 0
    torch.cuda.synchronize()
    return u_ref.cpu().numpy(), u_new.cpu().numpy()


def _solved(params, parts):
    pb = yq.Problem(params)
    pb.set_workload(parts)
    pb.set_boundary_data(pb.boundary_label())
    sigma, _ = pb.solve()
    return pb, sigma


def test_noalloc_potential_matches_two_calls_then_smaller():
    torch = _torch()
    big = workloads.random_ellipses(8, 14.0, 1.3, seed=5)
    pa, sa = _solved(yq.default_params(panels_per_particle=16, qbx_order=8, tol=1e-12), big)
    ua, na = _both(torch, pa, sa, _targets(big, 1500, 1, 14.0))
    assert np.all(np.isfinite(na))
    assert np.abs(na - ua).max() <= 1e-14 * np.abs(ua).max()
    small = workloads.two_ellipses(2, 0.8)
    pb, sb = _solved(yq.default_params(panels_per_particle=12, qbx_order=8, tol=1e-12), small)
    ub, nb = _both(torch, pb, sb, _targets(small, 100, 2, 3.0))
    assert np.all(np.isfinite(nb))
    assert np.abs(nb - ub).max() <= 1e-14 * np.abs(ub).max()
    # the first problem again, after the smaller one overwrote the shared scratch
    ua2, na2 = _both(torch, pa, sa, _targets(big, 300, 3, 14.0))
    assert np.abs(na2 - ua2).max() <= 1e-14 * np.abs(ua2).max()


def test_noalloc_potential_rejects_scratch_beyond_its_limit():
    torch = _torch()
    parts = workloads.two_ellipses(2, 0.8)
    pb, sigma = _solved(yq.default_params(panels_per_particle=12, qbx_order=8, tol=1e-10), parts)
    M = 9_000_000      # one chunk x M partial sums alone exceed 64 MiB
    t = torch.zeros(M, dtype=torch.float64, device="cuda")
    u = torch.zeros(M, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lib = yq._lib.load()
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    st = lib.yq_eval_potential_noalloc(pb.h, p(sigma), M, p(t), p(t), p(u))
    assert st == yq._lib.YQ_EINVAL
    assert b"scratch" in lib.yq_last_error(pb.h)
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0.0     # nothing was launched
