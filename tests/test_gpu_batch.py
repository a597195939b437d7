"""Batched solves (many configurations per fused launch) against the oracle, against
the single-configuration path, and alone vs in a mix; FMM configurations as trees
of the engine's forest (the default) and as worker-thread problems."""
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


P, ORDER = 12, 8


def _configs():
    # uneven sizes and screening constants; one config with a ragged node count
    return [
        workloads.random_ellipses(3, 9.0, 0.7, seed=1),
        workloads.two_ellipses(2, 1.6),
        workloads.random_ellipses(5, 12.0, 1.2, seed=3),
        workloads.single_disk(1.0, 0.5),
    ]


@pytest.fixture(scope="module")
def oracles():
    out = []
    for c in _configs():
        d = oracle.discretize(c, Params(panels=P, qbx_order=ORDER))
        A = oracle.build_matrices(d)
        f = oracle.arc_label(d)
        out.append(dict(d=d, A=A, f=f, sigma=oracle.lu_solve(A, f)))
    return out


def _batch(configs, **kw):
    _torch()
    b = yq.Batch(yq.default_params(panels_per_particle=P, qbx_order=ORDER, **kw))
    b.set_configs(configs)
    return b


def test_batch_operator_parity(oracles):
    b = _batch(_configs())
    sig = np.concatenate([workloads.random_density(o["d"].N, 7 + c) for c, o in enumerate(oracles)])
    out = _np(b.apply_operator(sig))
    out32 = _np(b.apply_operator(sig, yq.YQ_MIXED))
    for c, o in enumerate(oracles):
        s = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
        ref = o["A"] @ sig[s]
        assert _rel(out[s], ref) < 1e-12, c
        assert _rel(out32[s], ref) < 5e-6, c


@pytest.mark.parametrize("precision,tol,bound", [(0, 1e-13, 1e-10), (1, 1e-9, 1e-8)])
def test_batch_solve_parity(oracles, precision, tol, bound):
    b = _batch(_configs(), tol=tol, precision=precision)
    f = b.boundary_label()
    b.set_boundary_data(f)
    sig, infos = b.solve()
    sig = _np(sig)
    for c, o in enumerate(oracles):
        s = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
        assert _rel(_np(f)[s], o["f"]) < 1e-13
        assert infos[c]["residual"] <= tol, (c, infos[c])
        assert _rel(sig[s], o["sigma"]) < bound, c


def test_batch_alone_equals_mix_and_single_path():
    torch = _torch()
    cfgs = _configs()
    mix = _batch(cfgs, tol=1e-10, precision=1)
    mix.set_boundary_data(mix.boundary_label())
    sm, im = mix.solve()
    sm = _np(sm)
    for c, cfg in enumerate(cfgs):
        alone = _batch([cfg], tol=1e-10, precision=1)
        alone.set_boundary_data(alone.boundary_label())
        sa, ia = alone.solve()
        seg = sm[int(mix.offsets[c]):int(mix.offsets[c + 1])]
        # same arithmetic for a configuration alone and in the mix: bitwise equal
        assert np.array_equal(_np(sa), seg), c
        assert ia[0]["iterations"] == im[c]["iterations"]
        # and the single-problem path agrees within the solve tolerance
        pb = yq.Problem(yq.default_params(panels_per_particle=P, qbx_order=ORDER, tol=1e-10,
                                          precision=1))
        pb.set_workload(cfg)
        pb.set_boundary_data(pb.boundary_label())
        ss, _ = pb.solve()
        assert _rel(_np(ss), seg) < 1e-8


def test_batch_graph_replays_match_eager():
    torch = _torch()
    cfgs = _configs()
    g = _batch(cfgs, tol=1e-10, precision=1)
    e = _batch(cfgs, tol=1e-10, precision=1)
    e.use_graphs(False)
    for b in (g, e):
        b.set_boundary_data(b.boundary_label())
    se, _ = e.solve()
    se = _np(se)
    sig = np.random.default_rng(0).standard_normal(g.total)
    for rep in range(3):
        sg, _ = g.solve()              # every iteration is a graph replay
        assert np.array_equal(_np(sg), se), rep
        # eager work and synchronisation between replays
        o1 = _np(g.apply_operator(sig))
        o2 = _np(e.apply_operator(sig))
        assert np.array_equal(o1, o2)
        torch.cuda.synchronize()


def test_batch_forces_match_single():
    torch = _torch()
    cfgs = _configs()
    b = _batch(cfgs, tol=1e-10)
    b.set_boundary_data(b.boundary_label())
    sig, _ = b.solve()
    F, T, E = b.forces(sig)
    F, T = _np(F), _np(T)
    p0 = 0
    for c, cfg in enumerate(cfgs):
        pb = yq.Problem(yq.default_params(panels_per_particle=P, qbx_order=ORDER))
        pb.set_workload(cfg)
        pb.set_boundary_data(pb.boundary_label())
        Fs, Ts, Es = pb.forces(b.segment(sig, c))
        n = cfg.center.shape[0]
        assert np.array_equal(_np(Fs), F[p0:p0 + n]) and np.array_equal(_np(Ts), T[p0:p0 + n])
        assert Es == E[c]
        p0 += n


def test_batch_autotune_keeps_results_within_tolerance(oracles):
    b = _batch(_configs(), tol=1e-10, precision=1)
    pbk, fw = b.autotune()
    assert pbk in (1024, 2048, 4096, 8192) and fw in (2048, 4096, 8192)
    b.set_boundary_data(b.boundary_label())
    sig, infos = b.solve()
    sig = _np(sig)
    for c, o in enumerate(oracles):
        s = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
        assert _rel(sig[s], o["sigma"]) < 1e-8


def test_batch_fmm_lane_matches_oracle_single_and_direct_batch(oracles):
    torch = _torch()
    cfgs = _configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1)
    b = yq.Batch(yq.default_params(**prm))
    # the 5-particle configuration takes the FMM, as a worker-thread problem
    b.set_fmm(5 * P * 16, workers=2, in_engine=False)
    b.set_configs(cfgs)
    with pytest.raises(yq.YQError):
        b.set_fmm(0)                         # only before set_configs
    b.set_boundary_data(b.boundary_label())
    sig, infos = b.solve()
    sig = _np(sig)
    direct = _batch(cfgs, **{k: v for k, v in prm.items() if k not in ("panels_per_particle", "qbx_order")})
    direct.set_boundary_data(direct.boundary_label())
    sd, _ = direct.solve()
    sd = _np(sd)
    x = np.concatenate([workloads.random_density(o["d"].N, 40 + c) for c, o in enumerate(oracles)])
    op = _np(b.apply_operator(x))
    for c, o in enumerate(oracles):
        s = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
        assert infos[c]["residual"] <= 1e-10, (c, infos[c])
        assert _rel(sig[s], o["sigma"]) < 1e-8, c
        assert _rel(op[s], o["A"] @ x[s]) < 1e-12, c
        if c == 2:
            # the lane's configuration is exactly a standalone FMM solve
            pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, **prm))
            pb.set_workload(cfgs[c])
            pb.set_boundary_data(pb.boundary_label())
            ss, _ = pb.solve()
            assert np.array_equal(_np(ss), sig[s])
        else:
            # the engine members are unchanged by the lane next to them
            assert np.array_equal(sd[s], sig[s]), c
    F, T, E = b.forces(torch.as_tensor(sig, device="cuda"))
    Fd, Td, Ed = direct.forces(torch.as_tensor(sig, device="cuda"))
    sc = max(np.abs(_np(Fd)).max(), np.abs(_np(Td)).max())
    assert np.abs(_np(F) - _np(Fd)).max() < 1e-9 * sc and np.abs(_np(T) - _np(Td)).max() < 1e-9 * sc
    # every configuration in the lane (no engine members)
    allf = yq.Batch(yq.default_params(far_mode=yq.YQ_FAR_FMM, **prm))
    allf.set_fmm(0, workers=2, in_engine=False)
    allf.set_configs(cfgs[:2])
    allf.set_boundary_data(allf.boundary_label())
    sa, ia = allf.solve()
    for c in range(2):
        s = slice(int(allf.offsets[c]), int(allf.offsets[c + 1]))
        assert ia[c]["residual"] <= 1e-10 and _rel(_np(sa)[s], oracles[c]["sigma"]) < 1e-8


def _lane_batch(cfgs, graphs, in_engine=True, near=0, **prm):
    b = yq.Batch(yq.default_params(**prm))
    # the 5-particle configuration takes the FMM (a forest tree, or a lane problem);
    # near: the trees' near-field cache budget (0: the leaf passes evaluate every pair,
    # as a standalone FMM problem does)
    b.set_near_cache(near)
    b.set_fmm(5 * P * 16, workers=2, in_engine=in_engine)
    b.set_configs(cfgs)
    b.use_graphs(graphs)
    return b


def _forest_configs():
    # two FMM configurations of different tree depths between direct members
    return _configs() + [workloads.random_ellipses(9, 16.0, 0.9, seed=4)]


def test_batch_fmm_forest_matches_oracle_single_path_and_alone(oracles):
    torch = _torch()
    cfgs = _forest_configs()
    orc = list(oracles)
    d = oracle.discretize(cfgs[4], Params(panels=P, qbx_order=ORDER))
    A4 = oracle.build_matrices(d)
    f4 = oracle.arc_label(d)
    orc.append(dict(d=d, A=A4, f=f4, sigma=oracle.lu_solve(A4, f4)))
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1)
    b = _lane_batch(cfgs, True, **prm)
    b.set_boundary_data(b.boundary_label())
    sig, infos = b.solve()
    sig = _np(sig)
    direct = _batch(cfgs[:4], tol=1e-10, precision=1)
    direct.set_boundary_data(direct.boundary_label())
    sd = _np(direct.solve()[0])
    x = np.concatenate([workloads.random_density(o["d"].N, 60 + c) for c, o in enumerate(orc)])
    op32 = _np(b.apply_operator(x, yq.YQ_MIXED))
    op64 = _np(b.apply_operator(x, yq.YQ_FP64))
    for c, o in enumerate(orc):
        s = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
        assert infos[c]["residual"] <= 1e-10, (c, infos[c])
        assert _rel(sig[s], o["sigma"]) < 1e-8, c
        if c in (2, 4):
            # forest trees: the inner operator is the standalone FMM problem's up to the
            # engine's FP32 copy of the QBX correction, and the FP64 one the order-40
            # FMM's (operator error ~1e-10)
            pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, **prm))
            pb.set_workload(cfgs[c])
            assert _rel(op32[s], _np(pb.apply_operator(x[s], yq.YQ_MIXED))) < 1e-6, c
            assert _rel(op64[s], o["A"] @ x[s]) < 1e-9, c
            pb.set_boundary_data(pb.boundary_label())
            ss, _ = pb.solve()
            assert _rel(sig[s], _np(ss)) < 1e-8, c
            # alone (a batch of one tree) = in the mix, bitwise
            alone = _lane_batch([cfgs[c]], True, **prm)
            alone.set_boundary_data(alone.boundary_label())
            sa, ia = alone.solve()
            assert np.array_equal(_np(sa), sig[s]), c
            assert ia[0]["iterations"] == infos[c]["iterations"], c
        else:
            assert np.array_equal(sd[s], sig[s]), c          # direct members: unchanged
            assert _rel(op64[s], o["A"] @ x[s]) < 1e-12, c
    F, T, E = b.forces(torch.as_tensor(sig, device="cuda"))
    Fd, Td, Ed = direct.forces(torch.as_tensor(sig[:int(b.offsets[4])], device="cuda"))
    n4 = int(sum(c.center.shape[0] for c in cfgs[:4]))
    sc = max(np.abs(_np(Fd)).max(), np.abs(_np(Td)).max())
    assert np.abs(_np(F)[:n4] - _np(Fd)).max() < 1e-9 * sc
    assert np.abs(_np(T)[:n4] - _np(Td)).max() < 1e-9 * sc
    # a tree's forces (order-40 FMM gradient, batched) are the standalone FMM problem's
    poffs = np.concatenate([[0], np.cumsum([c.center.shape[0] for c in cfgs])])
    for c in (2, 4):
        pb = yq.Problem(yq.default_params(far_mode=yq.YQ_FAR_FMM, **prm))
        pb.set_workload(cfgs[c])
        pb.set_boundary_data(pb.boundary_label())
        Fs, Ts, Es = pb.forces(b.segment(torch.as_tensor(sig, device="cuda"), c))
        assert np.array_equal(_np(Fs), _np(F)[poffs[c]:poffs[c + 1]]), c
        assert np.array_equal(_np(Ts), _np(T)[poffs[c]:poffs[c + 1]]), c
        assert Es == E[c], c
    # every configuration a tree (no direct members), in FP64 precision too
    for precision, tol, bound in ((1, 1e-10, 1e-8), (0, 1e-11, 1e-8)):
        allf = yq.Batch(yq.default_params(far_mode=yq.YQ_FAR_FMM, panels_per_particle=P,
                                          qbx_order=ORDER, tol=tol, precision=precision))
        allf.set_configs([cfgs[0], cfgs[4]])
        allf.set_boundary_data(allf.boundary_label())
        sa, ia = allf.solve()
        for k, c in enumerate((0, 4)):
            s = slice(int(allf.offsets[k]), int(allf.offsets[k + 1]))
            assert ia[k]["residual"] <= tol and _rel(_np(sa)[s], orc[c]["sigma"]) < bound


@pytest.mark.parametrize("in_engine", [True, False])
def test_batch_graph_replay_equals_eager_with_fmm_configurations(in_engine):
    # the fused iteration stays graph-captured with forest trees in it, or while
    # lane workers solve beside it
    _torch()
    cfgs = _forest_configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1)
    e = _lane_batch(cfgs, False, in_engine, **prm)
    e.set_boundary_data(e.boundary_label())
    se, ie = e.solve()
    se = _np(se)
    g = _lane_batch(cfgs, True, in_engine, **prm)
    g.set_boundary_data(g.boundary_label())
    for rep in range(3):
        sg, ig = g.solve()
        assert np.array_equal(_np(sg), se), rep
        assert [i["iterations"] for i in ig] == [i["iterations"] for i in ie]


@pytest.mark.parametrize("in_engine,precision", [(True, 1), (False, 1), (True, 0)])
def test_batch_solve_forces_matches_solve_then_forces(in_engine, precision):
    # the mixed solves' last FP64 residual also gives the forces' gradient far field
    torch = _torch()
    cfgs = _forest_configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-9 if precision else 1e-11,
               precision=precision)
    a = _lane_batch(cfgs, True, in_engine, **prm)
    a.set_boundary_data(a.boundary_label())
    sa, ia = a.solve()
    Fa, Ta, Ea = a.forces(sa, gamma=1.3)
    f = _lane_batch(cfgs, True, in_engine, **prm)
    f.set_boundary_data(f.boundary_label())
    sf, inf_, Ff, Tf, Ef = f.solve_forces(gamma=1.3)
    assert [i["iterations"] for i in inf_] == [i["iterations"] for i in ia]
    assert max(i["residual"] for i in inf_) <= prm["tol"]
    assert _rel(_np(sf), _np(sa)) < 1e-13
    sc = max(np.abs(_np(Fa)).max(), np.abs(_np(Ta)).max())
    assert np.abs(_np(Ff) - _np(Fa)).max() < 1e-12 * sc
    assert np.abs(_np(Tf) - _np(Ta)).max() < 1e-12 * sc
    assert np.abs(Ef - Ea).max() < 1e-12 * np.abs(Ea).max()


def test_batch_raw_abi_without_device_sync_between_calls():
    # The batch calls are synchronous by contract: driven through the C ABI alone,
    # with no device-wide synchronisation between set-up, boundary data and solve,
    # the results equal those of the binding (which synchronises before each call).
    import ctypes
    torch = _torch()
    cfgs = _configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1)
    ref = _lane_batch(cfgs, True, near=-1, **prm)   # the library's default cache budget
    ref.set_boundary_data(ref.boundary_label())
    sref, _ = ref.solve()
    sref = _np(sref)

    lib = yq._lib.load()
    params = yq.default_params(**prm)
    h = ctypes.c_void_p()
    assert lib.yq_batch_create(ctypes.byref(params), ctypes.byref(h)) == 0
    try:
        assert lib.yq_batch_set_fmm(h, 5 * P * 16, 2) == 0
        npart = np.ascontiguousarray([c.center.shape[0] for c in cfgs], dtype=np.int32)
        cat = lambda k: np.ascontiguousarray(np.concatenate(
            [np.asarray(getattr(c, k), float).reshape(-1) for c in cfgs]))
        cen, ang, ax = cat("center"), cat("angle"), cat("axes")
        kap = np.ascontiguousarray([float(c.kappa) for c in cfgs])
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        assert lib.yq_batch_set_configs(h, len(cfgs), vp(npart), vp(cen), vp(ang), vp(ax),
                                        vp(kap)) == 0
        total = ctypes.c_int64()
        assert lib.yq_batch_num_nodes(h, ctypes.byref(total), None) == 0
        f = torch.empty(total.value, dtype=torch.float64, device="cuda")
        sig = torch.empty_like(f)
        torch.cuda.synchronize()            # the buffers exist before the library writes them
        assert lib.yq_batch_boundary_label(h, 0, ctypes.c_double(np.pi / 4),
                                           ctypes.c_double(0.1), ctypes.c_void_p(f.data_ptr())) == 0
        assert lib.yq_batch_set_boundary_data(h, ctypes.c_void_p(f.data_ptr())) == 0
        infos = (yq.yq_solve_info * len(cfgs))()
        assert lib.yq_batch_solve(h, ctypes.c_void_p(sig.data_ptr()), infos) == 0
        assert np.array_equal(_np(sig), sref)
    finally:
        lib.yq_batch_destroy(h)


def test_batch_far_field_timers_count_pairs_and_leave_results_unchanged():
    torch = _torch()
    cfgs = _configs()
    prm = dict(tol=1e-10, precision=1)
    ref = _batch(cfgs, **prm)
    ref.set_boundary_data(ref.boundary_label())
    s_ref, i_ref = ref.solve()
    b = _batch(cfgs, **prm)
    b.profile(True)
    x = np.random.default_rng(3).standard_normal(b.total)
    b.apply_operator(x, yq.YQ_MIXED)
    n, ms, pairs = b.profile_read(yq.YQ_MIXED)
    N = np.diff(b.offsets)
    assert n == 1 and ms > 0.0 and pairs == float((N * N).sum())
    b.apply_operator(x, yq.YQ_FP64)
    n64, ms64, pairs64 = b.profile_read(yq.YQ_FP64)
    assert n64 == 1 and ms64 > 0.0 and pairs64 == float((N * N).sum())
    b.set_boundary_data(b.boundary_label())
    s, infos = b.solve()                 # split graphs with events between them
    assert np.array_equal(_np(s), _np(s_ref))
    n, ms, pairs = b.profile_read(yq.YQ_MIXED)
    fp32_matvecs = sum(i["matvecs_fp32"] for i in infos)
    assert n >= max(i["matvecs_fp32"] for i in infos) and ms > 0.0
    # every evaluated pair belongs to a configuration's own N^2 block
    assert 0 < pairs <= float((N * N * np.array([i["matvecs_fp32"] + 2 for i in infos])).sum())
    assert fp32_matvecs > 0


def _sym_configs():
    # 2 chunks of 1,024 nodes at 12 panels (1,728 nodes); at 13 panels the 1,456 nodes
    # end in a ragged group of 48; one single-chunk configuration
    return [
        workloads.random_ellipses(9, 16.0, 0.9, seed=4),
        workloads.random_ellipses(7, 14.0, 1.1, seed=5),
        workloads.random_ellipses(3, 9.0, 0.7, seed=1),
    ]


@pytest.mark.parametrize("panels", [12, 13])
def test_batch_symmetric_far_field_matches_directed_and_oracle(panels):
    """One kernel evaluation per unordered pair (default) against one per directed pair
    and against the oracle's operator; the symmetric items of a configuration alone
    give the same bits as in the mix, and the timers count every directed pair."""
    torch = _torch()
    cfgs = _sym_configs()
    prm = yq.default_params(panels_per_particle=panels, qbx_order=ORDER)
    sym = yq.Batch(prm)
    sym.set_configs(cfgs)
    dirb = yq.Batch(prm).set_symmetric_far(False)
    dirb.set_configs(cfgs)
    assert np.array_equal(sym.offsets, dirb.offsets)
    N = np.diff(sym.offsets)
    assert N.max() > 1024 and (N % 64 != 0).any() == (panels == 13)
    sig = np.concatenate([workloads.random_density(int(n), 11 + c) for c, n in enumerate(N)])
    sym.profile(True)
    o_sym = _np(sym.apply_operator(sig, yq.YQ_MIXED))
    n, ms, pairs = sym.profile_read(yq.YQ_MIXED)
    assert n == 1 and ms > 0.0 and pairs == float((N * N).sum())
    o_dir = _np(dirb.apply_operator(sig, yq.YQ_MIXED))
    o_64 = _np(sym.apply_operator(sig))
    # the oracle's operator on one two-chunk configuration (ragged at 13 panels); the
    # FP64 engine operator, which matches the oracle to 1e-12, on all of them
    oc = 0 if panels == 12 else 1
    so = slice(int(sym.offsets[oc]), int(sym.offsets[oc + 1]))
    ref = oracle.build_matrices(oracle.discretize(cfgs[oc], Params(panels=panels,
                                                                   qbx_order=ORDER))) @ sig[so]
    assert _rel(o_64[so], ref) < 1e-12
    assert _rel(o_sym[so], ref) < 5e-6 and _rel(o_dir[so], ref) < 5e-6
    for c, cfg in enumerate(cfgs):
        s = slice(int(sym.offsets[c]), int(sym.offsets[c + 1]))
        ref = o_64[s]
        assert _rel(o_sym[s], ref) < 5e-6, c
        assert _rel(o_dir[s], ref) < 5e-6, c
        assert _rel(o_sym[s], o_dir[s]) < 5e-6, c
        alone = yq.Batch(prm)
        alone.set_configs([cfg])
        assert np.array_equal(_np(alone.apply_operator(sig[s], yq.YQ_MIXED)), o_sym[s]), c
    # the mixed solve with the symmetric inner operator reaches the FP64 tolerance
    sb = yq.Batch(yq.default_params(panels_per_particle=panels, qbx_order=ORDER, tol=1e-10,
                                    precision=1))
    sb.set_configs(cfgs)
    sb.set_boundary_data(sb.boundary_label())
    ss, infos = sb.solve()
    fb = yq.Batch(yq.default_params(panels_per_particle=panels, qbx_order=ORDER, tol=1e-12))
    fb.set_configs(cfgs)
    fb.set_boundary_data(fb.boundary_label())
    sf, _ = fb.solve()
    assert all(i["residual"] <= 1e-10 for i in infos)
    assert _rel(_np(ss), _np(sf)) < 1e-8
    torch.cuda.synchronize()


def test_batch_leaf_pass_timers_count_pairs_and_leave_results_unchanged():
    """The forest's leaf-pass timers: one timed launch per operator application, the
    same pair count at both orders (one tree), bounded by the members' N^2, and a
    profiled solve (iteration graph split into parts) equal to the plain one."""
    _torch()
    cfgs = _forest_configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1)
    ref = _lane_batch(cfgs, True, **prm)
    ref.set_boundary_data(ref.boundary_label())
    s_ref, i_ref = ref.solve()
    b = _lane_batch(cfgs, True, **prm)
    b.profile(True)
    N = np.diff(b.offsets)
    tree = N >= 5 * P * 16
    assert tree.sum() == 2
    x = np.random.default_rng(5).standard_normal(b.total)
    b.apply_operator(x, yq.YQ_MIXED)
    n1, ms1, p1, by1 = b.profile_read(yq.YQ_MIXED, reset=False, kernel="leaf")
    b.apply_operator(x, yq.YQ_MIXED)
    n2, ms2, p2, _ = b.profile_read(yq.YQ_MIXED, kernel="leaf")
    assert n1 == 1 and n2 == 2 and 0.0 < ms1 < ms2 and p2 == 2 * p1
    assert by1 == 0.0   # no near-field cache: no cached bytes
    assert float(N[tree].sum()) < p1 <= float((N[tree] ** 2).sum())
    b.apply_operator(x, yq.YQ_FP64)
    n64, ms64, p64, _ = b.profile_read(yq.YQ_FP64, kernel="leaf")
    assert n64 == 1 and ms64 > 0.0 and p64 == p1
    b.set_boundary_data(b.boundary_label())
    s, infos = b.solve()
    assert np.array_equal(_np(s), _np(s_ref))
    assert [i["iterations"] for i in infos] == [i["iterations"] for i in i_ref]
    n, ms, pairs, _ = b.profile_read(yq.YQ_MIXED, kernel="leaf")
    assert n >= max(i["matvecs_fp32"] for i in infos) and 0 < pairs <= n * p1


def test_batch_qbx_fold_with_panels_left_out():
    """QBX corrections folded into the near-field caches: with 16-node leaves many
    window panels (80 nodes per target) reach past the leaf's P2P list, so the finish
    applies those panels itself (the left-out list) while the rest ride in the cached
    coefficients; the operators agree with the passes that evaluate every pair."""
    _torch()
    cfgs = _forest_configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1, fmm_leaf_max=16)
    plain = _lane_batch(cfgs, True, near=0, **prm)
    cached = _lane_batch(cfgs, True, near=-1, **prm)
    assert cached.near_cache_info()[1:] == (2, 2)
    x = np.random.default_rng(12).standard_normal(cached.total)
    for prec, tol in ((yq.YQ_MIXED, 5e-6), (yq.YQ_FP64, 1e-12)):
        a = _np(cached.apply_operator(x, prec))
        b = _np(plain.apply_operator(x, prec))
        for c in range(len(cfgs)):
            s = slice(int(cached.offsets[c]), int(cached.offsets[c + 1]))
            assert _rel(a[s], b[s]) < tol, (prec, c)


def test_batch_leaves_over_64_nodes_stay_uncached():
    """The cached leaf pass hands a source leaf's densities to the lanes through one
    wavefront exchange (at most 64 nodes): trees built with larger leaves keep the
    passes that evaluate every pair, and their solves agree with the default trees'."""
    _torch()
    cfgs = _forest_configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1)
    big = _lane_batch(cfgs, True, near=-1, fmm_leaf_max=200, **prm)
    assert big.near_cache_info() == (0, 0, 0)
    ref = _lane_batch(cfgs, True, near=-1, **prm)
    for bt in (big, ref):
        bt.set_boundary_data(bt.boundary_label())
    sb, ib = big.solve()
    sr, _ = ref.solve()
    assert all(i["residual"] <= 1e-10 for i in ib)
    assert _rel(_np(sb), _np(sr)) < 1e-8


def test_batch_near_cache_matches_uncached_leaf_passes():
    """Forest trees with their near-field coefficients cached (FP32 inner, FP64
    residual operator) against the passes that evaluate every pair; the budget
    decides which trees hold a cache; a cached tree alone gives the bits it gives in
    the mix, and graph replays equal eager iterations."""
    torch = _torch()
    cfgs = _forest_configs()
    prm = dict(panels_per_particle=P, qbx_order=ORDER, tol=1e-10, precision=1)
    plain = _lane_batch(cfgs, True, near=0, **prm)
    cached = _lane_batch(cfgs, True, near=-1, **prm)
    held, t32, t64 = cached.near_cache_info()
    assert (t32, t64) == (2, 2) and held > 0 and plain.near_cache_info() == (0, 0, 0)
    # the cached pass's algorithmic bytes: 4 per pair, 16 per target, 8 per source of
    # each list entry (at least one pair each, so at most 8 per pair)
    cached.profile(True)
    xp = np.random.default_rng(8).standard_normal(cached.total)
    cached.apply_operator(xp, yq.YQ_MIXED)
    _, _, pr, by = cached.profile_read(yq.YQ_MIXED, kernel="leaf")
    Nt = float(np.diff(cached.offsets)[np.diff(cached.offsets) >= 5 * P * 16].sum())
    assert 4 * pr + 16 * Nt < by <= 12 * pr + 16 * Nt
    cached.profile(False)
    x = np.random.default_rng(9).standard_normal(cached.total)
    for prec, tol in ((yq.YQ_MIXED, 5e-6), (yq.YQ_FP64, 1e-12)):
        a = _np(cached.apply_operator(x, prec))
        b = _np(plain.apply_operator(x, prec))
        for c in range(len(cfgs)):
            s = slice(int(cached.offsets[c]), int(cached.offsets[c + 1]))
            assert _rel(a[s], b[s]) < tol, (prec, c)
    for bt in (plain, cached):
        bt.set_boundary_data(bt.boundary_label())
    sp, ip = plain.solve()
    sc, ic = cached.solve()
    assert all(i["residual"] <= 1e-10 for i in ic)
    assert _rel(_np(sc), _np(sp)) < 1e-8
    # graph replays equal eager iterations with the caches in use
    eager = _lane_batch(cfgs, False, near=-1, **prm)
    eager.set_boundary_data(eager.boundary_label())
    se, _ = eager.solve()
    assert np.array_equal(_np(se), _np(sc))
    # alone = in the mix, bitwise, for a cached tree
    alone = _lane_batch([cfgs[4]], True, near=-1, **prm)
    assert alone.near_cache_info()[1:] == (1, 1)
    alone.set_boundary_data(alone.boundary_label())
    sa, _ = alone.solve()
    assert np.array_equal(_np(sa), _np(sc)[int(cached.offsets[4]):int(cached.offsets[5])])
    # a budget one byte short of every cache: the last FP64 cache is left out
    short = _lane_batch(cfgs, True, near=held - 1, **prm)
    assert short.near_cache_info()[1:] == (2, 1)
    torch.cuda.synchronize()
