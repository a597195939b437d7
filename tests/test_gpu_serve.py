"""Continuous-batching server: every request's result matches the oracle and is
bitwise the same alone and in a mix; admission, cancellation and errors."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.geometry import Params

pytestmark = pytest.mark.gpu

yq = pytest.importorskip("paper_1810_04131_amd")

P, ORDER, TOL = 12, 8, 1e-9


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _requests():
    return [
        workloads.random_ellipses(4, 10.0, 0.8, seed=11),
        workloads.two_ellipses(5, 1.3),
        workloads.random_ellipses(2, 6.0, 2.0, seed=12),
        workloads.random_ellipses(6, 12.0, 0.6, seed=13),
        workloads.single_disk(1.0, 1.0),
    ]


def _server(**kw):
    _torch()
    prm = yq.default_params(panels_per_particle=P, qbx_order=ORDER, tol=TOL, precision=yq.YQ_MIXED)
    return yq.Server(prm, **kw)


def _alone(req):
    s = _server(node_capacity=20000, max_slots=2)
    t = s.submit(req)
    s.run_until_idle()
    return s.result(t)


@pytest.fixture(scope="module")
def mixed_run():
    s = _server(node_capacity=3 * 6 * P * 16, max_slots=3)   # room for ~3 requests at once
    reqs = _requests()
    tickets = [s.submit(r) for r in reqs[:3]]
    # later arrivals while the first ones are in flight
    for _ in range(3):
        s.step()
    tickets += [s.submit(r) for r in reqs[3:]]
    peak_running = 0
    for _ in range(100000):
        c, running, queued = s.step()
        peak_running = max(peak_running, running)
        if running == 0 and queued == 0:
            break
    return s, reqs, tickets, [s.result(t) for t in tickets], peak_running


def test_server_results_match_oracle(mixed_run):
    s, reqs, tickets, res, peak = mixed_run
    assert peak >= 2, "requests must overlap on the device"
    for req, r in zip(reqs, res):
        assert r["state"] == yq.Server.DONE
        assert r["info"]["residual"] <= TOL
        d = oracle.discretize(req, Params(panels=P, qbx_order=ORDER))
        A, Gx, Gy = oracle.build_matrices(d, gradient=True)
        f = oracle.arc_label(d)
        so = oracle.lu_solve(A, f)
        assert np.abs(r["sigma"] - so).max() / np.abs(so).max() < 1e-8
        Fo, To, _, Eo = oracle.forces_torques(d, f, oracle.surface_fields(Gx, Gy, so))
        sc = max(np.abs(Fo).max(), np.abs(To).max(), abs(Eo))
        assert np.abs(r["force"] - Fo).max() < 1e-7 * sc
        assert abs(r["energy"] - Eo) < 1e-7 * abs(Eo)
        assert r["latency"] > 0


def test_server_alone_equals_mix(mixed_run):
    s, reqs, tickets, res, _ = mixed_run
    for req, r in zip(reqs, res):
        a = _alone(req)
        assert np.array_equal(a["sigma"], r["sigma"])
        assert np.array_equal(a["force"], r["force"]) and a["energy"] == r["energy"]
        assert a["info"]["iterations"] == r["info"]["iterations"]


def test_server_admission_cancel_and_errors():
    torch = _torch()
    from paper_1810_04131_amd import _lib
    s = _server(node_capacity=4 * P * 16, max_slots=4)
    big = workloads.random_ellipses(5, 12.0, 1.0, seed=3)          # 5 particles > capacity of 4
    with pytest.raises(yq.YQError) as e:
        s.submit(big)
    assert e.value.status == _lib.YQ_EADMIT
    reqs = [workloads.random_ellipses(3, 9.0, 1.0, seed=20 + k) for k in range(3)]
    t = [s.submit(r) for r in reqs]
    s.step()
    # only one 3-particle request fits the 4-particle arena at a time
    states = [s.state(x)[0] for x in t]
    assert states.count(yq.Server.RUNNING) == 1 and states.count(yq.Server.QUEUED) == 2
    s.cancel(t[2])
    assert s.state(t[2])[0] == yq.Server.FAILED
    s.run_until_idle()
    assert s.state(t[0])[0] == yq.Server.DONE and s.state(t[1])[0] == yq.Server.DONE
    for x in t:
        s.release(x)
    with pytest.raises(yq.YQError):
        s.state(t[0])
    # memory budget admission: a budget below one request's estimate refuses it outright
    tiny = _server(node_capacity=100000, max_slots=4, mem_budget_bytes=1e6)
    with pytest.raises(yq.YQError) as e:
        tiny.submit(reqs[0])
    assert e.value.status == _lib.YQ_EADMIT


def _fmm_server(**kw):
    s = _server(**kw)
    s.set_fmm(900, workers=2)        # requests of >= 5 particles (960+ nodes) take the FMM lane
    return s


def test_server_fmm_lane_matches_oracle_and_alone():
    _torch()
    reqs = [
        workloads.random_ellipses(6, 12.0, 0.9, seed=31),     # FMM lane
        workloads.random_ellipses(2, 6.0, 1.4, seed=32),      # fused batch lane
        workloads.random_ellipses(7, 13.0, 1.2, seed=33),     # FMM lane
        workloads.random_ellipses(3, 9.0, 0.7, seed=34),      # fused batch lane
    ]
    s = _fmm_server(node_capacity=20000, max_slots=4)
    tickets = [s.submit(r) for r in reqs]
    peak = 0
    for _ in range(100000):
        c, running, queued = s.step()
        peak = max(peak, running)
        if running == 0 and queued == 0:
            break
    assert peak >= 3, "both lanes must run at once"
    for req, t in zip(reqs, tickets):
        r = s.result(t)
        assert r["state"] == yq.Server.DONE, r
        assert r["info"]["residual"] <= TOL
        d = oracle.discretize(req, Params(panels=P, qbx_order=ORDER))
        A, Gx, Gy = oracle.build_matrices(d, gradient=True)
        f = oracle.arc_label(d)
        so = oracle.lu_solve(A, f)
        assert np.abs(r["sigma"] - so).max() / np.abs(so).max() < 1e-8
        Fo, To, _, Eo = oracle.forces_torques(d, f, oracle.surface_fields(Gx, Gy, so))
        sc = max(np.abs(Fo).max(), np.abs(To).max(), abs(Eo))
        assert np.abs(r["force"] - Fo).max() < 1e-7 * sc
        assert abs(r["energy"] - Eo) < 1e-7 * abs(Eo)
        alone = _fmm_server(node_capacity=20000, max_slots=2)
        ta = alone.submit(req)
        alone.run_until_idle()
        a = alone.result(ta)
        assert np.array_equal(a["sigma"], r["sigma"])
        assert np.array_equal(a["force"], r["force"]) and a["energy"] == r["energy"]
        alone.close()
    with pytest.raises(yq.YQError):
        s.set_fmm(0)                 # only before the first submit
