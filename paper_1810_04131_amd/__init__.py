"""yqbx: MI355X-native Yukawa double-layer solver for many rigid ellipses.

Python binding of the C ABI in include/yqbx.h.  Every step of the solve runs
in the HIP library (libyqbx.so); this module only marshals arguments and uses
PyTorch for device memory and the current stream.  There is no CPU fallback:
the functions raise when the library is missing or no GPU is present.
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import _lib
from ._lib import (YQ_FAR_AUTO, YQ_FAR_CUTOFF, YQ_FAR_DIRECT, YQ_FAR_FMM, YQ_FMM64, YQ_FP64, YQ_LABEL_ARC,  # noqa: F401
                   YQ_LABEL_JANUS, YQ_M2L_MFMA, YQ_M2L_MFMA64, YQ_M2L_VALU, YQ_MIXED, YQError, yq_dynamics, yq_params,
                   yq_solve_info)

__all__ = ["Problem", "Batch", "Server", "default_params", "bessel", "YQError", "YQ_FP64", "YQ_MIXED"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("yqbx needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def default_params(**overrides) -> yq_params:
    lib = _lib.load()
    p = yq_params()
    lib.yq_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Problem:
    """One particle configuration on one GPU (a yq_problem handle)."""

    def __init__(self, params: Optional[yq_params] = None, device: str = "cuda:0", **overrides):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.lib = _lib.load()
        self.params = params if params is not None else default_params(**overrides)
        h = ctypes.c_void_p()
        _lib.check(self.lib.yq_create(ctypes.byref(self.params), ctypes.byref(h)))
        self.h = h
        self.stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.yq_set_stream(self.h, ctypes.c_void_p(self.stream.cuda_stream)))
        self.n = 0
        self.N = 0

    def _check(self, st):
        return _lib.check(st, self.h)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.yq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f64(self, *shape):
        return self.torch.empty(*shape, dtype=self.torch.float64, device=self.device)

    def _dev(self, t):
        t = self.torch.as_tensor(t, dtype=self.torch.float64, device=self.device)
        return t.contiguous()

    # -- set-up ---------------------------------------------------------------------------
    def set_particles(self, center, angle, axes, kappa):
        import numpy as np
        c = np.ascontiguousarray(np.asarray(center, dtype=np.float64).reshape(-1))
        a = np.ascontiguousarray(np.asarray(angle, dtype=np.float64).reshape(-1))
        x = np.ascontiguousarray(np.asarray(axes, dtype=np.float64).reshape(-1))
        n = a.size
        self._check(self.lib.yq_set_particles(self.h, n, c.ctypes.data_as(ctypes.c_void_p),
                                              a.ctypes.data_as(ctypes.c_void_p),
                                              x.ctypes.data_as(ctypes.c_void_p), float(kappa)))
        N = ctypes.c_int64()
        self._check(self.lib.yq_num_nodes(self.h, ctypes.byref(N)))
        self.n, self.N = n, int(N.value)
        return self

    def set_workload(self, particles):
        return self.set_particles(particles.center, particles.angle, particles.axes, particles.kappa)

    def nodes(self):
        out = [self._f64(self.N) for _ in range(5)]
        self._check(self.lib.yq_get_nodes(self.h, *[_ptr(t) for t in out]))
        return dict(zip(["x", "y", "nx", "ny", "w"], out))

    def near(self):
        tot = ctypes.c_int64()
        self._check(self.lib.yq_near_count(self.h, ctypes.byref(tot)))
        rp = self.torch.empty(self.N + 1, dtype=self.torch.int32, device=self.device)
        pn = self.torch.empty(max(int(tot.value), 1), dtype=self.torch.int32, device=self.device)
        self._check(self.lib.yq_get_near(self.h, _ptr(rp), _ptr(pn)))
        return rp, pn[: int(tot.value)]

    def boundary_label(self, kind=YQ_LABEL_ARC, a=0.7853981633974483, b=0.1):
        f = self._f64(self.N)
        self._check(self.lib.yq_boundary_label(self.h, kind, float(a), float(b), _ptr(f)))
        return f

    def set_boundary_data(self, f):
        f = self._dev(f)
        self._check(self.lib.yq_set_boundary_data(self.h, _ptr(f)))
        self._f = f
        return self

    # -- operator and solve ---------------------------------------------------------------
    def apply_far(self, sigma, precision=YQ_FP64, out=None):
        sigma = self._dev(sigma)
        out = self._f64(self.N) if out is None else out
        self._check(self.lib.yq_apply_far(self.h, _ptr(sigma), _ptr(out), precision))
        return out

    def apply_operator(self, sigma, precision=YQ_FP64, out=None):
        sigma = self._dev(sigma)
        out = self._f64(self.N) if out is None else out
        self._check(self.lib.yq_apply_operator(self.h, _ptr(sigma), _ptr(out), precision))
        return out

    def solve(self, sigma0=None, out=None, allow_noconv=False):
        s0 = self._dev(sigma0) if sigma0 is not None else None
        out = self._f64(self.N) if out is None else out
        info = yq_solve_info()
        st = self.lib.yq_solve(self.h, _ptr(s0), _ptr(out), ctypes.byref(info))
        if not (allow_noconv and st == _lib.YQ_ENOCONV):
            self._check(st)
        return out, {k: getattr(info, k) for k, _ in info._fields_}

    def surface_gradient(self, sigma):
        sigma = self._dev(sigma)
        gx, gy = self._f64(self.N), self._f64(self.N)
        self._check(self.lib.yq_surface_gradient(self.h, _ptr(sigma), _ptr(gx), _ptr(gy)))
        return gx, gy

    def forces(self, sigma, gamma=1.0):
        sigma = self._dev(sigma)
        F = self._f64(2 * self.n)
        T = self._f64(self.n)
        e = ctypes.c_double()
        self._check(self.lib.yq_forces(self.h, _ptr(sigma), float(gamma), _ptr(F), _ptr(T),
                                       ctypes.byref(e)))
        return F.view(self.n, 2), T, e.value

    def solve_forces(self, gamma=1.0, sigma0=None, out=None, allow_noconv=False):
        """solve() then forces() of its sigma in one call (yq_solve_forces)."""
        s0 = self._dev(sigma0) if sigma0 is not None else None
        out = self._f64(self.N) if out is None else out
        info = yq_solve_info()
        F = self._f64(2 * self.n)
        T = self._f64(self.n)
        e = ctypes.c_double()
        st = self.lib.yq_solve_forces(self.h, _ptr(s0), _ptr(out), ctypes.byref(info), float(gamma),
                                      _ptr(F), _ptr(T), ctypes.byref(e))
        if not (allow_noconv and st == _lib.YQ_ENOCONV):
            self._check(st)
        return out, {k: getattr(info, k) for k, _ in info._fields_}, F.view(self.n, 2), T, e.value

    # -- time stepping ----------------------------------------------------------------------
    def repulsion(self, c0, q=3):
        """Excluded-volume repulsion of the current particles (yq_repulsion): F (n, 2), tau, Phi_rep."""
        F = self._f64(2 * self.n)
        T = self._f64(self.n)
        e = ctypes.c_double()
        self._check(self.lib.yq_repulsion(self.h, float(c0), int(q), _ptr(F), _ptr(T),
                                          ctypes.byref(e)))
        return F.view(self.n, 2), T, e.value

    def step(self, sigma, dt, xi_x, xi_theta, c0, q=3, gamma=1.0, sigma_prev=None,
             allow_noconv=False):
        """One constant-drag time step (yq_step).

        sigma: device density of length N, the initial guess on entry (the previous
        step's density) and the density at the start configuration on return
        (updated in place).  sigma_prev: optional density of the step before; the
        guess is then 2 sigma - sigma_prev and sigma_prev takes sigma's old value.
        Returns (info, F_total (n, 2), tau_total, (Phi, Phi_rep)).
        """
        for t in (sigma, sigma_prev):
            if t is not None and not (t.is_contiguous() and t.dtype == self.torch.float64
                                      and t.device == self.device and t.numel() == self.N):
                raise ValueError("sigma and sigma_prev must be contiguous float64 device "
                                 "tensors of length N")
        dyn = yq_dynamics(float(dt), float(xi_x), float(xi_theta), float(gamma), float(c0), int(q))
        info = yq_solve_info()
        F = self._f64(2 * self.n)
        T = self._f64(self.n)
        e = (ctypes.c_double * 2)()
        st = self.lib.yq_step(self.h, ctypes.byref(dyn), _ptr(sigma), _ptr(sigma_prev),
                              ctypes.byref(info), _ptr(F),
                              _ptr(T), ctypes.cast(e, ctypes.c_void_p))
        if not (allow_noconv and st == _lib.YQ_ENOCONV):
            self._check(st)
        return {k: getattr(info, k) for k, _ in info._fields_}, F.view(self.n, 2), T, (e[0], e[1])

    def particles(self):
        """Current centres (n, 2) and angles (n,) as numpy arrays (yq_get_particles)."""
        import numpy as np
        c = np.empty(2 * self.n)
        a = np.empty(self.n)
        self._check(self.lib.yq_get_particles(self.h, c.ctypes.data_as(ctypes.c_void_p),
                                              a.ctypes.data_as(ctypes.c_void_p)))
        return c.reshape(self.n, 2), a

    def fmm_stats(self):
        """The FMM quadtree: depth, leaves, largest leaf, P2P pairs and M2L box pairs per pass."""
        d, nl, ml = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        pp, mp = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.yq_fmm_stats(self.h, ctypes.byref(d), ctypes.byref(nl), ctypes.byref(ml),
                                          ctypes.byref(pp), ctypes.byref(mp)))
        return dict(depth=d.value, leaves=nl.value, max_leaf=ml.value, p2p_pairs=pp.value,
                    m2l_pairs=mp.value)

    def eval_potential(self, sigma, targets):
        sigma = self._dev(sigma)
        t = self._dev(targets).reshape(-1, 2)
        tx, ty = t[:, 0].contiguous(), t[:, 1].contiguous()
        u = self._f64(t.shape[0])
        self._check(self.lib.yq_eval_potential(self.h, _ptr(sigma), t.shape[0], _ptr(tx), _ptr(ty),
                                               _ptr(u)))
        return u


class Batch:
    """Many independent configurations solved together (a yq_batch handle).

    Batch vectors concatenate the configurations' nodes (offsets[c]..offsets[c+1]).
    Batch calls are synchronous; the binding synchronises torch's stream first so
    that inputs written by torch are complete.
    """

    def __init__(self, params: Optional[yq_params] = None, device: str = "cuda:0", **overrides):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.lib = _lib.load()
        self.params = params if params is not None else default_params(**overrides)
        h = ctypes.c_void_p()
        _lib.check(self.lib.yq_batch_create(ctypes.byref(self.params), ctypes.byref(h)), None, True)
        self.h = h
        self.offsets = None
        self.total = 0
        self.nparticles = None

    def _check(self, st):
        return _lib.check(st, self.h, True)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.yq_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync(self):
        self.torch.cuda.synchronize(self.device)

    def set_fmm(self, min_nodes, workers=6, in_engine=True):
        """Configurations of at least min_nodes nodes take the FMM (before set_configs):
        as trees of the engine's forest (in_engine), else solved by worker threads."""
        self._check(self.lib.yq_batch_set_fmm(self.h, int(min_nodes), int(workers)))
        self._check(self.lib.yq_batch_set_fmm_engine(self.h, int(bool(in_engine))))
        return self

    def set_near_cache(self, max_bytes=-1):
        """Device memory for the FMM trees' near-field caches (before set_configs):
        -1 the free memory less a reserve (default), 0 none."""
        self._check(self.lib.yq_batch_set_near_cache(self.h, int(max_bytes)))
        return self

    def near_cache_info(self):
        """(bytes held, trees with an FP32 cache, trees with an FP64 cache)."""
        b, t32, t64 = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.yq_batch_near_cache_info(self.h, ctypes.byref(b), ctypes.byref(t32),
                                                      ctypes.byref(t64)))
        return int(b.value), int(t32.value), int(t64.value)

    def set_symmetric_far(self, enable=True):
        """Inner far field: one evaluation per unordered pair (default) or per directed
        pair (before set_configs)."""
        self._check(self.lib.yq_batch_set_symmetric_far(self.h, int(bool(enable))))
        return self

    def _f64(self, *shape):
        return self.torch.empty(*shape, dtype=self.torch.float64, device=self.device)

    def _dev(self, t):
        return self.torch.as_tensor(t, dtype=self.torch.float64, device=self.device).contiguous()

    def set_configs(self, configs):
        """configs: a list of workloads.Particles-like objects (center, angle, axes, kappa)."""
        import numpy as np
        npart = np.ascontiguousarray([c.center.shape[0] for c in configs], dtype=np.int32)
        cen = np.ascontiguousarray(np.concatenate([np.asarray(c.center, float).reshape(-1) for c in configs]))
        ang = np.ascontiguousarray(np.concatenate([np.asarray(c.angle, float).reshape(-1) for c in configs]))
        ax = np.ascontiguousarray(np.concatenate([np.asarray(c.axes, float).reshape(-1) for c in configs]))
        kap = np.ascontiguousarray([float(c.kappa) for c in configs], dtype=np.float64)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(self.lib.yq_batch_set_configs(self.h, len(configs), vp(npart), vp(cen), vp(ang),
                                                  vp(ax), vp(kap)))
        tot = ctypes.c_int64()
        offs = np.zeros(len(configs) + 1, dtype=np.int64)
        self._check(self.lib.yq_batch_num_nodes(self.h, ctypes.byref(tot), vp(offs)))
        self.total = int(tot.value)
        self.offsets = offs
        self.nparticles = npart
        return self

    def boundary_label(self, kind=YQ_LABEL_ARC, a=0.7853981633974483, b=0.1):
        f = self._f64(self.total)
        self._sync()
        self._check(self.lib.yq_batch_boundary_label(self.h, kind, float(a), float(b), _ptr(f)))
        return f

    def set_boundary_data(self, f):
        f = self._dev(f)
        self._sync()
        self._check(self.lib.yq_batch_set_boundary_data(self.h, _ptr(f)))
        return self

    def apply_operator(self, sigma, precision=YQ_FP64):
        sigma = self._dev(sigma)
        out = self._f64(self.total)
        self._sync()
        self._check(self.lib.yq_batch_apply_operator(self.h, _ptr(sigma), _ptr(out), precision))
        return out

    def solve(self, allow_noconv=False):
        out = self._f64(self.total)
        n = len(self.offsets) - 1
        infos = (yq_solve_info * n)()
        self._sync()
        st = self.lib.yq_batch_solve(self.h, _ptr(out), infos)
        if not (allow_noconv and st == _lib.YQ_ENOCONV):
            self._check(st)
        return out, [{k: getattr(x, k) for k, _ in x._fields_} for x in infos]

    def solve_forces(self, gamma=1.0, allow_noconv=False):
        """solve() then forces() of its sigma in one call (yq_batch_solve_forces)."""
        import numpy as np
        out = self._f64(self.total)
        n = len(self.offsets) - 1
        infos = (yq_solve_info * n)()
        npt = int(self.nparticles.sum())
        F = self._f64(2 * npt)
        T = self._f64(npt)
        E = np.zeros(n)
        self._sync()
        st = self.lib.yq_batch_solve_forces(self.h, _ptr(out), infos, float(gamma), _ptr(F), _ptr(T),
                                            E.ctypes.data_as(ctypes.c_void_p))
        if not (allow_noconv and st == _lib.YQ_ENOCONV):
            self._check(st)
        return (out, [{k: getattr(x, k) for k, _ in x._fields_} for x in infos], F.view(npt, 2), T,
                E)

    def forces(self, sigma, gamma=1.0):
        import numpy as np
        sigma = self._dev(sigma)
        npt = int(self.nparticles.sum())
        F = self._f64(2 * npt)
        T = self._f64(npt)
        E = np.zeros(len(self.offsets) - 1)
        self._sync()
        self._check(self.lib.yq_batch_forces(self.h, _ptr(sigma), float(gamma), _ptr(F), _ptr(T),
                                             E.ctypes.data_as(ctypes.c_void_p)))
        return F.view(npt, 2), T, E

    def autotune(self):
        pb, fw = ctypes.c_int32(), ctypes.c_int32()
        self._sync()
        self._check(self.lib.yq_batch_autotune(self.h, ctypes.byref(pb), ctypes.byref(fw)))
        return int(pb.value), int(fw.value)

    def use_graphs(self, enable=True):
        self._check(self.lib.yq_batch_use_graphs(self.h, int(bool(enable))))

    def profile(self, enable=True):
        """Timers of the fused far-field launches (see yq_batch_profile_enable)."""
        self._check(self.lib.yq_batch_profile_enable(self.h, int(bool(enable))))

    def profile_read(self, precision=YQ_MIXED, reset=True, kernel="direct"):
        """(launches, total ms, source-target pairs) of the timed far-field launches:
        kernel "direct" (the direct members' fused far field) or "leaf" (the FMM
        forest's leaf pass; then also the algorithmic bytes of its cached trees)."""
        n, ms, pairs, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        if kernel == "leaf":
            self._check(self.lib.yq_batch_profile_read_leaf(
                self.h, int(precision), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(pairs),
                ctypes.byref(by), int(bool(reset))))
            return int(n.value), float(ms.value), float(pairs.value), float(by.value)
        if kernel != "direct":
            raise KeyError(kernel)
        self._check(self.lib.yq_batch_profile_read(self.h, int(precision), ctypes.byref(n),
                                                   ctypes.byref(ms), ctypes.byref(pairs),
                                                   int(bool(reset))))
        return int(n.value), float(ms.value), float(pairs.value)

    def segment(self, v, c):
        return v[int(self.offsets[c]):int(self.offsets[c + 1])]


class Server:
    """Continuous-batching solve server (a yq_server handle); see include/yqbx.h."""

    QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3

    def __init__(self, params: Optional[yq_params] = None, node_capacity=1 << 20, max_slots=64,
                 mem_budget_bytes=64e9, device: str = "cuda:0", **overrides):
        torch = _torch()
        torch.cuda.set_device(torch.device(device))
        self.lib = _lib.load()
        self.params = params if params is not None else default_params(**overrides)
        h = ctypes.c_void_p()
        _lib.check(self.lib.yq_server_create(ctypes.byref(self.params), int(node_capacity),
                                             int(max_slots), float(mem_budget_bytes),
                                             ctypes.byref(h)), None, server=True)
        self.h = h
        self.sizes = {}

    def _check(self, st):
        return _lib.check(st, self.h, server=True)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.yq_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fmm(self, min_nodes, workers=2):
        """Requests of at least min_nodes nodes take the FMM lane (before the first submit)."""
        self._check(self.lib.yq_server_set_fmm(self.h, int(min_nodes), int(workers)))
        return self

    def submit(self, particles, label_kind=YQ_LABEL_ARC, a=0.7853981633974483, b=0.1):
        import numpy as np
        c = np.ascontiguousarray(np.asarray(particles.center, float).reshape(-1))
        an = np.ascontiguousarray(np.asarray(particles.angle, float).reshape(-1))
        ax = np.ascontiguousarray(np.asarray(particles.axes, float).reshape(-1))
        t = ctypes.c_int64()
        vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
        self._check(self.lib.yq_server_submit(self.h, an.size, vp(c), vp(an), vp(ax),
                                              float(particles.kappa), label_kind, float(a),
                                              float(b), ctypes.byref(t)))
        return int(t.value)

    def step(self):
        c, r, q = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.yq_server_step(self.h, ctypes.byref(c), ctypes.byref(r), ctypes.byref(q)))
        return int(c.value), int(r.value), int(q.value)

    def state(self, ticket):
        st, N, n = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        self._check(self.lib.yq_server_result(self.h, ticket, ctypes.byref(st), ctypes.byref(N),
                                              ctypes.byref(n), None, None, None, None, None, None))
        return int(st.value), int(N.value), int(n.value)

    def result(self, ticket):
        import numpy as np
        st, N, n = self.state(ticket)
        if st not in (self.DONE, self.FAILED):
            return None
        sig = np.zeros(N)
        F = np.zeros(2 * n)
        T = np.zeros(n)
        e = ctypes.c_double()
        info = yq_solve_info()
        lat = ctypes.c_double()
        stc, Nc, nc = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
        self._check(self.lib.yq_server_result(self.h, ticket, ctypes.byref(stc), ctypes.byref(Nc),
                                              ctypes.byref(nc), vp(sig), vp(F), vp(T),
                                              ctypes.byref(e), ctypes.byref(info), ctypes.byref(lat)))
        return dict(state=st, sigma=sig, force=F.reshape(n, 2), torque=T, energy=e.value,
                    info={k: getattr(info, k) for k, _ in info._fields_}, latency=lat.value)

    def release(self, ticket):
        self._check(self.lib.yq_server_release(self.h, ticket))

    def cancel(self, ticket):
        self._check(self.lib.yq_server_cancel(self.h, ticket))

    def run_until_idle(self, max_ticks=100000):
        for _ in range(max_ticks):
            c, r, q = self.step()
            if r == 0 and q == 0:
                return
        raise RuntimeError("server did not drain")


def bessel(kind, order, z, precision=YQ_FP64):
    """Device special functions: kind 0 K0, 1 K1, 2 K_order, 3 I_order."""
    torch = _torch()
    lib = _lib.load()
    z = torch.as_tensor(z, dtype=torch.float64, device="cuda").contiguous()
    out = torch.empty_like(z)
    torch.cuda.synchronize()
    _lib.check(lib.yq_bessel(kind, order, precision, z.numel(), _ptr(z), _ptr(out)))
    return out
