"""Benchmark of the full hot path on one MI355X.

One step = one complete solve of the 50-ellipse workload (N = 25,600 nodes,
kappa = 1, 32 panels x 16 nodes, QBX order 10): geometry + near lists + QBX
correction build, boundary label, mixed-precision GMRES (FP32 far field, FP64
Arnoldi and FP64 iterative refinement) to a relative residual of 1e-8, surface
gradient, forces/torques/energy, and the off-surface potential on a 32 x 32
grid.  Inputs are synthetic (seeded layouts, see workloads/).

Printed JSON line: value = dense-equivalent source-target interactions per
second over the whole step (N^2 per far-field pass, summed over every far-field
pass of the step, divided by the step's wall time); extra fields give the
per-matvec rate, solves/s and p50/p99 solve latency, the FP64-only path, the
roofline of the dominant kernel (FP32 far field, timed with hipEvents on the
problem's stream) and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic flops per source-target pair of the far-field kernels, counted
# from the source: an FMA counts 2, every other floating-point arithmetic
# operation (add, mul, rsq, exp2, log2, rcp, rint, ldexp) counts 1.  A pair's
# evaluation depends on the class of its (64-node target group, 256-node source
# tile) pair, kappa x (gap between their bounding circles):
#   FP32  >= 8: 2 differences, z^2 (3), rsq (1), Z (1), exp2 (1), rsq (1),
#               degree-3 Horner (6), 3 products (3), D.q' (3), accumulate (2) = 23
#         >= 4: the same with the degree-4 Horner (8)                          = 25
#         >= 2: the same with the degree-6 Horner (12)                         = 29
#         general (may be < 2): FP64 differences (2), z^2 (3), kappa^2 z^2 (1),
#               large branch rsq, z, exp2 argument + exp2, rsq, degree-6 Horner,
#               3 products (20), (x-y).q (3), accumulate (2); counted at the
#               cheaper branch                                                  = 31
#   FP64  >= 8: differences (2), r^2 (3), kappa^2 r^2 (1), two Newton-refined
#               rsqrt (2 x 12), z (1), s (1), degree-11 Horner (22), e^-z by
#               Cody-Waite + degree-13 Taylor (33), 3 products (3), (x-y).q (3),
#               product (1), accumulate (1)                                     = 95
#         >= 4: degree-15 Horner (30)                                          = 103
#         >= 2 and general: degree-20 Horner (40)                              = 113
F32_CLASS = {"z8": 23, "z4": 25, "z2": 29, "general": 31}
F64_CLASS = {"z8": 95, "z4": 103, "z2": 113, "general": 113}
# VALU instructions per pair in the pair loops of far32_kernel / far64_kernel,
# counted in their gfx950 assembly (hipcc -S of farfield.hip; the general path
# executes both branches of K1(z)/z), and the chip's VALU issue rate: 256 CUs x
# 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second (FP32 and FP64 alike).
F32_VALU = {"z8": 16, "z4": 17, "z2": 19, "general": 43}
F64_VALU = {"z8": 65, "z4": 69, "z2": 73, "general": 194}
VALU_ISSUE = 256 * 4 * 16 * 2.4e9


def far_class_mix(x, y, kappa, panels=False):
    """Fraction of the N^2 far-field pairs in each kernel class, from the same
    bounding circles as the kernels (bounding-box centre, largest distance):
    per (64-target group, 256-source tile), and with panels=True (the FP32
    and FP64 far-field kernels) per (group, 16-source panel) inside the tiles with close pairs."""
    import numpy as np
    n = len(x)

    def circles(g):
        out = []
        for a in range(0, n, g):
            px, py = x[a:a + g], y[a:a + g]
            cx, cy = 0.5 * (px.min() + px.max()), 0.5 * (py.min() + py.max())
            out.append((cx, cy, np.sqrt(((px - cx) ** 2 + (py - cy) ** 2).max()), len(px)))
        return np.array(out)

    def gap(a, b):
        return kappa * (np.hypot(a[:, None, 0] - b[None, :, 0], a[:, None, 1] - b[None, :, 1])
                        - a[:, None, 2] - b[None, :, 2])

    def split(z, w):
        masks = {"z8": z >= 8, "z4": (z >= 4) & (z < 8), "z2": (z >= 2) & (z < 4),
                 "general": z < 2}
        return {c: float(w[m].sum()) for c, m in masks.items()}

    t, g = circles(256), circles(64)
    zt = gap(g, t)
    wt = g[:, None, 3] * t[None, :, 3]
    tot = wt.sum()
    if not panels:
        return {c: v / tot for c, v in split(zt, wt).items()}
    far = np.where(zt >= 2, zt, -1.0)
    out = split(far, np.where(zt >= 2, wt, 0.0))
    p = circles(16)
    zp = gap(g, p)
    wp = g[:, None, 3] * p[None, :, 3]
    close = np.repeat(zt < 2, 16, axis=1)[:, :p.shape[0]]   # panels of the close tiles
    for c, v in split(zp, np.where(close, wp, 0.0)).items():
        out[c] += v
    return {c: v / tot for c, v in out.items()}


def flops_per_pair(mix, table):
    return sum(mix[c] * table[c] for c in table)


SRC_FOR_COUNTERS = ["paper_1810_04131_amd/csrc/farfield.hip",
                    "paper_1810_04131_amd/csrc/farfield_core.h", "paper_1810_04131_amd/csrc/bessel.h",
                    "paper_1810_04131_amd/csrc/bessel_tables.h"]
PH_FAR64, PH_FAR32 = 0, 1   # profiling phases of the library (yq_profile_enable)
PH_QBX, PH_FUSED, PH_REPULSION = 4, 6, 7
COUNTERS_FILE = "profiles/far32_kernel_50ellipses_N25600_counters.txt"
PEAK_FP32 = 157.3e12   # published MI355X FP32 vector peak (needs packed FP32)
PEAK_HBM = 8.0e12      # published MI355X HBM3E bandwidth (bytes/s)
PEAK_FP64 = 78.6e12    # published MI355X FP64 vector peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kappa", type=float, default=1.0)
    ap.add_argument("--tol", type=float, default=1e-9,
                    help="batch: relative residual tolerance of the mixed solves")
    ap.add_argument("--error-configs", type=int, default=16,
                    help="batch: configurations re-solved in FP64 to 1e-12 for the per-result errors")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1536)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--workload", choices=["medium", "batch", "serve", "large", "table2",
                                           "dynamics", "cutoff"],
                    default="batch",
                    help="batch: 1,024 configurations of 10-200 ellipses per batched solve "
                         "(default line); medium: the 50-ellipse solve; serve: Poisson-arrival "
                         "continuous batching")
    ap.add_argument("--configs", type=int, default=1024, help="batch: number of configurations")
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrival rate (1/s)")
    ap.add_argument("--nmax", type=int, default=None,
                    help="batch/serve: largest particle count (default 200 batch, 2000 serve)")
    ap.add_argument("--fmm-workers", type=int, default=6,
                    help="serve/batch: FMM-lane worker threads")
    ap.add_argument("--batch-lane", choices=["hybrid", "lane", "fused", "engine"], default="hybrid",
                    help="batch: hybrid = configurations from --fmm-min-nodes on take the FMM as "
                         "trees of the engine's forest (one captured iteration for the whole "
                         "batch); lane = they are standalone FMM problems solved by worker "
                         "threads beside the engine; fused = every configuration in the fused "
                         "direct engine; engine = only the configurations below "
                         "--fmm-min-nodes (the direct members of the hybrid run)")
    ap.add_argument("--far32", choices=["symmetric", "directed"], default="symmetric",
                    help="batch: inner far field of the direct members with one kernel "
                         "evaluation per unordered pair (bsym32_kernel) or per directed pair "
                         "(bfar32_kernel)")
    ap.add_argument("--fmm-order", type=int, default=15,
                    help="batch: inner FMM expansion order (default 15: with the FP64 "
                         "residuals the mixed solves take the same iterations and refinement "
                         "steps as at the library's 20, and 2 (p + 1) = 32 fills the MFMA "
                         "operand tiles without padding; 0: the library's)")
    ap.add_argument("--fmm-resid-order", type=int, default=31,
                    help="batch: order of the FP64 FMM of the refinement residuals and forces "
                         "(default 31: its operator differs from the library's order 40 by "
                         "1e-13 relative, far below the 1e-9 tolerance, and 2 (p + 1) = 64 "
                         "fills the MFMA operand tiles; 0: the library's)")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="batch: relative tolerance of each FP32-operator inner solve (default 0: "
                         "the library's, 1e-6)")
    ap.add_argument("--fmm-leaf", type=int, default=0,
                    help="batch: most nodes per FMM leaf (default 0: the library's, 64)")
    ap.add_argument("--near-cache-gb", type=float, default=None,
                    help="batch: device memory for the FMM trees' near-field caches (GB; 0 "
                         "none; default: the library's, the free memory less a reserve)")
    ap.add_argument("--fmm-min-nodes", type=int, default=None,
                    help="batch: configurations of at least this many nodes take the FMM "
                         "(default 0 for hybrid: every configuration is a tree of the forest, "
                         "measured fastest at every size of the workload; 20000 for lane and "
                         "engine); serve: requests of at least this many nodes take the FMM "
                         "lane (default 20000)")
    ap.add_argument("--fp64-requests", type=int, default=None,
                    help="serve: requests of the trace (from the start) replayed on the FP64 "
                         "one-at-a-time path (default all)")
    ap.add_argument("--single-baseline", type=int, default=128,
                    help="batch: configurations (every k-th) also solved one at a time on the "
                         "FP64 path for comparison")
    return ap.parse_args()


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SRC_FOR_COUNTERS:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def counters(key):
    """A per-launch figure from the committed counter summary, or None when the
    far-field source has changed since the counters were taken."""
    path = os.path.join(ROOT, COUNTERS_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != source_hash():
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


# the single-problem path's own crossover from the direct far field to the FMM (the
# library's automatic choice): the one-at-a-time baselines use it
SINGLE_FMM_NODES = 20000

BATCH_COUNTERS_FILE = {"symmetric": "profiles/bsym32_kernel_batch_engine_counters.txt",
                       "directed": "profiles/bfar32_kernel_batch_engine_counters.txt"}
BATCH_SRC = ["paper_1810_04131_amd/csrc/batch.hip", "paper_1810_04131_amd/csrc/farfield_core.h",
             "paper_1810_04131_amd/csrc/bessel.h", "paper_1810_04131_amd/csrc/bessel_tables.h"]


def batch_counters(kind):
    """Per-pair HBM bytes and VALU figures of the batch engine's FP32 far-field kernel
    (kind: symmetric or directed) from the committed counter summary, or {} when the
    kernel's source has changed since the counters were taken."""
    return _kv_counters(BATCH_COUNTERS_FILE[kind], BATCH_SRC)


LEAF_COUNTERS_FILE = "profiles/forest_cleaf_kernel_batch_counters.txt"
LEAF_SRC = ["paper_1810_04131_amd/csrc/fmm.hip", "paper_1810_04131_amd/csrc/farfield_core.h",
            "paper_1810_04131_amd/csrc/bessel.h", "paper_1810_04131_amd/csrc/bessel_tables.h"]


def leaf_counters():
    """Per-pair HBM bytes and VALU figures of the forest's FP32 leaf pass from the
    committed counter summary, or {} when its source has changed since."""
    return _kv_counters(LEAF_COUNTERS_FILE, LEAF_SRC)


def _kv_counters(path, srcs):
    import hashlib
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return {}
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != h.hexdigest()[:16]:
        return {}
    out = {}
    for k, v in kv.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def traffic_from_counters(launch_pairs):
    """HBM bytes per far32 launch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return counters("hbm_bytes_per_launch")


def copy_probe():
    import torch
    n = 64 * 1024 * 1024   # 256 MiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n,
                      "dispatches": 3}))


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def prof(pb, phase, reset=True):
    import ctypes
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    pb._check(pb.lib.yq_profile_read(pb.h, phase, ctypes.byref(n), ctypes.byref(ms), int(reset)))
    return int(n.value), float(ms.value)


def run_step(pb, parts, grid):
    pb.set_workload(parts)
    f = pb.boundary_label()
    pb.set_boundary_data(f)
    sigma, info, F, T, E = pb.solve_forces()
    u = pb.eval_potential(sigma, grid)
    return info, u


def cpu_baseline(cfg, rows):
    """The oracle's operator rows (plain q-point far sum + QBX rows), timed on the host."""
    import numpy as np

    import oracle
    from oracle.geometry import Params
    parts = cfg["particles"]
    d = oracle.discretize(parts, Params(panels=cfg["panels"], qbx_order=cfg["qbx_order"]))
    from threadpoolctl import threadpool_limits
    sig = np.random.default_rng(0).standard_normal(d.N)
    sel = np.linspace(0, d.N - 1, rows).astype(int).tolist()
    with threadpool_limits(limits=1):    # one core, so "cores" below is exact
        oracle.apply_rows(d, sel[:2], sig)   # warm-up
        t0 = time.perf_counter()
        oracle.apply_rows(d, sel, sig)
        dt = time.perf_counter() - t0
    return dict(value=rows * d.N / dt, unit="interactions/s", cores=1, kind="oracle",
                sample=f"{rows} of {d.N} operator rows of the same workload "
                       f"(each row: {d.N} far-field pairs + QBX window), single-threaded "
                       f"numpy/scipy, {dt:.1f} s")


def _batch_layout(item):
    import workloads
    return workloads.batched_layout(item)


def batch_layouts(plan):
    """Layouts of the batched workload's configurations, drawn in parallel host processes."""
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_batch_layout, plan, chunksize=8))


def _cpu_rows_job(job):
    """One worker's share of the CPU baseline: the oracle's operator rows of one
    configuration, timed on one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    import workloads
    from oracle.geometry import Params
    import warnings
    warnings.simplefilter("ignore", RuntimeWarning)   # the self pair's 0/0, masked out
    cfg, rows, seed = job
    d = oracle.discretize(cfg, Params(panels=32, qbx_order=10))
    sig = workloads.random_density(d.N, seed)
    rows = [r % d.N for r in rows]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.apply_rows(d, rows, sig)
        dt = time.perf_counter() - t0
    return len(rows) * d.N, dt


def cpu_baseline_batch(cfgs, matvecs_per_solve, n_configs=32, rows_per_config=96):
    """The oracle's operator rows (plain far sum + QBX rows) on rows drawn from
    n_configs of the batched workload's configurations, in one process per host
    core (16 at most); scaled to solves/s by the mean source-target pairs of one
    solve of the GPU run (its matvecs per solve times N^2 per configuration)."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    pick = np.linspace(0, len(cfgs) - 1, n_configs).astype(int)
    jobs = []
    for k, c in enumerate(pick):
        rows = np.random.default_rng(100 + k).integers(0, 1 << 30, rows_per_config).tolist()
        jobs.append((cfgs[c], rows, 200 + k))
    with ProcessPoolExecutor(workers) as ex:
        list(ex.map(_cpu_rows_job, [(cfgs[0], [0], 1)] * workers))    # warm-up (imports)
        t0 = time.perf_counter()
        res = list(ex.map(_cpu_rows_job, jobs))
        wall = time.perf_counter() - t0
    inter = sum(r[0] for r in res)
    rate = inter / wall
    N = np.array([c.n * 512 for c in cfgs], dtype=float)
    pairs_per_solve = float(np.mean(matvecs_per_solve * N * N))
    return dict(value=rate / pairs_per_solve, unit="solves/s (estimate)", cores=workers,
                kind="oracle", interactions_per_s=rate,
                sample=f"{len(jobs) * rows_per_config} operator rows (each: N far-field pairs + "
                       f"QBX window) from {len(jobs)} of the {len(cfgs)} configurations, one "
                       f"single-threaded oracle process per core, {wall:.1f} s; solves/s = "
                       f"interactions/s / {pairs_per_solve:.3e} pairs per solve (the GPU run's "
                       f"mean matvecs per solve x N^2)")


def errors_vs_oracle_c2(yq, tol):
    """Per-result errors of the 50-ellipse workload's mixed solve (kappa 1) against
    the oracle's stored dense-LU results (tests/golden/c2_kappa1.npz): density,
    potential, force and torque, each max |x - x*| / max |x*| (reading R15)."""
    import numpy as np
    import workloads
    path = os.path.join(ROOT, "tests", "golden", "c2_kappa1.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    cfg = workloads.config_medium(kappa=1.0, seed=0)
    pb = yq.Problem(yq.default_params(panels_per_particle=32, qbx_order=10, tol=tol,
                                      precision=yq.YQ_MIXED, maxiter=300))
    pb.set_workload(cfg["particles"])
    pb.set_boundary_data(pb.boundary_label())
    sig, info, F, T, E = pb.solve_forces()
    u = pb.eval_potential(sig, g["targets"])
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    return {"workload": "50 ellipses N=25600 kappa=1, mixed, tol %g" % tol,
            "density": rel(sig.cpu().numpy(), g["sigma"]),
            "potential": rel(u.cpu().numpy(), g["potential"]),
            "force": rel(F.cpu().numpy().reshape(-1, 2), g["force"]),
            "torque": rel(T.cpu().numpy(), g["torque"]),
            "energy": abs(E - float(g["energy"])) / abs(float(g["energy"]))}


def bench_batch(args):
    """The batched workload: many configurations of log-uniform 10..nmax ellipses.

    One step = one batched mixed-precision solve of every configuration plus the
    forces and torques of every particle.  Configurations below the FMM-lane
    threshold run in the fused engine (one persistent far-field launch per GMRES
    iteration for all of them, the iteration replayed from captured hipGraphs);
    larger ones are solved by lane workers with the FMM far field beside it.
    Set-up (geometry, near lists, QBX correction, trees) is done once before the
    timed region."""
    import numpy as np
    import torch

    import paper_1810_04131_amd as yq
    import workloads
    nmax = args.nmax or 200
    log = lambda msg: print(f"# {msg}", file=sys.stderr, flush=True)
    plan = workloads.batched_plan(args.configs, seed=0, nmax=nmax)
    t0 = time.perf_counter()
    cfgs = batch_layouts(plan)
    log(f"{len(cfgs)} configurations drawn in {time.perf_counter() - t0:.1f} s")
    engine_only = args.batch_lane == "engine"
    forest = args.batch_lane == "hybrid"
    min_nodes = args.fmm_min_nodes
    if min_nodes is None:
        min_nodes = 0 if forest else SINGLE_FMM_NODES
    if engine_only:
        cfgs = [c for c in cfgs if c.n * 512 < min_nodes]
    hybrid = args.batch_lane in ("hybrid", "lane")
    thr = min_nodes if hybrid else None
    tol = args.tol
    prm = yq.default_params(panels_per_particle=32, qbx_order=10, tol=tol,
                            precision=yq.YQ_MIXED, restart=60, maxiter=300)
    if args.fmm_order:
        prm.fmm_order = args.fmm_order
    if args.fmm_resid_order:
        prm.fmm_resid_order = args.fmm_resid_order
    if args.fmm_leaf:
        prm.fmm_leaf_max = args.fmm_leaf
    if args.inner_tol:
        prm.inner_tol = args.inner_tol
    inner_order = prm.fmm_order
    resid_order = prm.fmm_resid_order
    b = yq.Batch(prm)
    b.set_symmetric_far(args.far32 == "symmetric")
    if args.near_cache_gb is not None:
        b.set_near_cache(int(args.near_cache_gb * 1e9))
    if hybrid:
        b.set_fmm(thr, workers=args.fmm_workers, in_engine=forest)
    t0 = time.perf_counter()
    b.set_configs(cfgs)
    t_setup = time.perf_counter() - t0
    N = np.diff(b.offsets).astype(float)
    lane = N >= thr if hybrid else np.zeros(len(cfgs), dtype=bool)
    log(f"set-up {t_setup:.1f} s, {b.total} nodes, {int(lane.sum())} configurations take the FMM")
    near = b.near_cache_info()
    log(f"near-field caches: {near[0] / 1e9:.1f} GB, {near[1]} FP32 / {near[2]} FP64 trees")
    pblk, fwant = b.autotune()
    log(f"autotuned: persistent blocks {pblk}, far_want {fwant}")
    b.set_boundary_data(b.boundary_label())
    b.profile(True)      # events around every fused far-field launch (split iteration graphs)

    def step():
        return b.solve_forces()

    for k in range(max(args.warmup, 1)):
        step()
        log(f"warm-up step {k + 1} done")
    for prec in (yq.YQ_MIXED, yq.YQ_FP64):
        for kern in ("direct", "leaf"):
            b.profile_read(prec, reset=True, kernel=kern)
    lat = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        sig, infos, F, T, E = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        log(f"timed step {k + 1}: {lat[-1]:.2f} s")
    t_all = time.perf_counter() - t_all
    n32, ms32, pairs32 = b.profile_read(yq.YQ_MIXED)
    n64, ms64, pairs64 = b.profile_read(yq.YQ_FP64)
    nl32, msl32, pairsl32, bytesl32 = b.profile_read(yq.YQ_MIXED, kernel="leaf")
    nl64, msl64, pairsl64, bytesl64 = b.profile_read(yq.YQ_FP64, kernel="leaf")
    its = np.array([i["iterations"] for i in infos])
    ref = np.array([i["outer_steps"] for i in infos])
    mv = np.array([i["matvecs_fp32"] + i["matvecs_fp64"] for i in infos], dtype=float)
    resid = max(i["residual"] for i in infos)
    sig = sig.cpu().numpy()
    F, T = F.cpu().numpy().reshape(-1, 2), T.cpu().numpy()
    poff = np.concatenate([[0], np.cumsum(b.nparticles)])
    offs = b.offsets.copy()
    b.close()

    def single(c, p):
        pb = yq.Problem(p)
        pb.set_workload(cfgs[c])
        pb.set_boundary_data(pb.boundary_label())
        s, _ = pb.solve()
        Fs, Ts, _ = pb.forces(s)
        return s, Fs, Ts

    def p64(t, fmm):
        kw = dict(far_mode=yq.YQ_FAR_FMM) if fmm else {}
        return yq.default_params(panels_per_particle=32, qbx_order=10, tol=t,
                                 precision=yq.YQ_FP64, restart=60, maxiter=400, **kw)

    # FP64 one-at-a-time path: each configuration alone (FP64 solve to the same
    # tolerance with the direct far field below SINGLE_FMM_NODES and the FP64
    # FMM above, then its forces), on every k-th configuration
    stride = max(1, len(cfgs) // max(args.single_baseline, 1))
    sample = list(range(0, len(cfgs), stride))
    service = []
    for k, c in enumerate(sample):
        torch.cuda.synchronize()
        a = time.perf_counter()
        single(c, p64(tol, N[c] >= SINGLE_FMM_NODES))
        torch.cuda.synchronize()
        service.append(time.perf_counter() - a)
        if (k + 1) % 64 == 0:
            log(f"FP64 one at a time: {k + 1} of {len(sample)}")
    service = np.array(service)
    t_one = float(service.mean()) * len(cfgs)     # all configurations, one after another
    # per-result errors of the batch against FP64 solves to 1e-12 (the FP64 path
    # matches the oracle's LU to 1e-10 in the parity tests)
    err = {"density": 0.0, "force": 0.0, "torque": 0.0}
    ref_idx = list(range(0, len(cfgs), max(1, len(cfgs) // args.error_configs)))
    for c in ref_idx:
        s64, F64, T64 = single(c, p64(1e-12, N[c] >= SINGLE_FMM_NODES))
        s64, F64, T64 = s64.cpu().numpy(), F64.cpu().numpy().reshape(-1, 2), T64.cpu().numpy()
        err["density"] = max(err["density"], float(np.abs(sig[offs[c]:offs[c + 1]] - s64).max()
                                                   / np.abs(s64).max()))
        err["force"] = max(err["force"], float(np.abs(F[poff[c]:poff[c + 1]] - F64).max()
                                               / np.abs(F64).max()))
        err["torque"] = max(err["torque"], float(np.abs(T[poff[c]:poff[c + 1]] - T64).max()
                                                 / np.abs(T64).max()))
    t_step = percentile(lat, 0.5)
    # roofline of the fused FP32 far-field kernel: algorithmic flops = 40 per directed
    # source-target pair (35 for K1(z)/z with the pair's geometry, 5 for the directional
    # dot product and the accumulation); the symmetric kernel evaluates K1(z)/z once per
    # unordered pair: (35 + 2 x 5) / 2 = 22.5 per directed pair.  pairs = the directed
    # pairs the timed launches covered (configurations still iterating)
    sym = args.far32 == "symmetric"
    F32_ALG, F64_ALG = (22.5 if sym else 40.0), 50.0
    bc = batch_counters(args.far32)
    avg32 = ms32 / max(n32, 1)
    achieved = F32_ALG * pairs32 / (ms32 * 1e-3) if ms32 > 0 else 0.0
    direct = {"bound": "alu", "kernel": "bsym32_kernel" if sym else "bfar32_kernel",
              "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
              "frac": achieved / PEAK_FP32,
              "traffic": (bc["hbm_bytes_per_pair"] * pairs32 / max(n32, 1)
                          if "hbm_bytes_per_pair" in bc else None),
              "flops_per_pair": F32_ALG,
              "counter_flops_per_pair": bc.get("valu_flops_per_pair"),
              "counter_frac": (bc["valu_flops_per_pair"] * pairs32 / (ms32 * 1e-3) / PEAK_FP32
                               if "valu_flops_per_pair" in bc and ms32 > 0 else None),
              "pairs_per_launch": pairs32 / max(n32, 1), "avg_launch_ms": avg32,
              "launches": n32, "total_ms": ms32}
    # the forest's FP32 leaf pass (its launches of one operator application bracketed
    # together).  With the near-field caches it reads stored coefficients: HBM-bound,
    # achieved = the algorithmic bytes the launches report (4 per pair, 16 per target,
    # 8 per source of each list entry) / their time.  Without them it evaluates K1 per
    # pair: 40 flop per directed pair (the general FP32 path)
    lc = leaf_counters()
    if bytesl32 > 0:
        ach_l = bytesl32 / (msl32 * 1e-3) / 1e9 if msl32 > 0 else 0.0
        leaf = {"bound": "hbm", "kernel": "forest_cleaf_kernel", "achieved": ach_l,
                "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach_l * 1e9 / PEAK_HBM,
                "traffic": (lc["hbm_bytes_per_pair"] * pairsl32 / max(nl32, 1)
                            if "hbm_bytes_per_pair" in lc else None),
                "bytes_per_launch": bytesl32 / max(nl32, 1),
                "bytes_per_pair": bytesl32 / max(pairsl32, 1)}
    else:
        ach_l = 40.0 * pairsl32 / (msl32 * 1e-3) if msl32 > 0 else 0.0
        leaf = {"bound": "alu", "kernel": "forest_leaf_kernel", "achieved": ach_l / 1e12,
                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": ach_l / PEAK_FP32,
                "traffic": None, "flops_per_pair": 40.0}
    leaf.update({"pairs_per_launch": pairsl32 / max(nl32, 1),
                 "avg_launch_ms": msl32 / max(nl32, 1), "launches": nl32, "total_ms": msl32,
                 "launch_note": "one timed launch = the leaf pass of one operator application "
                                "(the local expansions' evaluation at the nodes runs before it, "
                                "outside the bracket)"})
    fp64 = {"direct_kernel": {"kernel": "bfar64_kernel", "launches": n64,
                              "avg_launch_ms": ms64 / max(n64, 1),
                              "achieved": F64_ALG * pairs64 / (ms64 * 1e-3) / 1e12
                              if ms64 > 0 else None,
                              "peak": PEAK_FP64 / 1e12,
                              "frac": F64_ALG * pairs64 / (ms64 * 1e-3) / PEAK_FP64
                              if ms64 > 0 else None},
            "forest_leaf": {"kernel": "forest_cleaf_kernel / forest_leaf_kernel (FP64)",
                            "launches": nl64, "avg_launch_ms": msl64 / max(nl64, 1),
                            "pairs_per_launch": pairsl64 / max(nl64, 1),
                            "bytes_per_launch": bytesl64 / max(nl64, 1),
                            "achieved_GBps": (bytesl64 / (msl64 * 1e-3) / 1e9
                                              if msl64 > 0 and bytesl64 > 0 else None)}}
    # the dominant FP32 kernel of the timed steps carries the roofline
    if msl32 > ms32:
        roof = dict(leaf, other_fp32_kernel=direct if n32 and pairs32 else None, fp64=fp64)
    else:
        roof = dict(direct, other_fp32_kernel=leaf if nl32 and pairsl32 else None, fp64=fp64)
    out = {
        "metric": "source-target interactions/s per matvec; solves/s + p50/p99 latency at 1e-8 rel err",
        "value": len(cfgs) / t_step, "unit": "solves/s", "n_gpus": 1, "steps": len(lat),
        "warmup": max(args.warmup, 1), "ms_per_step": t_all / len(lat) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {len(cfgs)} configurations of 10-{nmax} ellipses "
                               f"(log-uniform, box 30 sqrt(n/50), gap 0.2), 32x16 nodes per "
                               f"particle, kappa~U[0.5,2], QBX order 10, mixed FP32/FP64 to a "
                               f"relative residual of {tol:g}; one step = batched solve + "
                               f"forces/torques of every configuration; "
                               + (f"every configuration a tree of the engine's FMM forest (FMM "
                                  f"order {inner_order} inner / {resid_order} FP64 residuals; near-field "
                                  f"caches), one graph-replayed "
                                  f"iteration for the whole batch; the forces of every "
                                  f"configuration in one batched pass" if forest and thr == 0
                                  else f"every configuration in the fused engine, one graph-replayed "
                                  f"iteration for the whole batch: {int((~lane).sum())} below "
                                  f"{thr} nodes with the fused direct far field, {int(lane.sum())} "
                                  f"from {thr} nodes on as trees of the FMM forest (FMM order "
                                  f"{inner_order} inner / {resid_order} FP64 residuals); the forces of every "
                                  f"configuration in one batched pass" if forest
                                  else f"{int((~lane).sum())} configurations below {thr} nodes in the "
                                  f"fused direct engine (graph-replayed iteration), "
                                  f"{int(lane.sum())} from {thr} nodes on in the FMM lane "
                                  f"({args.fmm_workers} workers, FMM order {inner_order} inner / "
                                  f"{resid_order} FP64 residuals)" if hybrid
                                  else ("the configurations below %d nodes only, all in the fused "
                                        "direct engine" % min_nodes if engine_only
                                        else "every configuration in the fused direct engine")),
                   "configs": len(cfgs), "total_nodes": int(N.sum()),
                   "parallelism": "single GPU"},
        "solves_per_s": len(cfgs) / t_step,
        "latency_ms_p50": percentile(lat, 0.5) * 1e3, "latency_ms_p99": percentile(lat, 0.99) * 1e3,
        "setup_s": t_setup, "autotune": {"persist_blocks": pblk, "far_want": fwant},
        "near_cache": {"bytes": near[0], "trees_fp32": near[1], "trees_fp64": near[2]},
        "gmres_iterations_mean": float(its.mean()), "gmres_iterations_max": int(its.max()),
        "refine_steps_max": int(ref.max()), "residual_max": resid,
        "matvec_interactions_per_s_fp32": (pairs32 / (ms32 * 1e-3) if ms32 > 0 and pairs32 > 0
                                           else None),
        "leaf_pass_interactions_per_s_fp32": pairsl32 / (msl32 * 1e-3) if msl32 > 0 else None,
        "leaf_pass_cached_GBps_fp32": (bytesl32 / (msl32 * 1e-3) / 1e9
                                       if msl32 > 0 and bytesl32 > 0 else None),
        "matvec_interactions_per_s_fp64": (pairs64 / (ms64 * 1e-3) if ms64 > 0 and pairs64 > 0
                                           else None),
        "fp64_one_at_a_time": {"sample": len(sample), "of": len(cfgs),
                               "solves_per_s": len(cfgs) / t_one,
                               "latency_ms_p50": float(np.percentile(service, 50)) * 1e3,
                               "latency_ms_p99": float(np.percentile(service, 99)) * 1e3,
                               "all_configs_one_after_another_ms": t_one * 1e3},
        "errors_vs_fp64_path": dict(err, configs=len(ref_idx), reference="FP64 solve to 1e-12"),
        "errors_vs_oracle": errors_vs_oracle_c2(yq, tol),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(cfgs, mv)
    print(json.dumps(out), flush=True)


def _layout(req):
    import workloads
    return workloads.trace_particles(req)


def trace_layouts(trace):
    """Particle layouts of a request trace, drawn in parallel host processes."""
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_layout, trace, chunksize=8))


def bench_serve(args):
    """Poisson arrivals replayed in real time against the continuous-batching server
    (fused direct lane below 20,000 nodes, FMM lane above), and the FP64
    one-at-a-time path on the same trace (FCFS)."""
    import numpy as np
    import torch

    import paper_1810_04131_amd as yq
    import workloads
    nmax = args.nmax or 2000
    trace = workloads.serving_trace(args.requests, rate=args.rate, seed=1, nmax=nmax)
    t_lay = time.perf_counter()
    parts = trace_layouts(trace)
    t_lay = time.perf_counter() - t_lay
    print(f"# layouts of {len(parts)} requests in {t_lay:.1f} s", file=sys.stderr, flush=True)
    prm = yq.default_params(panels_per_particle=32, qbx_order=10, tol=1e-8, precision=yq.YQ_MIXED,
                            restart=60, maxiter=300, far_mode=yq.YQ_FAR_AUTO)
    srv = yq.Server(prm, node_capacity=2_000_000, max_slots=48, mem_budget_bytes=150e9)
    thr = args.fmm_min_nodes if args.fmm_min_nodes is not None else SINGLE_FMM_NODES
    srv.set_fmm(thr, workers=args.fmm_workers)
    # warm-up requests of both lanes (code paths, allocations)
    small = min(range(len(parts)), key=lambda k: parts[k].n)
    big = max(range(len(parts)), key=lambda k: parts[k].n)
    for k in (small, big):
        w = srv.submit(parts[k])
        srv.run_until_idle()
        srv.release(w)
    print("# warm-up done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    pending = list(zip(trace, parts))
    tickets = []
    peak = 0
    last_report = t0
    while True:
        now = time.perf_counter() - t0
        while pending and pending[0][0]["arrival"] <= now:
            r, p = pending.pop(0)
            tickets.append((r, srv.submit(p)))
        c, run, q = srv.step()
        peak = max(peak, run)
        if time.perf_counter() - last_report > 30:
            last_report = time.perf_counter()
            print(f"# t={now:.0f}s submitted {len(tickets)} running {run} queued {q}",
                  file=sys.stderr, flush=True)
        if run == 0 and q == 0:
            if not pending:
                break
            time.sleep(max(0.0, min(0.002, pending[0][0]["arrival"] - now)))
    wall = time.perf_counter() - t0
    lat, lat_fmm, lat_dir = [], [], []
    worst = 0.0
    for (r, t), p in zip(tickets, parts):
        res = srv.result(t)
        lat.append(res["latency"])
        (lat_fmm if p.n * 512 >= thr else lat_dir).append(res["latency"])
        worst = max(worst, res["info"]["residual"])
    print(f"# server: {len(tickets)} solves in {wall:.1f} s", file=sys.stderr, flush=True)
    # FP64 one-at-a-time path: each request solved alone, first come first served
    # (same far-field choice per size: direct below the lane threshold, FP64 FMM above)
    p64 = yq.default_params(panels_per_particle=32, qbx_order=10, tol=1e-8, precision=yq.YQ_FP64,
                            restart=60, maxiter=300)
    p64_fmm = yq.default_params(panels_per_particle=32, qbx_order=10, tol=1e-8,
                                precision=yq.YQ_FP64, restart=60, maxiter=300,
                                far_mode=yq.YQ_FAR_FMM)
    n64 = len(parts) if args.fp64_requests is None else min(args.fp64_requests, len(parts))
    service = []
    for k, p in enumerate(parts[:n64]):
        pb = yq.Problem(p64_fmm if p.n * 512 >= thr else p64)
        torch.cuda.synchronize()
        a = time.perf_counter()
        pb.set_workload(p)
        pb.set_boundary_data(pb.boundary_label())
        s, _ = pb.solve()
        pb.forces(s)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - a)
        del pb
        if (k + 1) % 200 == 0:
            print(f"# fp64 path: {k + 1} requests", file=sys.stderr, flush=True)
    tfree = 0.0
    lat64 = []
    for r, sv in zip(trace, service):
        start = max(tfree, r["arrival"])
        tfree = start + sv
        lat64.append(tfree - r["arrival"])
    out = {
        "metric": "source-target interactions/s per matvec; solves/s + p50/p99 latency at 1e-8 rel err",
        "value": len(tickets) / wall, "unit": "solves/s", "n_gpus": 1, "steps": len(tickets),
        "warmup": 2, "ms_per_step": wall / max(len(tickets), 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {args.rate:g}/s, {len(tickets)} "
                               f"requests of 10-{nmax} ellipses (log-uniform), kappa~U[0.5,2], "
                               f"32x16 nodes per particle, QBX order 10, mixed FP32/FP64 to 1e-8; "
                               f"fused direct lane below {thr} nodes, FMM lane "
                               f"({args.fmm_workers} workers) above",
                   "parallelism": "single GPU"},
        "latency_ms_p50": percentile(lat, 0.5) * 1e3, "latency_ms_p99": percentile(lat, 0.99) * 1e3,
        "solves_per_s": len(tickets) / wall, "peak_concurrent": peak, "residual_max": worst,
        "direct_lane": {"requests": len(lat_dir), "latency_ms_p50": percentile(lat_dir, 0.5) * 1e3,
                        "latency_ms_p99": percentile(lat_dir, 0.99) * 1e3},
        "fmm_lane": {"requests": len(lat_fmm), "latency_ms_p50": percentile(lat_fmm, 0.5) * 1e3,
                     "latency_ms_p99": percentile(lat_fmm, 0.99) * 1e3},
        "fp64_one_at_a_time": {"requests": n64,
                               "latency_ms_p50": percentile(lat64, 0.5) * 1e3,
                               "latency_ms_p99": percentile(lat64, 0.99) * 1e3,
                               "solves_per_s": len(service) / max(tfree - trace[0]["arrival"], 1e-9),
                               "mean_service_ms": float(np.mean(service)) * 1e3},
    }
    print(json.dumps(out), flush=True)


def bench_large(args):
    """500 ellipses (N = 256,000) with the FMM inner far field and FP64 FMM residuals."""
    import numpy as np
    import torch

    import paper_1810_04131_amd as yq
    import workloads
    cfg = workloads.config_large(seed=0)
    parts = cfg["particles"]
    prm = yq.default_params(far_mode=yq.YQ_FAR_FMM, fmm_order=20, fmm_leaf_max=64,
                            fmm_resid_order=40, precision=yq.YQ_MIXED, tol=1e-8, maxiter=400)
    pb = yq.Problem(prm)
    for _ in range(max(args.warmup, 1)):
        pb.set_workload(parts)
        pb.set_boundary_data(pb.boundary_label())
        pb.solve()
    pb.lib.yq_profile_enable(pb.h, (1 << PH_FAR32) | (1 << PH_FAR64))
    for ph in range(7):
        prof(pb, ph)
    lat, lat_setup = [], []
    for _ in range(max(args.steps, 1)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.set_workload(parts)
        pb.set_boundary_data(pb.boundary_label())
        t1 = time.perf_counter()
        sig, info = pb.solve()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        lat_setup.append(t1 - t0)
    n32, ms32 = prof(pb, PH_FAR32)
    n64, ms64 = prof(pb, PH_FAR64)
    N = pb.N
    out = {
        "metric": "source-target interactions/s per matvec; solves/s + p50/p99 latency at 1e-8 rel err",
        "value": float(N) * N / (ms32 / max(n32, 1) * 1e-3), "unit": "interactions/s (FMM, dense-equivalent)",
        "n_gpus": 1, "steps": len(lat), "warmup": args.warmup,
        "ms_per_step": percentile(lat, 0.5) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "500 ellipses A~U[0.8,1.2] B~U[0.4,0.6] in 100x100, N=256000, kappa=1, "
                               "QBX order 10, FMM order 20 (<=64 nodes/leaf) inner, FP64 FMM order 40 "
                               "residuals, tol 1e-8", "N": N, "parallelism": "single GPU"},
        "solves_per_s": 1.0 / percentile(lat, 0.5), "latency_ms_p50": percentile(lat, 0.5) * 1e3,
        "latency_ms_p99": percentile(lat, 0.99) * 1e3, "setup_ms_p50": percentile(lat_setup, 0.5) * 1e3,
        "gmres_iterations": info["iterations"], "refine_steps": info["outer_steps"],
        "residual": info["residual"], "fmm_inner_ms": ms32 / max(n32, 1),
        "fmm_resid_ms": ms64 / max(n64, 1),
    }
    print(json.dumps(out), flush=True)


# The paper's Table 2 (one time step on an 8-core Xeon E5-2650 v4, GIGAQBX FMM,
# 70 points per disk, GMRES tolerance 1e-5): disks, box side, T_total / T_ref with
# T_ref = 10 s, T_GMRES / T_total, GMRES iterations.
AUTO_FMM_NODES = 20000   # the library's YQ_FAR_AUTO switch to the FMM
PAPER_TABLE2 = [(250, 100.0, 9.7, 0.679, 32), (500, 200.0, 14.4, 0.663, 28),
                (1000, 200.0, 32.4, 0.701, 32), (2000, 400.0, 55.3, 0.647, 31)]


def bench_table2(args):
    """Context only: the paper's Table 2 collections (unit disks, kappa = 0.25,
    5 panels x 16 nodes per disk, tol 1e-5) solved here, beside the paper's times."""
    import torch

    import paper_1810_04131_amd as yq
    import workloads
    rows = []
    for n, box, ratio, gfrac, iters_paper in PAPER_TABLE2:
        parts = workloads.random_ellipses(n, box, 0.25, seed=0, axes=(1.0, 1.0),
                                          name=f"{n} unit disks in {box:g}x{box:g}")
        prm = yq.default_params(panels_per_particle=5, qbx_order=8, tol=1e-5,
                                precision=yq.YQ_MIXED, maxiter=300, far_mode=yq.YQ_FAR_AUTO)
        pb = yq.Problem(prm)
        lat, lat_setup, info = [], [], None
        for k in range(max(args.warmup, 1) + max(min(args.steps, 5), 1)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pb.set_workload(parts)
            pb.set_boundary_data(pb.boundary_label())
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info, _, _, _ = pb.solve_forces()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if k >= max(args.warmup, 1):
                lat.append(t2 - t0)
                lat_setup.append(t1 - t0)
        t_total = ratio * 10.0
        rows.append({"disks": n, "box": box, "N": pb.N,
                     "far_field": "FMM" if pb.N >= AUTO_FMM_NODES else "direct",
                     "ms_per_step": percentile(lat, 0.5) * 1e3,
                     "setup_ms": percentile(lat_setup, 0.5) * 1e3,
                     "gmres_iterations": info["iterations"], "residual": info["residual"],
                     "paper_T_total_s": t_total, "paper_T_gmres_s": t_total * gfrac,
                     "paper_gmres_iterations": iters_paper})
    last = rows[-1]
    out = {
        "metric": "source-target interactions/s per matvec; solves/s + p50/p99 latency at 1e-8 rel err",
        "value": 1e3 / last["ms_per_step"], "unit": "solves/s (2000 disks, tol 1e-5)",
        "n_gpus": 1, "steps": min(args.steps, 5), "warmup": max(args.warmup, 1),
        "ms_per_step": last["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "context: the paper's Table 2 collections (unit disks, kappa 0.25, "
                               "5 panels x 16 nodes, QBX order 8, mixed FP32/FP64, tol 1e-5, "
                               "FMM above 20000 nodes); one step = set-up + label + solve + forces",
                   "parallelism": "single GPU"},
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def bench_dynamics(args):
    """Constant-drag time stepping (eq. euler) of 100 ellipses on a 10 x 10 grid:
    each step is a warm-started solve, forces, repulsion, Euler update and the
    set-up rebuild at the new configuration."""
    import numpy as np
    import torch

    import paper_1810_04131_amd as yq
    import workloads
    cfg = workloads.config_dynamics(seed=0)
    parts = cfg["particles"]
    prm = yq.default_params(panels_per_particle=cfg["panels"], qbx_order=cfg["qbx_order"],
                            tol=cfg["tol"], precision=yq.YQ_MIXED, far_mode=yq.YQ_FAR_AUTO,
                            maxiter=300)
    pb = yq.Problem(prm)
    pb.set_workload(parts)
    pb.set_boundary_data(pb.boundary_label())
    dyn = dict(dt=cfg["dt"], xi_x=cfg["xi_x"], xi_theta=cfg["xi_theta"], c0=cfg["c0"],
               q=cfg["q"], gamma=cfg["gamma"])
    sigma = torch.zeros(pb.N, dtype=torch.float64, device="cuda")
    prev = sigma.clone()
    first = None
    for k in range(max(args.warmup, 2)):
        info, _, _, _ = pb.step(sigma, sigma_prev=prev, **dyn)
        first = first or info["iterations"]
    lat, its, energy = [], [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        info, F, T, E = pb.step(sigma, sigma_prev=prev, **dyn)   # synchronous
        lat.append(time.perf_counter() - t0)
        its.append(info["iterations"])
        energy.append(E[0] + E[1])
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t_all
    # two profiled steps for the breakdown; then a cold solve at the same configuration
    pb.lib.yq_profile_enable(pb.h, -1)
    for ph in range(8):
        prof(pb, ph)
    for _ in range(2):
        pb.step(sigma, sigma_prev=prev, **dyn)
    br = {name: prof(pb, ph) for name, ph in (("inner_far", PH_FAR32), ("fp64_far", PH_FAR64),
                                              ("fused", PH_FUSED), ("qbx_build", PH_QBX),
                                              ("repulsion", PH_REPULSION))}
    pb.lib.yq_profile_enable(pb.h, 0)
    _, cold = pb.solve()
    c, a = pb.particles()
    K = len(lat)
    out = {
        "metric": "time steps/s (warm-started solve, forces, repulsion, Euler update, set-up)",
        "value": K / t_all, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": max(args.warmup, 2),
        "ms_per_step": t_all / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "100 ellipses 1.0x0.5 on a 10x10 grid (spacing 2.5, random "
                               "orientations), N=51200, kappa=1, QBX order 10, mixed FP32/FP64 "
                               "tol 1e-8, FMM (far mode auto); dt 0.02, xi_x 1.5, xi_theta 2.0, "
                               "gamma 1, c0 0.02, q 3; guess 2 sigma_n - sigma_(n-1)",
                   "N": pb.N, "parallelism": "single GPU"},
        "latency_ms_p50": percentile(lat, 0.5) * 1e3, "latency_ms_p99": percentile(lat, 0.99) * 1e3,
        "gmres_iterations_mean": float(np.mean(its)), "gmres_iterations_first_step": first,
        "gmres_iterations_cold_same_config": cold["iterations"],
        "total_energy_first_last": [energy[0], energy[-1]],
        "profiled_step_ms": {k: v[1] / 2 for k, v in br.items()},
        "repulsion_us_per_launch": br["repulsion"][1] / max(br["repulsion"][0], 1) * 1e3,
        "particles_moved": float(np.abs(c - parts.center).max()),
    }
    print(json.dumps(out), flush=True)


def bench_cutoff(args):
    """The cutoff far field (sums truncated where exp(-kappa r) is below the bound,
    cutoff_tol 1e-12) beside the exact direct sum on the 50-ellipse workload at
    kappa 1, 2 and 4, and beside the FMM on the 500-ellipse workload at kappa 4.
    One step = set-up + label + mixed solve to 1e-8 + forces."""
    import numpy as np
    import torch

    import paper_1810_04131_amd as yq
    import workloads

    def run(parts, kw, steps):
        pb = yq.Problem(yq.default_params(**kw))
        lat, out = [], None
        for k in range(max(args.warmup, 1) + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pb.set_workload(parts)
            pb.set_boundary_data(pb.boundary_label())
            out = pb.solve_forces(allow_noconv=True)
            torch.cuda.synchronize()
            if k >= max(args.warmup, 1):
                lat.append(time.perf_counter() - t0)
        pb.lib.yq_profile_enable(pb.h, (1 << PH_FAR32) | (1 << PH_FAR64))
        for ph in range(8):
            prof(pb, ph)
        pb.set_workload(parts)
        pb.set_boundary_data(pb.boundary_label())
        pb.solve_forces(allow_noconv=True)
        n32, ms32 = prof(pb, PH_FAR32)
        n64, ms64 = prof(pb, PH_FAR64)
        info = out[1]
        return {"ms_per_step": percentile(lat, 0.5) * 1e3, "gmres_iterations": info["iterations"],
                "residual": info["residual"], "inner_far_ms": ms32 / max(n32, 1),
                "fp64_far_ms": ms64 / max(n64, 1)}, out[2].cpu().numpy()

    steps = max(min(args.steps, 5), 1)
    rows = []
    base = dict(panels_per_particle=32, qbx_order=10, tol=1e-8, precision=yq.YQ_MIXED, maxiter=300)
    for kappa in (1.0, 2.0, 4.0):
        parts = workloads.config_medium(kappa=kappa, seed=0)["particles"]
        rd, Fd = run(parts, base, steps)
        rc, Fc = run(parts, dict(base, far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=1e-12), steps)
        rows.append({"workload": f"50 ellipses N=25600 kappa={kappa:g}", "direct": rd, "cutoff": rc,
                     "force_rel_diff": float(np.abs(Fc - Fd).max() / np.abs(Fd).max())})
    large = workloads.config_large(seed=0)["particles"].copy()
    large.kappa = 4.0
    lbase = dict(base, maxiter=400)
    rf, Ff = run(large, dict(lbase, far_mode=yq.YQ_FAR_FMM, fmm_order=20, fmm_leaf_max=64,
                             fmm_resid_order=40), steps)
    rc, Fc = run(large, dict(lbase, far_mode=yq.YQ_FAR_CUTOFF, cutoff_tol=1e-12), steps)
    rows.append({"workload": "500 ellipses N=256000 kappa=4", "fmm": rf, "cutoff": rc,
                 "force_rel_diff": float(np.abs(Fc - Ff).max() / np.abs(Ff).max())})
    out = {
        "metric": "solve-and-forces steps/s with the cutoff far field (500 ellipses, N=256000, kappa 4)",
        "value": 1e3 / rc["ms_per_step"], "unit": "steps/s", "n_gpus": 1, "steps": steps,
        "warmup": max(args.warmup, 1), "ms_per_step": rc["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "cutoff far field (cutoff_tol 1e-12; FP32 inner operator 1e-7) vs the "
                               "exact direct sum (50 ellipses, kappa 1/2/4) and vs the FMM (500 "
                               "ellipses, kappa 4, order 20 inner / 40 residual); mixed tol 1e-8",
                   "parallelism": "single GPU"},
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU here; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "large":
        return bench_large(args)
    if args.workload == "table2":
        return bench_table2(args)
    if args.workload == "dynamics":
        return bench_dynamics(args)
    if args.workload == "cutoff":
        return bench_cutoff(args)
    import numpy as np
    import torch

    import paper_1810_04131_amd as yq
    import workloads

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    cfg = workloads.config_medium(kappa=args.kappa, seed=0)
    parts = cfg["particles"]
    gx, gy = np.meshgrid(np.linspace(0.5, 29.5, 32), np.linspace(0.5, 29.5, 32))
    grid = np.stack([gx.ravel(), gy.ravel()], 1)

    def make(precision):
        p = yq.default_params(panels_per_particle=cfg["panels"], qbx_order=cfg["qbx_order"],
                              tol=1e-8, precision=precision, restart=100, maxiter=300)
        return yq.Problem(p)

    pb = make(yq.YQ_MIXED)
    for _ in range(args.warmup):
        run_step(pb, parts, grid)
    torch.cuda.synchronize()
    # inside the timed region only the roofline kernel's launches carry events
    pb.lib.yq_profile_enable(pb.h, 1 << PH_FAR32)
    for ph in range(7):
        prof(pb, ph)
    lat = []
    far_passes = 0
    infos = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        info, _u = run_step(pb, parts, grid)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        infos.append(info)
        # far-field passes: operator applications + one gradient pass; the potential
        # grid is 1024 targets x N sources (counted as such)
        far_passes += info["matvecs_fp32"] + info["matvecs_fp64"] + 1
    t_all = time.perf_counter() - t_all
    N = pb.N
    n32, ms32 = prof(pb, PH_FAR32)
    # the other phases' durations from a separate profiled pass (not timed)
    pb.lib.yq_profile_enable(pb.h, -1)
    for _ in range(2):
        run_step(pb, parts, grid)
    nfin, msfin = prof(pb, 2)
    ngr, msgr = prof(pb, 3)
    nqb, msqb = prof(pb, 4)
    nfu, msfu = prof(pb, 6)
    pb.lib.yq_profile_enable(pb.h, 0)
    interactions = far_passes * float(N) * N + args.steps * grid.shape[0] * float(N)
    value = interactions / t_all
    avg32 = ms32 / max(n32, 1) * 1e-3
    pairs = float(N) * (N - 1)
    nd = pb.nodes()
    xn, yn = nd["x"].cpu().numpy(), nd["y"].cpu().numpy()
    mix = far_class_mix(xn, yn, args.kappa, panels=True)
    f32_pair = flops_per_pair(mix, F32_CLASS)
    mix64 = mix   # the FP64 kernels split close tiles into panels the same way
    f64_pair = flops_per_pair(mix64, F64_CLASS)
    f64_valu = flops_per_pair(mix64, F64_VALU)
    achieved32 = f32_pair * pairs / avg32
    ms_step = t_all / args.steps * 1e3

    # FP64-only path on the same workload (the reference for solve latency)
    p64 = make(yq.YQ_FP64)
    run_step(p64, parts, grid)
    torch.cuda.synchronize()
    p64.lib.yq_profile_enable(p64.h, 1 << PH_FAR64)
    prof(p64, PH_FAR64)
    lat64 = []
    it64 = []
    for _ in range(args.fp64_steps):
        t0 = time.perf_counter()
        info64, _ = run_step(p64, parts, grid)
        torch.cuda.synchronize()
        lat64.append(time.perf_counter() - t0)
        it64.append(info64["iterations"])
    n64b, ms64b = prof(p64, PH_FAR64)
    avg64b = ms64b / max(n64b, 1) * 1e-3

    out = {
        "metric": "source-target interactions/s per matvec; solves/s + p50/p99 latency at 1e-8 rel err",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"50 ellipses 1.0x0.5 in a 30x30 box, N={N}, kappa={args.kappa:g}, "
                               f"32 panels x 16 nodes, QBX order 10, direct far field, "
                               f"mixed FP32/FP64, tol 1e-8",
                   "N": N, "particles": parts.n, "kappa": args.kappa, "qbx_order": 10,
                   "parallelism": "single GPU"},
        "solves_per_s": 1.0 / (ms_step * 1e-3),
        "latency_ms_p50": percentile(lat, 0.5) * 1e3,
        "latency_ms_p99": percentile(lat, 0.99) * 1e3,
        "gmres_iterations": infos[-1]["iterations"],
        "refine_steps": infos[-1]["outer_steps"],
        "residual": infos[-1]["residual"],
        "matvec_interactions_per_s_fp32": pairs / avg32,
        "matvec_interactions_per_s_fp64": pairs / avg64b if n64b else None,
        "far32_ms": avg32 * 1e3,
        "far64_ms": avg64b * 1e3 if n64b else None,
        "finish_ms": msfin / max(nfin, 1),
        "grad_far_ms": msgr / ngr if ngr else None,
        "resid_grad_fused_ms": msfu / nfu if nfu else None,
        "grad_passes_unfused": ngr,
        "qbx_build_ms": msqb / max(nqb, 1),
        "fp64_path": {"latency_ms_p50": percentile(lat64, 0.5) * 1e3,
                      "solves_per_s": 1.0 / max(percentile(lat64, 0.5), 1e-12),
                      "gmres_iterations": it64[-1] if it64 else None,
                      "far64_achieved_tflops": f64_pair * pairs / avg64b / 1e12 if n64b else None,
                      "far64_frac_of_fp64_peak": f64_pair * pairs / avg64b / PEAK_FP64 if n64b else None,
                      "far64_flops_per_pair": f64_pair,
                      "far64_valu_issue_frac": pairs / avg64b * f64_valu / VALU_ISSUE if n64b else None,
                      "far64_counter_frac": (counters("far64_valu_flops_per_launch") / avg64b / PEAK_FP64
                                             if n64b and counters("far64_valu_flops_per_launch")
                                             else None)},
        "roofline": {"bound": "alu", "kernel": "far32_kernel", "achieved": achieved32 / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": achieved32 / PEAK_FP32,
                     "traffic": traffic_from_counters(pairs), "flops_per_pair": f32_pair,
                     "valu_instr_per_pair": flops_per_pair(mix, F32_VALU),
                     "valu_issue_frac": pairs / avg32 * flops_per_pair(mix, F32_VALU) / VALU_ISSUE,
                     # the same launch's flops from the VALU instruction counters
                     # (64 x (ADD + MUL + 2 FMA + TRANS) FP32 wave instructions)
                     "counter_flops_per_launch": counters("far32_valu_flops_per_launch"),
                     "counter_frac": (counters("far32_valu_flops_per_launch") / avg32 / PEAK_FP32
                                      if counters("far32_valu_flops_per_launch") else None),
                     "pair_classes": mix,
                     "source_sha256_16": source_hash(),
                     "pairs_per_launch": pairs, "avg_launch_ms": avg32 * 1e3},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
