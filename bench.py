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
# from the source of the large-argument branch (z >= 2) that almost every pair
# of this workload takes: an FMA counts 2, every other floating-point
# arithmetic operation (add, mul, rsq, exp2, rint, ldexp) counts 1.
#   FP32: 2 FP64 differences, r^2 (3), kappa^2 r^2 (1), rsq (1), z (1), rsq (1),
#         exp2 argument + exp2 (2), s (1), degree-8 Horner (16), 3 products (3),
#         (x-y).q (3), accumulate FMA (2)                                    = 36
#   FP64: differences (2), r^2 (3), kappa^2 r^2 (1), two Newton-refined rsqrt
#         (2 x 12), z (1), s (1), degree-20 Horner (40), e^-z by Cody-Waite +
#         degree-13 Taylor (33), 3 products (3), (x-y).q (3), product (1),
#         accumulate (1)                                                    = 113
F_DL32 = 36
F_DL64 = 113
SRC_FOR_COUNTERS = ["paper_1810_04131_amd/csrc/farfield.hip", "paper_1810_04131_amd/csrc/bessel.h",
                    "paper_1810_04131_amd/csrc/bessel_tables.h"]
COUNTERS_FILE = "profiles/far32_kernel_50ellipses_N25600_counters.txt"
PEAK_FP32 = 157.3e12   # published MI355X FP32 vector peak (needs packed FP32)
PEAK_FP64 = 78.6e12    # published MI355X FP64 vector peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kappa", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=384)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SRC_FOR_COUNTERS:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_counters(launch_pairs):
    """HBM bytes per far32 launch from the committed counter summary, or None when
    the kernel source has changed since the counters were taken."""
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
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    sigma, info = pb.solve()
    F, T, E = pb.forces(sigma)
    u = pb.eval_potential(sigma, grid)
    return info, u


def cpu_baseline(cfg, rows):
    """The oracle's operator rows (plain q-point far sum + QBX rows), timed on the host."""
    import numpy as np

    import oracle
    from oracle.geometry import Params
    parts = cfg["particles"]
    d = oracle.discretize(parts, Params(panels=cfg["panels"], qbx_order=cfg["qbx_order"]))
    sig = np.random.default_rng(0).standard_normal(d.N)
    sel = np.linspace(0, d.N - 1, rows).astype(int).tolist()
    oracle.apply_rows(d, sel[:2], sig)   # warm-up
    t0 = time.perf_counter()
    oracle.apply_rows(d, sel, sig)
    dt = time.perf_counter() - t0
    return dict(value=rows * d.N / dt, unit="interactions/s", cores=1, kind="oracle",
                sample=f"{rows} of {d.N} operator rows of the same workload "
                       f"(each row: {d.N} far-field pairs + QBX window), single-threaded "
                       f"numpy/scipy, {dt:.1f} s")


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
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
    pb.lib.yq_profile_enable(pb.h, 1)
    for ph in range(6):
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
    n32, ms32 = prof(pb, 1)
    n64, ms64 = prof(pb, 0)
    nfin, msfin = prof(pb, 2)
    ngr, msgr = prof(pb, 3)
    nqb, msqb = prof(pb, 4)
    pb.lib.yq_profile_enable(pb.h, 0)
    interactions = far_passes * float(N) * N + args.steps * grid.shape[0] * float(N)
    value = interactions / t_all
    avg32 = ms32 / max(n32, 1) * 1e-3
    avg64 = ms64 / max(n64, 1) * 1e-3
    pairs = float(N) * (N - 1)
    achieved32 = F_DL32 * pairs / avg32
    ms_step = t_all / args.steps * 1e3

    # FP64-only path on the same workload (the reference for solve latency)
    p64 = make(yq.YQ_FP64)
    run_step(p64, parts, grid)
    torch.cuda.synchronize()
    p64.lib.yq_profile_enable(p64.h, 1)
    prof(p64, 0)
    lat64 = []
    it64 = []
    for _ in range(args.fp64_steps):
        t0 = time.perf_counter()
        info64, _ = run_step(p64, parts, grid)
        torch.cuda.synchronize()
        lat64.append(time.perf_counter() - t0)
        it64.append(info64["iterations"])
    n64b, ms64b = prof(p64, 0)
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
        "grad_far_ms": msgr / max(ngr, 1),
        "qbx_build_ms": msqb / max(nqb, 1),
        "fp64_path": {"latency_ms_p50": percentile(lat64, 0.5) * 1e3,
                      "solves_per_s": 1.0 / max(percentile(lat64, 0.5), 1e-12),
                      "gmres_iterations": it64[-1] if it64 else None,
                      "far64_achieved_tflops": F_DL64 * pairs / avg64b / 1e12 if n64b else None,
                      "far64_frac_of_fp64_peak": F_DL64 * pairs / avg64b / PEAK_FP64 if n64b else None},
        "roofline": {"bound": "alu", "kernel": "far32_kernel", "achieved": achieved32 / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": achieved32 / PEAK_FP32,
                     "traffic": traffic_from_counters(pairs), "flops_per_pair": F_DL32,
                     "source_sha256_16": source_hash(),
                     "pairs_per_launch": pairs, "avg_launch_ms": avg32 * 1e3},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
