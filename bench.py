"""Benchmark: float64 PCG preconditioned by one non-nested multigrid V-cycle.

Workload (default): 3D Poisson on the unit cube, Q2, four independent
hexahedral meshes of 64^3, 29^3, 13^3 and 6^3 cells with interior vertices
perturbed by +-0.15 h, zero Dirichlet data, f = sum of 8 Gaussian bumps of
width 0.1; the V-cycle in float64 (plain) and, for comparison, in float32.

A step is one pcg_solve to a relative residual of 1e-8 from x0 = 0 with the
hierarchy resident on the GPU.  value = fine DoFs x CG iterations / solve
time, in MDoF/s per PCG iteration (DoFs counted with the boundary, as the
paper does).  Each solve's wall time gives the p50/p99 latency.

Also reported: setup times, the float32-MG solve, the operator kernel's HBM
roofline (algorithmic bytes / measured kernel time) and the CPU oracle timed
on a bounded sample of the same workload on this machine's host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MDoF/s per PCG iteration and solve time to 1e-8 (FP32-MG vs FP64-MG); p50/p99 latency"
UNIT = "MDoF/s per PCG iteration"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, p):
    """Nearest-rank percentile."""
    s = sorted(xs)
    k = max(1, int(-(-p * len(s) // 100)))
    return s[min(k, len(s)) - 1]


def vmult_bytes(level, word):
    """Algorithmic bytes of one operator application: read src, write dst,
    the int32 cell-to-DoF map and the merged metric (d(d+1)/2 words per Gauss point)."""
    q = (level.degree + 1) ** level.dim
    m = level.dim * (level.dim + 1) // 2
    return 2 * word * level.n_dofs + 4 * level.n_cells * q + word * level.n_cells * q * m


def cpu_baseline(cells, cfg):
    """Oracle PCG on a reduced instance of the same workload recipe, 1 thread."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    code = f"""
import json, time, sys
sys.path.insert(0, {ROOT!r})
import numpy as np
from oracle import assemble, multigrid, space, transfer
from workloads import config_levels, config_source, random_vector
meshes = config_levels({cfg!r}, cells={cells!r})
k = {2}
sps = [space.Space(m, k) for m in meshes]
As = [assemble.stiffness(s) for s in sps]
Ps = [transfer.prolongation(sps[i + 1], sps[i])[0] for i in range(len(sps) - 1)]
H = multigrid.Hierarchy(As, [s.free for s in sps], Ps,
                        eig_start=[random_vector(s.n_dofs, 100 + i) for i, s in enumerate(sps)])
b = assemble.load_vector(sps[-1], config_source({cfg!r}))
t0 = time.perf_counter()
x, it, hist = H.pcg(b, rtol=1e-8)
t = time.perf_counter() - t0
print(json.dumps(dict(n=sps[-1].n_dofs, it=it, t=t)))
"""
    t0 = time.perf_counter()
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    wall = time.perf_counter() - t0
    if out.returncode != 0:
        log(out.stderr[-2000:])
        return None
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return dict(value=round(r["n"] * r["it"] / r["t"] / 1e6, 4), unit=UNIT, cores=1, kind="oracle",
                sample=(f"oracle float64 PCG + float64 V-cycle (scipy CSR) on the same recipe at "
                        f"{'/'.join(str(c) for c in cells[::-1])} cells per direction "
                        f"({r['n']} fine DoFs), {r['it']} iterations in {r['t']:.2f} s; "
                        f"setup excluded; {wall:.1f} s wall including setup"),
                cpu=_cpu_model(), host_cpus=os.cpu_count())


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true", help="also print the per-component V-cycle times")
    ap.add_argument("--roofline-reps", type=int, default=100)
    ap.add_argument("--geometry", choices=["trilinear", "metric"], default=None,
                    help="operator geometry source (default: the library's choice)")
    args = ap.parse_args()
    if args.geometry:
        os.environ["NNMG_GEOMETRY"] = args.geometry
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2412_10910_amd as nn
    from workloads import config_levels, config_source

    cfg = 1
    cells = [6, 13, 29, 64]
    degree = 2
    dev = "cuda:0"
    torch.cuda.init()
    ctx = nn.Context(0)

    log("generating meshes")
    meshes = config_levels(cfg, cells=cells)
    t0 = time.perf_counter()
    levels = [nn.Level.from_mesh(ctx, m, degree) for m in meshes]
    t_levels = time.perf_counter() - t0
    t0 = time.perf_counter()
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    t_transfers = time.perf_counter() - t0
    t0 = time.perf_counter()
    H = nn.Hierarchy(ctx, levels, transfers)
    t_hier = time.perf_counter() - t0
    fine = levels[-1]
    f = config_source(cfg)
    b = fine.assemble_rhs(torch.tensor(f(fine.quadrature_points()).reshape(-1), dtype=torch.float64, device=dev))
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    log(f"setup: levels {t_levels:.2f} s, transfers {t_transfers:.2f} s, hierarchy {t_hier:.2f} s; "
        f"fine DoFs {fine.n_dofs}")

    def run(dtype, steps, warmup):
        for _ in range(warmup):
            H.pcg_solve(b, x, rtol=1e-8, vcycle_dtype=dtype, history=False)
        torch.cuda.synchronize()
        lat, its = [], []
        t_start = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            _, info = H.pcg_solve(b, x, rtol=1e-8, vcycle_dtype=dtype, history=False)
            lat.append(time.perf_counter() - t1)
            its.append(info["iterations"])
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        return total, lat, its, info

    log("timing float64-MG PCG")
    tot64, lat64, its64, info64 = run(torch.float64, args.steps, args.warmup)
    log("timing float32-MG PCG")
    tot32, lat32, its32, info32 = run(torch.float32, args.steps, args.warmup)
    value = fine.n_dofs * sum(its64) / tot64 / 1e6
    value32 = fine.n_dofs * sum(its32) / tot32 / 1e6

    # operator kernel on the fine level: one launch per call, timed with events
    log("timing the operator kernel")
    reps = args.roofline_reps
    src = torch.rand(fine.n_dofs, dtype=torch.float64, device=dev)
    dst = torch.zeros_like(src)
    for _ in range(5):
        fine.vmult_add(src, dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fine.vmult_add(src, dst)
    e1.record()
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    bytes64 = vmult_bytes(fine, 8)
    achieved = bytes64 / (k_ms * 1e-3) / 1e9
    src32, dst32 = src.float(), dst.float()
    e0.record()
    for _ in range(reps):
        fine.vmult_add(src32, dst32)
    e1.record()
    torch.cuda.synchronize()
    k32_ms = e0.elapsed_time(e1) / reps
    achieved32 = vmult_bytes(fine, 4) / (k32_ms * 1e-3) / 1e9

    profile = None
    if args.profile:
        H.set_profiling(True)
        H.pcg_solve(b, x, rtol=1e-8, vcycle_dtype=torch.float64, history=False)
        ms = H.profile()
        H.set_profiling(False)
        profile = {name: [round(float(v), 4) for v in ms[:, j]] for j, name in enumerate(H.COMPONENTS)}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline([3, 6, 13, 29], cfg)

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tot64 / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3D Poisson Q2 on the unit cube, non-nested perturbed hex levels "
                        "64^3/29^3/13^3/6^3 (+-0.15h), 8 Gaussian bumps, float64 V-cycle in float64 PCG to 1e-8",
            "fine_dofs": fine.n_dofs,
            "level_dofs": [lv.n_dofs for lv in levels],
            "iterations": its64[-1],
        },
        "latency_ms": {"p50": round(percentile(lat64, 50) * 1e3, 4), "p99": round(percentile(lat64, 99) * 1e3, 4)},
        "fp32_mg": {
            "value": round(value32, 2),
            "ms_per_step": round(tot32 / args.steps * 1e3, 4),
            "iterations": its32[-1],
            "relres": info32["relres"],
            "latency_ms": {"p50": round(percentile(lat32, 50) * 1e3, 4),
                           "p99": round(percentile(lat32, 99) * 1e3, 4)},
            "speedup_vs_fp64_mg": round((tot64 / sum(its64) * its64[-1]) / (tot32 / sum(its32) * its32[-1]), 3),
        },
        "setup_s": {"levels": round(t_levels, 3), "transfers": round(t_transfers, 3), "hierarchy": round(t_hier, 3)},
        "roofline": {
            "bound": "hbm",
            "kernel": "vmult3_kernel<3,double> (fine level, 262144 cells)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_launch": bytes64,
            "kernel_ms": round(k_ms, 5),
            "fp32": {"kernel_ms": round(k32_ms, 5), "achieved": round(achieved32, 1),
                     "frac": round(achieved32 / HBM_PEAK_GBS, 4)},
        },
        "cpu_baseline": cpu,
    }
    if profile is not None:
        line["vcycle_profile_ms"] = profile
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
