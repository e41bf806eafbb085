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

import numpy as np

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


def vmult_bytes(level, word, nr=1):
    """Algorithmic bytes of one operator application dst = A src: read src and
    write dst (N words each), the int32 cell-to-node map (q per cell) and the
    stored geometry per Gauss point: the merged metric, d(d+1)/2 words, for the
    Laplacian; J^{-1} and w det J, d^2 + 1 words, for elasticity (the
    stored-geometry form of the operator; the library rebuilds the geometry
    from the trilinear map instead, which moves fewer bytes, so this is the
    method's figure, not a count of ours).  With nr fused right-hand sides the
    vectors count nr times, the map and the geometry once."""
    q = (level.degree + 1) ** level.dim
    m = level.dim * (level.dim + 1) // 2 if level.ncomp == 1 else level.dim * level.dim + 1
    return 2 * word * level.n_dofs * nr + 4 * level.n_cells * q + word * level.n_cells * q * m


def transfer_bytes(coarse, n_points, word, prolong, nr=1):
    """Algorithmic bytes of one prolongation (fine += P coarse) or restriction
    (coarse += P^T fine): per fine point its index (int32), its d reference
    coordinates and the fine values of its nc components (read and written for
    prolongation, read for restriction); per coarse cell the two point-range
    offsets it reads, its q int32 node indices and the nc q coarse values (read
    for prolongation, read and written for restriction); values nr times with
    nr fused right-hand sides."""
    q = (coarse.degree + 1) ** coarse.dim
    d, nc = coarse.dim, coarse.ncomp * nr
    per_point = 4 + d * word + (2 if prolong else 1) * nc * word
    per_cell = 8 + 4 * q + (1 if prolong else 2) * nc * word * q
    return n_points * per_point + coarse.n_cells * per_cell


# main-run workloads: config, cells per direction (coarse -> fine), degree,
# operator, the oracle sample of the CPU baseline, and a description
WORKLOADS = {
    "cube_q2": dict(cfg=1, cells=[6, 13, 29, 64], degree=2, operator="laplace", cpu_cells=[3, 6, 13, 29],
                    roofline="cube_q2_64",
                    text="3D Poisson Q2 on the unit cube, non-nested perturbed hex levels 64^3/29^3/13^3/6^3 "
                         "(+-0.15h), 8 Gaussian bumps, float64 V-cycle in float64 PCG to 1e-8"),
    "ball_q4": dict(cfg="2q4", cells=[5, 7, 15, 34, 75], degree=4, operator="laplace", roofline="ball_q4_75",
                    pmg=True, cpu_cells=[5, 7, 11],
                    text="3D Poisson Q4 on the ball, non-nested levels 75^3/34^3/15^3/7^3/5^3 (27.3M fine DoFs), "
                         "bumps in the radius-0.8 ball; coarse solver: polynomial coarsening Q4->Q3->Q2->Q1 on the "
                         "5^3 mesh, then the dense inverse on Q1 (compared with the dense inverse on 5^3 Q4); "
                         "float64 V-cycle in float64 PCG to 1e-8"),
    "beam_q2": dict(cfg=3, cells=[(14, 3, 3), (33, 7, 7), (80, 16, 16)], degree=2, operator="elasticity", rhs=4,
                    roofline="beam_q2",
                    cpu_cells=[(10, 2, 2), (22, 5, 5), (50, 10, 10)],
                    text="3D linear elasticity, vector Q2, lambda = mu = 1, beam [0,5]x[0,1]^2 clamped at x = 0, "
                         "body load (0,0,-1) and three random smooth loads fused as 4 right-hand sides, "
                         "non-nested perturbed hex levels 80x16x16/33x7x7/14x3x3 (+-0.1h), "
                         "float64 V-cycle in float64 PCG to 1e-8"),
}

def run_serving(args, ctx, nn, torch, log):
    """The serving stream: requests with Poisson arrivals on a pool of resident
    hierarchies (0.1M..8M DoFs, 3-5 levels), 1..8 bump right-hand sides each,
    float32-MG in float64 PCG to 1e-8.  The same arrival trace is replayed
    with one request at a time and with continuous batching."""
    from workloads import SERVING_POOL, config_levels, config_source
    dev = "cuda:0"
    t0 = time.perf_counter()
    pool = []
    for cfg, cells, k in SERVING_POOL:
        meshes = config_levels(cfg, cells=cells)
        levels = [nn.Level.from_mesh(ctx, m, k) for m in meshes]
        trs = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
        H = nn.Hierarchy(ctx, levels, trs)
        if not args.no_tune:
            H.tune(torch.float32, reps=5)
        # replicas over the same levels and transfers, so a mesh can serve several requests at a time
        reps = [H] + [nn.Hierarchy(ctx, levels, trs) for _ in range(args.serving_replicas - 1)]
        fine = levels[-1]
        qp = fine.quadrature_points()
        cols = [fine.assemble_rhs(torch.tensor(config_source(cfg, 50 + r)(qp), dtype=torch.float64,
                                               device=dev).reshape(-1)) for r in range(8)]
        bank = {r: (cols[0] if r == 1 else torch.stack(cols[:r], dim=1).contiguous()) for r in range(1, 9)}
        pool.append(dict(H=H, reps=reps, levels=levels, trs=trs, n=fine.n_dofs, bank=bank, cfg=cfg, cells=cells,
                         k=k))
        log(f"pool: cfg {cfg} Q{k} {cells} -> {fine.n_dofs} DoFs")
    t_setup = time.perf_counter() - t0
    # warm-up (grows the buffers to 8 right-hand sides and captures every graph), then
    # the one-at-a-time service time of each hierarchy, averaged over 1..8 right-hand sides
    service = []
    for P in pool:
        for Hr in P["reps"]:
            for r in range(1, 9):
                Hr.pcg_solve(P["bank"][r], rtol=1e-8, vcycle_dtype=torch.float32, history=False)
        torch.cuda.synchronize()
        ts = []
        for r in (1, 4, 8):
            t1 = time.perf_counter()
            P["H"].pcg_solve(P["bank"][r], rtol=1e-8, vcycle_dtype=torch.float32, history=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        service.append(sum(ts) / len(ts))
    mean_service = sum(service) / len(service)
    rate = args.serving_load / mean_service
    rng = np.random.default_rng(4000)
    n_req = args.serving_requests
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    which = rng.integers(len(pool), size=n_req)
    nrs = rng.integers(1, 9, size=n_req)
    log(f"serving: {n_req} requests at {rate:.1f}/s (offered load {args.serving_load} of one-at-a-time capacity)")

    def replay(max_active):
        srv = nn.Server(ctx, max_active=max_active)
        torch.cuda.synchronize()
        tickets = []
        t_start = time.perf_counter()
        for a, h, r in zip(arrivals, which, nrs):
            now = time.perf_counter() - t_start
            if a > now:
                time.sleep(a - now)
            P = pool[int(h)]
            tickets.append((int(h), int(r), time.perf_counter() - t_start,
                            srv.submit(P["reps"], P["bank"][int(r)], vcycle_dtype=torch.float32)))
        lat, ends, work, its_all, queued = [], [], 0, [], []
        for h, r, ts, t in tickets:
            _, info, tm = t.wait()
            infos = info if isinstance(info, list) else [info]
            assert all(i["status"] == "OK" for i in infos)
            its = sum(i["iterations"] for i in infos)
            work += pool[h]["n"] * its
            its_all.append(its / r)
            lat.append(tm["total_ms"])
            queued.append(tm["queued_ms"])
            ends.append(ts + tm["total_ms"] * 1e-3)
        st = srv.stats()
        srv.close()
        makespan = max(ends)
        return dict(value=work / makespan / 1e6, makespan_s=round(makespan, 4),
                    latency_ms={"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3)},
                    mean_queued_ms=round(sum(queued) / len(queued), 3), max_running=st["max_running"],
                    mean_iterations=round(sum(its_all) / len(its_all), 2))

    log("replay: one request at a time")
    serial = replay(1)
    log(f"replay: continuous batching, {args.serving_slots} slots")
    batched = replay(args.serving_slots)
    big = pool[-1]
    log("timing the operator and transfer kernels of the largest hierarchy")
    k = kernel_rooflines(big["levels"][-1], big["levels"][-2], big["trs"][-1], args.roofline_reps)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline([3, 6, 13, 29], 1, "laplace")
    op = k["operator_fp32"]

    def entry(name):
        v = k[name]
        return {"ms": round(v["ms"], 5), "bytes": v["bytes"], "achieved": round(v["gbs"], 1),
                "frac": round(v["frac"], 4), "traffic": None}

    line = {
        "metric": METRIC,
        "value": round(batched["value"], 2),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": n_req,
        "warmup": 8 * len(pool),
        "ms_per_step": round(batched["makespan_s"] / n_req * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("serving stream: Poisson Q2 (perturbed cubes) and Q3 (balls) solves, 0.1M-8M fine DoFs "
                         "log-uniform over 6 resident meshes with 3-5 non-nested levels, Poisson arrivals, "
                         "1-8 Gaussian-bump right-hand sides per request, float32-MG in float64 PCG to 1e-8"),
            "pool_dofs": [P["n"] for P in pool],
            "requests": n_req,
            "arrival_rate_per_s": round(rate, 3),
            "offered_load": args.serving_load,
            "slots": args.serving_slots,
            "replicas_per_mesh": args.serving_replicas,
        },
        "latency_ms": batched["latency_ms"],
        "serving": {"continuous_batching": batched, "one_at_a_time": serial,
                    "speedup": round(batched["value"] / serial["value"], 3),
                    "service_ms_alone": [round(t * 1e3, 3) for t in service]},
        "setup_s": {"pool": round(t_setup, 3)},
        "roofline": {
            "bound": "hbm", "achieved": round(op["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(op["frac"], 4), "traffic": None,
            "kernel": (f"operator application on the largest resident level ({big['n']} DoFs), float32 (the "
                       "V-cycle precision): vmult_kernel + gather_kernel"),
            "bytes_per_launch": op["bytes"], "ms_per_launch": round(op["ms"], 5),
            "kernels": {n: entry(n) for n in k},
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# level pairs (fine <- coarse) for --roofline-only: workload, cells per direction, degree
ROOFLINE_WORKLOADS = {
    "cube_q2_64": (1, [6, 13, 29, 64], 2, "laplace"),      # 64^3 <- 29^3, 2.1M DoFs
    "ball_q3_96": (2, [5, 9, 19, 43, 96], 3, "laplace"),   # 96^3 <- 43^3, 24.1M DoFs
    "ball_q4_75": ("2q4", [5, 7, 15, 34, 75], 4, "laplace"),  # 75^3 <- 34^3, 27.3M DoFs
    "beam_q2": (3, [(14, 3, 3), (33, 7, 7), (80, 16, 16)], 2, "elasticity"),  # 525,987 DoFs
}

KERNEL_SOURCES = ("paper_2412_10910_amd/csrc/kernels/vmult.hip", "paper_2412_10910_amd/csrc/kernels/gather.hip",
                  "paper_2412_10910_amd/csrc/kernels/transfer.hip", "paper_2412_10910_amd/csrc/kernels/common.hpp")
# recorded HBM traffic of the roofline workloads (profiles/traffic_operator_transfer_<workload>.txt)
def traffic_file(tag):
    return os.path.join(ROOT, "profiles", f"traffic_operator_transfer_{tag}.txt")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(tag):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary,
    or {} when it is missing or was taken on kernel sources that have changed."""
    try:
        lines = open(traffic_file(tag)).read().splitlines()
    except OSError:
        return {}
    kv = {}
    for line in lines:
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256_16") != kernel_source_hash():
        return {}
    return {k[len("traffic_bytes."):]: float(v) for k, v in kv.items() if k.startswith("traffic_bytes.")}


def time_launches(fn, reps):
    """Average duration of fn() in ms from HIP events recorded on the current
    stream (the stream the library launches on), after 5 untimed calls."""
    import torch
    for _ in range(5):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def kernel_rooflines(fine, coarse, transfer, reps, nr=1):
    """Operator and transfer kernels of the two finest levels, FP64 and FP32;
    with nr > 1 also the launches that carry nr right-hand sides (suffix _x<nr>)."""
    import torch
    dev = "cuda:0"
    npts = transfer.n_points
    out = {}
    for dt, word, tag in ((torch.float64, 8, "fp64"), (torch.float32, 4, "fp32")):
        for r in sorted({1, nr}):
            sfx = "" if r == 1 else f"_x{r}"
            shape_f = (fine.n_dofs,) if r == 1 else (fine.n_dofs, r)
            shape_c = (coarse.n_dofs,) if r == 1 else (coarse.n_dofs, r)
            src = torch.rand(shape_f, dtype=torch.float64, device=dev).to(dt)
            dst = torch.zeros_like(src)
            csrc = torch.rand(shape_c, dtype=torch.float64, device=dev).to(dt)
            cdst = torch.zeros_like(csrc)
            ms = time_launches(lambda: fine.vmult_add(src, dst), reps)
            out[f"operator_{tag}{sfx}"] = dict(ms=ms, bytes=vmult_bytes(fine, word, r))
            ms = time_launches(lambda: transfer.prolongate(csrc, dst), reps)
            out[f"prolongate_{tag}{sfx}"] = dict(ms=ms, bytes=transfer_bytes(coarse, npts, word, True, r))
            ms = time_launches(lambda: transfer.restrict(src, cdst), reps)
            out[f"restrict_{tag}{sfx}"] = dict(ms=ms, bytes=transfer_bytes(coarse, npts, word, False, r))
    for v in out.values():
        v["gbs"] = v["bytes"] / (v["ms"] * 1e-3) / 1e9
        v["frac"] = v["gbs"] / HBM_PEAK_GBS
    return out


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size: its FETCH_SIZE/WRITE_SIZE readings
    scale the counters of the other kernels to bytes."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return nbytes


def cpu_baseline(cells, cfg, operator="laplace", degree=2, pmg=False):
    """Oracle PCG on a reduced instance of the same workload recipe, 1 thread."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    code = f"""
import json, time, sys
sys.path.insert(0, {ROOT!r})
import numpy as np
from oracle import assemble, elasticity, multigrid, space, transfer
from workloads import config_levels, config_source, random_vector
meshes = config_levels({cfg!r}, cells={cells!r})
k = {degree}
specs = ([(meshes[0], d) for d in range(1, k)] if {pmg!r} else []) + [(m, k) for m in meshes]
sps = [space.Space(m, d) for m, d in specs]
if {operator!r} == "elasticity":
    nc = 3
    As = [elasticity.stiffness(s, 1.0, 1.0) for s in sps]
    Ps = [elasticity.vector_prolongation(transfer.prolongation(sps[i + 1], sps[i])[0], 3) for i in range(len(sps) - 1)]
    frees = [elasticity.vector_free(s) for s in sps]
    b = elasticity.load_vector(sps[-1], config_source({cfg!r}))
else:
    nc = 1
    As = [assemble.stiffness(s) for s in sps]
    Ps = [transfer.prolongation(sps[i + 1], sps[i])[0] for i in range(len(sps) - 1)]
    frees = [s.free for s in sps]
    b = assemble.load_vector(sps[-1], config_source({cfg!r}))
H = multigrid.Hierarchy(As, frees, Ps, eig_start=[random_vector(s.n_dofs * nc, 100 + i) for i, s in enumerate(sps)])
t0 = time.perf_counter()
x, it, hist = H.pcg(b, rtol=1e-8)
t = time.perf_counter() - t0
print(json.dumps(dict(n=sps[-1].n_dofs * nc, it=it, t=t)))
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
                        f"{' / '.join(str(c) for c in cells[::-1])} cells, Q{degree}"
                        + (f" with polynomial coarsening to Q1 on the coarsest mesh" if pmg else "")
                        + f" ({r['n']} fine DoFs), {r['it']} iterations in {r['t']:.2f} s; "
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
    ap.add_argument("--roofline-rhs", type=int, default=1,
                    help="--roofline-only: also time the launches that carry this many right-hand sides")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the operator/transfer kernel loops of the two finest levels and a copy of "
                         "known size (the run that rocprofv3 traces and counts)")
    ap.add_argument("--serving-requests", type=int, default=120)
    ap.add_argument("--serving-load", type=float, default=1.0,
                    help="arrival rate as a fraction of the one-request-at-a-time service rate")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-replicas", type=int, default=2, help="hierarchies per resident mesh")
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["serving"], default="cube_q2",
                    help="the PCG workload (default: the 3D Poisson cube the metric is quoted on)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (operator variant per level, restriction team per transfer)")
    ap.add_argument("--rhs", type=int, default=None,
                    help="right-hand sides fused per solve (default: the workload's, 1 for the cube, 4 for the beam)")
    ap.add_argument("--roofline-workload", choices=sorted(ROOFLINE_WORKLOADS), default="cube_q2_64",
                    help="level pair of --roofline-only")
    ap.add_argument("--geometry", choices=["trilinear", "metric"], default=None,
                    help="operator geometry source (default: the library's choice)")
    args = ap.parse_args()
    if args.geometry:
        os.environ["NNMG_GEOMETRY"] = args.geometry
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2412_10910_amd as nn
    from workloads import config_levels, config_source, random_load

    dev = "cuda:0"
    torch.cuda.init()
    ctx = nn.Context(0)
    if args.workload == "serving" and not args.roofline_only:
        return run_serving(args, ctx, nn, torch, log)
    wl = WORKLOADS[args.workload]
    cfg, cells, degree, operator = wl["cfg"], wl["cells"], wl["degree"], wl["operator"]

    log("generating meshes")
    meshes = config_levels(cfg, cells=cells) if not args.roofline_only else None

    if args.roofline_only:
        rcfg, rcells, rdeg, rop = ROOFLINE_WORKLOADS[args.roofline_workload]
        rmeshes = config_levels(rcfg, cells=rcells)
        fine = nn.Level.from_mesh(ctx, rmeshes[-1], rdeg, rop)
        coarse = nn.Level.from_mesh(ctx, rmeshes[-2], rdeg, rop)
        tr = nn.Transfer(ctx, fine, coarse)
        nbytes = copy_calibration()
        k = kernel_rooflines(fine, coarse, tr, args.roofline_reps, args.roofline_rhs)
        print(json.dumps({"roofline_only": True, "workload": args.roofline_workload, "copy_bytes": nbytes, "reps": args.roofline_reps,
                          "kernels": {n: {"ms": round(v["ms"], 5), "bytes": v["bytes"], "GB/s": round(v["gbs"], 1),
                                          "frac": round(v["frac"], 4)} for n, v in k.items()}}), flush=True)
        return

    t0 = time.perf_counter()
    levels = [nn.Level.from_mesh(ctx, m, degree, operator) for m in meshes]
    t_levels = time.perf_counter() - t0
    t0 = time.perf_counter()
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    t_transfers = time.perf_counter() - t0
    t0 = time.perf_counter()
    H = nn.Hierarchy(ctx, levels, transfers)
    t_hier = time.perf_counter() - t0
    H_mesh, t_hier_mesh = None, None
    if wl.get("pmg"):
        # polynomial coarsening below the coarsest mesh level, sharing the mesh levels and transfers;
        # the hierarchy with the dense inverse on the coarsest mesh is kept for the comparison
        t0 = time.perf_counter()
        plevels = [nn.Level.from_mesh(ctx, meshes[0], d, operator) for d in range(1, degree)]
        ptrs = [nn.Transfer(ctx, (plevels + [levels[0]])[i + 1], plevels[i]) for i in range(len(plevels))]
        H_mesh, t_hier_mesh = H, t_hier
        H = nn.Hierarchy(ctx, plevels + levels, ptrs + transfers)
        t_hier = time.perf_counter() - t0
    tuned = None
    t_tune = 0.0
    if not args.no_tune:
        t0 = time.perf_counter()
        rep = H.tune(torch.float64, reps=10)
        t_tune = time.perf_counter() - t0
        tuned = dict(levels=[r["chosen"] for r in rep["levels"]], restriction_teams=[r["chosen"] for r in rep["transfers"]])
    fine = levels[-1]
    nr = args.rhs if args.rhs is not None else wl.get("rhs", 1)
    if operator == "elasticity":
        srcs = [config_source(cfg)] + [random_load(i) for i in range(1, nr)]
    else:
        srcs = [config_source(cfg, i) for i in range(nr)]
    qp = fine.quadrature_points()
    cols = [fine.assemble_rhs(torch.tensor(f(qp).reshape(-1), dtype=torch.float64, device=dev)) for f in srcs]
    b = cols[0] if nr == 1 else torch.stack(cols, dim=1).contiguous()
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    log(f"setup: levels {t_levels:.2f} s, transfers {t_transfers:.2f} s, hierarchy {t_hier:.2f} s; "
        f"fine DoFs {fine.n_dofs}")

    def run(dtype, steps, warmup, H=H):
        for _ in range(warmup):
            H.pcg_solve(b, x, rtol=1e-8, vcycle_dtype=dtype, history=False)
        torch.cuda.synchronize()
        lat, its = [], []
        t_start = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            _, info = H.pcg_solve(b, x, rtol=1e-8, vcycle_dtype=dtype, history=False)
            lat.append(time.perf_counter() - t1)
            infos = info if isinstance(info, list) else [info]
            its.append(sum(i["iterations"] for i in infos))
            info = dict(iterations=[i["iterations"] for i in infos] if nr > 1 else infos[0]["iterations"],
                        relres=max(i["relres"] for i in infos))
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        return total, lat, its, info

    log("timing float64-MG PCG")
    tot64, lat64, its64, info64 = run(torch.float64, args.steps, args.warmup)
    log("timing float32-MG PCG")
    tot32, lat32, its32, info32 = run(torch.float32, args.steps, args.warmup)
    value = fine.n_dofs * sum(its64) / tot64 / 1e6
    value32 = fine.n_dofs * sum(its32) / tot32 / 1e6
    dense = None
    if H_mesh is not None:
        log("timing the dense coarse inverse on the coarsest mesh for comparison")
        dsteps = max(1, args.steps // 5)
        d64, _, dits64, dinfo64 = run(torch.float64, dsteps, 1, H_mesh)
        d32, _, dits32, dinfo32 = run(torch.float32, dsteps, 1, H_mesh)
        dense = {"setup_hierarchy_s": round(t_hier_mesh, 3), "coarse_free_dofs": H_mesh.coarse_free_dofs,
                 "float64_mg": {"value": round(fine.n_dofs * sum(dits64) / d64 / 1e6, 2),
                                "ms_per_step": round(d64 / dsteps * 1e3, 4), "iterations": dinfo64["iterations"]},
                 "float32_mg": {"value": round(fine.n_dofs * sum(dits32) / d32 / 1e6, 2),
                                "ms_per_step": round(d32 / dsteps * 1e3, 4), "iterations": dinfo32["iterations"]}}

    log("timing the operator and transfer kernels")
    k = kernel_rooflines(fine, levels[-2], transfers[-1], args.roofline_reps, nr)
    traffic = recorded_traffic(wl["roofline"])

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
        cpu = cpu_baseline(wl["cpu_cells"], cfg, operator, degree, bool(wl.get("pmg")))

    op_key = "operator_fp64" if nr == 1 else f"operator_fp64_x{nr}"
    op = k[op_key]

    def entry(name):
        v = k[name]
        return {"ms": round(v["ms"], 5), "bytes": v["bytes"], "achieved": round(v["gbs"], 1),
                "frac": round(v["frac"], 4), "traffic": traffic.get(name)}

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
            "workload": wl["text"],
            "fine_dofs": fine.n_dofs,
            "level_dofs": [lv.n_dofs for lv in levels],
            "rhs": nr,
            "iterations": info64["iterations"],
        },
        "latency_ms": {"p50": round(percentile(lat64, 50) * 1e3, 4), "p99": round(percentile(lat64, 99) * 1e3, 4)},
        "fp32_mg": {
            "value": round(value32, 2),
            "ms_per_step": round(tot32 / args.steps * 1e3, 4),
            "iterations": info32["iterations"],
            "relres": info32["relres"],
            "latency_ms": {"p50": round(percentile(lat32, 50) * 1e3, 4),
                           "p99": round(percentile(lat32, 99) * 1e3, 4)},
            "speedup_vs_fp64_mg": round(tot64 / tot32, 3),
        },
        "setup_s": {"levels": round(t_levels, 3), "transfers": round(t_transfers, 3), "hierarchy": round(t_hier, 3),
                    "tune": round(t_tune, 3)},
        "tuned": tuned,
        "roofline": {
            "bound": "hbm",
            "achieved": round(op["gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(op["frac"], 4),
            "traffic": traffic.get(op_key),
            "kernel": (f"operator application on the finest level ({fine.n_dofs} DoFs"
                       + (f", {nr} fused right-hand sides" if nr > 1 else "") + "), float64: "
                       + (f"vmult_kernel<3,3,double,1,0,{1 if nr == 1 else 0}>" if operator == "laplace"
                          else f"elasticity_kernel<3,double,{1 if nr == 1 else 0}>")
                       + " (per-cell sum factorization) + gather_kernel (per-DoF sum of the cell "
                         "contributions), back to back on one stream"),
            "bytes_per_launch": op["bytes"],
            "ms_per_launch": round(op["ms"], 5),
            "kernels": {n: entry(n) for n in k},
        },
        "cpu_baseline": cpu,
    }
    if profile is not None:
        line["vcycle_profile_ms"] = profile
    if dense is not None:
        line["config"]["levels"] = [f"{lv.n_dofs}@Q{lv.degree}" for lv in H.levels]
        line["coarse_dense_inverse"] = dense
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
