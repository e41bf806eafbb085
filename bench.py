"""Benchmark: float64 PCG preconditioned by one non-nested multigrid V-cycle.

Workload (default): 3D Poisson on the ball (a structured cube mapped by
x -> x |x|_inf / |x|_2), Q4 on five independent non-nested meshes of
75^3/34^3/15^3/7^3/5^3 cells (27,270,901 fine DoFs, the largest configuration
of the paper's ball experiment that fits one GPU), zero Dirichlet data,
f = sum of 8 Gaussian bumps of width 0.1 in the radius-0.8 ball; coarse
solver: polynomial coarsening Q4->Q3->Q2->Q1 on the 5^3 mesh, then the dense
float64 inverse on Q1.  The V-cycle runs in float64 (the plain method: the
headline value) and in float32 inside the float64 CG (paper §4), and both
reach 1e-8.  The Q3 ball on 96^3/43^3/19^3/9^3/5^3 (24,137,569 DoFs) is
measured in the same run and reported under "extra_workloads".

A step is one pcg_solve to a relative residual of 1e-8 from x0 = 0 with the
hierarchy resident on the GPU.  value = fine DoFs x CG iterations / solve
time, in MDoF/s per PCG iteration (DoFs counted with the boundary, as the
paper does).  Each solve's wall time gives the p50/p99 latency.

Also reported: setup times; the per-component V-cycle times of one solve
(pre-smoother, residual, restriction, coarse solve, prolongation,
post-smoother, per level); the operator and transfer kernels against the HBM
roofline (model bytes and, where recorded, measured HBM bytes per launch);
the error against the float64 oracle, quoted from the oracle's stored
whole-solve goldens (tests/golden/pcg_*.txt) re-solved here at the reduced
size the oracle can solve; and the CPU oracle timed on a bounded sample of
the same workload on this machine's host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload W] [--no-cpu-baseline]
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
# published vector peaks of MI355X (float32 with packed math, which this build
# does not use: its float32 vector issue rate equals the float64 one)
FP64_PEAK_GFLOPS = 78_600.0
FP32_PEAK_GFLOPS = 157_300.0


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


def vmult_flops(level, nr=1):
    """Algorithmic flops of one Laplace operator application: per cell and
    right-hand side 4d sum-factorization sweeps of 2 n^(d+1) flops (d
    interpolations and d collocation derivatives forward, their transposes
    backward) and the symmetric d x d metric times the gradient at each of the
    n^d Gauss points (d^2 multiplications and d(d-1) additions).  None for
    elasticity (no single count of its stress evaluation is used here)."""
    if level.ncomp != 1:
        return None
    n, d = level.degree + 1, level.dim
    return nr * level.n_cells * (4 * d * 2 * n ** (d + 1) + (2 * d * d - d) * n ** d)


def transfer_flops(coarse, n_points, nr=1):
    """Algorithmic flops of one prolongation or restriction: per fine point the
    d 1D Lagrange bases at its reference coordinates (5n - 1 flops each: the
    differences, the prefix and suffix products and the barycentric scaling)
    and, per value, the tensor-product contraction of n^d + ... + n
    multiply-adds (2 flops each)."""
    n, d = coarse.degree + 1, coarse.dim
    contraction = 2 * sum(n ** e for e in range(1, d + 1))
    return n_points * (d * (5 * n - 1) + coarse.ncomp * nr * contraction)


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


# PCG workloads: config, cells per direction (coarse -> fine), degree, operator,
# polynomial coarsening on the coarsest mesh, the level pair whose recorded
# traffic applies, the oracle's whole-solve golden of the same recipe at a
# size the oracle solves, the oracle sample of the CPU baseline, a description
WORKLOADS = {
    "ball_q4": dict(cfg="2q4", cells=[5, 7, 15, 34, 75], degree=4, operator="laplace", pmg=True,
                    roofline="ball_q4_75", golden="ball_q4_24", cpu_cells=[5, 7, 11],
                    text="3D Poisson Q4 on the ball (cube mapped by x|x|_inf/|x|_2), non-nested levels "
                         "75^3/34^3/15^3/7^3/5^3 (27,270,901 fine DoFs), 8 Gaussian bumps in the radius-0.8 ball, "
                         "zero Dirichlet; coarse solver: polynomial coarsening Q4->Q3->Q2->Q1 on the 5^3 mesh, "
                         "then the dense float64 inverse on Q1; float64 V-cycle in float64 PCG to 1e-8 (value) "
                         "and float32 V-cycle in float64 PCG to 1e-8 (fp32_mg)"),
    "ball_q3": dict(cfg=2, cells=[5, 9, 19, 43, 96], degree=3, operator="laplace", pmg=False,
                    roofline="ball_q3_96", golden="ball_q3_32", cpu_cells=[3, 5, 9],
                    text="3D Poisson Q3 on the ball (cube mapped by x|x|_inf/|x|_2), non-nested levels "
                         "96^3/43^3/19^3/9^3/5^3 (24,137,569 fine DoFs), 8 Gaussian bumps in the radius-0.8 ball, "
                         "zero Dirichlet; dense float64 inverse on 5^3 Q3; float64 V-cycle in float64 PCG to 1e-8 "
                         "(value) and float32 V-cycle in float64 PCG to 1e-8 (fp32_mg)"),
    "cube_q2": dict(cfg=1, cells=[6, 13, 29, 64], degree=2, operator="laplace", pmg=False,
                    roofline="cube_q2_64", golden="cube_q2_64", cpu_cells=[3, 6, 13, 29],
                    text="3D Poisson Q2 on the unit cube, non-nested perturbed hex levels 64^3/29^3/13^3/6^3 "
                         "(+-0.15h), 8 Gaussian bumps, float64 V-cycle in float64 PCG to 1e-8"),
    "beam_q2": dict(cfg=3, cells=[(14, 3, 3), (33, 7, 7), (80, 16, 16)], degree=2, operator="elasticity", rhs=4,
                    pmg=False, roofline="beam_q2", golden=None,
                    cpu_cells=[(10, 2, 2), (22, 5, 5), (50, 10, 10)],
                    text="3D linear elasticity, vector Q2, lambda = mu = 1, beam [0,5]x[0,1]^2 clamped at x = 0, "
                         "body load (0,0,-1) and three random smooth loads fused as 4 right-hand sides, "
                         "non-nested perturbed hex levels 80x16x16/33x7x7/14x3x3 (+-0.1h), "
                         "float64 V-cycle in float64 PCG to 1e-8"),
}
DEFAULT_WORKLOAD = "ball_q4"
# measured in the same run as a workload and reported beside it
EXTRA_WORKLOADS = {"ball_q4": ["ball_q3"]}


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
    n_req = args.serving_requests
    rng = np.random.default_rng(4000)
    # one trace shape for every load: unit-rate exponential gaps, scaled by the load's rate
    gaps = rng.exponential(1.0, n_req)
    which = rng.integers(len(pool), size=n_req)
    nrs = rng.integers(1, 9, size=n_req)
    # size-aware admission: a request of at least this many fine DoFs x right-hand
    # sides is large (here: every 8.1M-DoF request, the 2.1M/1.8M ones with several
    # right-hand sides), and large requests run one at a time beside small ones
    large_work = 4e6
    MODES = {"one_at_a_time": dict(max_active=1),
             "batching_arrival": dict(max_active=args.serving_slots),
             "batching_sized": dict(max_active=args.serving_slots, policy="smallest", aging_ms=250.0,
                                    large_work=large_work, max_large=1)}

    def replay(mode, load):
        rate = load / mean_service
        arrivals = np.cumsum(gaps / rate)
        srv = nn.Server(ctx, **MODES[mode])
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
        return dict(value=round(work / makespan / 1e6, 2), makespan_s=round(makespan, 4),
                    latency_ms={"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3)},
                    mean_queued_ms=round(sum(queued) / len(queued), 3), max_running=st["max_running"],
                    mean_iterations=round(sum(its_all) / len(its_all), 2))

    # offered-load sweep: the same request sequence at each load, replayed in each mode
    loads = sorted({0.5, 1.0, 1.5, args.serving_load})
    sweep = {}
    for load in loads:
        sweep[str(load)] = {}
        for mode in MODES:
            log(f"replay: load {load}, {mode}")
            sweep[str(load)][mode] = replay(mode, load)
    at = sweep[str(args.serving_load)]
    serial, batched = at["one_at_a_time"], at["batching_sized"]
    rate = args.serving_load / mean_service
    big = pool[-1]
    log("timing the operator and transfer kernels of the largest hierarchy")
    k = kernel_rooflines(big["levels"][-1], big["levels"][-2], big["trs"][-1], args.roofline_reps)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline([3, 6, 13, 29], 1, "laplace")
    op = k["operator_fp32"]

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
            "admission": ("smallest expected work (fine DoFs x right-hand sides) first, aging bound 250 ms, "
                          f"requests of >= {large_work:.0f} DoF x rhs run one at a time"),
        },
        "latency_ms": batched["latency_ms"],
        "serving": {"continuous_batching": batched, "one_at_a_time": serial,
                    "speedup": round(batched["value"] / serial["value"], 3),
                    "load_sweep": sweep,
                    "service_ms_alone": [round(t * 1e3, 3) for t in service]},
        "setup_s": {"pool": round(t_setup, 3)},
        "roofline": roofline_entry(k, "operator_fp32", {}, big["levels"][-1], 4, 1,
                                   f"operator application on the largest resident level ({big['n']} DoFs), "
                                   "float32 (the V-cycle precision)"),
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
    or {} when it is missing or was taken on kernel sources that have changed.
    Keys: the roofline entries (operator_fp64, ...) and, per kernel, the
    operator kernels of every variant the tuner ran ("kernel:<name>", the
    fine-level gather as "kernel:<name>@fine"), so that an operator entry is
    priced by the variant the tuner chose in this run."""
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
    out = {k[len("traffic_bytes."):]: float(v) for k, v in kv.items() if k.startswith("traffic_bytes.")}
    out.update({"kernel:" + k[len("traffic_kernel."):]: float(v) for k, v in kv.items()
                if k.startswith("traffic_kernel.")})
    return out


def entry_traffic(traffic, key, v):
    """Measured bytes of one roofline entry: the sum over its launches where
    the per-kernel values were recorded (operators), else the entry's value."""
    names = v.get("launches")
    if names:
        keys = ["kernel:" + names[0]] + ["kernel:" + n + "@fine" for n in names[1:]]
        if all(k in traffic for k in keys):
            return sum(traffic[k] for k in keys)
        return None
    return traffic.get(key)


def operator_kernel_names(level, word, nr=1):
    """The kernels one operator application (Level.vmult, dst = A src) launches, named
    as the kernel trace names them, for the level's degree and operator variant
    (vmult_kernel<dim, n, T, geometry, scatter, nrt, index layout, sweep, layout
    blocks per workgroup>), with the operator variant of the precision of that
    word size."""
    T = "double" if word == 8 else "float"
    n = level.degree + 1
    nrt = 1 if nr == 1 else 0
    if level.operator == "elasticity":
        return [f"elasticity_kernel<{n}, {T}, {nrt}>", f"gather_kernel<3, {nr}, {T}>", f"copy_idx_kernel<{T}>"]
    import torch
    dt = torch.float64 if word == 8 else torch.float32
    variant = level.VARIANTS[level.variant_of(dt)]
    geo = 1 if variant.startswith("trilinear") else 0
    sw = 1 if variant.endswith("+transposed") else 0
    if variant.endswith("atomic"):
        return [f"vmult_kernel<{level.dim}, {n}, {T}, {geo}, 1, {nrt}, 0, 0, 1>", f"fill_kernel<{T}>",
                f"copy_idx_kernel<{T}>"]
    idx = 1 if "+entity" in variant else 0
    cells, base = level.cells_per_block(dt)[:2]
    return [f"vmult_kernel<{level.dim}, {n}, {T}, {geo}, 0, {nrt}, {idx}, {sw}, {cells // base}>",
            f"gather_kernel<1, {nr}, {T}>", f"copy_idx_kernel<{T}>"]


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
            # the operator application dst = A src (nnmg_vmult): the cell
            # kernel, the gather that writes dst, the identity on constrained rows
            peak = FP64_PEAK_GFLOPS if word == 8 else FP32_PEAK_GFLOPS
            ms = time_launches(lambda: fine.vmult(src, dst), reps)
            out[f"operator_{tag}{sfx}"] = dict(ms=ms, bytes=vmult_bytes(fine, word, r), flops=vmult_flops(fine, r),
                                               flop_peak=peak, launches=operator_kernel_names(fine, word, r))
            ms = time_launches(lambda: transfer.prolongate(csrc, dst), reps)
            out[f"prolongate_{tag}{sfx}"] = dict(ms=ms, bytes=transfer_bytes(coarse, npts, word, True, r),
                                                 flops=transfer_flops(coarse, npts, r), flop_peak=peak)
            ms = time_launches(lambda: transfer.restrict(src, cdst), reps)
            out[f"restrict_{tag}{sfx}"] = dict(ms=ms, bytes=transfer_bytes(coarse, npts, word, False, r),
                                               flops=transfer_flops(coarse, npts, r), flop_peak=peak)
            del src, dst, csrc, cdst
    for v in out.values():
        v["gbs"] = v["bytes"] / (v["ms"] * 1e-3) / 1e9
        v["frac"] = v["gbs"] / HBM_PEAK_GBS
    return out


def kernel_entry(v, traffic):
    """One kernel of the roofline table: time, model bytes and their rate, and
    the measured HBM bytes and their rate where recorded for these sources."""
    e = {"ms": round(v["ms"], 5), "bytes": v["bytes"], "achieved": round(v["gbs"], 1),
         "frac": round(v["frac"], 4), "traffic": traffic}
    if traffic:
        rate = traffic / (v["ms"] * 1e-3) / 1e9
        e["traffic_rate"] = round(rate, 1)
        e["traffic_frac"] = round(rate / HBM_PEAK_GBS, 4)
    if v.get("flops"):
        # the arithmetic side of the same launch, against the published vector
        # peak of its precision (float32: the packed-math figure)
        e["flops"] = v["flops"]
        e["gflops"] = round(v["flops"] / (v["ms"] * 1e-3) / 1e9, 1)
        e["flop_frac"] = round(e["gflops"] / v["flop_peak"], 4)
    if "launches" in v:
        e["launches"] = v["launches"]
    return e


def roofline_entry(k, key, traffic, fine, word, nr, what):
    """The roofline object of the line for the dominant kernel `key`."""
    op = k[key]
    t = entry_traffic(traffic, key, op)
    names = op.get("launches", [])
    out = {
        "bound": "hbm",
        "achieved": round(op["gbs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(op["frac"], 4),
        "traffic": t,
        "kernel": (what + ": " + " + ".join(names) + ", back to back on one stream; HIP events over "
                   "the repeated launches"),
        "model": ("algorithmic bytes of the stored-geometry operator: 2 s N vectors + 4 q C int32 map + "
                  "s q C metric words (the library rebuilds the geometry from the trilinear map and does not "
                  "read a metric, so achieved/frac are effective rates; traffic_rate is the measured one)"),
        "bytes_per_launch": op["bytes"],
        "ms_per_launch": round(op["ms"], 5),
        "kernels": {n: kernel_entry(v, entry_traffic(traffic, n, v)) for n, v in k.items()},
    }
    if t:
        out["traffic_rate"] = round(t / (op["ms"] * 1e-3) / 1e9, 1)
        out["traffic_frac"] = round(out["traffic_rate"] / HBM_PEAK_GBS, 4)
    if op.get("flops"):
        out["flops_per_launch"] = op["flops"]
        out["gflops"] = round(op["flops"] / (op["ms"] * 1e-3) / 1e9, 1)
        out["flop_frac"] = round(out["gflops"] / op["flop_peak"], 4)
    return out


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size, three times: its FETCH_SIZE/WRITE_SIZE
    readings scale the counters of the other kernels to bytes, and its rate
    (bytes read plus written over the median time, HIP events) is what HBM
    gives a streaming kernel on this GPU.  Returns (bytes, GB/s)."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    times = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del a, b
    return nbytes, 2 * nbytes / (sorted(times)[1] * 1e-3) / 1e9


def cpu_baseline(cells, cfg, operator="laplace", degree=2, pmg=False, runs=3):
    """The oracle (scipy CSR, 1 thread) on a reduced instance of the same
    workload recipe: the median of `runs` PCG solves, and beside it the
    median time of one CSR product per level and of one V-cycle."""
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
def med(f, n):
    ts = []
    for _ in range(n):
        t0 = time.perf_counter(); f(); ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], ts
mv = []
for A in As:
    v = random_vector(A.shape[0], 5)
    mv.append(med(lambda: A @ v, 5)[0])
tv, _ = med(lambda: H.vcycle(b), 3)
its = []
def solve():
    x, it, hist = H.pcg(b, rtol=1e-8)
    its.append(it)
t, ts = med(solve, {runs})
print(json.dumps(dict(n=sps[-1].n_dofs * nc, it=its[0], t=t, ts=ts, mv=mv, vcycle=tv,
                      levels=[s.n_dofs * nc for s in sps], nnz=[int(A.nnz) for A in As])))
"""
    t0 = time.perf_counter()
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)
    wall = time.perf_counter() - t0
    if out.returncode != 0:
        log(out.stderr[-2000:])
        return None
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return dict(value=round(r["n"] * r["it"] / r["t"] / 1e6, 4), unit=UNIT, cores=1, kind="oracle",
                sample=(f"oracle float64 PCG + float64 V-cycle (scipy CSR, one thread) on the same recipe at "
                        f"{' / '.join(str(c) for c in cells[::-1])} cells, Q{degree}"
                        + (" with polynomial coarsening to Q1 on the coarsest mesh" if pmg else "")
                        + f" ({r['n']} fine DoFs), {r['it']} iterations, median of {runs} solves "
                        f"{r['t']:.3f} s; setup excluded; {wall:.1f} s wall including setup (the full-size "
                        "oracle needs tens of GB of CSR and minutes of setup per level, beyond this run's budget)"),
                solve_s=[round(t, 4) for t in r["ts"]],
                matvec_ms_per_level=[round(t * 1e3, 3) for t in r["mv"]],
                vcycle_ms=round(r["vcycle"] * 1e3, 2),
                level_dofs=r["levels"], level_nnz=r["nnz"],
                cpu=_cpu_model(), host_cpus=os.cpu_count())


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def load_golden(name):
    """The oracle's stored whole-solve golden (tests/golden/pcg_<name>.txt)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("_golden_io", os.path.join(ROOT, "tests", "golden", "golden_io.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load_golden(name)


def _cfg_key(s):
    return int(s) if s.isdigit() else s


def golden_check(ctx, nn, torch, name):
    """Solve the golden's case with the library (bounds injected from the
    golden, as the GPU parity test does) and compare: iteration counts, the
    float64-MG residual history, and the solution at the stored points."""
    from scipy.spatial import cKDTree

    from workloads import config_levels, config_source
    dev = "cuda:0"
    g = load_golden(name)
    cfg = _cfg_key(g["cfg"])
    cells = [int(c) for c in g["cells"].split()]
    k = int(g["degree"])
    meshes = config_levels(cfg, cells=cells)
    levels, transfers = nn.build_levels(ctx, meshes, k, p_coarsening=bool(int(g["pmg"])))
    assert [lv.n_dofs for lv in levels] == [int(v) for v in g["level_dofs"].split()]
    H = nn.Hierarchy(ctx, levels, transfers)
    for l in range(1, len(levels)):
        lo, hi = (float(v) for v in g[f"bounds.{l}"].split())
        H.set_cheb_bounds(l, lo, hi)
    fine = levels[-1]
    b = fine.assemble_rhs(torch.tensor(config_source(cfg)(fine.quadrature_points()).reshape(-1),
                                       dtype=torch.float64, device=dev))
    samples = g["samples"]
    dist, idx = cKDTree(fine.support_points()).query(samples[:, :3])
    assert dist.max() <= 1e-12
    u = samples[:, 3]
    out = {"dofs": fine.n_dofs, "oracle_iterations_fp64": int(g["iterations_fp64"]),
           "oracle_iterations_fp32": int(g["iterations_fp32"]), "samples": int(u.size)}
    hist_orc = np.array([float(v) for v in g["history_fp64"].split()])
    for dt, tag in ((torch.float64, "fp64"), (torch.float32, "fp32")):
        x, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=dt)
        xs = x[torch.tensor(idx, device=dev)].cpu().numpy()
        out[f"iterations_{tag}"] = info["iterations"]
        out[f"max_rel_err_{tag}"] = float(np.abs(xs - u).max() / np.abs(u).max())
        if dt == torch.float64 and info["iterations"] == hist_orc.size - 1:
            out["history_max_abs_diff_fp64"] = float(np.abs(info["history"] - hist_orc).max())
    H.close()
    for t in transfers:
        t.close()
    for lv in levels:
        lv.close()
    return out


def run_pcg_workload(name, args, ctx, nn, torch, steps, warmup, with_cpu):
    """Build, tune and time one PCG workload; returns the fields of its line."""
    from workloads import config_levels, config_source, random_load
    dev = "cuda:0"
    wl = WORKLOADS[name]
    cfg, cells, degree, operator = wl["cfg"], wl["cells"], wl["degree"], wl["operator"]
    log(f"[{name}] generating meshes")
    meshes = config_levels(cfg, cells=cells)
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
    all_levels, all_transfers = levels, transfers
    if wl.get("pmg"):
        # polynomial coarsening below the coarsest mesh level, sharing the mesh levels and transfers;
        # the hierarchy with the dense inverse on the coarsest mesh is kept for the comparison
        t0 = time.perf_counter()
        plevels = [nn.Level.from_mesh(ctx, meshes[0], d, operator) for d in range(1, degree)]
        ptrs = [nn.Transfer(ctx, (plevels + [levels[0]])[i + 1], plevels[i]) for i in range(len(plevels))]
        H_mesh, t_hier_mesh = H, t_hier
        H = nn.Hierarchy(ctx, plevels + levels, ptrs + transfers)
        t_hier = time.perf_counter() - t0
        all_levels, all_transfers = plevels + levels, ptrs + transfers
    tuned = None
    t_tune = 0.0
    if not args.no_tune:
        t0 = time.perf_counter()
        # each precision has its own operator variant: float64 for the plain
        # method, float32 for the float32 V-cycle
        rep = H.tune(torch.float64, reps=10)
        rep32 = [lv.tune(torch.float32, reps=10) for lv in H.levels]
        t_tune = time.perf_counter() - t0
        tuned = dict(levels_fp64=[r["chosen"] for r in rep["levels"]],
                     levels_fp32=[r["chosen"] for r in rep32],
                     cells_per_block_fp64=[r["cells_per_block"] for r in rep["levels"]],
                     cells_per_block_fp32=[r["cells_per_block"] for r in rep32],
                     fine_ms_cells_fp64=rep["levels"][-1]["ms_cells"], fine_ms_cells_fp32=rep32[-1]["ms_cells"],
                     rhs_split_fp64=[r["rhs_split"] for r in rep["levels"]],
                     rhs_split_fp32=[r["rhs_split"] for r in rep32],
                     restriction_teams=[r["chosen"] for r in rep["transfers"]])
    fine = levels[-1]
    nr = args.rhs if args.rhs is not None else wl.get("rhs", 1)
    if operator == "elasticity":
        srcs = [config_source(cfg)] + [random_load(i) for i in range(1, nr)]
    else:
        srcs = [config_source(cfg, i) for i in range(nr)]
    qp = fine.quadrature_points()
    cols = [fine.assemble_rhs(torch.tensor(f(qp).reshape(-1), dtype=torch.float64, device=dev)) for f in srcs]
    del qp
    b = cols[0] if nr == 1 else torch.stack(cols, dim=1).contiguous()
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    log(f"[{name}] setup: levels {t_levels:.2f} s, transfers {t_transfers:.2f} s, hierarchy {t_hier:.2f} s; "
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
        # the true residual of the last solution, with the library's float64 operator
        true = float((b - fine.vmult(x)).norm() / b.norm())
        return total, lat, its, info, true

    log(f"[{name}] timing float64-MG PCG")
    tot64, lat64, its64, info64, true64 = run(torch.float64, steps, warmup)
    log(f"[{name}] timing float32-MG PCG")
    tot32, lat32, its32, info32, true32 = run(torch.float32, steps, warmup)
    value = fine.n_dofs * sum(its64) / tot64 / 1e6
    value32 = fine.n_dofs * sum(its32) / tot32 / 1e6
    dense = None
    if H_mesh is not None:
        log(f"[{name}] timing the dense coarse inverse on the coarsest mesh for comparison")
        dsteps = max(1, steps // 5)
        d64, _, dits64, dinfo64, _ = run(torch.float64, dsteps, 1, H_mesh)
        d32, _, dits32, dinfo32, _ = run(torch.float32, dsteps, 1, H_mesh)
        dense = {"setup_hierarchy_s": round(t_hier_mesh, 3), "coarse_free_dofs": H_mesh.coarse_free_dofs,
                 "float64_mg": {"value": round(fine.n_dofs * sum(dits64) / d64 / 1e6, 2),
                                "ms_per_step": round(d64 / dsteps * 1e3, 4), "iterations": dinfo64["iterations"]},
                 "float32_mg": {"value": round(fine.n_dofs * sum(dits32) / d32 / 1e6, 2),
                                "ms_per_step": round(d32 / dsteps * 1e3, 4), "iterations": dinfo32["iterations"]}}
        H_mesh.close()

    profile = None
    if not args.no_profile:
        # the six components of Algorithm V_cycle per level, one solve each,
        # events around every component (slower than the graph-replayed solve)
        profile = {}
        for dt, tag in ((torch.float64, "fp64_mg"), (torch.float32, "fp32_mg")):
            H.set_profiling(True)
            H.pcg_solve(b, x, rtol=1e-8, vcycle_dtype=dt, history=False)
            ms = H.profile()
            H.set_profiling(False)
            tot = {c: float(ms[:, j].sum()) for j, c in enumerate(H.COMPONENTS)}
            s = sum(tot.values())
            profile[tag] = {
                "ms_per_level": {c: [round(float(v), 4) for v in ms[:, j]] for j, c in enumerate(H.COMPONENTS)},
                "ms_total": {c: round(v, 4) for c, v in tot.items()},
                "share": {c: round(v / s, 4) for c, v in tot.items()} if s > 0 else None,
                "levels": [f"{lv.n_dofs}@Q{lv.degree}" for lv in all_levels],
            }

    log(f"[{name}] timing the operator and transfer kernels")
    k = kernel_rooflines(fine, levels[-2], transfers[-1], args.roofline_reps, nr)
    traffic = recorded_traffic(wl["roofline"])
    _, copy_gbs = copy_calibration()

    golden = None
    if wl.get("golden") and not args.no_golden:
        log(f"[{name}] re-solving the oracle's golden {wl['golden']}")
        golden = golden_check(ctx, nn, torch, wl["golden"])

    cpu = None
    if with_cpu:
        log(f"[{name}] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(wl["cpu_cells"], cfg, operator, degree, bool(wl.get("pmg")))

    op_key = "operator_fp64" if nr == 1 else f"operator_fp64_x{nr}"
    res = {
        "value": round(value, 2),
        "ms_per_step": round(tot64 / steps * 1e3, 4),
        "config": {
            "workload": wl["text"],
            "fine_dofs": fine.n_dofs,
            "level_dofs": [lv.n_dofs for lv in all_levels],
            "level_degrees": [lv.degree for lv in all_levels],
            "rhs": nr,
            "iterations": info64["iterations"],
        },
        "latency_ms": {"p50": round(percentile(lat64, 50) * 1e3, 4), "p99": round(percentile(lat64, 99) * 1e3, 4)},
        "relres": info64["relres"],
        "true_relres": true64,
        "fp32_mg": {
            "value": round(value32, 2),
            "ms_per_step": round(tot32 / steps * 1e3, 4),
            "iterations": info32["iterations"],
            "relres": info32["relres"],
            "true_relres": true32,
            "latency_ms": {"p50": round(percentile(lat32, 50) * 1e3, 4),
                           "p99": round(percentile(lat32, 99) * 1e3, 4)},
            "speedup_vs_fp64_mg": round(tot64 / tot32, 3),
        },
        "setup_s": {"levels": round(t_levels, 3), "transfers": round(t_transfers, 3), "hierarchy": round(t_hier, 3),
                    "tune": round(t_tune, 3)},
        "tuned": tuned,
        "roofline": dict(roofline_entry(k, op_key, traffic, fine, 8, nr,
                                        f"operator application on the finest level ({fine.n_dofs} DoFs"
                                        + (f", {nr} fused right-hand sides" if nr > 1 else "") + "), float64"),
                         copy_gbs=round(copy_gbs, 1)),
        "error_vs_oracle": {
            "golden": golden,
            "note": ("the full-size solve is beyond the oracle (tens of GB of CSR); the same recipe at the size "
                     "of the oracle's stored golden is re-solved here with the golden's smoother bounds and "
                     "compared with it; true_relres is ||b - A x|| / ||b|| of the full-size solution with the "
                     "library's float64 operator") if golden else None,
        },
        "cpu_baseline": cpu,
    }
    if profile is not None:
        res["vcycle_profile"] = profile
    if dense is not None:
        res["coarse_dense_inverse"] = dense
    H.close()
    for t in all_transfers:
        t.close()
    for lv in all_levels:
        lv.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-component V-cycle times")
    ap.add_argument("--no-golden", action="store_true", help="skip the re-solve of the oracle's golden")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra workloads measured beside the default")
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
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["serving"], default=DEFAULT_WORKLOAD,
                    help="the PCG workload (default: the Q4 ball, the largest single-GPU configuration)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (operator variant per level, restriction team per transfer)")
    ap.add_argument("--rhs", type=int, default=None,
                    help="right-hand sides fused per solve (default: the workload's, 1 for Poisson, 4 for the beam)")
    ap.add_argument("--roofline-workload", choices=sorted(ROOFLINE_WORKLOADS), default="ball_q4_75",
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
    from workloads import config_levels

    torch.cuda.init()
    ctx = nn.Context(0)
    if args.workload == "serving" and not args.roofline_only:
        return run_serving(args, ctx, nn, torch, log)

    if args.roofline_only:
        rcfg, rcells, rdeg, rop = ROOFLINE_WORKLOADS[args.roofline_workload]
        rmeshes = config_levels(rcfg, cells=rcells)
        fine = nn.Level.from_mesh(ctx, rmeshes[-1], rdeg, rop)
        coarse = nn.Level.from_mesh(ctx, rmeshes[-2], rdeg, rop)
        tr = nn.Transfer(ctx, fine, coarse)
        if not args.no_tune:
            # the kernels the tuned solve runs: one operator variant per precision
            # the fine level's operator variants only: the restriction team
            # stays at its default, so that every profiling pass of this
            # command launches the same transfer kernels
            for dt in (torch.float64, torch.float32):
                fine.tune(dt, reps=10)
        nbytes, copy_gbs = copy_calibration()
        k = kernel_rooflines(fine, coarse, tr, args.roofline_reps, args.roofline_rhs)
        print(json.dumps({"roofline_only": True, "workload": args.roofline_workload, "copy_bytes": nbytes,
                          "copy_gbs": round(copy_gbs, 1), "reps": args.roofline_reps,
                          "kernels": {n: {"ms": round(v["ms"], 5), "bytes": v["bytes"], "GB/s": round(v["gbs"], 1),
                                          "frac": round(v["frac"], 4), "launches": v.get("launches")}
                                      for n, v in k.items()}}), flush=True)
        return

    main_res = run_pcg_workload(args.workload, args, ctx, nn, torch, args.steps, args.warmup,
                                not args.no_cpu_baseline)
    extras = {}
    if not args.no_extra:
        for name in EXTRA_WORKLOADS.get(args.workload, []):
            torch.cuda.empty_cache()
            r = run_pcg_workload(name, args, ctx, nn, torch, args.steps, args.warmup, False)
            r.pop("cpu_baseline", None)
            extras[name] = r
    line = {
        "metric": METRIC,
        "value": main_res.pop("value"),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": main_res.pop("config"),
    }
    line.update(main_res)
    if extras:
        line["extra_workloads"] = extras
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
