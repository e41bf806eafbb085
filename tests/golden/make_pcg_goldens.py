"""Write the oracle's whole-solve goldens at the parity sizes of the solver.

Usage: python tests/golden/make_pcg_goldens.py [case ...]   (default: every case)

For each case the oracle (``oracle/``, float64 NumPy/SciPy) builds the
hierarchy from the seeded meshes of ``workloads/``, estimates the Chebyshev
bounds of every level from the seeded Lanczos start vectors, and solves the
workload's right-hand side with PCG to 1e-8, preconditioned by one float64
V-cycle (Algorithm ``V_cycle``; paper §4 solver settings) and, separately, by a
float32 V-cycle.  It writes ``pcg_<case>.txt`` beside this script:

* per-level DoF counts and the Chebyshev interval [lo, hi] of every smoothed
  level (the GPU test injects these, so both sides smooth with one interval);
* the float64-MG iteration count and relative residual history;
* the float32-MG iteration count;
* norms of the solution and its value at sampled free support points, keyed by
  the point's coordinates (the two numberings differ; points identify DoFs).

Nothing here runs the HIP library: every stored value comes from ``oracle/``.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import assemble, multigrid, space, transfer  # noqa: E402
from workloads import config_levels, config_source, random_vector  # noqa: E402

# name: (workload config, cells per direction coarse -> fine, degree,
#        polynomial coarsening Q1..Q(k-1) below the coarsest mesh)
CASES = {
    # the 3D Poisson cube at full size: 64^3/29^3/13^3/6^3, Q2, 2,146,689 DoFs
    "cube_q2_64": (1, [6, 13, 29, 64], 2, False),
    # the ball reduced for the oracle: Q3 32^3/15^3/7^3/4^3 (912,673 DoFs)
    "ball_q3_32": ("2p3", [4, 7, 15, 32], 3, False),
    # Q4 24^3/11^3/5^3 (912,673 DoFs) with polynomial coarsening Q4->Q3->Q2->Q1
    # on the 5^3 mesh, the coarse solver of the Q4 ball benchmark
    "ball_q4_24": ("2p4", [5, 11, 24], 4, True),
}

N_SAMPLES = 1024
EIG_SEED = 100     # Lanczos start vector of level l: random_vector(n_l, EIG_SEED + l), oracle DoF order
SAMPLE_SEED = 7


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"pcg_{name}.txt")


def build(cfg, cells, k, pmg):
    meshes = config_levels(cfg, cells=cells)
    specs = ([(meshes[0], d) for d in range(1, k)] if pmg else []) + [(m, k) for m in meshes]
    spaces = [space.Space(m, d) for m, d in specs]
    As = [assemble.stiffness(s) for s in spaces]
    Ps = [transfer.prolongation(spaces[i + 1], spaces[i])[0] for i in range(len(spaces) - 1)]
    return spaces, As, Ps


def make(name: str) -> str:
    cfg, cells, k, pmg = CASES[name]
    t0 = time.perf_counter()
    spaces, As, Ps = build(cfg, cells, k, pmg)
    t_setup = time.perf_counter() - t0
    print(f"[{name}] levels {[s.n_dofs for s in spaces]}, setup {t_setup:.1f} s", flush=True)
    frees = [s.free for s in spaces]
    starts = [random_vector(s.n_dofs, EIG_SEED + i) for i, s in enumerate(spaces)]
    H64 = multigrid.Hierarchy(As, frees, Ps, eig_start=starts)
    fine = spaces[-1]
    b = assemble.load_vector(fine, config_source(cfg))
    t1 = time.perf_counter()
    x, it, hist = H64.pcg(b, rtol=1e-8)
    t_pcg = time.perf_counter() - t1
    print(f"[{name}] float64-MG: {it} iterations in {t_pcg:.1f} s", flush=True)
    H32 = multigrid.Hierarchy(As, frees, Ps, bounds=H64.bounds, dtype=np.float32)
    x32, it32, hist32 = H32.pcg(b, rtol=1e-8)
    print(f"[{name}] float32-MG: {it32} iterations", flush=True)
    rng = np.random.default_rng(SAMPLE_SEED)
    free = np.nonzero(fine.free)[0]
    pick = np.sort(rng.choice(free, size=min(N_SAMPLES, free.size), replace=False))
    lines = [
        "# Whole-solve golden of the non-nested multigrid PCG (Algorithm V_cycle; paper §4 solver settings).",
        "# Written by tests/golden/make_pcg_goldens.py from oracle/ (float64 NumPy/SciPy) and workloads/ only.",
        "# Chebyshev bounds: Lanczos from random_vector(n_l, 100 + l) in the oracle's DoF order.",
        "# samples: x y z u_h(x) at free support points of the finest level (float64-MG solution).",
        f"case = {name}",
        f"cfg = {cfg}",
        f"cells = {' '.join(str(c) for c in cells)}",
        f"degree = {k}",
        f"pmg = {int(pmg)}",
        f"level_degrees = {' '.join(str(s.k) for s in spaces)}",
        f"level_dofs = {' '.join(str(s.n_dofs) for s in spaces)}",
        f"level_free = {' '.join(str(int(s.free.sum())) for s in spaces)}",
    ]
    for l in range(1, len(spaces)):
        lo, hi = H64.bounds[l]
        lines.append(f"bounds.{l} = {float(lo)!r} {float(hi)!r}")
    lines += [
        f"rtol = 1e-08",
        f"iterations_fp64 = {it}",
        f"history_fp64 = {' '.join(repr(float(h)) for h in hist)}",
        f"iterations_fp32 = {it32}",
        f"relres_fp32 = {float(hist32[-1])!r}",
        f"x_norm2 = {float(np.linalg.norm(x))!r}",
        f"x_max = {float(np.abs(x).max())!r}",
        f"b_norm2 = {float(np.linalg.norm(b))!r}",
        f"oracle_seconds = setup {t_setup:.1f} pcg {t_pcg:.1f}",
        f"samples = {pick.size}",
    ]
    for i in pick:
        p = fine.support_points[i]
        lines.append(" ".join(repr(float(v)) for v in (p[0], p[1], p[2], x[i])))
    path = golden_path(name)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"[{name}] wrote {path} ({time.perf_counter() - t0:.1f} s)", flush=True)
    return path


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(CASES)):
        make(nm)
