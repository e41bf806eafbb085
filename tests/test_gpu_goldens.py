"""The whole solve against the oracle at the sizes assigned to parity.

The oracle's float64 PCG (Algorithm V_cycle as the preconditioner; paper §4
solver settings) is too slow to run inside a GPU test at these sizes, so its
results are stored as goldens by tests/golden/make_pcg_goldens.py, which calls
only oracle/ and workloads/:

* cube_q2_64: the 3D Poisson cube at full size, Q2 on 64^3/29^3/13^3/6^3
  (2,146,689 DoFs);
* ball_q3_32: the ball reduced for the oracle, Q3 on 32^3/15^3/7^3/4^3
  (912,673 DoFs, curved boundary: eq. closest_point);
* ball_q4_24: Q4 on 24^3/11^3/5^3 with polynomial coarsening Q4->Q3->Q2->Q1
  on the 5^3 mesh (912,673 DoFs), the coarse solver of the Q4 ball benchmark.

The library builds the same hierarchy from the same seeded meshes, takes the
oracle's Chebyshev intervals (parity injection: both sides then smooth with
one interval), and must give
* float64-MG: the same iteration count, a residual history within 1e-12 of
  the oracle's, the solution within 1e-10 (relative to its largest sampled
  value) at the stored support points and in the 2-norm;
* float32-MG (paper §4: V-cycle in single precision inside double CG):
  relative residual <= 1e-8, iterations within +-1 of the oracle's float64-MG
  and float32-MG counts, solution within 1e-6 of the oracle's.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from workloads import config_levels, config_source

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from golden_io import load_golden  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CASES = ["cube_q2_64", "ball_q3_32", "ball_q4_24"]


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


@pytest.mark.parametrize("name", CASES)
def test_pcg_matches_the_oracle_golden(ctx, name):
    import paper_2412_10910_amd as nn
    g = load_golden(name)
    cfg = int(g["cfg"]) if g["cfg"].isdigit() else g["cfg"]
    cells = [int(c) for c in g["cells"].split()]
    k = int(g["degree"])
    t0 = time.perf_counter()
    levels, transfers = nn.build_levels(ctx, config_levels(cfg, cells=cells), k, p_coarsening=bool(int(g["pmg"])))
    assert [lv.n_dofs for lv in levels] == [int(v) for v in g["level_dofs"].split()]
    assert [lv.n_free for lv in levels] == [int(v) for v in g["level_free"].split()]
    assert [lv.degree for lv in levels] == [int(v) for v in g["level_degrees"].split()]
    H = nn.Hierarchy(ctx, levels, transfers)
    for l in range(1, len(levels)):
        lo, hi = (float(v) for v in g[f"bounds.{l}"].split())
        H.set_cheb_bounds(l, lo, hi)
    fine = levels[-1]
    b = fine.assemble_rhs(torch.tensor(config_source(cfg)(fine.quadrature_points()).reshape(-1),
                                       dtype=torch.float64, device=DEV))
    bn = float(g["b_norm2"])
    assert abs(float(b.norm()) - bn) <= 1e-12 * bn
    samples = g["samples"]
    dist, idx = cKDTree(fine.support_points()).query(samples[:, :3])
    assert dist.max() <= 1e-12, "stored points are not support points of the library's level"
    u = samples[:, 3]
    sel = torch.tensor(idx, device=DEV)
    log(f"[{name}] {len(levels)} levels, fine DoFs {fine.n_dofs}, setup {time.perf_counter() - t0:.1f} s")

    it_orc = int(g["iterations_fp64"])
    hist_orc = np.array([float(v) for v in g["history_fp64"].split()])
    x, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float64)
    err = float(np.abs(x[sel].cpu().numpy() - u).max() / np.abs(u).max())
    dnorm = abs(float(x.norm()) - float(g["x_norm2"])) / float(g["x_norm2"])
    hdiff = float(np.abs(info["history"] - hist_orc).max()) if info["iterations"] == it_orc else float("inf")
    log(f"[{name}] float64-MG: {info['iterations']} iterations (oracle {it_orc}), history diff {hdiff:.2e}, "
        f"sampled error {err:.2e}, norm difference {dnorm:.2e}")
    assert info["iterations"] == it_orc
    assert hdiff <= 1e-12
    assert err <= 1e-10
    assert dnorm <= 1e-10

    x32, info32 = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32)
    err32 = float(np.abs(x32[sel].cpu().numpy() - u).max() / np.abs(u).max())
    log(f"[{name}] float32-MG: {info32['iterations']} iterations (oracle float64 {it_orc}, float32 "
        f"{g['iterations_fp32']}), relres {info32['relres']:.2e}, sampled error {err32:.2e}")
    assert info32["relres"] <= 1e-8
    assert abs(info32["iterations"] - it_orc) <= 1
    assert abs(info32["iterations"] - int(g["iterations_fp32"])) <= 1
    assert err32 <= 1e-6
    H.close()
