"""GPU parity of the smoother bounds, the V-cycle and PCG against the oracle.

Bars:
* Chebyshev bounds (Lanczos from the same start vector): relative 1e-10;
* one float64 V-cycle: 1e-12 relative to the largest entry;
* float64-MG PCG: same iteration count, residual histories within 1e-12
  (absolute, the history is already divided by ||b||), solutions within 1e-10
  relative;
* float32-MG PCG (paper §4: V-cycle in single precision, CG in double):
  reaches the 1e-8 tolerance with an iteration count within +-1 of the
  float64 oracle; its error against the float64 oracle solution is below
  100 x the tolerance relative to the solution.
"""

import numpy as np
import pytest
import torch

from oracle import assemble
from workloads import config_levels, config_source, random_vector

from _parity import DEV, build_pairs, eig_starts, oracle_hierarchy, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _setup(ctx, cfg, cells, k):
    import paper_2412_10910_amd as nn
    meshes = config_levels(cfg, cells=cells)
    pairs = build_pairs(ctx, meshes, k)
    starts = eig_starts(pairs)
    H_orc = oracle_hierarchy(pairs, starts)
    transfers = [nn.Transfer(ctx, pairs[i + 1].lib, pairs[i].lib) for i in range(len(pairs) - 1)]
    H_lib = nn.Hierarchy(ctx, [p.lib for p in pairs], transfers,
                         eig_start=[p.to_lib(s) for p, s in zip(pairs, starts)])
    b_orc = assemble.load_vector(pairs[-1].orc, config_source(cfg))
    fine = pairs[-1]
    fq = torch.tensor(config_source(cfg)(fine.lib.quadrature_points()).reshape(-1), dtype=torch.float64, device=DEV)
    b_lib = fine.lib.assemble_rhs(fq)
    assert rel_err(fine.to_orc(b_lib), b_orc) <= 1e-12
    return pairs, H_orc, H_lib, b_orc, b_lib


SETUPS = [
    ("cfg0_full", 0, [9, 23, 64], 1),
    ("cfg1_small", 1, [3, 6, 13], 2),
    ("ball_q3_small", 2, [3, 5, 9], 3),
    ("ball_q4_small", 2, [3, 7], 4),
]


@pytest.mark.parametrize("name,cfg,cells,k", SETUPS, ids=[s[0] for s in SETUPS])
def test_bounds_vcycle_pcg_parity(ctx, name, cfg, cells, k):
    pairs, H_orc, H_lib, b_orc, b_lib = _setup(ctx, cfg, cells, k)
    for l in range(1, len(pairs)):
        lo, hi = H_lib.cheb_bounds(l)
        assert abs(hi - H_orc.bounds[l][1]) <= 1e-10 * H_orc.bounds[l][1]
        assert abs(lo - H_orc.bounds[l][0]) <= 1e-10 * H_orc.bounds[l][0]
        # use identical bounds for the bitwise-comparable parts below
        H_lib.set_cheb_bounds(l, *H_orc.bounds[l])
    fine = pairs[-1]
    r = np.where(fine.orc.free, random_vector(fine.orc.n_dofs, 77), 0.0)
    z = H_lib.vcycle(fine.to_lib(r))
    assert rel_err(fine.to_orc(z), H_orc.vcycle(r)) <= 1e-12
    # float64 multigrid inside float64 CG
    x_orc, it_orc, hist_orc = H_orc.pcg(b_orc, rtol=1e-8)
    x_lib, info = H_lib.pcg_solve(b_lib, rtol=1e-8, vcycle_dtype=torch.float64)
    assert info["iterations"] == it_orc
    assert np.abs(info["history"] - np.array(hist_orc)).max() <= 1e-12
    assert rel_err(fine.to_orc(x_lib), x_orc) <= 1e-10
    # float32 multigrid inside float64 CG
    x32, info32 = H_lib.pcg_solve(b_lib, rtol=1e-8, vcycle_dtype=torch.float32)
    assert info32["relres"] <= 1e-8
    assert abs(info32["iterations"] - it_orc) <= 1
    err = rel_err(fine.to_orc(x32), x_orc)
    assert err <= 1e-6, err


SMOOTHERS = [(1, "slots"), (2, "slots"), (4, "slots"), (2, "atomic"), (3, "atomic")]


@pytest.mark.parametrize("cheb,scatter", SMOOTHERS, ids=[f"degree{c}-{s}" for c, s in SMOOTHERS])
def test_smoother_degree_and_scatter_against_the_oracle(ctx, cheb, scatter):
    """Chebyshev smoothers of degree 1, 2 and 4 (the default is 3), and the
    float-atomic operator with its separate smoothing step: the steps read a
    zero or x in place of the previous direction and do not store the last
    one, which must leave the oracle's V-cycle (1e-12) and float64-MG PCG
    (same iterations, histories within 1e-12) unchanged; float32-MG converges
    within one iteration of it."""
    import paper_2412_10910_amd as nn
    meshes = config_levels(1, cells=[3, 6, 13])
    pairs = build_pairs(ctx, meshes, 2)
    starts = eig_starts(pairs)
    H_orc = oracle_hierarchy(pairs, starts, cheb_degree=cheb)
    if scatter == "atomic":
        for p in pairs:
            p.lib.set_variant(1)  # trilinear geometry, float atomics, both precisions
    transfers = [nn.Transfer(ctx, pairs[i + 1].lib, pairs[i].lib) for i in range(len(pairs) - 1)]
    H_lib = nn.Hierarchy(ctx, [p.lib for p in pairs], transfers,
                         eig_start=[p.to_lib(s) for p, s in zip(pairs, starts)], cheb_degree=cheb)
    for l in range(1, len(pairs)):
        H_lib.set_cheb_bounds(l, *H_orc.bounds[l])
    fine = pairs[-1]
    r = np.where(fine.orc.free, random_vector(fine.orc.n_dofs, 78), 0.0)
    z = H_lib.vcycle(fine.to_lib(r))
    assert rel_err(fine.to_orc(z), H_orc.vcycle(r)) <= 1e-12
    b_orc = assemble.load_vector(fine.orc, config_source(1))
    fq = torch.tensor(config_source(1)(fine.lib.quadrature_points()).reshape(-1), dtype=torch.float64, device=DEV)
    b_lib = fine.lib.assemble_rhs(fq)
    x_orc, it_orc, hist_orc = H_orc.pcg(b_orc, rtol=1e-8)
    x_lib, info = H_lib.pcg_solve(b_lib, rtol=1e-8, vcycle_dtype=torch.float64)
    assert info["iterations"] == it_orc
    assert np.abs(info["history"] - np.array(hist_orc)).max() <= 1e-12
    assert rel_err(fine.to_orc(x_lib), x_orc) <= 1e-10
    x32, info32 = H_lib.pcg_solve(b_lib, rtol=1e-8, vcycle_dtype=torch.float32)
    assert info32["relres"] <= 1e-8
    assert abs(info32["iterations"] - it_orc) <= 1


def test_zero_rhs_and_not_converged(ctx):
    import paper_2412_10910_amd as nn
    pairs, H_orc, H_lib, b_orc, b_lib = _setup(ctx, 0, [4, 9], 1)
    x, info = H_lib.pcg_solve(torch.zeros_like(b_lib))
    assert info["iterations"] == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(nn.NNMGError) as e:
        H_lib.pcg_solve(b_lib, rtol=1e-14, max_it=1)
    assert e.value.name == "NOT_CONVERGED"
    x, info = H_lib.pcg_solve(b_lib, rtol=1e-14, max_it=1, raise_on_failure=False)
    assert info["status"] == "NOT_CONVERGED" and info["iterations"] == 1
    bad = b_lib.clone()
    bad[pairs[-1].lib.constrained().argmin()] = float("nan")
    with pytest.raises(nn.NNMGError) as e:
        H_lib.pcg_solve(bad)
    assert e.value.name == "BREAKDOWN"
    # an infinite entry passes the start (|b| = inf is not NaN) and breaks down
    # at the first p.q (NaN); the returned iterate is the last good one (x0 = 0)
    bad = b_lib.clone()
    bad[pairs[-1].lib.constrained().argmin()] = float("inf")
    x, info = H_lib.pcg_solve(bad, raise_on_failure=False)
    assert info["status"] == "BREAKDOWN" and info["iterations"] == 1
    assert bool(torch.isfinite(x).all()) and float(x.abs().max()) == 0.0


def test_profile_components(ctx):
    pairs, H_orc, H_lib, b_orc, b_lib = _setup(ctx, 1, [3, 6, 13], 2)
    H_lib.set_profiling(True)
    _, info = H_lib.pcg_solve(b_lib)
    ms = H_lib.profile()
    H_lib.set_profiling(False)
    assert ms.shape == (3, 6)
    assert ms[0, 3] > 0 and np.all(ms[1:, [0, 1, 2, 4, 5]] > 0)
    assert np.all(ms[0, [0, 1, 2, 4, 5]] == 0)


def test_graph_replays_match_eager_launches(ctx):
    """The captured preconditioner graph, replayed over several solves with
    eager work and synchronisations in between, gives bitwise the results of
    launching the V-cycle kernel by kernel (both precisions), also after the
    smoother bounds change (which rebuilds the graph)."""
    import paper_2412_10910_amd as nn
    meshes = config_levels(1, cells=[3, 6, 13])
    levels = [nn.Level.from_mesh(ctx, m, 2) for m in meshes]
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    H = nn.Hierarchy(ctx, levels, transfers)
    fine = levels[-1]
    con = torch.tensor(fine.constrained(), device=DEV)
    for rep in range(4):
        if rep == 2:
            lo, hi = H.cheb_bounds(2)
            H.set_cheb_bounds(2, lo * 1.1, hi * 1.05)
        b = torch.tensor(random_vector(fine.n_dofs, 200 + rep), device=DEV)
        b[con] = 0
        for dt in (torch.float64, torch.float32):
            xg, ig = H.pcg_solve(b, rtol=1e-10, vcycle_dtype=dt, use_graph=True)
            y = fine.vmult(b)  # eager work between replays
            torch.cuda.synchronize()
            xe, ie = H.pcg_solve(b, rtol=1e-10, vcycle_dtype=dt, use_graph=False)
            torch.cuda.synchronize()
            assert ig["iterations"] == ie["iterations"]
            assert np.array_equal(ig["history"], ie["history"])
            assert torch.equal(xg, xe)
            assert torch.isfinite(y).all()


@pytest.mark.parametrize("cfg,cells,k", [(0, [9], 1), (1, [6], 2), (2, [3], 3)])
def test_coarse_solve_alone(ctx, cfg, cells, k):
    """With one level the V-cycle is the coarse solve: A^{-1} r (float64, one
    refinement step) against a dense solve of the oracle's reduced system,
    and the float32 V-cycle (float64 inverse applied once, float32 input and
    output)."""
    import paper_2412_10910_amd as nn
    from _parity import Pair
    (m,) = config_levels(cfg, cells=cells)
    p = Pair(ctx, m, k)
    H = nn.Hierarchy(ctx, [p.lib], [])
    free = p.orc.free
    r = np.where(free, random_vector(p.orc.n_dofs, 91), 0.0)
    A = p.A.toarray()
    expect = np.zeros_like(r)
    expect[free] = np.linalg.solve(A[np.ix_(free, free)], r[free])
    z = p.to_orc(H.vcycle(p.to_lib(r)))
    assert rel_err(z, expect) <= 1e-12
    assert np.all(z[~free] == 0)
    # float32 V-cycle: the input is rounded to float32, the solve is float64,
    # the output is rounded to float32 (one rounding, 6e-8 relative)
    r32 = r.astype(np.float32).astype(np.float64)
    expect32 = np.zeros_like(r)
    expect32[free] = np.linalg.solve(A[np.ix_(free, free)], r32[free])
    z32 = p.to_orc(H.vcycle(p.to_lib(r, torch.float32)))
    assert rel_err(z32, expect32) <= 2e-7
