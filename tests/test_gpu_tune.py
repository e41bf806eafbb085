"""The autotuner: every operator variant, both cells-per-workgroup sizes and
every restriction team size must give the oracle's result (float64 within 1e-12, float32 within 2e-5 of the
largest entry; the variants only reorder floating-point sums), tuning must
keep the fastest variant it timed, and a hierarchy must re-capture its V-cycle
graph when a variant under it changes.
"""

import numpy as np
import pytest
import torch

from workloads import config_levels, config_source, random_vector

from _parity import DEV, Pair, oracle_prolongation, rel_err

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 2e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


@pytest.mark.parametrize("cfg,cells,k", [(0, [13], 1), (1, [5], 2), (2, [4], 3), (2, [3], 4)])
def test_operator_variants_match_oracle(ctx, cfg, cells, k):
    (m,) = config_levels(cfg, cells=cells)
    p = Pair(ctx, m, k)
    x = random_vector(p.orc.n_dofs, 5)
    ref = p.A @ x
    variants = [0, 1, 2, 3, 6, 8] + ([4, 5, 10, 11] if (k >= 3 and p.lib.dim == 3) else [])
    for v in variants:
        p.lib.set_variant(v)
        assert p.lib.variant == v
        for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
            assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x, dt))), ref) <= tol, (v, dt)


@pytest.mark.parametrize("cfg,cells,k", [(0, [13], 1), (0, [9], 4), (1, [5], 2), (1, [4], 1), (1, [3], 2),
                                         (2, [4], 3), (2, [3], 4), (2, [5], 4)])
def test_two_layout_blocks_per_workgroup(ctx, cfg, cells, k):
    """Cells per workgroup: a workgroup of two layout blocks gives the oracle's
    product, and bitwise the product of one layout block per workgroup, for
    every slot variant, with one and with three right-hand sides (looping and
    split); the cases include odd numbers of layout blocks (the last
    workgroup then has a block past the end, which must store nothing)."""
    (m,) = config_levels(cfg, cells=cells)
    p = Pair(ctx, m, k)
    x = random_vector(p.orc.n_dofs, 5)
    ref = p.A @ x
    cells1, base, nblk = p.lib.cells_per_block()
    assert cells1 == base and nblk >= 1
    variants = [0, 2, 6, 8] + ([4, 5, 10, 11] if (k >= 3 and p.lib.dim == 3) else [])
    for v in variants:
        p.lib.set_variant(v)
        for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
            xl = p.to_lib(x, dt)
            X = torch.stack([p.to_lib(random_vector(p.orc.n_dofs, 30 + r), dt) for r in range(3)], 1).contiguous()
            p.lib.set_cells_per_block(base, dt)
            y1 = p.lib.vmult(xl)
            Y1 = p.lib.vmult(X)
            p.lib.set_cells_per_block(2 * base, dt)
            assert p.lib.cells_per_block(dt)[0] == 2 * base
            y2 = p.lib.vmult(xl)
            assert torch.equal(y1, y2), (v, dt, nblk)
            assert rel_err(p.to_orc(y2), ref) <= tol, (v, dt)
            for split in (False, True):
                p.lib.set_rhs_split(split, dt)
                assert torch.equal(p.lib.vmult(X), Y1), (v, dt, split)
            p.lib.set_rhs_split(False, dt)
            p.lib.set_cells_per_block(base, dt)
    # the other sizes are refused; the atomic variants run one block and say so
    import paper_2412_10910_amd as nn
    for bad in (base + 1, 3 * base, 0):
        with pytest.raises(nn.NNMGError):
            p.lib.set_cells_per_block(bad)
    p.lib.set_cells_per_block(2 * base)
    p.lib.set_variant(1)
    assert p.lib.cells_per_block()[0] == base
    p.lib.set_variant(0)
    assert p.lib.cells_per_block()[0] == 2 * base
    p.lib.set_cells_per_block(base)


def test_elasticity_runs_one_layout_block_per_workgroup(ctx):
    import paper_2412_10910_amd as nn
    (m,) = config_levels(3, cells=[(3, 1, 1)])
    lv = nn.Level.from_mesh(ctx, m, 2, "elasticity")
    c, base, _ = lv.cells_per_block()
    assert c == base
    with pytest.raises(nn.NNMGError):
        lv.set_cells_per_block(2 * base)


@pytest.mark.parametrize("cfg,cells,k", [(1, [3, 7], 2), (2, [3, 6], 3), (3, [(3, 1, 1), (7, 2, 2)], 2)])
def test_restriction_teams_match_oracle(ctx, cfg, cells, k):
    import paper_2412_10910_amd as nn
    op = "elasticity" if cfg == 3 else "laplace"
    cm, fm = config_levels(cfg, cells=cells)
    f, c = Pair(ctx, fm, k, op), Pair(ctx, cm, k, op)
    tr = nn.Transfer(ctx, f.lib, c.lib)
    P = oracle_prolongation(f, c)
    rf = np.where(f.free, random_vector(f.orc.n_dofs * f.nc, 6), 0.0)
    ref = P.T @ rf
    for team in (4, 8, 16, 32, 64):
        tr.set_team(team)
        assert tr.team == team
        for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
            out = c.to_orc(tr.restrict(f.to_lib(rf, dt), torch.zeros(c.lib.n_dofs, dtype=dt, device=DEV)))
            assert rel_err(out, ref) <= tol, (team, dt)


def test_tune_keeps_the_fastest_and_the_solver_still_converges(ctx):
    import paper_2412_10910_amd as nn
    meshes = config_levels(1, cells=[3, 6, 13, 29])
    levels = [nn.Level.from_mesh(ctx, m, 2) for m in meshes]
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    H = nn.Hierarchy(ctx, levels, transfers)
    fine = levels[-1]
    b = fine.assemble_rhs(torch.tensor(config_source(1)(fine.quadrature_points()), device=DEV).reshape(-1))
    _, before = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32)
    report = H.tune(torch.float32, reps=5)
    for lv, r in zip(levels, report["levels"]):
        ms = r["ms"]
        # the float-atomic variants are not reproducible and never timed
        assert set(ms) == {"trilinear+slots", "metric+slots", "trilinear+slots+transposed", "metric+slots+transposed"} and all(t > 0 for t in ms.values())
        assert r["chosen"] == min(ms, key=ms.get)
        assert lv.VARIANTS[lv.variant_of(torch.float32)] == r["chosen"]
        # cells per workgroup: both timed for the variant kept, the faster in use
        mc = r["ms_cells"]
        base = lv.cells_per_block(torch.float32)[1]
        assert mc is not None and all(t > 0 for t in mc.values())
        want = 2 * base if mc["two blocks"] < mc["one block"] else base
        assert r["cells_per_block"] == want == lv.cells_per_block(torch.float32)[0]
    for tr, r in zip(transfers, report["transfers"]):
        assert r["chosen"] == min(r["ms"], key=r["ms"].get) and tr.team == r["chosen"]
    for dt in (torch.float32, torch.float64):
        x, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=dt)
        assert info["status"] == "OK" and abs(info["iterations"] - before["iterations"]) <= 1
        true = float((b - fine.vmult(x)).norm() / b.norm())
        assert true <= 1.01e-8


def test_graph_recaptured_after_a_variant_change(ctx):
    """The captured preconditioner bakes in the kernels and buffers of the
    variant in use; after a change the next solve must use the new variant:
    graph and kernel-by-kernel solves agree bitwise (slot variants are
    deterministic)."""
    import paper_2412_10910_amd as nn
    meshes = config_levels(1, cells=[3, 6, 13])
    levels = [nn.Level.from_mesh(ctx, m, 2) for m in meshes]
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    H = nn.Hierarchy(ctx, levels, transfers)
    fine = levels[-1]
    b = fine.assemble_rhs(torch.tensor(config_source(1)(fine.quadrature_points()), device=DEV).reshape(-1))
    H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32)  # captures the graph with variant 0
    for v, team in ((2, 8), (0, 32), (2, 4)):
        fine.set_variant(v)
        transfers[-1].set_team(team)
        xg, ig = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32, use_graph=True)
        xe, ie = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32, use_graph=False)
        assert ig["iterations"] == ie["iterations"]
        assert torch.equal(xg, xe), v


def test_elasticity_has_one_variant(ctx):
    import paper_2412_10910_amd as nn
    (m,) = config_levels(3, cells=[(3, 1, 1)])
    lv = nn.Level.from_mesh(ctx, m, 2, "elasticity")
    with pytest.raises(nn.NNMGError):
        lv.set_variant(1)
    r = lv.tune(torch.float64, reps=3)
    assert list(r["ms"]) == ["trilinear+slots"] and lv.variant == 0
