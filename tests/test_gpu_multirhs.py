"""Several right-hand sides in one launch (interleaved [DoF][nrhs] vectors).

Every fused call must give, for each right-hand side, exactly what the
single-vector call gives on that right-hand side alone: the fused kernels
carry out the same arithmetic in the same order per right-hand side, so the
comparison is bitwise (operator, transfers, V-cycle, and the iterates and
iteration counts of PCG, where a converged right-hand side is frozen while
the others go on).  The single-vector path is itself pinned to the oracle by
the other GPU tests; one direct oracle comparison of the fused PCG is made
here as well, and the beam workload with four loads is solved at full size.
"""

import numpy as np
import pytest
import torch

from workloads import config_levels, config_source, random_load, random_vector

from _parity import DEV, Pair, eig_starts, oracle_hierarchy, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _columns(n, nr, seed, dtype=torch.float64, mask=None):
    cols = [random_vector(n, seed + r) for r in range(nr)]
    if mask is not None:
        cols = [np.where(mask, c, 0.0) for c in cols]
    return torch.tensor(np.stack(cols, axis=1), dtype=dtype, device=DEV).contiguous()


def _same(a: torch.Tensor, b: torch.Tensor):
    assert a.dtype == b.dtype and a.shape == b.shape
    assert torch.equal(a, b), f"max difference {float((a.double() - b.double()).abs().max()):.3e}"


@pytest.mark.parametrize("operator,cfg,cells,k", [("laplace", 1, [5, 11], 2), ("laplace", 2, [3, 7], 3),
                                                  ("laplace", 0, [6, 13], 1), ("elasticity", 3, [(3, 1, 1), (7, 2, 2)], 2)])
@pytest.mark.parametrize("nr", [2, 3, 8])
@pytest.mark.parametrize("split", [False, True], ids=["loop", "split"])
def test_operator_and_transfers_match_single(ctx, operator, cfg, cells, k, nr, split):
    """split: one row of workgroups per right-hand side instead of a loop."""
    import paper_2412_10910_amd as nn
    coarse_m, fine_m = config_levels(cfg, cells=cells)
    fine = nn.Level.from_mesh(ctx, fine_m, k, operator)
    coarse = nn.Level.from_mesh(ctx, coarse_m, k, operator)
    for dt in (torch.float64, torch.float32):
        fine.set_rhs_split(split, dt)
    tr = nn.Transfer(ctx, fine, coarse)
    for dt in (torch.float64, torch.float32):
        X = _columns(fine.n_dofs, nr, 11, dt)
        Y = fine.vmult(X)
        for r in range(nr):
            _same(Y[:, r], fine.vmult(X[:, r].contiguous()))
        Z = torch.ones_like(X)
        fine.vmult_add(X, Z)
        for r in range(nr):
            z = torch.ones(fine.n_dofs, dtype=dt, device=DEV)
            _same(Z[:, r], fine.vmult_add(X[:, r].contiguous(), z))
        cmask = ~coarse.constrained()
        V = _columns(coarse.n_dofs, nr, 21, dt, cmask)
        P = tr.prolongate(V, torch.zeros(fine.n_dofs, nr, dtype=dt, device=DEV))
        R = tr.restrict(X, torch.zeros(coarse.n_dofs, nr, dtype=dt, device=DEV))
        for r in range(nr):
            _same(P[:, r], tr.prolongate(V[:, r].contiguous(), torch.zeros(fine.n_dofs, dtype=dt, device=DEV)))
            _same(R[:, r], tr.restrict(X[:, r].contiguous(), torch.zeros(coarse.n_dofs, dtype=dt, device=DEV)))


def _hierarchy(ctx, cfg, cells, k, operator="laplace"):
    import paper_2412_10910_amd as nn
    meshes = config_levels(cfg, cells=cells)
    levels = [nn.Level.from_mesh(ctx, m, k, operator) for m in meshes]
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    return nn.Hierarchy(ctx, levels, transfers), levels


@pytest.mark.parametrize("operator,cfg,cells,k", [("laplace", 1, [3, 6, 13], 2),
                                                  ("elasticity", 3, [(3, 1, 1), (7, 2, 2), (14, 3, 3)], 2)])
@pytest.mark.parametrize("split", [False, True], ids=["loop", "split"])
def test_vcycle_and_pcg_match_single(ctx, operator, cfg, cells, k, split):
    H, levels = _hierarchy(ctx, cfg, cells, k, operator)
    for lv in levels:
        for dt in (torch.float64, torch.float32):
            lv.set_rhs_split(split, dt)
    fine = levels[-1]
    free = ~fine.constrained()
    nr = 4
    R = _columns(fine.n_dofs, nr, 31, mask=free)
    for dt in (torch.float64, torch.float32):
        Z = H.vcycle(R.to(dt))
        for r in range(nr):
            _same(Z[:, r], H.vcycle(R[:, r].to(dt).contiguous()))
    # right-hand sides of different difficulty, one of them zero
    B = torch.zeros(fine.n_dofs, nr, dtype=torch.float64, device=DEV)
    q = torch.tensor(random_load(3)(fine.quadrature_points()) if operator == "elasticity"
                     else config_source(cfg)(fine.quadrature_points()), device=DEV).reshape(-1)
    B[:, 0] = fine.assemble_rhs(q)
    B[:, 1] = R[:, 1]
    B[:, 3] = R[:, 3] * 1e-3 + B[:, 0]
    for dt in (torch.float64, torch.float32):
        for graph in (True, False):
            X, infos = H.pcg_solve(B, rtol=1e-8, vcycle_dtype=dt, use_graph=graph)
            assert [i["status"] for i in infos] == ["OK"] * nr
            assert infos[2]["iterations"] == 0 and float(X[:, 2].abs().max()) == 0.0
            for r in range(nr):
                x, info = H.pcg_solve(B[:, r].contiguous(), rtol=1e-8, vcycle_dtype=dt, use_graph=graph)
                assert info["iterations"] == infos[r]["iterations"], (dt, graph, r)
                assert np.array_equal(info["history"], infos[r]["history"])
                _same(X[:, r], x)


def test_pcg_multi_against_oracle(ctx):
    """The fused float64-MG PCG against the oracle's PCG, right-hand side by
    right-hand side: same iteration counts, residual histories within 1e-12."""
    import paper_2412_10910_amd as nn
    meshes = config_levels(1, cells=[3, 6, 13])
    pairs = [Pair(ctx, m, 2) for m in meshes]
    starts = eig_starts(pairs)
    H_orc = oracle_hierarchy(pairs, starts)
    transfers = [nn.Transfer(ctx, pairs[i + 1].lib, pairs[i].lib) for i in range(len(pairs) - 1)]
    H = nn.Hierarchy(ctx, [p.lib for p in pairs], transfers, eig_start=[p.to_lib(s) for p, s in zip(pairs, starts)])
    for l in range(1, len(pairs)):
        H.set_cheb_bounds(l, *H_orc.bounds[l])
    fine = pairs[-1]
    nr = 3
    bs = [np.where(fine.free, random_vector(fine.orc.n_dofs, 400 + r), 0.0) for r in range(nr)]
    B = torch.stack([fine.to_lib(b) for b in bs], dim=1).contiguous()
    X, infos = H.pcg_solve(B, rtol=1e-8, vcycle_dtype=torch.float64)
    for r in range(nr):
        x_orc, it_orc, hist_orc = H_orc.pcg(bs[r], rtol=1e-8)
        assert infos[r]["iterations"] == it_orc
        assert np.abs(infos[r]["history"] - np.array(hist_orc)).max() <= 1e-12
        assert rel_err(fine.to_orc(X[:, r]), x_orc) <= 1e-10


def test_bad_rhs_counts(ctx):
    import paper_2412_10910_amd as nn
    H, levels = _hierarchy(ctx, 1, [3, 6], 2)
    fine = levels[-1]
    for nr in (9, 12):
        X = torch.zeros(fine.n_dofs, nr, dtype=torch.float64, device=DEV)
        with pytest.raises(nn.NNMGError):
            fine.vmult(X)
        with pytest.raises(nn.NNMGError):
            H.vcycle(X)
        with pytest.raises(nn.NNMGError):
            H.pcg_solve(X)


def test_beam_four_loads_full_size(ctx):
    """The beam workload at full size (525,987 DoFs) with the gravity load and
    three random loads fused: every solve reaches 1e-8 in both V-cycle
    precisions with the iterations of its single solve, and the float32-MG
    columns equal their single solves bitwise."""
    H, levels = _hierarchy(ctx, 3, None, 2, "elasticity")
    fine = levels[-1]
    assert fine.n_dofs == 525987
    pts = fine.quadrature_points()
    srcs = [config_source(3)] + [random_load(i) for i in (1, 2, 3)]
    B = torch.stack([fine.assemble_rhs(torch.tensor(f(pts), device=DEV).reshape(-1)) for f in srcs],
                    dim=1).contiguous()
    for dt in (torch.float32, torch.float64):
        X, infos = H.pcg_solve(B, rtol=1e-8, vcycle_dtype=dt)
        for r, info in enumerate(infos):
            b = B[:, r].contiguous()
            true = float((b - fine.vmult(X[:, r].contiguous())).norm() / b.norm())
            assert info["relres"] <= 1e-8 and true <= 1.01e-8, (dt, r, info, true)
            x, single = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=dt)
            assert single["iterations"] == info["iterations"]
            if dt == torch.float32:
                _same(X[:, r], x)
