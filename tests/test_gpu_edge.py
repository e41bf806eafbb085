"""Degenerate and edge cases on the GPU, against the oracle where there is
something to compare: single-cell meshes, levels whose every DoF is
constrained (empty free set, empty transfers), meshes one cell thick (the
operator's x-runs shorter than a block, padding in every block), a
one-level hierarchy (the exact coarse solve as the preconditioner: CG stops
after one iteration), zero and out-of-range right-hand-side counts.
"""

import numpy as np
import pytest
import torch

from workloads import config_source, dirichlet_face, perturb_interior, random_vector, structured_box, structured_brick

from _parity import DEV, Pair, oracle_prolongation, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (3, 1), (3, 2), (3, 4)])
def test_single_cell(ctx, dim, k):
    """One cell with every boundary face Dirichlet: only the (k-1)^d interior
    nodes are free (none for Q1: an empty free set, an empty transfer, the
    identity operator).  The operator matches the oracle with and without the
    Dirichlet marks; a one-level solve of a zero right-hand side stops at
    iteration 0 and of a bump source after one iteration (exact coarse solve)."""
    import paper_2412_10910_amd as nn
    m = structured_box(dim, 1, 0.0, 1.0)
    p = Pair(ctx, m, k)
    assert p.lib.n_free == (k - 1) ** dim
    x = random_vector(p.orc.n_dofs, 3)
    assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x))), p.A @ x) <= 1e-12
    if k == 1:
        xt = torch.tensor(x, device=DEV)
        assert torch.equal(p.lib.vmult(xt), xt)
    H = nn.Hierarchy(ctx, [p.lib], [])
    xs, info = H.pcg_solve(torch.zeros(p.lib.n_dofs, dtype=torch.float64, device=DEV))
    assert info["iterations"] == 0 and info["status"] == "OK" and float(xs.abs().max()) == 0.0
    if k > 1:
        b = p.lib.assemble_rhs(torch.tensor(config_source(1)(p.lib.quadrature_points()), device=DEV).reshape(-1)) \
            if dim == 3 else p.to_lib(np.where(p.free, 1.0, 0.0))
        _, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float64)
        assert info["iterations"] == 1 and info["relres"] <= 1e-8
        # nested transfer to Q1 on the same cell: the coarse space has no free DoF
        coarse = Pair(ctx, m, 1)
        tr = nn.Transfer(ctx, p.lib, coarse.lib)
        assert tr.points()["owner"].size == (k - 1) ** dim
        out = tr.prolongate(torch.ones(coarse.lib.n_dofs, dtype=torch.float64, device=DEV),
                            torch.zeros(p.lib.n_dofs, dtype=torch.float64, device=DEV))
        assert float(out.abs().max()) == 0.0
    m.dirichlet[:] = 0
    q = Pair(ctx, m, k)
    y = q.to_orc(q.lib.vmult(q.to_lib(random_vector(q.orc.n_dofs, 4))))
    assert rel_err(y, q.A @ random_vector(q.orc.n_dofs, 4)) <= 1e-12


@pytest.mark.parametrize("cells", [(1, 5, 4), (2, 3, 3), (13, 1, 2)])
def test_thin_meshes(ctx, cells):
    """Meshes one or two cells thick: x-runs shorter than a block of the
    operator, so blocks mix rows and hold padding."""
    import paper_2412_10910_amd as nn
    hi = tuple(0.3 * c for c in cells)
    m = structured_brick(cells, (0.0, 0.0, 0.0), hi)
    m = perturb_interior(m, 0.2, [hi[a] / cells[a] for a in range(3)], np.random.default_rng(sum(cells)))
    m.dirichlet[:] = 0
    m = dirichlet_face(m, 2, 0.0)
    for k in (1, 2, 3):
        p = Pair(ctx, m, k)
        x = random_vector(p.orc.n_dofs, 8)
        for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
            assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x, dt))), p.A @ x) <= tol, (k, dt)
    f, c = Pair(ctx, m, 3), Pair(ctx, m, 2)
    tr = nn.Transfer(ctx, f.lib, c.lib, nested_p=0)
    P = oracle_prolongation(f, c)
    v = np.where(c.free, random_vector(c.orc.n_dofs, 9), 0.0)
    out = f.to_orc(tr.prolongate(c.to_lib(v), torch.zeros(f.lib.n_dofs, dtype=torch.float64, device=DEV)))
    assert rel_err(out, P @ v) <= 1e-12


def test_one_level_hierarchy_is_an_exact_solve(ctx):
    """With one level the preconditioner is the exact coarse solve: CG
    reaches the tolerance in one iteration, in both V-cycle precisions (the
    float32 cycle rounds r and z, so it needs at most three)."""
    import paper_2412_10910_amd as nn
    from workloads import config_levels
    (m,) = config_levels(1, cells=[4])
    lv = nn.Level.from_mesh(ctx, m, 2)
    H = nn.Hierarchy(ctx, [lv], [])
    b = lv.assemble_rhs(torch.tensor(config_source(1)(lv.quadrature_points()), device=DEV).reshape(-1))
    _, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float64)
    assert info["iterations"] == 1 and info["relres"] <= 1e-8
    _, info32 = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32)
    assert info32["iterations"] <= 3 and info32["relres"] <= 1e-8


def test_rhs_counts_out_of_range(ctx):
    import paper_2412_10910_amd as nn
    from workloads import config_levels
    (m,) = config_levels(1, cells=[3])
    lv = nn.Level.from_mesh(ctx, m, 2)
    H = nn.Hierarchy(ctx, [lv], [])
    for nr in (0, 9):
        X = torch.zeros(lv.n_dofs, nr, dtype=torch.float64, device=DEV)
        with pytest.raises(nn.NNMGError):
            lv.vmult(X)
        with pytest.raises(nn.NNMGError):
            H.vcycle(X)


@pytest.mark.parametrize("cells", [(1, 1, 1), (1, 5, 4), (2, 3, 3), (13, 1, 2)])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_operator_variants_on_edge_meshes(ctx, cells, dirichlet):
    """Every operator variant (per-node or entity-compressed indices, base or
    transposed sweeps, trilinear or stored geometry) on single cells and on
    meshes one or two cells thick, where x-runs are shorter than a block and
    many entities are constrained or shared by few cells."""
    hi = tuple(0.3 * c for c in cells)
    m = structured_brick(cells, (0.0, 0.0, 0.0), hi)
    m = perturb_interior(m, 0.2, [hi[a] / cells[a] for a in range(3)], np.random.default_rng(7 + sum(cells)))
    if not dirichlet:
        m.dirichlet[:] = 0
    for k in (3, 4):
        p = Pair(ctx, m, k)
        x = random_vector(p.orc.n_dofs, 9)
        ref = p.A @ x
        for v in (0, 2, 4, 5, 6, 8, 10, 11):
            p.lib.set_variant(v)
            for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
                assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x, dt))), ref) <= tol, (k, v, dt)
