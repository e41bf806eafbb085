"""Polynomial coarsening on the coarsest mesh (paper §2, Coarse grid solvers):
the nested polynomial transfer against the oracle's P (built by point
location, the definition P_ij = phi_j(x_i)), and V-cycles and PCG of
hierarchies whose coarsest mesh carries degrees 1..k against the oracle.

Bars: float64 1e-12 and float32 2e-5 relative to the largest reference
entry (the transfer is the same interpolation as the located one, by sum
factorization); V-cycles 1e-12 (max(1e-12, kappa 1e-15) for elasticity);
PCG with the oracle's iteration count and residual history.
"""

import numpy as np
import pytest
import torch

from workloads import config_levels, config_source, dirichlet_face, perturb_interior, random_vector, scramble
from workloads import structured_box, structured_brick

from _parity import DEV, Pair, eig_starts, oracle_hierarchy, oracle_prolongation, rel_err

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 2e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _mesh(dim, n, seed, scram):
    m = structured_box(dim, n, 0.0, 1.0)
    m = perturb_interior(m, 0.2, 1.0 / n, np.random.default_rng(seed))
    if scram:
        m = scramble(m, np.random.default_rng(seed + 1))
    return m


CASES = [(2, 5, 2, 1, False), (2, 4, 4, 3, True), (3, 3, 2, 1, True), (3, 3, 3, 2, False), (3, 2, 4, 3, True),
         (3, 2, 4, 2, False)]


@pytest.mark.parametrize("dim,n,kf,kc,scram", CASES)
def test_nested_transfer_matches_oracle(ctx, dim, n, kf, kc, scram):
    import paper_2412_10910_amd as nn
    m = _mesh(dim, n, 10 * kf + kc, scram)
    f, c = Pair(ctx, m, kf), Pair(ctx, m, kc)
    tr = nn.Transfer(ctx, f.lib, c.lib)
    general = nn.Transfer(ctx, f.lib, c.lib, nested_p=0)
    P = oracle_prolongation(f, c)
    vc = np.where(c.free, random_vector(c.orc.n_dofs, 5), 0.0)
    rf = np.where(f.free, random_vector(f.orc.n_dofs, 6), 0.0)
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        for t in (tr, general):
            out = f.to_orc(t.prolongate(c.to_lib(vc, dt), torch.zeros(f.lib.n_dofs, dtype=dt, device=DEV)))
            assert rel_err(out, P @ vc) <= tol
            rc = c.to_orc(t.restrict(f.to_lib(rf, dt), torch.zeros(c.lib.n_dofs, dtype=dt, device=DEV)))
            assert rel_err(rc, P.T @ rf) <= tol
    # several right-hand sides at once equal the single calls bitwise
    V = torch.stack([c.to_lib(np.where(c.free, random_vector(c.orc.n_dofs, 20 + r), 0.0)) for r in range(3)],
                    dim=1).contiguous()
    F = tr.prolongate(V, torch.zeros(f.lib.n_dofs, 3, dtype=torch.float64, device=DEV))
    R = tr.restrict(F, torch.zeros(c.lib.n_dofs, 3, dtype=torch.float64, device=DEV))
    for r in range(3):
        fr = tr.prolongate(V[:, r].contiguous(), torch.zeros(f.lib.n_dofs, dtype=torch.float64, device=DEV))
        assert torch.equal(F[:, r], fr)
        assert torch.equal(R[:, r], tr.restrict(fr, torch.zeros(c.lib.n_dofs, dtype=torch.float64, device=DEV)))


def test_nested_points_are_the_fine_support_points(ctx):
    """The recorded owner and reference position of every point map back to its fine support point."""
    import paper_2412_10910_amd as nn
    from oracle import space
    m = _mesh(3, 3, 77, True)
    f, c = Pair(ctx, m, 3), Pair(ctx, m, 2)
    pts = nn.Transfer(ctx, f.lib, c.lib).points()
    assert pts["n_projected"] == 0
    V = space.Space(m, 2)
    sup = f.lib.support_points()
    for i in range(0, len(pts["owner"]), 7):
        xi = pts["xi"][i][None, :]
        xq = V.map_points(xi, np.array([pts["owner"][i]]))[0, 0]
        assert np.abs(xq - sup[pts["fine_dof"][i]]).max() <= 1e-13


def test_elasticity_nested_transfer(ctx):
    import paper_2412_10910_amd as nn
    m = structured_brick((3, 2, 2), (0.0, 0.0, 0.0), (2.0, 1.0, 1.0))
    m = dirichlet_face(perturb_interior(m, 0.2, [2 / 3, 0.5, 0.5], np.random.default_rng(4)), 0, 0.0)
    f, c = Pair(ctx, m, 2, "elasticity"), Pair(ctx, m, 1, "elasticity")
    tr = nn.Transfer(ctx, f.lib, c.lib)
    P = oracle_prolongation(f, c)
    vc = np.where(c.free, random_vector(c.orc.n_dofs * 3, 8), 0.0)
    rf = np.where(f.free, random_vector(f.orc.n_dofs * 3, 9), 0.0)
    out = f.to_orc(tr.prolongate(c.to_lib(vc), torch.zeros(f.lib.n_dofs, dtype=torch.float64, device=DEV)))
    assert rel_err(out, P @ vc) <= TOL64
    rc = c.to_orc(tr.restrict(f.to_lib(rf), torch.zeros(c.lib.n_dofs, dtype=torch.float64, device=DEV)))
    assert rel_err(rc, P.T @ rf) <= TOL64


@pytest.mark.parametrize("cfg,cells,k", [(1, [3, 7], 2), ("2p3", [3, 6], 3), ("2p4", [3, 5], 4)])
def test_pmg_vcycle_and_pcg(ctx, cfg, cells, k):
    """Degrees 1..k on the coarsest mesh, then the non-nested mesh levels: the
    V-cycle and PCG match the oracle's hierarchy built from the same levels."""
    import paper_2412_10910_amd as nn
    meshes = config_levels(cfg, cells=cells)
    specs = [(meshes[0], d) for d in range(1, k)] + [(m, k) for m in meshes]
    pairs = [Pair(ctx, m, d) for m, d in specs]
    starts = eig_starts(pairs)
    H_orc = oracle_hierarchy(pairs, starts)
    levels, transfers = nn.build_levels(ctx, meshes, k, p_coarsening=True)
    assert [lv.degree for lv in levels] == [d for _, d in specs]
    H = nn.Hierarchy(ctx, [p.lib for p in pairs],
                     [nn.Transfer(ctx, pairs[i + 1].lib, pairs[i].lib) for i in range(len(pairs) - 1)],
                     eig_start=[p.to_lib(s) for p, s in zip(pairs, starts)])
    for l in range(1, len(pairs)):
        H.set_cheb_bounds(l, *H_orc.bounds[l])
    fine = pairs[-1]
    r = np.where(fine.free, random_vector(fine.orc.n_dofs, 31), 0.0)
    assert rel_err(fine.to_orc(H.vcycle(fine.to_lib(r))), H_orc.vcycle(r)) <= 1e-12
    from oracle import assemble
    src = config_source(cfg)
    b_orc = assemble.load_vector(fine.orc, src)
    b = fine.lib.assemble_rhs(torch.tensor(src(fine.lib.quadrature_points()), device=DEV).reshape(-1))
    x_orc, it_orc, hist_orc = H_orc.pcg(b_orc, rtol=1e-8)
    x, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float64)
    assert info["iterations"] == it_orc
    assert np.abs(info["history"] - np.array(hist_orc)).max() <= 1e-12
    x32, info32 = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32)
    assert info32["relres"] <= 1e-8 and abs(info32["iterations"] - it_orc) <= 1
    # the helper's hierarchy (its own Lanczos bounds) converges as well
    H2 = nn.Hierarchy(ctx, levels, transfers)
    _, info2 = H2.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32)
    assert info2["status"] == "OK" and info2["iterations"] <= it_orc + 2
