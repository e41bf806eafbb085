"""GPU parity of the linear elasticity path (paper §4, Applications to FEA)
against the oracle: operator, diagonal, load vector, transfers, V-cycle and
PCG, on small perturbed and scrambled meshes and on the beam workload.

Bars as for the Laplace path: float64 within 1e-12 relative to the largest
reference entry, float32 within 2e-5; float64-MG PCG with the same iteration
count and residual history within 1e-12; float32-MG within +-1 iteration.
"""

import numpy as np
import pytest
import torch

from oracle import elasticity
from workloads import config_levels, config_source, dirichlet_face, perturb_interior, random_load, random_vector
from workloads import scramble, structured_brick

from _parity import DEV, Pair, eig_starts, oracle_hierarchy, oracle_prolongation, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _brick(cells, hi, alpha, seed, scram, clamp=True):
    m = structured_brick(cells, (0.0, 0.0, 0.0), hi)
    m = perturb_interior(m, alpha, [hi[a] / cells[a] for a in range(3)], np.random.default_rng(seed))
    if clamp:
        m = dirichlet_face(m, 0, 0.0)
    else:
        m.dirichlet[:] = 0  # free boundary everywhere
    if scram:
        m = scramble(m, np.random.default_rng(seed + 1))
    return m


CASES = [(1, (5, 3, 2), False), (2, (4, 3, 2), True), (2, (7, 2, 2), False), (3, (3, 2, 2), True),
         (4, (2, 2, 2), False)]


@pytest.mark.parametrize("k,cells,scram", CASES)
def test_operator_diagonal_rhs(ctx, k, cells, scram):
    m = _brick(cells, (2.0, 1.0, 0.8), 0.2, 40 + k, scram)
    p = Pair(ctx, m, k, "elasticity")
    A = p.A
    x = random_vector(p.orc.n_dofs * 3, 3)
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        y = p.to_orc(p.lib.vmult(p.to_lib(x, dt)))
        assert rel_err(y, A @ x) <= tol, (k, dt)
    assert rel_err(p.to_orc(p.lib.diagonal()), A.diagonal()) <= TOL64
    # load vector of a smooth random body force
    f = random_load(7)
    fq = torch.tensor(f(p.lib.quadrature_points()).reshape(-1), device=DEV)
    b = p.to_orc(p.lib.assemble_rhs(fq))
    assert rel_err(b, elasticity.load_vector(p.orc, f)) <= TOL64


def test_rigid_motion_in_kernel_without_clamp(ctx):
    """With no clamped face, A applied to a rigid-body motion vanishes on the GPU too."""
    m = _brick((3, 3, 2), (1.0, 1.0, 0.6), 0.2, 77, True, clamp=False)
    p = Pair(ctx, m, 2, "elasticity")
    for r in elasticity.rigid_body_modes(p.orc):
        y = p.to_orc(p.lib.vmult(p.to_lib(r)))
        assert np.abs(y).max() <= 1e-12 * np.abs(p.A).max() * np.abs(r).max()


@pytest.mark.parametrize("k", [2, 3])
def test_transfer(ctx, k):
    import paper_2412_10910_amd as nn
    fm = _brick((7, 3, 3), (2.0, 1.0, 1.0), 0.2, 50 + k, True)
    cm = _brick((3, 2, 2), (2.0, 1.0, 1.0), 0.2, 60 + k, False)
    f, c = Pair(ctx, fm, k, "elasticity"), Pair(ctx, cm, k, "elasticity")
    tr = nn.Transfer(ctx, f.lib, c.lib)
    P = oracle_prolongation(f, c)
    vc = np.where(c.free, random_vector(c.orc.n_dofs * 3, 5), 0.0)
    rf = np.where(f.free, random_vector(f.orc.n_dofs * 3, 6), 0.0)
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        out = f.to_orc(tr.prolongate(c.to_lib(vc, dt), f.to_lib(np.zeros(f.orc.n_dofs * 3), dt)))
        assert rel_err(out, P @ vc) <= tol
        rc = c.to_orc(tr.restrict(f.to_lib(rf, dt), c.to_lib(np.zeros(c.orc.n_dofs * 3), dt)))
        assert rel_err(rc, P.T @ rf) <= tol


def test_beam_vcycle_and_pcg(ctx):
    import paper_2412_10910_amd as nn
    meshes = config_levels(3, cells=[(5, 1, 1), (10, 2, 2), (20, 4, 4)])
    pairs = [Pair(ctx, m, 2, "elasticity") for m in meshes]
    starts = eig_starts(pairs)
    H_orc = oracle_hierarchy(pairs, starts)
    transfers = [nn.Transfer(ctx, pairs[i + 1].lib, pairs[i].lib) for i in range(len(pairs) - 1)]
    H = nn.Hierarchy(ctx, [p.lib for p in pairs], transfers, eig_start=[p.to_lib(s) for p, s in zip(pairs, starts)])
    for l in range(1, len(pairs)):
        lo, hi = H.cheb_bounds(l)
        assert abs(hi - H_orc.bounds[l][1]) <= 1e-10 * H_orc.bounds[l][1]
        H.set_cheb_bounds(l, *H_orc.bounds[l])
    fine = pairs[-1]
    r = np.where(fine.free, random_vector(fine.orc.n_dofs * 3, 77), 0.0)
    # The exact coarse solve amplifies the rounding differences between the two
    # assembled coarse operators (entries summed in different orders, ~1e-15
    # relative) by the coarse condition number, which is large for a clamped
    # beam: the V-cycle bar is max(1e-12, kappa * 1e-15).
    A0 = pairs[0].A.toarray()[np.ix_(pairs[0].free, pairs[0].free)]
    ev = np.linalg.eigvalsh(A0)
    kappa = ev[-1] / ev[0]
    tol_v = max(1e-12, kappa * 1e-15)
    assert rel_err(fine.to_orc(H.vcycle(fine.to_lib(r))), H_orc.vcycle(r)) <= tol_v
    src = config_source(3)
    b_orc = elasticity.load_vector(fine.orc, src)
    b = fine.lib.assemble_rhs(torch.tensor(src(fine.lib.quadrature_points()).reshape(-1), device=DEV))
    assert rel_err(fine.to_orc(b), b_orc) <= 1e-12
    x_orc, it_orc, hist_orc = H_orc.pcg(b_orc, rtol=1e-8)
    x, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float64)
    assert info["iterations"] == it_orc
    assert np.abs(info["history"] - np.array(hist_orc)).max() <= max(1e-12, tol_v)
    assert rel_err(fine.to_orc(x), x_orc) <= 1e-10
    x32, info32 = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=torch.float32)
    assert info32["relres"] <= 1e-8 and abs(info32["iterations"] - it_orc) <= 1
    assert rel_err(fine.to_orc(x32), x_orc) <= 1e-6


def test_beam_full_size(ctx):
    """The beam workload at full size (80 x 16 x 16 cells, 525,987 DoFs):
    sampled operator rows recomputed by the oracle on the cells around them,
    V-cycle symmetry, and PCG in both V-cycle precisions (true residual,
    iterations within +-1)."""
    import time

    import paper_2412_10910_amd as nn
    from scipy.spatial import cKDTree

    from oracle import space
    from workloads import Mesh
    t0 = time.perf_counter()
    meshes = config_levels(3)
    levels = [nn.Level.from_mesh(ctx, m, 2, "elasticity") for m in meshes]
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    H = nn.Hierarchy(ctx, levels, transfers)
    fine = levels[-1]
    assert fine.n_dofs == 525987
    print(f"[beam full size] setup {time.perf_counter() - t0:.1f} s", flush=True)
    # sampled rows: the oracle's elasticity operator on a sub-mesh around them
    pts = fine.support_points()[::3]
    con = fine.constrained()[::3]
    rng = np.random.default_rng(17)
    nodes = np.sort(rng.choice(np.nonzero(~con)[0], size=60, replace=False))
    m = meshes[-1]
    cv = m.vertices[m.cells]
    lo, hi = cv.min(axis=1) - 1e-9, cv.max(axis=1) + 1e-9
    cells = np.unique(np.concatenate([np.nonzero(np.all((lo <= p) & (p <= hi), axis=1))[0] for p in pts[nodes]]))
    verts, inv = np.unique(m.cells[cells].reshape(-1), return_inverse=True)
    sub = space.Space(Mesh(m.vertices[verts], inv.reshape(cells.size, -1).astype(np.int32), m.dirichlet[verts]), 2)
    K = elasticity.stiffness(sub, 1.0, 1.0, constrain=False).tocsr()
    dist, s2l = cKDTree(pts).query(sub.support_points)
    assert dist.max() <= 1e-12
    assert np.array_equal(sub.constrained, con[s2l])
    x = random_vector(fine.n_dofs, 31)
    xs = np.where(np.repeat(sub.free, 3), x.reshape(-1, 3)[s2l].reshape(-1), 0.0)
    l2s = {int(g): i for i, g in enumerate(s2l)}
    rows = np.array([3 * l2s[int(n)] + c for n in nodes for c in range(3)])
    ref = K[rows] @ xs
    lib_rows = np.array([3 * int(n) + c for n in nodes for c in range(3)])
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        y = fine.vmult(torch.tensor(x, dtype=dt, device=DEV))
        got = y[torch.tensor(lib_rows, device=DEV)].double().cpu().numpy()
        assert rel_err(got, ref) <= tol, dt
    # V-cycle symmetry and PCG
    cmask = torch.tensor(fine.constrained(), device=DEV)
    r = torch.tensor(random_vector(fine.n_dofs, 61), device=DEV)
    s = torch.tensor(random_vector(fine.n_dofs, 62), device=DEV)
    r[cmask] = 0
    s[cmask] = 0
    vr, vs = H.vcycle(r), H.vcycle(s)
    assert abs(float(torch.dot(vr, s)) - float(torch.dot(r, vs))) <= 1e-11 * float(vr.norm() * s.norm())
    src = config_source(3)
    b = fine.assemble_rhs(torch.tensor(src(fine.quadrature_points()).reshape(-1), device=DEV))
    its = {}
    for dt in (torch.float64, torch.float32):
        t1 = time.perf_counter()
        xs_, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=dt)
        torch.cuda.synchronize()
        true = float((b - fine.vmult(xs_)).norm() / b.norm())
        print(f"[beam full size] PCG {dt}: {info['iterations']} iterations, relres {info['relres']:.2e}, true "
              f"{true:.2e}, {1e3 * (time.perf_counter() - t1):.1f} ms", flush=True)
        assert info["relres"] <= 1e-8 and true <= 1.01e-8
        its[dt] = info["iterations"]
    assert abs(its[torch.float64] - its[torch.float32]) <= 1
