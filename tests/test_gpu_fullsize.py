"""Parity at the workloads' full sizes, on sampled outputs, in every launch
configuration the benchmark can time: the operator rows are checked for each
deterministic operator variant the autotuner chooses from, with one and two
layout blocks per workgroup.

The oracle cannot assemble a 2M-24M DoF operator or locate every fine point
within a test's time, so it recomputes sampled outputs one by one:

* operator rows: the cells around sampled DoFs form a sub-mesh; the oracle
  builds its own Q_k space and element matrices there, and row i of
  K_sub x_sub equals row i of A x for a DoF i whose cells are all included;
* prolongation: fine support points of sampled fine regions (from the
  oracle's own space on those cells) are located in the full coarse space by
  the oracle, then P v is evaluated per point from the coarse basis;
* restriction: for sampled coarse DoFs j, every fine point that can own a
  cell around j is located by the oracle, and (P^T r)_j is summed directly.

Only support-point coordinates identify DoFs between the two numberings
(matched within 1e-12, as in the small-size tests).  The solver is checked at
full size through properties that hold at any size: V-cycle symmetry, the
true residual of the PCG solution, and float32-MG iterations within +-1 of
float64-MG.
"""

from __future__ import annotations

import time

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from oracle import assemble, basis, space, transfer
from workloads import Mesh, config_levels, config_source, random_vector

from _parity import DEV, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5

# (id, workload, level sizes coarse -> fine, degree)
CASES = [
    ("cube_q2_64", 1, [6, 13, 29, 64], 2),
    ("ball_q3_96", 2, [5, 9, 19, 43, 96], 3),
    ("ball_q4_75", "2q4", [5, 7, 15, 34, 75], 4),
]


def log(msg):
    print(msg, flush=True)


class CellBoxes:
    """Vertex bounding boxes of a mesh's cells, for finding the cells around points."""

    def __init__(self, mesh: Mesh):
        cv = mesh.vertices[mesh.cells]
        self.lo = cv.min(axis=1) - 1e-9
        self.hi = cv.max(axis=1) + 1e-9
        self.rad = 0.5 * float(np.linalg.norm(self.hi - self.lo, axis=1).max())
        self.tree = cKDTree(0.5 * (self.lo + self.hi))

    def around(self, pts: np.ndarray) -> np.ndarray:
        """Cells whose box contains one of the points (a superset of the cells holding them)."""
        cand = self.tree.query_ball_point(pts, r=self.rad * 1.001)
        sel = set()
        for p, cs in zip(pts, cand):
            cs = np.asarray(cs, dtype=np.int64)
            ok = np.all((self.lo[cs] <= p) & (p <= self.hi[cs]), axis=1)
            sel.update(cs[ok].tolist())
        return np.array(sorted(sel), dtype=np.int64)


def _submesh(mesh: Mesh, cells: np.ndarray) -> Mesh:
    verts, inv = np.unique(mesh.cells[cells].reshape(-1), return_inverse=True)
    return Mesh(vertices=mesh.vertices[verts], cells=inv.reshape(cells.size, -1).astype(np.int32),
                dirichlet=mesh.dirichlet[verts])


def _match_into(lib_points: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Index of the library DoF at each point (checked to 1e-12)."""
    lo, hi = pts.min(axis=0) - 1e-9, pts.max(axis=0) + 1e-9
    idx = np.nonzero(np.all((lib_points >= lo) & (lib_points <= hi), axis=1))[0]
    dist, j = cKDTree(lib_points[idx]).query(pts)
    assert dist.max() <= 1e-12 * max(1.0, float(np.abs(pts).max())), f"points differ by {dist.max():.3e}"
    return idx[j]


class FullLevels:
    """The two finest levels and their transfer, built as the benchmark builds them."""

    def __init__(self, ctx, cfg, cells, k):
        import paper_2412_10910_amd as nn
        t0 = time.perf_counter()
        self.meshes = config_levels(cfg, cells=cells)
        self.k = k
        self.cfg = cfg
        self.fine = nn.Level.from_mesh(ctx, self.meshes[-1], k)
        self.coarse = nn.Level.from_mesh(ctx, self.meshes[-2], k)
        t1 = time.perf_counter()
        self.tr = nn.Transfer(ctx, self.fine, self.coarse)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        self.fine_pts = self.fine.support_points()
        self.coarse_pts = self.coarse.support_points()
        self.fine_con = self.fine.constrained()
        self.coarse_con = self.coarse.constrained()
        self.fine_boxes = CellBoxes(self.meshes[-1])
        log(f"[fullsize cfg {cfg} cells {cells[-2]}->{cells[-1]} Q{k}] levels {t1 - t0:.1f} s, transfer "
            f"{t2 - t1:.1f} s; fine DoFs {self.fine.n_dofs}, points {self.tr.n_points}")
        self._coarse_orc = None

    @property
    def coarse_orc(self):
        if self._coarse_orc is None:
            self._coarse_orc = space.Space(self.meshes[-2], self.k)
        return self._coarse_orc


_CACHE: dict = {}


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _levels(ctx, case):
    name, cfg, cells, k = case
    if name not in _CACHE:
        _CACHE[name] = FullLevels(ctx, cfg, cells, k)
    return _CACHE[name]


def _sample_free(n_dofs, constrained, count, seed):
    rng = np.random.default_rng(seed)
    free = np.nonzero(~constrained)[0]
    return np.sort(rng.choice(free, size=min(count, free.size), replace=False))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_operator_rows_full_size(ctx, case):
    F = _levels(ctx, case)
    lib = F.fine
    free = np.nonzero(~F.fine_con)[0]
    rows = _sample_free(lib.n_dofs, F.fine_con, 160, 5)
    # also the first and last free DoF of the numbering and the free DoF
    # nearest to each corner of the domain's bounding box
    lo, hi = F.fine_pts.min(axis=0), F.fine_pts.max(axis=0)
    corners = np.array([[hi[a] if (b >> a) & 1 else lo[a] for a in range(3)] for b in range(8)])
    _, near = cKDTree(F.fine_pts[free]).query(corners)
    rows = np.unique(np.concatenate([rows, free[[0, -1]], free[near]]))
    cells = F.fine_boxes.around(F.fine_pts[rows])
    sub = space.Space(_submesh(F.meshes[-1], cells), F.k)
    K = assemble.stiffness(sub, constrain=False).tocsr()
    sub2lib = _match_into(F.fine_pts, sub.support_points)
    # the sub-space's Dirichlet DoFs are the library's on every sub-space DoF
    assert np.array_equal(sub.constrained, F.fine_con[sub2lib])
    lib2sub = {int(g): i for i, g in enumerate(sub2lib)}
    rs = np.array([lib2sub[int(r)] for r in rows])
    x_all = random_vector(lib.n_dofs, 31)
    x_sub = np.where(sub.free, x_all[sub2lib], 0.0)
    ref = K[rs] @ x_sub
    # every deterministic variant the autotuner may keep, with one and two
    # layout blocks per workgroup
    variants = [v for v, name in enumerate(lib.VARIANTS)
                if name is not None and "atomic" not in name and ("entity" not in name or (F.k >= 3))]
    base = lib.cells_per_block()[1]
    idx = torch.tensor(rows, device=DEV)
    worst = {}
    for v in variants:
        lib.set_variant(v)
        for cpb in (base, 2 * base):
            lib.set_cells_per_block(cpb)
            for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
                x = torch.tensor(x_all, dtype=dt, device=DEV)
                got = lib.vmult(x)[idx].double().cpu().numpy()
                err = rel_err(got, ref)
                worst[dt] = max(worst.get(dt, 0.0), err)
                assert err <= tol, (lib.VARIANTS[v], cpb, dt, err)
    lib.set_variant(0)
    lib.set_cells_per_block(base)
    for dt, e in worst.items():
        log(f"  operator {case[0]} {dt}: {rows.size} rows over {cells.size} cells, {len(variants)} variants x 2 "
            f"workgroup sizes, largest rel err {e:.2e}")


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_prolongation_points_full_size(ctx, case):
    F = _levels(ctx, case)
    C = F.coarse_orc
    perm_c = _match_into(F.coarse_pts, C.support_points)  # oracle coarse DoF -> library DoF
    assert np.array_equal(C.constrained, F.coarse_con[perm_c])
    # sampled fine regions: the oracle's own fine space on a few hundred fine cells
    rng = np.random.default_rng(9)
    fcells = np.unique(rng.choice(F.meshes[-1].n_cells, size=300, replace=False))
    fsub = space.Space(_submesh(F.meshes[-1], fcells), F.k)
    pts = fsub.support_points[fsub.free]
    fine_ids = _match_into(F.fine_pts, pts)
    assert not F.fine_con[fine_ids].any()
    owner, ref, _ = transfer.locate(pts, C)
    lib = F.tr.points()
    pos = np.searchsorted(lib["fine_dof"], fine_ids)
    assert np.array_equal(lib["fine_dof"][pos], fine_ids)
    assert np.array_equal(lib["owner"][pos], owner), "owner cells differ"
    assert np.abs(lib["xi"][pos] - ref).max() <= 1e-12
    v_orc = random_vector(C.n_dofs, 41) * C.free
    vals = basis.shape_values(F.k, 3, ref)  # [P, q]
    expect = np.einsum("pa,pa->p", vals, v_orc[C.cell_dofs[owner]])
    v_lib = np.zeros(F.coarse.n_dofs)
    v_lib[perm_c] = v_orc
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        out = torch.zeros(F.fine.n_dofs, dtype=dt, device=DEV)
        F.tr.prolongate(torch.tensor(v_lib, dtype=dt, device=DEV), out)
        got = out[torch.tensor(fine_ids, device=DEV)].double().cpu().numpy()
        err = rel_err(got, expect)
        log(f"  prolongation {case[0]} {dt}: {pts.shape[0]} points, rel err {err:.2e}")
        assert err <= tol


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_restriction_dofs_full_size(ctx, case):
    F = _levels(ctx, case)
    C = F.coarse_orc
    perm_c = _match_into(F.coarse_pts, C.support_points)
    rng = np.random.default_rng(13)
    # (the oracle locates every candidate point of a sampled DoF's cells:
    # about 3.5 s per coarse DoF at Q4, so fewer of them there)
    js = np.sort(rng.choice(np.nonzero(C.free)[0], size=24 if F.k <= 3 else 10, replace=False))
    r_all = random_vector(F.fine.n_dofs, 43)
    r_gpu = {dt: torch.tensor(r_all, dtype=dt, device=DEV) for dt in (torch.float64, torch.float32)}
    outs = {}
    for dt in r_gpu:
        o = torch.zeros(F.coarse.n_dofs, dtype=dt, device=DEV)
        F.tr.restrict(r_gpu[dt], o)
        outs[dt] = o.double().cpu().numpy()
    expect = np.zeros(js.size)
    for t, j in enumerate(js):
        kcells = np.nonzero((C.cell_dofs == j).any(axis=1))[0]
        # every fine point a cell around j can own lies in its grown bounding box
        cv = C.cell_vertices[kcells]
        lo, hi = cv.min(axis=1), cv.max(axis=1)
        g = (transfer.EXPAND * np.linalg.norm(hi - lo, axis=1))[:, None]
        corners = np.concatenate([lo - g, hi + g])
        box_lo, box_hi = corners.min(axis=0), corners.max(axis=0)
        inside = np.nonzero(np.all((F.fine_pts >= box_lo) & (F.fine_pts <= box_hi), axis=1))[0]
        fcells = F.fine_boxes.around(F.fine_pts[inside])
        fsub = space.Space(_submesh(F.meshes[-1], fcells), F.k)
        pts = fsub.support_points[fsub.free]
        sel = np.all((pts >= box_lo) & (pts <= box_hi), axis=1)
        pts = pts[sel]
        owner, ref, _ = transfer.locate(pts, C)
        hit = np.isin(owner, kcells)
        vals = basis.shape_values(F.k, 3, ref[hit])
        local = np.argmax(C.cell_dofs[owner[hit]] == j, axis=1)
        ids = _match_into(F.fine_pts, pts[hit])
        expect[t] = np.sum(vals[np.arange(local.size), local] * r_all[ids])
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        got = outs[dt][perm_c[js]]
        err = rel_err(got, expect)
        log(f"  restriction {case[0]} {dt}: {js.size} coarse DoFs, rel err {err:.2e}")
        assert err <= tol


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_transfer_adjoint_full_size(ctx, case):
    F = _levels(ctx, case)
    v = torch.tensor(random_vector(F.coarse.n_dofs, 51), device=DEV)
    r = torch.tensor(random_vector(F.fine.n_dofs, 52), device=DEV)
    v[torch.tensor(F.coarse_con, device=DEV)] = 0
    r[torch.tensor(F.fine_con, device=DEV)] = 0
    pv = F.tr.prolongate(v, torch.zeros_like(r))
    ptr = F.tr.restrict(r, torch.zeros_like(v))
    a, b = float(torch.dot(pv, r)), float(torch.dot(v, ptr))
    scale = float(pv.norm() * r.norm())
    log(f"  adjoint {case[0]}: <Pv,r> = {a:.15e}, <v,P^T r> = {b:.15e}")
    assert abs(a - b) <= 1e-12 * scale


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_solver_properties_full_size(ctx, case):
    import paper_2412_10910_amd as nn
    _CACHE.clear()
    torch.cuda.empty_cache()
    name, cfg, cells, k = case
    t0 = time.perf_counter()
    meshes = config_levels(cfg, cells=cells)
    levels = [nn.Level.from_mesh(ctx, m, k) for m in meshes]
    transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    H = nn.Hierarchy(ctx, levels, transfers)
    fine = levels[-1]
    fq = torch.tensor(config_source(cfg)(fine.quadrature_points()).reshape(-1), dtype=torch.float64, device=DEV)
    b = fine.assemble_rhs(fq)
    torch.cuda.synchronize()
    log(f"  [{name}] hierarchy of {len(levels)} levels in {time.perf_counter() - t0:.1f} s")
    con = torch.tensor(fine.constrained(), device=DEV)
    # V-cycle symmetry <V r, s> = <r, V s> (float64, exact coarse solve)
    r = torch.tensor(random_vector(fine.n_dofs, 61), device=DEV)
    s = torch.tensor(random_vector(fine.n_dofs, 62), device=DEV)
    r[con] = 0
    s[con] = 0
    vr, vs = H.vcycle(r), H.vcycle(s)
    a, c = float(torch.dot(vr, s)), float(torch.dot(r, vs))
    assert abs(a - c) <= 1e-12 * float(vr.norm() * s.norm())
    assert float(torch.dot(vr, r)) > 0
    # PCG in both V-cycle precisions: converged, true residual, iterations within +-1
    res = {}
    for dt in (torch.float64, torch.float32):
        t1 = time.perf_counter()
        x, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=dt)
        torch.cuda.synchronize()
        t = time.perf_counter() - t1
        true = float((b - fine.vmult(x)).norm() / b.norm())
        log(f"  [{name}] PCG with {dt} V-cycle: {info['iterations']} iterations, relres {info['relres']:.3e}, "
            f"true {true:.3e}, {t * 1e3:.1f} ms")
        assert info["relres"] <= 1e-8
        assert true <= 1.01e-8
        res[dt] = (x, info["iterations"])
    assert abs(res[torch.float64][1] - res[torch.float32][1]) <= 1
    # both solutions agree to the solver tolerance (relative, A-norm-free bound)
    d = float((res[torch.float64][0] - res[torch.float32][0]).norm() / res[torch.float64][0].norm())
    log(f"  [{name}] |x64 - x32| / |x64| = {d:.2e}")
    assert d <= 1e-6
