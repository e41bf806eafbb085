"""Mesh generators for the synthetic Poisson workloads.

Every level of a multigrid hierarchy is an independent quadrilateral or
hexahedral mesh of the same domain (paper §2: the levels T_1 .. T_L are
non-nested partitions with C h_l <= h_{l+1} <= h_l).  The paper's own meshes
(gmsh / Cubit / CAD) are not available, so structured meshes with randomly
perturbed interior vertices and a mapped-cube ball stand in for them.

Conventions (shared by every consumer):

* ``vertices``: float64 ``[V, dim]``.
* ``cells``: int32 ``[C, 2**dim]``; the local vertex ``b`` of a cell sits at
  the reference corner whose coordinate along axis ``a`` is bit ``a`` of ``b``
  (lexicographic, x fastest).  Cells have positive orientation.
* ``dirichlet``: uint8 ``[V]``, 1 for vertices on the Dirichlet boundary.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class Mesh:
    vertices: np.ndarray  # float64 [V, dim]
    cells: np.ndarray  # int32 [C, 2**dim]
    dirichlet: np.ndarray  # uint8 [V]

    @property
    def dim(self) -> int:
        return int(self.vertices.shape[1])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


def structured_box(dim: int, n: int, lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """Structured n^dim mesh of [lo, hi]^dim, every boundary vertex Dirichlet."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n < 1:
        raise ValueError("n must be >= 1")
    coords = np.linspace(lo, hi, n + 1)
    # vertex index = ix + (n+1) * iy + (n+1)^2 * iz  (x fastest)
    idx = np.indices([n + 1] * dim)  # idx[a] = index along axis a, arrays indexed [i0, i1, ...]
    flat = [idx[a].reshape(-1, order="F") for a in range(dim)]
    verts = np.stack([coords[f] for f in flat], axis=1)
    stride = [(n + 1) ** a for a in range(dim)]
    cidx = np.indices([n] * dim)
    cflat = [cidx[a].reshape(-1, order="F") for a in range(dim)]
    base = sum(cflat[a] * stride[a] for a in range(dim))
    cells = np.empty((base.size, 2 ** dim), dtype=np.int64)
    for b in range(2 ** dim):
        off = sum(((b >> a) & 1) * stride[a] for a in range(dim))
        cells[:, b] = base + off
    on_bnd = np.zeros(verts.shape[0], dtype=bool)
    for a in range(dim):
        on_bnd |= (flat[a] == 0) | (flat[a] == n)
    return Mesh(verts.astype(np.float64), cells.astype(np.int32), on_bnd.astype(np.uint8))


def structured_brick(cells, lo, hi) -> Mesh:
    """Structured hexahedral mesh of the box [lo, hi] with cells[a] cells along
    axis a (x fastest, as structured_box); every boundary vertex Dirichlet."""
    nx, ny, nz = (int(c) for c in cells)
    if min(nx, ny, nz) < 1:
        raise ValueError("cells must be >= 1")
    axes = [np.linspace(lo[a], hi[a], cells[a] + 1) for a in range(3)]
    n1 = [nx + 1, ny + 1, nz + 1]
    iv = np.arange(n1[0] * n1[1] * n1[2])
    ix, iy, iz = iv % n1[0], (iv // n1[0]) % n1[1], iv // (n1[0] * n1[1])
    verts = np.stack([axes[0][ix], axes[1][iy], axes[2][iz]], axis=1)
    ic = np.arange(nx * ny * nz)
    cx, cy, cz = ic % nx, (ic // nx) % ny, ic // (nx * ny)
    base = cx + n1[0] * (cy + n1[1] * cz)
    cells_ = np.empty((ic.size, 8), dtype=np.int64)
    for b in range(8):
        cells_[:, b] = base + (b & 1) + n1[0] * (((b >> 1) & 1) + n1[1] * ((b >> 2) & 1))
    on_bnd = (ix == 0) | (ix == nx) | (iy == 0) | (iy == ny) | (iz == 0) | (iz == nz)
    return Mesh(verts.astype(np.float64), cells_.astype(np.int32), on_bnd.astype(np.uint8))


def dirichlet_face(mesh: Mesh, axis: int, value: float) -> Mesh:
    """The same mesh with only the vertices on the plane x_axis = value Dirichlet."""
    tol = 1e-12 * max(1.0, float(np.ptp(mesh.vertices)))
    d = (np.abs(mesh.vertices[:, axis] - value) < tol).astype(np.uint8)
    return Mesh(mesh.vertices.copy(), mesh.cells.copy(), d)


def perturb_interior(mesh: Mesh, alpha: float, h, rng: np.random.Generator) -> Mesh:
    """Move every coordinate of every non-boundary vertex by U(-alpha*h, alpha*h)
    (h a number or one cell size per axis)."""
    v = mesh.vertices.copy()
    # the boundary is found geometrically (a vertex on a facet of the bounding
    # box), so the result does not depend on the Dirichlet flags
    lo = mesh.vertices.min(axis=0)
    hi = mesh.vertices.max(axis=0)
    tol = 1e-12 * max(1.0, float(np.max(hi - lo)))
    geo_bnd = np.any((np.abs(mesh.vertices - lo) < tol) | (np.abs(mesh.vertices - hi) < tol), axis=1)
    interior = ~geo_bnd
    hh = np.broadcast_to(np.asarray(h, dtype=np.float64), (v.shape[1],))
    delta = rng.uniform(-1.0, 1.0, size=v.shape) * (alpha * hh)
    v[interior] += delta[interior]
    return Mesh(v, mesh.cells.copy(), mesh.dirichlet.copy())


def ball_map(mesh: Mesh) -> Mesh:
    """Map a mesh of [-1,1]^d onto the unit ball by x -> x |x|_inf / |x|_2 (0 -> 0)."""
    v = mesh.vertices
    ninf = np.max(np.abs(v), axis=1)
    n2 = np.linalg.norm(v, axis=1)
    scale = np.where(n2 > 0, ninf / np.where(n2 > 0, n2, 1.0), 0.0)
    return Mesh(v * scale[:, None], mesh.cells.copy(), mesh.dirichlet.copy())


def _orientation_preserving_symmetries(dim: int):
    """All symmetries of the reference square/cube with determinant +1.

    Each symmetry is returned as a permutation ``perm`` of the 2**dim local
    vertices: new local vertex b takes old local vertex perm[b].
    """
    out = []
    for axes in itertools.permutations(range(dim)):
        for flips in itertools.product((0, 1), repeat=dim):
            m = np.zeros((dim, dim))
            for i, a in enumerate(axes):
                m[i, a] = -1.0 if flips[i] else 1.0
            if np.linalg.det(m) < 0:
                continue
            perm = []
            for b in range(2 ** dim):
                # corner of the new cell in reference coords
                x = np.array([(b >> a) & 1 for a in range(dim)], dtype=float)
                # new coordinate i is old coordinate axes[i] (flipped if requested)
                old = np.zeros(dim)
                for i, a in enumerate(axes):
                    old[a] = 1.0 - x[i] if flips[i] else x[i]
                perm.append(int(sum(int(round(old[a])) << a for a in range(dim))))
            out.append(perm)
    return out


def scramble(mesh: Mesh, rng: np.random.Generator, rotate: bool = True,
             renumber_cells: bool = True, renumber_vertices: bool = True) -> Mesh:
    """Same geometric mesh with random cell order, cell orientation and vertex ids."""
    cells = mesh.cells.copy()
    verts = mesh.vertices.copy()
    diri = mesh.dirichlet.copy()
    dim = mesh.dim
    if rotate:
        syms = np.array(_orientation_preserving_symmetries(dim), dtype=np.int64)
        pick = rng.integers(0, syms.shape[0], size=cells.shape[0])
        cells = np.take_along_axis(cells, syms[pick], axis=1)
    if renumber_cells:
        cells = cells[rng.permutation(cells.shape[0])]
    if renumber_vertices:
        perm = rng.permutation(verts.shape[0])  # new id of old vertex i is perm[i]
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.size)
        verts = verts[inv]
        diri = diri[inv]
        cells = perm[cells]
    return Mesh(verts, cells.astype(np.int32), diri)


# ---------------------------------------------------------------------------
# The synthetic workloads.  Levels are listed coarse -> fine.
# ---------------------------------------------------------------------------

CONFIGS = {
    # 2D Poisson, f = 1, Q1, 64^2 / 23^2 / 9^2 quads, interior vertices +-0.2h
    0: dict(dim=2, degree=1, domain="square", cells=[9, 23, 64], alpha=0.2, source="one"),
    # 3D Poisson, Q2, 64^3 / 29^3 / 13^3 / 6^3 hexes, interior vertices +-0.15h,
    # f = sum of 8 Gaussian bumps of width 0.1
    1: dict(dim=3, degree=2, domain="cube", cells=[6, 13, 29, 64], alpha=0.15, source="bumps"),
    # 3D Poisson on the mapped-cube ball, Q3, 96^3 .. 5^3 hexes
    2: dict(dim=3, degree=3, domain="ball", cells=[5, 9, 19, 43, 96], alpha=0.0, source="bumps_ball"),
    # the same ball with Q4 (27.3M fine DoFs)
    "2q4": dict(dim=3, degree=4, domain="ball", cells=[5, 7, 15, 34, 75], alpha=0.0, source="bumps_ball"),
    # reduced ball hierarchies that the oracle can solve in seconds
    "2p3": dict(dim=3, degree=3, domain="ball", cells=[4, 7, 15, 32], alpha=0.0, source="bumps_ball"),
    "2p4": dict(dim=3, degree=4, domain="ball", cells=[5, 11, 24], alpha=0.0, source="bumps_ball"),
    # 3D linear elasticity (vector Q2, lambda = mu = 1) on the beam [0,5] x [0,1]^2
    # clamped at x = 0, body load (0, 0, -1); cells per level (x, y, z),
    # interior vertices +-0.1h
    3: dict(dim=3, degree=2, domain="beam", cells=[(14, 3, 3), (33, 7, 7), (80, 16, 16)], alpha=0.1,
            source="gravity", operator="elasticity", lam=1.0, mu=1.0),
}

BEAM_LENGTH = 5.0


def _seed_base(cfg) -> int:
    return {0: 0, 1: 1, 2: 2, "2q4": 2, "2p3": 2, "2p4": 2, 3: 3}.get(cfg, 9)


def level_mesh(domain: str, dim: int, n: int, alpha: float, seed: int) -> Mesh:
    if domain == "square" or domain == "cube":
        m = structured_box(dim, n, 0.0, 1.0)
        if alpha > 0:
            m = perturb_interior(m, alpha, 1.0 / n, np.random.default_rng(seed))
        return m
    if domain == "ball":
        m = structured_box(dim, n, -1.0, 1.0)
        if alpha > 0:
            m = perturb_interior(m, alpha, 2.0 / n, np.random.default_rng(seed))
        return ball_map(m)
    if domain == "beam":
        # n = (cells along x, y, z); clamped (Dirichlet) on the face x = 0 only
        hi = (BEAM_LENGTH, 1.0, 1.0)
        m = structured_brick(n, (0.0, 0.0, 0.0), hi)
        if alpha > 0:
            h = [hi[a] / n[a] for a in range(3)]
            m = perturb_interior(m, alpha, h, np.random.default_rng(seed))
        return dirichlet_face(m, 0, 0.0)
    raise ValueError(domain)


# Resident hierarchies of the serving stream: Poisson on perturbed cubes (Q2,
# the recipe of the 64^3 cube workload) and on balls (Q3, the recipe of the
# 96^3 ball), fine sizes spread log-uniformly over 0.1M..8M DoFs, 3 to 5
# independent levels each: (config key, cells per direction coarse -> fine,
# degree).
SERVING_POOL = [
    (1, [5, 11, 23], 2),           # 103,823 DoFs
    (2, [4, 9, 20], 3),            # 226,981
    (1, [4, 8, 17, 36], 2),        # 389,017
    (2, [5, 10, 20, 40], 3),       # 1,771,561
    (1, [6, 13, 29, 64], 2),       # 2,146,689
    (1, [5, 10, 22, 46, 100], 2),  # 8,120,601
]


def config_levels(cfg, cells=None):
    """Meshes of a workload, coarse -> fine; ``cells`` overrides the per-level sizes.

    Level l (0-based, coarse -> fine) is perturbed with
    ``numpy.random.default_rng(1000 * cfg_seed + l)``.
    """
    c = CONFIGS[cfg]
    sizes = list(cells) if cells is not None else c["cells"]
    base = _seed_base(cfg)
    return [level_mesh(c["domain"], c["dim"], n, c["alpha"], 1000 * base + l)
            for l, n in enumerate(sizes)]
