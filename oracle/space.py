"""Continuous Q_k space on a quad/hex mesh (paper §2: V_l with Q^p on each cell).

Geometry is the bi/trilinear (Q1) map of each cell's 2^d vertices.  Global
degrees of freedom are identified by their physical support points: two local
nodes of different cells are the same DoF iff they map to the same point
(paper §2, eq. ``pointwise``: one DoF per support point).  A DoF is
constrained (homogeneous Dirichlet) iff it lies in the closure of a boundary
face all of whose vertices carry the Dirichlet flag.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
from scipy.spatial import cKDTree

from . import basis


def vertex_shape(dim: int, xi: np.ndarray):
    """Q1 vertex functions and their reference gradients at points xi [P, dim].

    Returns (N [P, 2^dim], dN [P, 2^dim, dim]); vertex b sits at the corner whose
    coordinate along axis a is bit a of b.
    """
    xi = np.atleast_2d(xi)
    P = xi.shape[0]
    nv = 2 ** dim
    N = np.ones((P, nv))
    dN = np.ones((P, nv, dim))
    for b in range(nv):
        for a in range(dim):
            bit = (b >> a) & 1
            f = xi[:, a] if bit else 1.0 - xi[:, a]
            df = 1.0 if bit else -1.0
            N[:, b] *= f
            for c in range(dim):
                dN[:, b, c] *= df if c == a else f
    return N, dN


class Space:
    """Q_k space on one mesh level."""

    def __init__(self, mesh, degree: int):
        self.mesh = mesh
        self.dim = mesh.dim
        self.k = int(degree)
        self.n = self.k + 1
        self.nodes1d = basis.gauss_lobatto_nodes(self.k)
        self.node_ref = basis.tensor_points(self.nodes1d, self.dim)  # [q, dim]
        self.cell_vertices = mesh.vertices[mesh.cells]  # [C, 2^d, d]
        self._number_dofs()
        self._constrain()

    # -- geometry -----------------------------------------------------------
    def map_points(self, xi: np.ndarray, cells=None) -> np.ndarray:
        """Physical points F_K(xi) for every cell K: [C, P, dim]."""
        N, _ = vertex_shape(self.dim, xi)
        cv = self.cell_vertices if cells is None else self.cell_vertices[cells]
        return np.einsum("pb,cbi->cpi", N, cv)

    def jacobians(self, xi: np.ndarray, cells=None) -> np.ndarray:
        """J[c, p, i, a] = d x_i / d xi_a at points xi: [C, P, dim, dim]."""
        _, dN = vertex_shape(self.dim, xi)
        cv = self.cell_vertices if cells is None else self.cell_vertices[cells]
        return np.einsum("pba,cbi->cpia", dN, cv)

    # -- DoFs ---------------------------------------------------------------
    def _number_dofs(self):
        pts = self.map_points(self.node_ref)  # [C, q, d]
        C, q, d = pts.shape
        flat = pts.reshape(-1, d)
        ext = np.ptp(self.mesh.vertices, axis=0).max()
        tol = 1e-8 * max(ext, 1e-300)
        tree = cKDTree(flat)
        pairs = tree.query_pairs(r=tol, output_type="ndarray")
        m = flat.shape[0]
        g = sp.coo_matrix((np.ones(pairs.shape[0]), (pairs[:, 0], pairs[:, 1])), shape=(m, m))
        ncomp, label = csgraph.connected_components(g, directed=False)
        # number DoFs by first appearance in (cell, local node) order
        first = np.full(ncomp, m, dtype=np.int64)
        np.minimum.at(first, label, np.arange(m))
        order = np.argsort(first, kind="stable")
        new_id = np.empty(ncomp, dtype=np.int64)
        new_id[order] = np.arange(ncomp)
        self.cell_dofs = new_id[label].reshape(C, q)
        self.n_dofs = int(ncomp)
        self.support_points = np.zeros((ncomp, d))
        self.support_points[self.cell_dofs.reshape(-1)] = flat

    def _constrain(self):
        dim, k = self.dim, self.k
        cells = self.mesh.cells
        C = cells.shape[0]
        mi = basis.multi_indices(self.n, dim)
        keys, tags = [], []
        for a in range(dim):
            for s in (0, 1):
                verts_local = [b for b in range(2 ** dim) if ((b >> a) & 1) == s]
                keys.append(np.sort(cells[:, verts_local], axis=1))
                tags.append(np.stack([np.arange(C), np.full(C, a), np.full(C, s)], axis=1))
        keys = np.concatenate(keys)
        tags = np.concatenate(tags)
        _, inverse, counts = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
        inverse = inverse.reshape(-1)
        on_boundary = counts[inverse] == 1  # a face owned by a single cell
        diri = self.mesh.dirichlet.astype(bool)
        marked = on_boundary & np.all(diri[keys], axis=1)
        constrained = np.zeros(self.n_dofs, dtype=bool)
        for c, a, s in tags[marked]:
            local = np.nonzero(mi[:, a] == s * k)[0]
            constrained[self.cell_dofs[c, local]] = True
        self.constrained = constrained
        self.free = ~constrained

    # -- quadrature ---------------------------------------------------------
    def quadrature(self, nq: int | None = None):
        """Gauss rule with nq points per direction (default k+1): ref points, weights."""
        nq = self.n if nq is None else nq
        x, w = basis.gauss_legendre(nq)
        return basis.tensor_points(x, self.dim), basis.tensor_weights(w, self.dim)

    def interpolate(self, func) -> np.ndarray:
        """Nodal interpolant I_l u = sum_i u(x_i) phi_i (paper §2, eq. ``pointwise``)."""
        return np.asarray(func(self.support_points), dtype=np.float64)
