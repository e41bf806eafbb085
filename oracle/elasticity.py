"""Linear elasticity for vector-valued Q_k elements (paper §4, Applications
to FEA, eq. ``linear_elasticity``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The displacement u has d components, each in the scalar Q_k space of
``space.Space``.  Vector DoFs are interleaved by node: DoF d * i + c is
component c at scalar node i.  The bilinear form is

    a(u, v) = (sigma(u), eps(v)),  sigma(u) = lam tr(eps(u)) I + 2 mu eps(u),
    eps(u)  = (grad u + grad u^T) / 2,

so for u = phi_b e_d and v = phi_a e_c

    K_(a,c),(b,d) = int lam d_c phi_a d_d phi_b
                        + mu (delta_cd grad phi_a . grad phi_b + d_d phi_a d_c phi_b),

integrated with the (k+1)^d Gauss rule like the Laplacian.  A node whose
scalar DoF is constrained (it lies on a face all of whose vertices carry the
Dirichlet flag: the clamped part of the boundary) has all d components fixed
at zero; every other boundary face is traction free.  The load vector is
b_(a,c) = int f_c phi_a.

Rigid-body motions (the kernel of a with free boundary, eq. ``rbm``):
translations e_c and rotations about the coordinate axes.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis

_CHUNK = 5000


def vector_free(space) -> np.ndarray:
    """Free mask of the interleaved vector DoFs."""
    return np.repeat(space.free, space.dim)


def element_matrices(space, cells: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """Local elasticity matrices [len(cells), d q, d q] in (node, component) order."""
    d = space.dim
    xq, wq = space.quadrature()
    grad_ref = basis.shape_gradients(space.k, d, xq)  # [Q, q, d]
    J = space.jacobians(xq, cells)  # [c, Q, d, d]
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0):
        raise ValueError("cell with non-positive Jacobian determinant")
    Jinv = np.linalg.inv(J)
    g = np.einsum("Qja,cQax->cQjx", grad_ref, Jinv)  # physical gradients [c, Q, q, d]
    s = detJ * wq[None, :]  # [c, Q]
    nc, nQ, q, _ = g.shape
    # L[a,i,b,j] = sum_Q s d_i phi_a d_j phi_b, as a batched product over cells
    G = g.reshape(nc, nQ, q * d)
    L = (G.transpose(0, 2, 1) @ (G * s[:, :, None])).reshape(nc, q, d, q, d)
    K = lam * L                                # lam d_c phi_a d_d phi_b
    K = K + mu * L.transpose(0, 1, 4, 3, 2)    # mu d_d phi_a d_c phi_b
    lap = np.einsum("caibi->cab", L)           # grad phi_a . grad phi_b
    for i in range(d):
        K[:, :, i, :, i] += mu * lap
    return K.reshape(nc, q * d, q * d)


def vector_cell_dofs(space) -> np.ndarray:
    """[C, q * d] vector DoFs of every cell in (node, component) order."""
    d = space.dim
    return (d * space.cell_dofs[:, :, None] + np.arange(d)[None, None, :]).reshape(space.cell_dofs.shape[0], -1)


def stiffness(space, lam: float, mu: float, constrain: bool = True) -> sp.csr_matrix:
    """Global elasticity matrix as CSR; identity on constrained rows/columns."""
    cd = vector_cell_dofs(space)
    C, nq = cd.shape
    rows, cols, vals = [], [], []
    for s in range(0, C, _CHUNK):
        cells = np.arange(s, min(C, s + _CHUNK))
        Ke = element_matrices(space, cells, lam, mu)
        dofs = cd[cells]
        rows.append(np.repeat(dofs, nq, axis=1).reshape(-1))
        cols.append(np.tile(dofs, (1, nq)).reshape(-1))
        vals.append(Ke.reshape(-1))
    N = space.n_dofs * space.dim
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    if constrain:
        free = vector_free(space)
        keep = sp.diags(free.astype(np.float64))
        A = (keep @ A @ keep + sp.diags((~free).astype(np.float64))).tocsr()
    return A


def load_vector(space, func, constrain: bool = True) -> np.ndarray:
    """b_(a,c) = int f_c phi_a with the (k+1)^d Gauss rule; func maps x [..., d] to f [..., d]."""
    d = space.dim
    xq, wq = space.quadrature()
    vals_ref = basis.shape_values(space.k, d, xq)  # [Q, q]
    cd = vector_cell_dofs(space)
    C = cd.shape[0]
    b = np.zeros(space.n_dofs * d)
    for s in range(0, C, _CHUNK):
        cells = np.arange(s, min(C, s + _CHUNK))
        x = space.map_points(xq, cells)  # [c, Q, d]
        detJ = np.linalg.det(space.jacobians(xq, cells))
        fq = np.asarray(func(x), dtype=np.float64) * (detJ * wq[None, :])[..., None]  # [c, Q, d]
        be = np.einsum("cQk,Qa->cak", fq, vals_ref)  # [c, q, d]
        np.add.at(b, cd[cells].reshape(-1), be.reshape(-1))
    if constrain:
        b[~vector_free(space)] = 0.0
    return b


def vector_prolongation(P: sp.spmatrix, dim: int) -> sp.csr_matrix:
    """P acting on every component: (P_vec)_(i,c),(j,c) = P_ij (interleaved DoFs)."""
    P = sp.coo_matrix(P)
    rows = (dim * P.row[:, None] + np.arange(dim)[None, :]).reshape(-1)
    cols = (dim * P.col[:, None] + np.arange(dim)[None, :]).reshape(-1)
    vals = np.repeat(P.data, dim)
    return sp.coo_matrix((vals, (rows, cols)), shape=(P.shape[0] * dim, P.shape[1] * dim)).tocsr()


def rigid_body_modes(space) -> np.ndarray:
    """The six rigid-body motions of 3D (three of 2D) interpolated at the nodes: [m, N d]."""
    x = space.support_points
    d = space.dim
    modes = []
    for c in range(d):
        m = np.zeros((space.n_dofs, d))
        m[:, c] = 1.0
        modes.append(m)
    if d == 3:
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        zero = np.zeros_like(X)
        modes += [np.stack([zero, Z, -Y], 1), np.stack([-Z, zero, X], 1), np.stack([Y, -X, zero], 1)]
    else:
        modes.append(np.stack([x[:, 1], -x[:, 0]], 1))
    return np.array([m.reshape(-1) for m in modes])
