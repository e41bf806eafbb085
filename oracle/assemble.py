"""Assembled stiffness matrix and load vector (paper §2, eqs. ``problem``,
``discrete_problem`` and ``linear_system``; §4: Poisson, Gauss rule with
(p+1)^d points).

K_ij = sum_K sum_q grad(phi_i) . grad(phi_j) |det J_q| w_q,
b_i  = sum_K sum_q f(x_q) phi_i(x_q) |det J_q| w_q.

Homogeneous Dirichlet DoFs are eliminated by replacing their rows and columns
by the identity, and their load entries by zero.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis

_CHUNK = 20000


def _chunk(space) -> int:
    """Cells per batch: at most 20,000, fewer at high degree so that a batch's
    gradient arrays stay within a few hundred MB (memory only: every cell is
    computed on its own)."""
    Q = space.n ** space.dim
    return max(64, min(_CHUNK, int(3e7 // (Q * Q))))


def element_matrices(space, cells: np.ndarray) -> np.ndarray:
    """Local stiffness matrices of the given cells: [len(cells), q, q]."""
    xq, wq = space.quadrature()
    grad_ref = basis.shape_gradients(space.k, space.dim, xq)  # [Q, q, d]
    J = space.jacobians(xq, cells)  # [c, Q, d, d]
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0):
        raise ValueError("cell with non-positive Jacobian determinant")
    Jinv = np.linalg.inv(J)  # [c, Q, a, i]: d xi_a / d x_i
    # physical gradient: grad phi = J^{-T} grad_ref  -> g[c, Q, i_dof, x]
    g = np.einsum("Qja,cQax->cQjx", grad_ref, Jinv)
    scale = detJ * wq[None, :]
    # K_ij = sum_{Q,x} g[Q,i,x] g[Q,j,x] scale[Q], as a batched product over cells
    c, Q, q, d = g.shape
    gt = g.transpose(0, 2, 1, 3).reshape(c, q, Q * d)
    gs = (g * scale[:, :, None, None]).transpose(0, 2, 1, 3).reshape(c, q, Q * d)
    return gt @ gs.transpose(0, 2, 1)


def stiffness(space, constrain: bool = True) -> sp.csr_matrix:
    """Global stiffness matrix as CSR; identity on constrained rows/columns."""
    C, q = space.cell_dofs.shape
    rows, cols, vals = [], [], []
    step = _chunk(space)
    for s in range(0, C, step):
        cells = np.arange(s, min(C, s + step))
        Ke = element_matrices(space, cells)
        dofs = space.cell_dofs[cells]
        rows.append(np.repeat(dofs, q, axis=1).reshape(-1))
        cols.append(np.tile(dofs, (1, q)).reshape(-1))
        vals.append(Ke.reshape(-1))
    N = space.n_dofs
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    if constrain:
        keep = sp.diags(space.free.astype(np.float64))
        A = (keep @ A @ keep + sp.diags(space.constrained.astype(np.float64))).tocsr()
    return A


def load_vector(space, func, constrain: bool = True) -> np.ndarray:
    """b_i = int f phi_i with the (k+1)^d Gauss rule; zero on constrained DoFs."""
    xq, wq = space.quadrature()
    vals_ref = basis.shape_values(space.k, space.dim, xq)  # [Q, q]
    C, q = space.cell_dofs.shape
    b = np.zeros(space.n_dofs)
    step = _chunk(space)
    for s in range(0, C, step):
        cells = np.arange(s, min(C, s + step))
        x = space.map_points(xq, cells)  # [c, Q, d]
        detJ = np.linalg.det(space.jacobians(xq, cells))
        fq = np.asarray(func(x), dtype=np.float64) * detJ * wq[None, :]
        be = np.einsum("cQ,Qi->ci", fq, vals_ref)
        np.add.at(b, space.cell_dofs[cells].reshape(-1), be.reshape(-1))
    if constrain:
        b[space.constrained] = 0.0
    return b


def quadrature_points(space) -> np.ndarray:
    """Physical Gauss points of every cell: [C, (k+1)^d, d]."""
    xq, _ = space.quadrature()
    return space.map_points(xq)


def l2_error(space, u: np.ndarray, exact, nq: int | None = None) -> float:
    """|| u_h - u ||_{L2} with an (nq)^d Gauss rule (default k+3)."""
    nq = space.k + 3 if nq is None else nq
    xq, wq = space.quadrature(nq)
    vals_ref = basis.shape_values(space.k, space.dim, xq)
    C = space.cell_dofs.shape[0]
    err2 = 0.0
    step = _chunk(space)
    for s in range(0, C, step):
        cells = np.arange(s, min(C, s + step))
        x = space.map_points(xq, cells)
        detJ = np.linalg.det(space.jacobians(xq, cells))
        uh = np.einsum("Qi,ci->cQ", vals_ref, u[space.cell_dofs[cells]])
        err2 += float(np.sum((uh - exact(x)) ** 2 * detJ * wq[None, :]))
    return float(np.sqrt(err2))
