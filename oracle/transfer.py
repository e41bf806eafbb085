"""Non-nested transfer: point location and the explicit prolongation matrix.

Paper §2 (after eq. ``residual2``): P_ij = phi_j^{l-1}(x_i), rows indexed by
fine DoFs, columns by coarse DoFs; restriction is the transpose P^T.
Paper §3.1: the owning coarse cell of each fine support point is found by a
geometric search, and its reference position by inverting the cell map with
Newton's method.  Paper §3.3, eq. ``closest_point``: a point outside every
coarse cell is evaluated at the point of the closed reference cell nearest to
its pre-image.

Rules fixed here where the paper leaves details open:

* candidate cells of a point x are the cells whose vertex bounding box, grown
  on every side by ``expand`` times its diagonal, contains x;
* Newton starts at the cell centre, stops when the update's max-norm is at
  most ``newton_tol`` (the update is applied first) and gives up after
  ``newton_max_it`` steps; a candidate whose Newton does not stop is skipped;
* the owner is the lowest-numbered candidate whose pre-image lies within
  ``inside_tol`` (max-norm) of [0,1]^d; if there is none, the candidate whose
  pre-image is nearest to [0,1]^d in the Euclidean reference distance (lowest
  number on ties);
* the stored reference position is the pre-image clamped to [0,1]^d;
* only unconstrained fine DoFs are located, and only unconstrained coarse DoFs
  receive columns (constrained DoFs are fixed at zero).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis
from .space import vertex_shape

EXPAND = 0.25
INSIDE_TOL = 1e-10
NEWTON_TOL = 1e-12
NEWTON_MAX_IT = 50


class PointNotFound(RuntimeError):
    pass


def newton_inverse(cell_vertices: np.ndarray, x: np.ndarray, tol=NEWTON_TOL, max_it=NEWTON_MAX_IT):
    """Invert the Q1 cell maps: for each pair m, find xi with F_{K_m}(xi) = x_m.

    cell_vertices [M, 2^d, d], x [M, d].  Returns (xi [M, d], converged [M] bool).
    """
    M, nv, d = cell_vertices.shape
    xi = np.full((M, d), 0.5)
    done = np.zeros(M, dtype=bool)
    failed = np.zeros(M, dtype=bool)
    for _ in range(max_it):
        act = np.nonzero(~done & ~failed)[0]
        if act.size == 0:
            break
        N, dN = _vertex_shape_batched(d, xi[act])
        cv = cell_vertices[act]
        F = np.einsum("mb,mbi->mi", N, cv)
        J = np.einsum("mba,mbi->mia", dN, cv)
        det = np.linalg.det(J)
        ok = np.abs(det) > 0
        delta = np.zeros((act.size, d))
        delta[ok] = np.linalg.solve(J[ok], (F - x[act])[ok][..., None])[..., 0]
        xi[act] -= delta
        bad = ~ok | ~np.all(np.isfinite(xi[act]), axis=1) | (np.max(np.abs(xi[act]), axis=1) > 1e6)
        failed[act[bad]] = True
        conv = ~bad & (np.max(np.abs(delta), axis=1) <= tol)
        done[act[conv]] = True
    return xi, done


def _vertex_shape_batched(dim, xi):
    """Q1 vertex functions at one point per pair: N [M, 2^d], dN [M, 2^d, d]."""
    M = xi.shape[0]
    nv = 2 ** dim
    N = np.ones((M, nv))
    dN = np.ones((M, nv, dim))
    for b in range(nv):
        for a in range(dim):
            bit = (b >> a) & 1
            f = xi[:, a] if bit else 1.0 - xi[:, a]
            df = 1.0 if bit else -1.0
            N[:, b] *= f
            for c in range(dim):
                dN[:, b, c] *= df if c == a else f
    return N, dN


def expanded_boxes(space, expand=EXPAND):
    cv = space.cell_vertices
    lo = cv.min(axis=1)
    hi = cv.max(axis=1)
    diag = np.linalg.norm(hi - lo, axis=1)
    return lo - expand * diag[:, None], hi + expand * diag[:, None]


def candidate_pairs_bruteforce(points, space, expand=EXPAND):
    """All (point, cell) pairs whose grown box contains the point, by testing every pair."""
    lo, hi = expanded_boxes(space, expand)
    inside = np.all((points[:, None, :] >= lo[None]) & (points[:, None, :] <= hi[None]), axis=2)
    p, c = np.nonzero(inside)
    return p, c


def candidate_pairs_bucketed(points, space, expand=EXPAND):
    """Same pairs as the brute-force search; a uniform grid only prefilters them."""
    lo, hi = expanded_boxes(space, expand)
    d = points.shape[1]
    glo = np.minimum(lo.min(axis=0), points.min(axis=0))
    ghi = np.maximum(hi.max(axis=0), points.max(axis=0))
    size = np.median(hi - lo, axis=0)
    nb = np.maximum(1, np.minimum(512, np.ceil((ghi - glo) / size))).astype(np.int64)
    step = (ghi - glo) / nb

    def bucket(x):
        return np.clip(np.floor((x - glo) / step).astype(np.int64), 0, nb - 1)

    blo = bucket(lo)
    bhi = bucket(hi)
    strides = np.cumprod(np.concatenate([[1], nb[:-1]]))
    # every (cell, bucket) pair with the bucket inside the cell's bucket range
    span = bhi - blo + 1
    count = np.prod(span, axis=1)
    cell_ids = np.repeat(np.arange(lo.shape[0]), count)
    local = np.arange(cell_ids.size) - np.repeat(np.cumsum(count) - count, count)
    coords = np.empty((cell_ids.size, d), dtype=np.int64)
    rem = local.copy()
    for a in range(d):
        sa = span[cell_ids, a]
        coords[:, a] = blo[cell_ids, a] + rem % sa
        rem //= sa
    bucket_ids = [coords @ strides]
    cell_ids = [cell_ids]
    bucket_ids = np.concatenate(bucket_ids)
    cell_ids = np.concatenate(cell_ids)
    order = np.lexsort((cell_ids, bucket_ids))
    bucket_ids, cell_ids = bucket_ids[order], cell_ids[order]
    nbt = int(np.prod(nb))
    offs = np.searchsorted(bucket_ids, np.arange(nbt + 1))
    pb = bucket(points) @ strides
    cnt = offs[pb + 1] - offs[pb]
    p = np.repeat(np.arange(points.shape[0]), cnt)
    start = np.repeat(offs[pb], cnt)
    local = np.arange(p.size) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    c = cell_ids[start + local]
    keep = np.all((points[p] >= lo[c]) & (points[p] <= hi[c]), axis=1)
    p, c = p[keep], c[keep]
    order = np.lexsort((c, p))
    return p[order], c[order]


POINT_CHUNK = 100000


def locate(points, coarse, bruteforce=False, expand=EXPAND, inside_tol=INSIDE_TOL,
           newton_tol=NEWTON_TOL, newton_max_it=NEWTON_MAX_IT):
    """Owner cell, clamped reference position and projection flag of each point.

    Every point is located on its own, so large point sets are processed in
    slices of POINT_CHUNK points (memory only; the result is the same)."""
    points = np.asarray(points, dtype=np.float64)
    if points.shape[0] > POINT_CHUNK:
        parts = [_locate(points[s:s + POINT_CHUNK], coarse, bruteforce, expand, inside_tol, newton_tol,
                         newton_max_it) for s in range(0, points.shape[0], POINT_CHUNK)]
        return tuple(np.concatenate([pt[i] for pt in parts]) for i in range(3))
    return _locate(points, coarse, bruteforce, expand, inside_tol, newton_tol, newton_max_it)


def _locate(points, coarse, bruteforce, expand, inside_tol, newton_tol, newton_max_it):
    P, d = points.shape
    if bruteforce:
        p, c = candidate_pairs_bruteforce(points, coarse, expand)
    else:
        p, c = candidate_pairs_bucketed(points, coarse, expand)
    order = np.lexsort((c, p))
    p, c = p[order], c[order]
    xi, conv = newton_inverse(coarse.cell_vertices[c], points[p], newton_tol, newton_max_it)
    clamped = np.clip(xi, 0.0, 1.0)
    dist_inf = np.max(np.abs(xi - clamped), axis=1)
    dist_2 = np.linalg.norm(xi - clamped, axis=1)
    owner = np.full(P, -1, dtype=np.int64)
    ref = np.zeros((P, d))
    projected = np.zeros(P, dtype=bool)
    # pass 1: inside candidates, lowest cell number (pairs are sorted by (p, c))
    ins = conv & (dist_inf <= inside_tol)
    idx = np.nonzero(ins)[0]
    first = np.unique(p[idx], return_index=True)
    sel = idx[first[1]]
    owner[p[sel]] = c[sel]
    ref[p[sel]] = clamped[sel]
    # pass 2: nearest pre-image for the rest
    rest = conv & (owner[p] < 0)
    idx = np.nonzero(rest)[0]
    if idx.size:
        o = np.lexsort((c[idx], dist_2[idx], p[idx]))
        idx = idx[o]
        first = np.unique(p[idx], return_index=True)
        sel = idx[first[1]]
        owner[p[sel]] = c[sel]
        ref[p[sel]] = clamped[sel]
        projected[p[sel]] = True
    if np.any(owner < 0):
        raise PointNotFound(f"{int(np.sum(owner < 0))} points have no owning coarse cell")
    return owner, ref, projected


def prolongation(fine, coarse, bruteforce=False):
    """Sparse P [N_fine, N_coarse] with P_ij = phi_j(x_i) (free rows and columns only)."""
    free_f = np.nonzero(fine.free)[0]
    owner, ref, projected = locate(fine.support_points[free_f], coarse, bruteforce)
    vals = basis.shape_values(coarse.k, coarse.dim, ref)  # [P, q_c]
    cols = coarse.cell_dofs[owner]  # [P, q_c]
    rows = np.repeat(free_f, cols.shape[1]).reshape(cols.shape)
    keep = coarse.free[cols]
    P = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])),
                      shape=(fine.n_dofs, coarse.n_dofs)).tocsr()
    P.sum_duplicates()
    info = dict(owner=owner, ref=ref, projected=projected, points=free_f)
    return P, info
