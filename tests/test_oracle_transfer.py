"""Pins of the oracle's non-nested transfer (point location and P).

* Linear functions are reproduced exactly across non-nested perturbed levels
  (Q1 geometry reproduces linear fields, so the coarse interpolant of a linear
  g evaluated at fine points is g itself).
* Q_k polynomials are reproduced across non-nested axis-aligned levels.
* Nested levels: P equals the Kronecker product of 1D embedding matrices
  obtained from a Vandermonde solve (the canonical injection, paper §4.1).
* Partition of unity, agreement of the bucketed and all-pairs searches, the
  pre-image property F_K(xi) = x, and the projection rule of eq.
  ``closest_point`` on the ball.
"""

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import basis, space, transfer
from workloads import ball_map, perturb_interior, scramble, structured_box


def _free_mesh(dim, n, alpha, seed, scram=False):
    m = structured_box(dim, n)
    if alpha:
        m = perturb_interior(m, alpha, 1.0 / n, np.random.default_rng(seed))
    if scram:
        m = scramble(m, np.random.default_rng(seed + 100))
    m.dirichlet[:] = 0
    return m


@pytest.mark.parametrize("dim,k,nf,nc", [(2, 1, 9, 4), (2, 2, 7, 3), (2, 4, 6, 4), (3, 1, 5, 2), (3, 2, 4, 3), (3, 3, 3, 2)])
def test_linear_exactness_nonnested_perturbed(dim, k, nf, nc):
    f = space.Space(_free_mesh(dim, nf, 0.2, 1, scram=True), k)
    c = space.Space(_free_mesh(dim, nc, 0.2, 2, scram=True), k)
    P, info = transfer.prolongation(f, c, bruteforce=True)
    for coef in ([1.0, 0.0, 0.0], [0.4, -1.3, 2.0]):
        g = lambda x: x @ np.array(coef[:dim]) + 0.7
        assert np.abs(P @ g(c.support_points) - g(f.support_points)).max() < 1e-13
    assert np.abs(P @ np.ones(c.n_dofs) - 1.0).max() < 1e-13
    assert not info["projected"].any()


@pytest.mark.parametrize("dim,k,nf,nc", [(2, 2, 7, 3), (2, 3, 5, 2), (3, 2, 5, 2)])
def test_qk_exactness_axis_aligned(dim, k, nf, nc):
    f = space.Space(_free_mesh(dim, nf, 0.0, 0), k)
    c = space.Space(_free_mesh(dim, nc, 0.0, 0), k)
    P, _ = transfer.prolongation(f, c, bruteforce=True)
    rng = np.random.default_rng(3)
    coef = rng.normal(size=[k + 1] * dim)

    def g(x):
        out = np.zeros(x.shape[0])
        for idx in np.ndindex(*coef.shape):
            out += coef[idx] * np.prod([x[:, a] ** idx[a] for a in range(dim)], axis=0)
        return out
    assert np.abs(P @ g(c.support_points) - g(f.support_points)).max() < 1e-12


@pytest.mark.parametrize("dim,k,nc", [(2, 1, 2), (2, 3, 2), (3, 2, 2)])
def test_nested_equals_kronecker_embedding(dim, k, nc):
    f = space.Space(structured_box(dim, 2 * nc), k)
    c = space.Space(structured_box(dim, nc), k)
    P, _ = transfer.prolongation(f, c, bruteforce=True)
    # 1D global node positions (GLL nodes per cell)
    gl = basis.gauss_lobatto_nodes(k)

    def nodes1d(n):
        x = np.unique(np.concatenate([(i + gl) / n for i in range(n)]).round(14))
        return x
    xf, xc = nodes1d(2 * nc), nodes1d(nc)
    # 1D embedding: each coarse global basis function is a piecewise polynomial of
    # degree k; on each coarse cell solve a Vandermonde system for its coefficients
    E = np.zeros((xf.size, xc.size))
    for cell in range(nc):
        loc = np.arange(cell * k, cell * k + k + 1)
        V = np.vander(xc[loc], k + 1, increasing=True)
        coef = np.linalg.solve(V, np.eye(k + 1))  # column j: coefficients of basis j
        inside = (xf >= cell / nc - 1e-14) & (xf <= (cell + 1) / nc + 1e-14)
        Vf = np.vander(xf[inside], k + 1, increasing=True)
        E[np.ix_(np.nonzero(inside)[0], loc)] = Vf @ coef
    Pk = E
    for _ in range(dim - 1):
        Pk = np.kron(E, Pk)  # lexicographic, first coordinate fastest
    # map tensor-grid order to each space's DoF order by coordinates
    def grid_order(sp, x1):
        pts = basis.tensor_points(x1, dim)
        dist, idx = cKDTree(sp.support_points).query(pts)
        assert dist.max() < 1e-12
        return idx
    of, oc = grid_order(f, xf), grid_order(c, xc)
    Pd = P.toarray()[np.ix_(of, oc)]
    freef = f.free[of]
    freec = c.free[oc]
    expect = Pk * freef[:, None] * freec[None, :]
    assert np.abs(Pd - expect).max() < 1e-13


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 1), (3, 3)])
def test_bucketed_equals_bruteforce_and_preimage(dim, k):
    f = space.Space(_free_mesh(dim, 5, 0.2, 7, scram=True), k)
    c = space.Space(_free_mesh(dim, 3, 0.2, 8, scram=True), k)
    pts = f.support_points
    o1, r1, p1 = transfer.locate(pts, c, bruteforce=True)
    o2, r2, p2 = transfer.locate(pts, c, bruteforce=False)
    assert np.array_equal(o1, o2) and np.array_equal(r1, r2) and np.array_equal(p1, p2)
    from oracle.space import vertex_shape
    for i in range(pts.shape[0]):
        N, _ = vertex_shape(dim, r1[i][None])
        x = N[0] @ c.cell_vertices[o1[i]]
        assert np.abs(x - pts[i]).max() < 1e-13


def test_ball_projection_rule():
    """Fine points outside the coarse polyhedral ball are evaluated at the
    nearest point of the closed reference cell (eq. ``closest_point``)."""
    fm = ball_map(structured_box(3, 7, -1.0, 1.0))
    cm = ball_map(structured_box(3, 3, -1.0, 1.0))
    fm.dirichlet[:] = 0  # locate boundary points too
    f = space.Space(fm, 2)
    c = space.Space(cm, 2)
    o1, r1, p1 = transfer.locate(f.support_points, c, bruteforce=True)
    o2, r2, p2 = transfer.locate(f.support_points, c, bruteforce=False)
    assert np.array_equal(o1, o2) and np.array_equal(r1, r2)
    assert p1.any(), "the polyhedral fine ball reaches outside the coarse one"
    assert np.all((r1 >= 0) & (r1 <= 1))
    # for a projected point, no candidate cell contains it and the chosen cell
    # minimises the reference distance among candidates
    pts = f.support_points
    pp, cc = transfer.candidate_pairs_bruteforce(pts, c)
    xi, conv = transfer.newton_inverse(c.cell_vertices[cc], pts[pp])
    dist = np.linalg.norm(xi - np.clip(xi, 0, 1), axis=1)
    for i in np.nonzero(p1)[0][:50]:
        sel = (pp == i) & conv
        assert dist[sel].min() > transfer.INSIDE_TOL
        best = cc[sel][np.argmin(dist[sel])]
        assert best == o1[i]


def test_point_outside_every_box_is_an_error():
    c = space.Space(_free_mesh(2, 3, 0.0, 0), 1)
    with pytest.raises(transfer.PointNotFound):
        transfer.locate(np.array([[3.0, 3.0]]), c, bruteforce=True)


@pytest.mark.parametrize("dim,kf,kc", [(2, 2, 1), (2, 4, 3), (3, 2, 1), (3, 3, 2), (3, 4, 2), (3, 4, 3)])
def test_nested_polynomial_transfer_galerkin_identity(dim, kf, kc):
    """Polynomial coarsening on one mesh (paper §2, Coarse grid solvers): the
    spaces are nested, and on affine cells the Gauss rule integrates both
    operators exactly, so P^T A_f P = A_c on the free block.  Independent of
    how P is formed; a wrong or missing entry of P breaks it.  P also
    reproduces Q_kc polynomials exactly."""
    from oracle import assemble
    n = 3 if dim == 2 else 2
    m = structured_box(dim, n, 0.0, 1.0)
    Vf, Vc = space.Space(m, kf), space.Space(m, kc)
    P, _ = transfer.prolongation(Vf, Vc)
    Af, Ac = assemble.stiffness(Vf), assemble.stiffness(Vc)
    G = (P.T @ Af @ P).toarray()[np.ix_(Vc.free, Vc.free)]
    R = Ac.toarray()[np.ix_(Vc.free, Vc.free)]
    assert np.abs(G - R).max() <= 1e-12 * np.abs(R).max()
    # exact for a polynomial of degree kc in each variable (no Dirichlet mask)
    m.dirichlet[:] = 0
    Vf, Vc = space.Space(m, kf), space.Space(m, kc)
    P, _ = transfer.prolongation(Vf, Vc)
    g = lambda x: np.prod([(x[..., a] + 0.3) ** kc - 0.5 * x[..., a] for a in range(dim)], axis=0)
    assert np.abs(P @ g(Vc.support_points) - g(Vf.support_points)).max() <= 1e-13
