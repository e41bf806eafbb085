"""Pins of the elasticity oracle (paper §4, Applications to FEA): what the
mathematics fixes for the vector Q_k discretization of linear elasticity.

* The six rigid-body motions (eq. ``rbm``) are exactly representable and lie
  in the kernel of the operator with free boundary, and the kernel has
  exactly that dimension; with a clamped face the operator is definite.
* Symmetry, and the patch test: a linear displacement (constant strain) has
  zero residual at every node off the boundary on perturbed, scrambled meshes.
* A displacement field in Q_2 that vanishes on the boundary is reproduced
  exactly when its body force is integrated (affine cells).
* O(h^{k+1}) L2 convergence for a smooth solution on perturbed meshes.
* Rigid-body motions are transferred exactly by the non-nested prolongation.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import assemble, elasticity as el, space, transfer
from workloads import config_levels, dirichlet_face, perturb_interior, scramble, structured_brick

LAM, MU = 1.0, 1.0


def _brick(cells, hi, alpha=0.0, seed=0, scram=False):
    m = structured_brick(cells, (0.0, 0.0, 0.0), hi)
    if alpha > 0:
        m = perturb_interior(m, alpha, [hi[a] / cells[a] for a in range(3)], np.random.default_rng(seed))
    if scram:
        m = scramble(m, np.random.default_rng(seed + 1))
    return m


@pytest.mark.parametrize("k,scram", [(1, True), (2, False), (2, True), (3, True)])
def test_rigid_body_modes_span_the_kernel(k, scram):
    m = _brick((3, 2, 2), (1.5, 1.0, 1.0), alpha=0.2, seed=k, scram=scram)
    V = space.Space(m, k)
    K = el.stiffness(V, LAM, MU, constrain=False)
    scale = abs(K).max()
    for r in el.rigid_body_modes(V):
        assert np.abs(K @ r).max() <= 1e-12 * scale * np.abs(r).max()
    if k == 1:
        # the kernel is exactly six-dimensional (no spurious zero-energy modes)
        ev = sla.eigvalsh(K.toarray())
        assert np.all(np.abs(ev[:6]) <= 1e-10 * ev[-1])
        assert ev[6] > 1e-6 * ev[-1]


def test_symmetric_and_definite_with_a_clamped_face():
    m = dirichlet_face(_brick((3, 2, 2), (1.5, 1.0, 1.0), alpha=0.2, seed=3), 0, 0.0)
    V = space.Space(m, 2)
    K = el.stiffness(V, LAM, MU)
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    free = el.vector_free(V)
    ev = sla.eigvalsh(K.toarray()[np.ix_(free, free)])
    assert ev[0] > 0


@pytest.mark.parametrize("k", [1, 2, 3])
def test_patch_test_constant_strain(k):
    m = _brick((3, 3, 2), (1.0, 1.0, 0.7), alpha=0.25, seed=10 + k, scram=True)
    V = space.Space(m, k)
    K = el.stiffness(V, LAM, MU, constrain=False)
    rng = np.random.default_rng(20 + k)
    A, b = rng.normal(size=(3, 3)), rng.normal(size=3)
    u = (V.support_points @ A.T + b).reshape(-1)
    # nodes off the boundary of the box
    x = V.support_points
    inner = np.all((x > 1e-9) & (x < np.array([1.0, 1.0, 0.7]) - 1e-9), axis=1)
    r = (K @ u).reshape(-1, 3)[inner]
    assert np.abs(r).max() <= 1e-12 * abs(K).max() * np.abs(u).max()


def _poly_solution():
    """u = (1, -2, 3/2) g with g = p(x) p(y) p(z), p(t) = t (1 - t): in Q_2,
    zero on the boundary of the unit cube; f = -mu lap u - (lam + mu) grad div u."""
    a = np.array([1.0, -2.0, 1.5])

    def parts(x):
        t = [x[..., i] for i in range(3)]
        p = [ti * (1 - ti) for ti in t]
        dp = [1 - 2 * ti for ti in t]
        return p, dp

    def u(x):
        p, _ = parts(x)
        g = p[0] * p[1] * p[2]
        return g[..., None] * a

    def f(x):
        p, dp = parts(x)
        H = np.empty(x.shape[:-1] + (3, 3))
        for i in range(3):
            for j in range(3):
                if i == j:
                    prod = -2.0 * np.prod([p[m] for m in range(3) if m != i], axis=0)
                else:
                    other = [m for m in range(3) if m not in (i, j)][0]
                    prod = dp[i] * dp[j] * p[other]
                H[..., i, j] = prod
        lap = np.trace(H, axis1=-2, axis2=-1)
        graddiv = H @ a
        return -MU * lap[..., None] * a - (LAM + MU) * graddiv

    return u, f


def test_exact_reproduction_of_a_q2_displacement():
    u, f = _poly_solution()
    V = space.Space(_brick((3, 2, 3), (1.0, 1.0, 1.0)), 2)  # every boundary vertex clamped
    K = el.stiffness(V, LAM, MU)
    b = el.load_vector(V, f)
    uh = spla.spsolve(K.tocsc(), b)
    uI = u(V.support_points).reshape(-1) * el.vector_free(V)
    assert np.abs(uh - uI).max() <= 1e-12 * np.abs(uI).max()


def test_l2_convergence_rate_q2():
    a = np.array([1.0, 2.0, -1.0])
    pi = np.pi

    def u(x):
        s = np.sin(pi * x[..., 0]) * np.sin(pi * x[..., 1]) * np.sin(pi * x[..., 2])
        return s[..., None] * a

    def f(x):
        sx, sy, sz = (np.sin(pi * x[..., i]) for i in range(3))
        cx, cy, cz = (np.cos(pi * x[..., i]) for i in range(3))
        S = sx * sy * sz
        H = np.empty(x.shape[:-1] + (3, 3))
        H[..., 0, 0] = H[..., 1, 1] = H[..., 2, 2] = -pi * pi * S
        H[..., 0, 1] = H[..., 1, 0] = pi * pi * cx * cy * sz
        H[..., 0, 2] = H[..., 2, 0] = pi * pi * cx * sy * cz
        H[..., 1, 2] = H[..., 2, 1] = pi * pi * sx * cy * cz
        return -MU * (-3 * pi * pi * S)[..., None] * a - (LAM + MU) * (H @ a)

    errs = []
    for n in (2, 4):
        V = space.Space(_brick((n, n, n), (1.0, 1.0, 1.0), alpha=0.15, seed=30 + n), 2)
        K = el.stiffness(V, LAM, MU)
        uh = spla.spsolve(K.tocsc(), el.load_vector(V, f)).reshape(-1, 3)
        e2 = sum(assemble.l2_error(V, uh[:, c], lambda x, c=c: u(x)[..., c]) ** 2 for c in range(3))
        errs.append(np.sqrt(e2))
    rate = np.log2(errs[0] / errs[1])
    assert 2.6 <= rate <= 3.6, (errs, rate)


def test_prolongation_transfers_rigid_motions_exactly():
    coarse, fine = config_levels(3, cells=[(3, 1, 1), (7, 2, 2)])
    Vc, Vf = space.Space(coarse, 2), space.Space(fine, 2)
    P, _ = transfer.prolongation(Vf, Vc)
    # rigid motions are linear: exact across non-nested levels on every free row
    # (columns of constrained coarse nodes are dropped, so compare where the
    # coarse motion vanishes on the clamped face: translations along x are not)
    Pv = el.vector_prolongation(P, 3)
    free_f = el.vector_free(Vf)
    for rc, rf in zip(el.rigid_body_modes(Vc), el.rigid_body_modes(Vf)):
        rc = rc * el.vector_free(Vc)
        got = Pv @ rc
        # fine points whose owner cell touches the clamped face see the dropped columns
        ok = free_f & (np.repeat(Vf.support_points[:, 0], 3) > 5.0 / 3 + 1e-9)
        assert np.abs(got[ok] - rf[ok]).max() <= 1e-12 * np.abs(rf).max()


def test_cantilever_tip_deflection_and_multigrid():
    """Beam [0,5] x [0,1]^2 clamped at x = 0 under the body load (0, 0, -1),
    lam = mu = 1 (E = 2.5, nu = 0.25, G = 1): the mean tip deflection lies
    between the Euler-Bernoulli value q L^4 / (8 E I) = 375 and the Timoshenko
    value with shear factor 5/6, 375 + q L^2 / (2 (5/6) G A) = 390 (a soft,
    physical pin), and the non-nested V-cycle preconditions CG to 1e-8 in a
    few iterations with the solution of the direct solve."""
    from oracle import multigrid
    from workloads import config_source
    ms = config_levels(3, cells=[(5, 1, 1), (10, 2, 2), (20, 4, 4)])
    Vs = [space.Space(m, 2) for m in ms]
    As = [el.stiffness(V, LAM, MU) for V in Vs]
    b = el.load_vector(Vs[-1], config_source(3))
    u = spla.spsolve(As[-1].tocsc(), b)
    x = Vs[-1].support_points
    w = u.reshape(-1, 3)[np.isclose(x[:, 0], 5.0), 2].mean()
    assert 0.97 * 375.0 <= -w <= 1.03 * 390.0
    Ps = [el.vector_prolongation(transfer.prolongation(Vs[i + 1], Vs[i])[0], 3) for i in range(2)]
    starts = [np.random.default_rng(i).uniform(-1, 1, V.n_dofs * 3) for i, V in enumerate(Vs)]
    H = multigrid.Hierarchy(As, [el.vector_free(V) for V in Vs], Ps, eig_start=starts)
    xh, it, hist = H.pcg(b, rtol=1e-8)
    assert it <= 15 and hist[-1] <= 1e-8
    assert np.abs(xh - u).max() <= 1e-6 * np.abs(u).max()
