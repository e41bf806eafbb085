"""Pins of the oracle's smoother, eigenvalue estimate, coarse solve, V-cycle and PCG.

* Chebyshev: on A = diag(lambda), D = I the error after one sweep is
  T_3((theta - lambda)/delta) / T_3(theta/delta) times the initial error.
* Lanczos: with as many steps as distinct eigenvalues, the tridiagonal
  matrix reproduces them exactly; with 12 steps the estimate is a lower bound
  of lambda_max(D^{-1}A) within a few percent.
* Coarse solve: residual at rounding level.
* V-cycle: linear, symmetric and positive definite (R = P^T, polynomial
  smoother, exact coarse solve).
* PCG: same iterates as SciPy's CG with the same preconditioner; converges.
* Paper §4.1, tables ``nested_2D`` / ``nested_3D``: 3 iterations on nested
  hierarchies for a 10^4 reduction (soft pin: the coarse solver differs).
"""

import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assemble, multigrid, space, transfer
from workloads import config_levels, config_source, random_vector, structured_box

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "nested_tables.txt")


def _cheb_T3(x):
    return 4 * x ** 3 - 3 * x


@pytest.mark.parametrize("start", ["zero", "nonzero"])
def test_chebyshev_error_polynomial_closed_form(start):
    lam = np.array([0.05, 0.1, 0.3, 0.7, 1.0, 1.4, 1.9])
    A = sp.diags(lam).tocsr()
    dinv = np.ones(lam.size)
    rng = np.random.default_rng(0)
    xs = rng.normal(size=lam.size)
    f = A @ xs
    hi = 2.0
    lo = hi / 20
    x0 = None if start == "zero" else rng.normal(size=lam.size)
    x = multigrid.chebyshev(A, dinv, f, x0, lo, hi)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    factor = _cheb_T3((theta - lam) / delta) / _cheb_T3(theta / delta)
    e0 = xs - (0 if x0 is None else x0)
    assert np.allclose(xs - x, factor * e0, atol=1e-14, rtol=1e-12)


@pytest.mark.parametrize("degree", [1, 2, 4, 5])
@pytest.mark.parametrize("start", ["zero", "nonzero"])
def test_chebyshev_error_polynomial_any_degree(start, degree):
    # after k steps the error is T_k((theta - lambda)/delta) / T_k(theta/delta)
    # times the initial one, T_k from numpy's Chebyshev series
    lam = np.array([0.05, 0.1, 0.3, 0.7, 1.0, 1.4, 1.9])
    A = sp.diags(lam).tocsr()
    rng = np.random.default_rng(degree)
    xs = rng.normal(size=lam.size)
    f = A @ xs
    hi = 2.0
    lo = hi / 20
    x0 = None if start == "zero" else rng.normal(size=lam.size)
    x = multigrid.chebyshev(A, np.ones(lam.size), f, x0, lo, hi, degree=degree)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Tk = np.polynomial.chebyshev.Chebyshev.basis(degree)
    factor = Tk((theta - lam) / delta) / Tk(theta / delta)
    e0 = xs - (0 if x0 is None else x0)
    assert np.allclose(xs - x, factor * e0, atol=1e-14, rtol=1e-12)


def test_lanczos_exact_on_few_eigenvalues():
    lam = np.array([1.0, 2.0, 2.0, 3.0, 3.0, 3.0, 5.0])
    A = sp.diags(lam).tocsr()
    T = multigrid.lanczos_tridiagonal(A, np.ones(lam.size), np.ones(lam.size), iters=12)
    assert T.shape == (4, 4)  # four distinct eigenvalues: CG stops after 4 steps
    assert np.allclose(np.sort(np.linalg.eigvalsh(T)), [1.0, 2.0, 3.0, 5.0], atol=1e-12)


def test_lanczos_estimate_is_a_tight_lower_bound():
    sps = [space.Space(m, 2) for m in config_levels(1, cells=[3, 6])]
    A = assemble.stiffness(sps[1])
    free = sps[1].free
    dinv = multigrid.inverse_diagonal(A, free)
    v0 = np.where(free, random_vector(sps[1].n_dofs, 3), 0.0)
    est = multigrid.estimate_max_eigenvalue(A, dinv, v0)
    Af = A[free][:, free].toarray()
    d = np.sqrt(dinv[free])
    lam_max = np.linalg.eigvalsh(d[:, None] * Af * d[None, :]).max()
    assert est <= lam_max * (1 + 1e-12)
    assert est >= 0.9 * lam_max


def _hierarchy(cfg, cells, degree, dtype=np.float64, cheb_degree=multigrid.CHEB_DEGREE):
    sps = [space.Space(m, degree) for m in config_levels(cfg, cells=cells)]
    As = [assemble.stiffness(s) for s in sps]
    Ps = [transfer.prolongation(sps[i + 1], sps[i])[0] for i in range(len(sps) - 1)]
    starts = [random_vector(s.n_dofs, 17 + i) for i, s in enumerate(sps)]
    H = multigrid.Hierarchy(As, [s.free for s in sps], Ps, eig_start=starts, dtype=dtype, cheb_degree=cheb_degree)
    return sps, H


def test_coarse_solve_residual():
    sps, H = _hierarchy(1, [3, 6], 2)
    r = np.where(sps[0].free, random_vector(sps[0].n_dofs, 5), 0.0)
    x = H.coarse.solve(r)
    assert np.linalg.norm(H.A64[0] @ x - r) <= 1e-14 * np.linalg.norm(r)


@pytest.mark.parametrize("cfg,cells,k,cheb", [(0, [3, 7, 16], 1, 3), (1, [2, 4, 7], 2, 3), (1, [2, 4, 7], 2, 1),
                                              (1, [2, 4, 7], 2, 2), (1, [2, 4, 7], 2, 4)])
def test_vcycle_linear_symmetric_positive(cfg, cells, k, cheb):
    # the same smoothing polynomial before and after the coarse correction makes
    # the V-cycle symmetric for every smoother degree
    sps, H = _hierarchy(cfg, cells, k, cheb_degree=cheb)
    free = sps[-1].free
    n = sps[-1].n_dofs
    r = np.where(free, random_vector(n, 1), 0.0)
    s = np.where(free, random_vector(n, 2), 0.0)
    Vr, Vs = H.vcycle(r), H.vcycle(s)
    assert abs(Vr @ s - r @ Vs) <= 1e-13 * abs(Vr @ s)
    assert Vr @ r > 0 and Vs @ s > 0
    assert np.allclose(H.vcycle(2.0 * r - 3.0 * s), 2.0 * Vr - 3.0 * Vs, atol=1e-13 * np.abs(Vr).max())
    assert np.all(Vr[~free] == 0)


def test_pcg_matches_scipy_cg_with_same_preconditioner():
    sps, H = _hierarchy(0, [4, 9, 20], 1)
    b = assemble.load_vector(sps[-1], config_source(0))
    x, it, hist = H.pcg(b, rtol=1e-8)
    assert hist[-1] <= 1e-8
    M = spla.LinearOperator(H.A64[-1].shape, matvec=lambda v: H.vcycle(np.asarray(v).ravel()))
    count = [0]

    def cb(_):
        count[0] += 1
    xs, info = spla.cg(H.A64[-1], b, rtol=1e-8, atol=0.0, M=M, callback=cb)
    assert info == 0
    assert count[0] == it
    assert np.linalg.norm(xs - x) <= 1e-10 * np.linalg.norm(x)


def test_pcg_a_norm_error_decreases():
    sps, H = _hierarchy(1, [2, 4, 7], 2)
    A = H.A64[-1]
    b = assemble.load_vector(sps[-1], config_source(1))
    xstar = spla.spsolve(A.tocsc(), b)
    errs = []
    for m in range(1, 8):
        x, it, _ = H.pcg(b, rtol=0.0, max_it=m)
        e = x - xstar
        errs.append(float(e @ (A @ e)))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1) if errs[i] > 1e-26)


def test_fp32_vcycle_iterations_within_one():
    sps, H = _hierarchy(1, [2, 4, 8], 2)
    H32 = multigrid.Hierarchy(H.A64, [s.free for s in sps], [p for p in H.P], bounds=H.bounds,
                              dtype=np.float32)
    b = assemble.load_vector(sps[-1], config_source(1))
    _, it64, h64 = H.pcg(b)
    _, it32, h32 = H32.pcg(b)
    assert h32[-1] <= 1e-8 and abs(it32 - it64) <= 1


def _nested(dim, k, level):
    sps = [space.Space(structured_box(dim, 2 ** (i - 1), -1.0, 1.0), k) for i in range(1, level + 1)]
    As = [assemble.stiffness(s) for s in sps]
    Ps = [transfer.prolongation(sps[i + 1], sps[i])[0] for i in range(len(sps) - 1)]
    starts = [random_vector(s.n_dofs, 31 + i) for i, s in enumerate(sps)]
    H = multigrid.Hierarchy(As, [s.free for s in sps], Ps, eig_start=starts)
    b = assemble.load_vector(sps[-1], lambda x: np.ones(x.shape[:-1]))
    return H, b


def _golden_iterations():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            dim, k, level, dofs, its = (int(t) for t in line.split())
            if dofs <= 40000:
                out.append((dim, k, level, its))
    return out


@pytest.mark.parametrize("dim,k,level,its", _golden_iterations())
def test_nested_iteration_counts_soft_pin(dim, k, level, its):
    if k == 1 and level == 2:
        pytest.skip("a single unknown: CG terminates after one step whatever the preconditioner")
    H, b = _nested(dim, k, level)
    _, it, hist = H.pcg(b, rtol=1e-4)
    assert hist[-1] <= 1e-4
    assert abs(it - its) <= 1, (it, its)
