"""Smoother, coarse solver, V-cycle and preconditioned CG (paper §2, Algorithm
``V_cycle``; §4 solver settings).

* Point-Jacobi Chebyshev smoother of degree 3 (paper §4).  The recurrence is
  the three-term Chebyshev semi-iteration (Saad, Iterative Methods for Sparse
  Linear Systems, 2nd ed., Algorithm 12.1) applied to D^{-1} A on
  [lambda_max / 20, lambda_max], with the residual recomputed as f - A x at
  every step.  One smoothing sweep performs three updates of x; from a zero
  initial guess the first residual is f itself.
* lambda_max is 1.2 times the largest eigenvalue of the Lanczos tridiagonal
  matrix built from 12 steps of Jacobi-preconditioned CG (paper §4).
* Coarse-grid solve: exact, by a dense Cholesky factorisation of the
  unconstrained block plus one step of iterative refinement (stands in for
  the paper's AMG coarse solver).
* V-cycle: pre-smooth from zero, residual, restrict with P^T, recurse,
  prolongate and add, post-smooth starting from the current iterate.
* PCG (Saad, Algorithm 9.1) with one V-cycle as the preconditioner, x0 = 0,
  stopping when ||r_k||_2 <= rtol ||r_0||_2.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

CHEB_DEGREE = 3
SMOOTHING_RANGE = 20.0
EIG_SAFETY = 1.2
EIG_ITERS = 12


def inverse_diagonal(A, free) -> np.ndarray:
    d = A.diagonal().copy()
    out = np.zeros_like(d)
    out[free] = 1.0 / d[free]
    return out


def lanczos_tridiagonal(A, dinv, v0, iters=EIG_ITERS):
    """Tridiagonal Lanczos matrix from `iters` steps of Jacobi-PCG on A y = v0.

    With CG coefficients alpha_j, beta_j:
    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = sqrt(beta_j)/alpha_j.
    The iteration stops early if the residual vanishes (relative 1e-14).
    """
    r = v0.astype(np.float64).copy()
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    r0 = float(np.sqrt(r @ r))
    alphas, betas = [], []
    for _ in range(iters):
        q = A @ p
        pq = float(p @ q)
        if pq <= 0:
            break
        alpha = rz / pq
        alphas.append(alpha)
        r = r - alpha * q
        if np.sqrt(r @ r) <= 1e-14 * r0:
            break
        z = dinv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return T


def estimate_max_eigenvalue(A, dinv, v0, iters=EIG_ITERS) -> float:
    T = lanczos_tridiagonal(A, dinv, v0, iters)
    return float(np.max(np.linalg.eigvalsh(T)))


def chebyshev_bounds(lam_est: float, safety=EIG_SAFETY, ratio=SMOOTHING_RANGE):
    hi = safety * lam_est
    return hi / ratio, hi


def chebyshev(A, dinv, f, x0, lo, hi, degree=CHEB_DEGREE, dtype=np.float64):
    """Degree-`degree` Chebyshev semi-iteration on D^{-1}A over [lo, hi].

    x0 = None means a zero initial guess (then r_0 = f needs no product).
    """
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x0 is None:
        x = np.zeros_like(f)
        r = f.copy()
    else:
        x = x0.copy()
        r = f - A @ x
    d = (dinv * r) / dtype(theta)
    x = x + d
    for _ in range(1, degree):
        r = f - A @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = dtype(rho_new * rho) * d + dtype(2.0 * rho_new / delta) * (dinv * r)
        x = x + d
        rho = rho_new
    return x


class CoarseSolver:
    """Exact solve on the unconstrained block, plus one refinement step."""

    def __init__(self, A, free):
        self.A = A
        self.free = np.nonzero(free)[0]
        Aff = A[self.free][:, self.free].toarray()
        self.factor = sla.cho_factor(Aff, lower=True)

    def _solve_once(self, r):
        x = np.zeros_like(r, dtype=np.float64)
        if self.free.size:
            x[self.free] = sla.cho_solve(self.factor, r[self.free].astype(np.float64))
        return x

    def solve(self, r):
        r = r.astype(np.float64)
        x = self._solve_once(r)
        x = x + self._solve_once(r - self.A @ x)
        return x


class Hierarchy:
    """Levels coarse -> fine: operators A_l, free masks, P_l (level l-1 -> l)."""

    def __init__(self, operators, frees, prolongations, eig_start=None, bounds=None,
                 dtype=np.float64, cheb_degree=CHEB_DEGREE):
        self.L = len(operators)
        self.cheb_degree = cheb_degree  # smoothing steps (operator applications) per smoother call
        assert len(prolongations) == self.L - 1
        self.dtype = dtype
        self.A64 = operators
        self.frees = frees
        self.A = [a.astype(dtype) for a in operators]
        self.P = [p.astype(dtype) for p in prolongations]
        self.R = [p.T.tocsr() for p in self.P]
        self.dinv64 = [inverse_diagonal(a, f) for a, f in zip(operators, frees)]
        self.dinv = [d.astype(dtype) for d in self.dinv64]
        self.coarse = CoarseSolver(operators[0], frees[0])
        self.bounds = [None] * self.L
        for l in range(1, self.L):
            if bounds is not None and bounds[l] is not None:
                self.bounds[l] = tuple(bounds[l])
                continue
            v0 = eig_start[l] if eig_start is not None else None
            if v0 is None:
                raise ValueError("a Lanczos start vector is required for every level above the coarsest")
            v0 = np.where(frees[l], v0, 0.0)
            lam = estimate_max_eigenvalue(operators[l], self.dinv64[l], v0)
            self.bounds[l] = chebyshev_bounds(lam)

    def vcycle(self, f, l=None):
        """z = V(l, f) with a zero initial guess (Algorithm ``V_cycle``)."""
        if l is None:
            l = self.L - 1
        f = f.astype(self.dtype)
        if l == 0:
            return self.coarse.solve(f).astype(self.dtype)
        A, dinv = self.A[l], self.dinv[l]
        lo, hi = self.bounds[l]
        x = chebyshev(A, dinv, f, None, lo, hi, degree=self.cheb_degree, dtype=self.dtype)
        r = f - A @ x
        rc = self.R[l - 1] @ r
        dc = self.vcycle(rc, l - 1)
        x = x + self.P[l - 1] @ dc
        x = chebyshev(A, dinv, f, x, lo, hi, degree=self.cheb_degree, dtype=self.dtype)
        return x

    def pcg(self, b, rtol=1e-8, max_it=200, precondition=True):
        """PCG from x0 = 0; returns x, iterations, history of ||r_k|| / ||r_0||."""
        A = self.A64[-1]
        x = np.zeros_like(b)
        r = b.copy()
        r0 = float(np.linalg.norm(r))
        hist = [1.0]
        if r0 == 0.0:
            return x, 0, hist
        z = self.vcycle(r).astype(np.float64) if precondition else r.copy()
        p = z.copy()
        rz = float(r @ z)
        it = 0
        while it < max_it:
            q = A @ p
            alpha = rz / float(p @ q)
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            rel = float(np.linalg.norm(r)) / r0
            hist.append(rel)
            if rel <= rtol:
                break
            z = self.vcycle(r).astype(np.float64) if precondition else r.copy()
            rz_new = float(r @ z)
            beta = rz_new / rz
            p = z + beta * p
            rz = rz_new
        return x, it, hist
