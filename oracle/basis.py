"""1D ingredients of tensor-product Q_k elements on the reference cell [0,1]^d.

* Gauss-Legendre rule with k+1 points (paper §4 uses (p+1)^d Gauss points).
* Gauss-Lobatto support points (paper §3.2, figure ``GaussLobatto``).
* Lagrange polynomials through a node set, their values and derivatives,
  evaluated with the plain product formula.

Multi-indices are lexicographic with the first coordinate fastest:
``a = a_0 + n a_1 + n^2 a_2``.
"""

from __future__ import annotations

import itertools

import numpy as np


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [0, 1]: points, weights."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def gauss_lobatto_nodes(k: int) -> np.ndarray:
    """k+1 Gauss-Lobatto points on [0, 1]: the end points and the roots of P_k'."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if k == 1:
        inner = np.array([])
    else:
        inner = np.sort(np.polynomial.legendre.Legendre.basis(k).deriv().roots().real)
    t = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (t + 1.0)


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """V[j, i] = phi_i(x_j) for the Lagrange polynomials phi_i through ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    out = np.ones((x.size, n))
    for i in range(n):
        for m in range(n):
            if m != i:
                out[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return out


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[j, i] = phi_i'(x_j), by the product rule applied to the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    out = np.zeros((x.size, n))
    for i in range(n):
        for l in range(n):
            if l == i:
                continue
            term = np.full(x.size, 1.0 / (nodes[i] - nodes[l]))
            for m in range(n):
                if m != i and m != l:
                    term *= (x - nodes[m]) / (nodes[i] - nodes[m])
            out[:, i] += term
    return out


def multi_indices(n: int, dim: int) -> np.ndarray:
    """All multi-indices of {0..n-1}^dim in lexicographic order, first index fastest."""
    out = [tuple(reversed(t)) for t in itertools.product(range(n), repeat=dim)]
    return np.array(out, dtype=np.int64)


def tensor_points(x1d: np.ndarray, dim: int) -> np.ndarray:
    """Tensor grid of a 1D point set: [n^dim, dim], lexicographic."""
    mi = multi_indices(x1d.size, dim)
    return x1d[mi]


def tensor_weights(w1d: np.ndarray, dim: int) -> np.ndarray:
    mi = multi_indices(w1d.size, dim)
    return np.prod(w1d[mi], axis=1)


def shape_values(k: int, dim: int, xi: np.ndarray) -> np.ndarray:
    """phi_a(xi_p) for the Q_k Lagrange basis on Gauss-Lobatto nodes: [P, (k+1)^dim]."""
    nodes = gauss_lobatto_nodes(k)
    xi = np.atleast_2d(xi)
    mi = multi_indices(k + 1, dim)
    out = np.ones((xi.shape[0], mi.shape[0]))
    for a in range(dim):
        v = lagrange_values(nodes, xi[:, a])  # [P, n]
        out *= v[:, mi[:, a]]
    return out


def shape_gradients(k: int, dim: int, xi: np.ndarray) -> np.ndarray:
    """Reference gradients d phi_a / d xi_c at points xi: [P, (k+1)^dim, dim]."""
    nodes = gauss_lobatto_nodes(k)
    xi = np.atleast_2d(xi)
    mi = multi_indices(k + 1, dim)
    vals = [lagrange_values(nodes, xi[:, a]) for a in range(dim)]
    ders = [lagrange_derivatives(nodes, xi[:, a]) for a in range(dim)]
    out = np.ones((xi.shape[0], mi.shape[0], dim))
    for c in range(dim):
        for a in range(dim):
            f = ders[a] if a == c else vals[a]
            out[:, :, c] *= f[:, mi[:, a]]
    return out
