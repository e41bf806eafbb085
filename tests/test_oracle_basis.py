"""Pins of the oracle's 1D and tensor-product ingredients against closed forms."""

import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_rule_exact_to_degree_2n_minus_1(n):
    x, w = basis.gauss_legendre(n)
    for m in range(2 * n):
        assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-13
    # and not beyond (degree 2n is integrated with an error)
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-9


def test_gauss_lobatto_closed_forms():
    s5 = 1.0 / np.sqrt(5.0)
    s37 = np.sqrt(3.0 / 7.0)
    expect = {
        1: [0.0, 1.0],
        2: [0.0, 0.5, 1.0],
        3: [0.0, 0.5 * (1 - s5), 0.5 * (1 + s5), 1.0],
        4: [0.0, 0.5 * (1 - s37), 0.5, 0.5 * (1 + s37), 1.0],
    }
    for k, e in expect.items():
        assert np.allclose(basis.gauss_lobatto_nodes(k), e, atol=1e-15, rtol=0)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_lagrange_cardinal_and_reproduction(k):
    nodes = basis.gauss_lobatto_nodes(k)
    V = basis.lagrange_values(nodes, nodes)
    assert np.allclose(V, np.eye(k + 1), atol=1e-14)
    x = np.linspace(-0.3, 1.3, 37)
    V = basis.lagrange_values(nodes, x)
    D = basis.lagrange_derivatives(nodes, x)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-12)
    # polynomials of degree <= k are reproduced, with their derivatives
    for m in range(k + 1):
        assert np.allclose(V @ nodes ** m, x ** m, atol=1e-12)
        dm = m * x ** (m - 1) if m > 0 else 0 * x
        assert np.allclose(D @ nodes ** m, dm, atol=1e-11)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (3, 2), (3, 4)])
def test_tensor_gradient_matches_finite_differences(dim, k):
    rng = np.random.default_rng(5)
    xi = rng.uniform(0.05, 0.95, size=(4, dim))
    g = basis.shape_gradients(k, dim, xi)
    h = 1e-6
    for c in range(dim):
        e = np.zeros(dim)
        e[c] = h
        fd = (basis.shape_values(k, dim, xi + e) - basis.shape_values(k, dim, xi - e)) / (2 * h)
        assert np.allclose(g[:, :, c], fd, atol=1e-7)


def test_multi_index_order_is_first_index_fastest():
    mi = basis.multi_indices(3, 3)
    assert mi[1].tolist() == [1, 0, 0]
    assert mi[3].tolist() == [0, 1, 0]
    assert mi[9].tolist() == [0, 0, 1]
