"""CPU oracle for the matrix-free non-nested multigrid method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle is a plain, slow, obviously correct implementation written from the
paper's definitions, in float64 NumPy/SciPy:

* ``basis``       -- Gauss-Legendre quadrature, Gauss-Lobatto support points and
                     1D Lagrange polynomials (paper §4: Q^p elements with a
                     (p+1)^d Gauss rule).
* ``space``       -- Q_k spaces on a quad/hex mesh with a bi/trilinear geometry
                     map, DoFs identified by their physical support point
                     (paper §2, eq. ``pointwise``), homogeneous Dirichlet DoFs.
* ``assemble``    -- assembled sparse stiffness matrix and load vector (paper §2,
                     eqs. ``problem`` to ``linear_system``).
* ``transfer``    -- brute-force point location with Newton inversion of the cell
                     map and the explicit sparse prolongation matrix
                     P_ij = phi_j^{l-1}(x_i) (paper §2 after eq. ``residual2``;
                     §3.1; §3.3 eq. ``closest_point``).  Restriction is P^T
                     (paper §2, eq. ``residual2``).
* ``multigrid``   -- Jacobi diagonal, Lanczos eigenvalue estimate, Chebyshev
                     smoother, dense coarse solve, the V-cycle of Algorithm
                     ``V_cycle`` and preconditioned CG (paper §2 and §4).

It shares no code with the HIP path.  Inputs come from the ``workloads``
package only.
"""

from . import basis, space, assemble, transfer, multigrid  # noqa: F401
