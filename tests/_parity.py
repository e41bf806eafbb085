"""Helpers shared by the GPU parity tests: build the same level on both sides
and map between the oracle's DoF order and the library's.

The DoF permutation is found by matching support points; the match itself is
checked (bijective, within 1e-12) before any value is compared, so it pins the
library's support points against the oracle's independently computed ones.
"""

from __future__ import annotations

import numpy as np
import torch
from scipy.spatial import cKDTree

from oracle import assemble, multigrid, space, transfer
from workloads import random_vector

DEV = "cuda:0"


def match_dofs(lib_points: np.ndarray, orc_points: np.ndarray) -> np.ndarray:
    """perm[i_lib] = i_orc such that the support points coincide."""
    dist, perm = cKDTree(orc_points).query(lib_points)
    scale = max(1.0, float(np.abs(orc_points).max()))
    assert dist.max() <= 1e-12 * scale, f"support points differ by {dist.max():.3e}"
    assert np.unique(perm).size == perm.size == orc_points.shape[0], "support points are not a bijection"
    return perm


class Pair:
    """One mesh level on both sides (Laplace, or linear elasticity with
    lam = mu = 1 and DoF 3 i + c for component c of node i on both sides)."""

    def __init__(self, ctx, mesh, degree, operator="laplace", lam=1.0, mu=1.0):
        import paper_2412_10910_amd as nn
        self.mesh = mesh
        self.k = degree
        self.operator, self.lam, self.mu = operator, lam, mu
        self.orc = space.Space(mesh, degree)
        self.lib = nn.Level.from_mesh(ctx, mesh, degree, operator, lam, mu)
        self.nc = self.lib.ncomp
        assert self.lib.n_dofs == self.orc.n_dofs * self.nc
        node_perm = match_dofs(self.lib.support_points()[:: self.nc], self.orc.support_points)
        self.perm = (self.nc * node_perm[:, None] + np.arange(self.nc)[None, :]).reshape(-1)
        self.free = np.repeat(self.orc.free, self.nc)  # oracle order
        assert np.array_equal(self.lib.constrained(), ~self.free[self.perm])
        self._A = None

    @property
    def A(self):
        if self._A is None:
            if self.operator == "elasticity":
                from oracle import elasticity
                self._A = elasticity.stiffness(self.orc, self.lam, self.mu)
            else:
                self._A = assemble.stiffness(self.orc)
        return self._A

    def to_lib(self, v_orc: np.ndarray, dtype=torch.float64) -> torch.Tensor:
        return torch.tensor(v_orc[self.perm], dtype=dtype, device=DEV)

    def to_orc(self, t: torch.Tensor) -> np.ndarray:
        out = np.empty(self.orc.n_dofs * self.nc)
        out[self.perm] = t.double().cpu().numpy()
        return out


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| (the elementwise bar of the parity tests)."""
    den = float(np.abs(b).max())
    return float(np.abs(a - b).max()) / (den if den > 0 else 1.0)


def build_pairs(ctx, meshes, degree, operator="laplace"):
    return [Pair(ctx, m, degree, operator) for m in meshes]


def oracle_prolongation(fine, coarse):
    P = transfer.prolongation(fine.orc, coarse.orc)[0]
    if fine.nc > 1:
        from oracle import elasticity
        P = elasticity.vector_prolongation(P, fine.nc)
    return P


def oracle_hierarchy(pairs, eig_start_orc, dtype=np.float64, bounds=None, cheb_degree=multigrid.CHEB_DEGREE):
    Ps = [oracle_prolongation(pairs[i + 1], pairs[i]) for i in range(len(pairs) - 1)]
    return multigrid.Hierarchy([p.A for p in pairs], [p.free for p in pairs], Ps, eig_start=eig_start_orc,
                               bounds=bounds, dtype=dtype, cheb_degree=cheb_degree)


def eig_starts(pairs, seed=100):
    return [random_vector(p.orc.n_dofs * p.nc, seed + i) for i, p in enumerate(pairs)]
