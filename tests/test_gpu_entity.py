"""GPU parity of the operator with entity-compressed indices (autotuner
variants 4 and 5: one record of entity DoF bases, slot bases, writer counts
and orientations per cell) against the oracle.

The variants change where the operator reads its indices and in which order
the cell contributions of a DoF are summed, never what is summed, so the bars
are the operator's: float64 within 1e-12 of the oracle relative to the
largest entry, float32 within 2e-5; V-cycle within 1e-12; float64-MG PCG with
the oracle's iteration count and residual history within 1e-12.  Scrambled
meshes (random orientation-preserving vertex rotations per cell, renumbered
vertices and cells) exercise every edge and face orientation code.
"""

import numpy as np
import pytest
import torch

from workloads import config_levels, perturb_interior, random_vector, scramble, structured_box

from _parity import DEV, Pair, rel_err
from test_gpu_solver import _setup

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _mesh(n, seed, scram):
    m = perturb_interior(structured_box(3, n), 0.2, 1.0 / n, np.random.default_rng(seed))
    if scram:
        m = scramble(m, np.random.default_rng(seed + 1))
    return m


@pytest.mark.parametrize("k,n", [(3, 6), (4, 5)])
@pytest.mark.parametrize("scram", [False, True])
def test_entity_variants_match_assembled_operator(ctx, k, n, scram):
    p = Pair(ctx, _mesh(n, 31 * n + k, scram), k)
    x = random_vector(p.orc.n_dofs, 8)
    ref = p.A @ x
    free = p.orc.free
    base = random_vector(p.orc.n_dofs, 9)
    expect_add = base + np.where(free, p.A @ np.where(free, x, 0.0), 0.0)
    for v in (4, 5, 10, 11):
        p.lib.set_variant(v)
        assert p.lib.variant == v
        for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
            assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x, dt))), ref) <= tol, (v, dt)
        acc = p.lib.vmult_add(p.to_lib(x), p.to_lib(base))
        assert rel_err(p.to_orc(acc), expect_add) <= TOL64, v


def test_entity_variant_several_right_hand_sides(ctx):
    p = Pair(ctx, config_levels(2, cells=[6])[0], 4)
    p.lib.set_variant(4)
    X = np.stack([random_vector(p.orc.n_dofs, 20 + r) for r in range(3)], axis=1)
    ref = p.A @ X
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        src = torch.stack([p.to_lib(X[:, r], dt) for r in range(3)], dim=1).contiguous()
        out = p.lib.vmult(src)
        for r in range(3):
            assert rel_err(p.to_orc(out[:, r]), ref[:, r]) <= tol, (r, dt)


def test_each_precision_keeps_its_own_variant(ctx):
    """float64 on the per-node layout, float32 on the entity records (and the
    reverse): each precision's product uses its own kernels and slot offsets."""
    p = Pair(ctx, _mesh(5, 77, True), 3)
    x = random_vector(p.orc.n_dofs, 10)
    ref = p.A @ x
    for v64, v32 in ((0, 4), (5, 2), (4, 0)):
        p.lib.set_variant(v64, torch.float64)
        p.lib.set_variant(v32, torch.float32)
        assert (p.lib.variant_of(torch.float64), p.lib.variant_of(torch.float32)) == (v64, v32)
        assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x, torch.float64))), ref) <= TOL64
        assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x, torch.float32))), ref) <= TOL32
    r = p.lib.tune(torch.float32, reps=2)
    assert set(r["ms"]) == {"trilinear+slots", "metric+slots", "trilinear+slots+transposed", "metric+slots+transposed"} | {"trilinear+entity", "metric+entity", "trilinear+entity+transposed", "metric+entity+transposed"}
    assert p.lib.VARIANTS[p.lib.variant_of(torch.float32)] == r["chosen"]
    assert p.lib.variant_of(torch.float64) == 4  # untouched by the float32 tuning


def test_entity_variant_not_offered_below_degree_3(ctx):
    import paper_2412_10910_amd as nn
    lv = nn.Level.from_mesh(ctx, config_levels(1, cells=[4])[0], 2)
    with pytest.raises(nn.NNMGError):
        lv.set_variant(4)
    r = lv.tune(torch.float32, reps=2)
    assert set(r["ms"]) == {"trilinear+slots", "metric+slots", "trilinear+slots+transposed", "metric+slots+transposed"}


@pytest.mark.parametrize("cells,k", [([3, 5, 9], 3), ([3, 7], 4)])
def test_entity_variant_vcycle_and_pcg_parity(ctx, cells, k):
    pairs, H_orc, H_lib, b_orc, b_lib = _setup(ctx, 2, cells, k)
    for l in range(1, len(pairs)):
        H_lib.set_cheb_bounds(l, *H_orc.bounds[l])
    for p in pairs[1:]:
        p.lib.set_variant(4)
    fine = pairs[-1]
    r = np.where(fine.orc.free, random_vector(fine.orc.n_dofs, 78), 0.0)
    assert rel_err(fine.to_orc(H_lib.vcycle(fine.to_lib(r))), H_orc.vcycle(r)) <= 1e-12
    x_orc, it_orc, hist_orc = H_orc.pcg(b_orc, rtol=1e-8)
    x_lib, info = H_lib.pcg_solve(b_lib, rtol=1e-8, vcycle_dtype=torch.float64)
    assert info["iterations"] == it_orc
    assert np.abs(info["history"] - np.array(hist_orc)).max() <= 1e-12
    assert rel_err(fine.to_orc(x_lib), x_orc) <= 1e-10
    x32, info32 = H_lib.pcg_solve(b_lib, rtol=1e-8, vcycle_dtype=torch.float32)
    assert info32["relres"] <= 1e-8 and abs(info32["iterations"] - it_orc) <= 1
    # tuned: the tuner may pick any deterministic variant; the solve stays
    # within the same bars
    H_lib.tune(torch.float32, reps=2)
    x_t, info_t = H_lib.pcg_solve(b_lib, rtol=1e-8, vcycle_dtype=torch.float64)
    assert info_t["iterations"] == it_orc and rel_err(fine.to_orc(x_t), x_orc) <= 1e-10
