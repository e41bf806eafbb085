"""GPU parity of the level setup and the sum-factorisation operator against the oracle.

Bar: float64 results within 1e-12 of the oracle relative to the largest entry
of the reference (max |gpu - oracle| <= 1e-12 max |oracle|); float32 within
2e-5 (a few units of float32 rounding, amplified by the ~27-125 term sums).
"""

import numpy as np
import pytest
import torch

from oracle import assemble
from workloads import config_levels, config_source, perturb_interior, random_vector, scramble, structured_box

from _parity import DEV, Pair, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _mesh(dim, n, alpha, seed, scram):
    m = structured_box(dim, n)
    if alpha:
        m = perturb_interior(m, alpha, 1.0 / n, np.random.default_rng(seed))
    if scram:
        m = scramble(m, np.random.default_rng(seed + 1))
    return m


CASES = [(2, 1, 9), (2, 2, 7), (2, 3, 5), (2, 4, 5), (3, 1, 9), (3, 2, 7), (3, 3, 5), (3, 4, 4)]


@pytest.mark.parametrize("dim,k,n", CASES)
@pytest.mark.parametrize("scram", [False, True])
def test_vmult_matches_assembled_operator(ctx, dim, k, n, scram):
    p = Pair(ctx, _mesh(dim, n, 0.2, 7 * n + k, scram), k)
    x = random_vector(p.orc.n_dofs, 3)
    ref = p.A @ x
    y = p.lib.vmult(p.to_lib(x))
    assert rel_err(p.to_orc(y), ref) <= TOL64
    y32 = p.lib.vmult(p.to_lib(x, torch.float32))
    assert rel_err(p.to_orc(y32), ref) <= TOL32
    # accumulate form: unconstrained block only, added to dst
    free = p.orc.free
    xf = np.where(free, x, 0.0)
    base = random_vector(p.orc.n_dofs, 4)
    acc = p.lib.vmult_add(p.to_lib(x), p.to_lib(base))
    expect = base + np.where(free, p.A @ xf, 0.0)
    assert rel_err(p.to_orc(acc), expect) <= TOL64


@pytest.mark.parametrize("dim,k,n", CASES)
def test_diagonal_and_rhs(ctx, dim, k, n):
    p = Pair(ctx, _mesh(dim, n, 0.2, 11 * n + k, True), k)
    d = p.to_orc(p.lib.diagonal())
    assert rel_err(d, p.A.diagonal()) <= TOL64
    f = config_source(1) if dim == 3 else (lambda x: 1.0 + np.sin(3 * x[..., 0]) * x[..., 1])
    qp = p.lib.quadrature_points()
    fq = torch.tensor(f(qp).reshape(-1), dtype=torch.float64, device=DEV)
    b = p.to_orc(p.lib.assemble_rhs(fq))
    assert rel_err(b, assemble.load_vector(p.orc, f)) <= TOL64


def test_quadrature_points_match(ctx):
    m = _mesh(3, 4, 0.2, 5, True)
    p = Pair(ctx, m, 3)
    assert np.abs(p.lib.quadrature_points() - assemble.quadrature_points(p.orc)).max() < 1e-14


def test_config1_level_sizes_and_vmult(ctx):
    """The 13^3 level of the 3D Q2 workload, several blocks and a ragged tail."""
    p = Pair(ctx, config_levels(1, cells=[13])[0], 2)
    assert p.lib.n_dofs == 27 ** 3 and p.lib.n_free == 25 ** 3
    x = random_vector(p.orc.n_dofs, 9)
    assert rel_err(p.to_orc(p.lib.vmult(p.to_lib(x))), p.A @ x) <= TOL64


def test_errors_are_reported(ctx):
    import paper_2412_10910_amd as nn
    m = structured_box(2, 2)
    with pytest.raises(nn.NNMGError) as e:
        nn.Level.from_mesh(ctx, m, 5)
    assert e.value.name == "UNSUPPORTED"
    bad = structured_box(2, 2)
    bad.cells = bad.cells[:, [1, 0, 3, 2]].copy()  # mirrored cells: negative Jacobian
    with pytest.raises(nn.NNMGError) as e:
        nn.Level.from_mesh(ctx, bad, 1)
    assert e.value.name == "MESH"
    bad = structured_box(2, 2)
    bad.cells[0, 0] = 99
    with pytest.raises(nn.NNMGError) as e:
        nn.Level.from_mesh(ctx, bad, 1)
    assert e.value.name == "MESH"
    lv = nn.Level.from_mesh(ctx, m, 1)
    x = lv.empty()
    with pytest.raises(nn.NNMGError):
        lv.vmult(x, x)


@pytest.mark.parametrize("dim,k,n", [(2, 2, 9), (3, 2, 7), (3, 4, 4)])
def test_slot_scatter_is_deterministic_and_matches_atomics(ctx, dim, k, n, monkeypatch):
    """The default scatter (per-cell contributions summed per DoF in a fixed
    order) gives bitwise identical results on repeated calls, and agrees with
    the float-atomic scatter and with the stored-metric geometry to 1e-13."""
    import paper_2412_10910_amd as nn
    m = _mesh(dim, n, 0.2, 13 * n + k, True)
    lv = nn.Level.from_mesh(ctx, m, k)
    x = torch.tensor(random_vector(lv.n_dofs, 21), device=DEV)
    y1 = lv.vmult(x)
    y2 = lv.vmult(x)
    assert torch.equal(y1, y2)
    monkeypatch.setenv("NNMG_SCATTER", "atomic")
    la = nn.Level.from_mesh(ctx, m, k)
    ya = la.vmult(x)
    assert float((ya - y1).abs().max()) <= 1e-13 * float(y1.abs().max())
    monkeypatch.setenv("NNMG_SCATTER", "slots")
    monkeypatch.setenv("NNMG_GEOMETRY", "metric")
    lm = nn.Level.from_mesh(ctx, m, k)
    ym = lm.vmult(x)
    assert float((ym - y1).abs().max()) <= 1e-13 * float(y1.abs().max())
