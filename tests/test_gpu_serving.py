"""The serving loop: requests on resident hierarchies of different sizes and
operators, with 1 to 8 right-hand sides, submitted together and admitted as
slots and memory free up.  Each result must be the same in the mix as alone
(bitwise: a request makes exactly the launches of a blocking solve), the
admission limits must hold, and requests on distinct hierarchies must run at
the same time.
"""

import numpy as np
import pytest
import torch

from workloads import config_levels, config_source, random_load, random_vector

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def setup():
    import paper_2412_10910_amd as nn
    ctx = nn.Context(0)
    specs = [(1, [3, 6, 13], 2, "laplace"), (2, [3, 5, 9], 3, "laplace"),
             (3, [(3, 1, 1), (7, 2, 2), (14, 3, 3)], 2, "elasticity"), (0, [9, 23, 64], 1, "laplace")]
    hs = []
    for cfg, cells, k, op in specs:
        meshes = config_levels(cfg, cells=cells)
        levels = [nn.Level.from_mesh(ctx, m, k, op) for m in meshes]
        transfers = [nn.Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
        hs.append((cfg, op, nn.Hierarchy(ctx, levels, transfers)))
    return nn, ctx, hs


def _rhs(cfg, op, H, nr, seed):
    fine = H.fine
    qp = fine.quadrature_points()
    cols = []
    for r in range(nr):
        f = random_load(seed + r) if op == "elasticity" else config_source(cfg, seed + r)
        cols.append(fine.assemble_rhs(torch.tensor(f(qp), device=DEV).reshape(-1)))
    return cols[0] if nr == 1 else torch.stack(cols, dim=1).contiguous()


def _requests(hs):
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(14):
        h = int(rng.integers(len(hs)))
        nr = int(rng.integers(1, 9))
        reqs.append((h, nr, 100 + 10 * i))
    return reqs


def _alone(hs, reqs, dt):
    out = []
    for h, nr, seed in reqs:
        cfg, op, H = hs[h]
        b = _rhs(cfg, op, H, nr, seed)
        x, info = H.pcg_solve(b, rtol=1e-8, vcycle_dtype=dt, history=False)
        out.append((b, x.clone(), info))
    return out


def _iters(info):
    return [i["iterations"] for i in info] if isinstance(info, list) else [info["iterations"]]


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_mix_equals_alone(setup, dt):
    nn, ctx, hs = setup
    reqs = _requests(hs)
    ref = _alone(hs, reqs, dt)
    srv = nn.Server(ctx, max_active=4)
    tickets = [srv.submit(hs[h][2], b, vcycle_dtype=dt) for (h, nr, seed), (b, _, _) in zip(reqs, ref)]
    for t, (b, x_ref, info_ref) in zip(tickets, ref):
        x, info, times = t.wait()
        assert _iters(info) == _iters(info_ref)
        assert torch.equal(x, x_ref)
        assert times["total_ms"] >= times["run_ms"] >= 0 and times["queued_ms"] >= 0
    st = srv.stats()
    assert st["submitted"] == st["completed"] == len(reqs)
    assert st["running"] == st["pending"] == 0 and st["reserved"] == 0
    assert 2 <= st["max_running"] <= 4  # distinct hierarchies ran at the same time
    srv.close()


def test_memory_budget_admits_one_at_a_time(setup):
    nn, ctx, hs = setup
    reqs = [(0, 3, 7), (1, 2, 9), (2, 4, 11), (0, 1, 13)]
    ref = _alone(hs, reqs, torch.float32)
    budget = min(hs[h][2].footprint(nr) for h, nr, _ in reqs)  # no two requests fit together
    srv = nn.Server(ctx, max_active=4, memory_budget=budget)
    tickets = [srv.submit(hs[h][2], b) for (h, nr, seed), (b, _, _) in zip(reqs, ref)]
    for t, (b, x_ref, info_ref) in zip(tickets, ref):
        x, info, _ = t.wait()
        assert torch.equal(x, x_ref) and _iters(info) == _iters(info_ref)
    st = srv.stats()
    assert st["max_running"] == 1 and st["completed"] == len(reqs)
    srv.close()


def test_admission_while_running(setup):
    """Requests submitted while others run are admitted as slots free up."""
    nn, ctx, hs = setup
    srv = nn.Server(ctx, max_active=2)
    first = [(3, 1, 21), (1, 8, 23)]
    later = [(0, 5, 25), (2, 2, 27), (3, 3, 29)]
    ref = _alone(hs, first + later, torch.float32)
    tickets = [srv.submit(hs[h][2], b) for (h, _, _), (b, _, _) in zip(first, ref[:2])]
    x0, _, _ = tickets[0].wait()
    tickets += [srv.submit(hs[h][2], b) for (h, _, _), (b, _, _) in zip(later, ref[2:])]
    assert torch.equal(x0, ref[0][1])
    for t, (b, x_ref, info_ref) in zip(tickets[1:], ref[1:]):
        x, info, _ = t.wait()
        assert torch.equal(x, x_ref) and _iters(info) == _iters(info_ref)
    assert srv.stats()["max_running"] <= 2
    srv.close()


def test_errors(setup):
    nn, ctx, hs = setup
    srv = nn.Server(ctx, max_active=1)
    H = hs[0][2]
    with pytest.raises(nn.NNMGError):
        srv.submit(H, torch.zeros(H.fine.n_dofs, 9, dtype=torch.float64, device=DEV))
    b = torch.tensor(random_vector(H.fine.n_dofs, 3), device=DEV)
    b[torch.tensor(H.fine.constrained(), device=DEV)] = 0
    t = srv.submit(H, b, max_it=1)
    with pytest.raises(nn.NNMGError):  # not converged in one iteration
        t.wait()
    with pytest.raises(nn.NNMGError):  # the ticket is retired
        t.wait()
    srv.close()


def test_hierarchies_sharing_levels_and_transfers(setup):
    """Two hierarchies over the same levels and transfers (replicas for a busy
    mesh: each holds its own work and restriction buffers) serve requests at
    the same time with the results of a lone solve."""
    nn, ctx, hs = setup
    cfg, op, H = hs[0]
    twin = nn.Hierarchy(ctx, H.levels, H.transfers)
    reqs = [(0, 4, 31), (0, 2, 33), (0, 8, 35), (0, 1, 37)]
    ref = _alone(hs, reqs, torch.float32)
    srv = nn.Server(ctx, max_active=2)
    tickets = [srv.submit([H, twin], b) for b, _, _ in ref]  # whichever replica is idle
    for t, (b, x_ref, info_ref) in zip(tickets, ref):
        x, info, _ = t.wait()
        assert torch.equal(x, x_ref) and _iters(info) == _iters(info_ref)
    assert srv.stats()["max_running"] == 2
    srv.close()


def test_mix_matches_the_oracle():
    """Every right-hand side of every request in a mix on Laplace Q1/Q2/Q3 and
    elasticity hierarchies is the float64 oracle's float64-MG PCG solution:
    the same iteration count and the solution within 1e-10 relative to its
    largest entry.  The library's hierarchies start Lanczos from the oracle's
    vectors and then take the oracle's Chebyshev bounds, so both sides run the
    same method."""
    import paper_2412_10910_amd as nn
    from oracle import assemble, elasticity
    from _parity import build_pairs, eig_starts, oracle_hierarchy, rel_err

    ctx = nn.Context(0)
    specs = [(0, [9, 23, 64], 1, "laplace"), (1, [3, 6, 13], 2, "laplace"), (2, [3, 5, 9], 3, "laplace"),
             (3, [(5, 1, 1), (10, 2, 2), (20, 4, 4)], 2, "elasticity")]
    sides = []
    for cfg, cells, k, op in specs:
        pairs = build_pairs(ctx, config_levels(cfg, cells=cells), k, op)
        starts = eig_starts(pairs)
        H_orc = oracle_hierarchy(pairs, starts)
        trs = [nn.Transfer(ctx, pairs[i + 1].lib, pairs[i].lib) for i in range(len(pairs) - 1)]
        H = nn.Hierarchy(ctx, [p.lib for p in pairs], trs, eig_start=[p.to_lib(s) for p, s in zip(pairs, starts)])
        for l in range(1, len(pairs)):
            H.set_cheb_bounds(l, *H_orc.bounds[l])
        sides.append((cfg, op, pairs, H_orc, H))
    # requests: (hierarchy, number of right-hand sides), sources by seed
    rng = np.random.default_rng(11)
    reqs = [(int(rng.integers(len(sides))), int(rng.integers(1, 4))) for _ in range(10)]
    bs, refs = [], []
    for i, (h, nr) in enumerate(reqs):
        cfg, op, pairs, H_orc, H = sides[h]
        fine = pairs[-1]
        cols_lib, cols_orc = [], []
        qp = fine.lib.quadrature_points()
        for r in range(nr):
            f = random_load(200 + 10 * i + r) if op == "elasticity" else config_source(cfg, 200 + 10 * i + r)
            cols_lib.append(fine.lib.assemble_rhs(torch.tensor(f(qp), device=DEV).reshape(-1)))
            cols_orc.append(elasticity.load_vector(fine.orc, f) if op == "elasticity"
                            else assemble.load_vector(fine.orc, f))
        bs.append(cols_lib[0] if nr == 1 else torch.stack(cols_lib, dim=1).contiguous())
        refs.append((h, cols_orc))
    # every request submitted at once, so that they share the device
    srv = nn.Server(ctx, max_active=4)
    tickets = [srv.submit(sides[h][4], b, vcycle_dtype=torch.float64) for (h, _), b in zip(reqs, bs)]
    for t, (h, cols_orc) in zip(tickets, refs):
        x, info, _ = t.wait()
        infos = info if isinstance(info, list) else [info]
        fine, H_orc = sides[h][2][-1], sides[h][3]
        for r, b_orc in enumerate(cols_orc):
            x_orc, it_orc, _ = H_orc.pcg(b_orc, rtol=1e-8)
            xr = x if x.dim() == 1 else x[:, r]
            assert infos[r]["iterations"] == it_orc, (h, r)
            assert rel_err(fine.to_orc(xr), x_orc) <= 1e-10, (h, r)
    assert srv.stats()["max_running"] >= 2
    srv.close()


def test_size_aware_admission(setup):
    """Smallest expected work first, large requests one at a time: every result
    is still the lone solve's, bitwise, and no two large requests ran at once."""
    import time
    nn, ctx, hs = setup
    reqs = [(3, 8, 31), (3, 6, 33), (0, 1, 35), (1, 1, 37), (3, 7, 39), (2, 2, 41), (1, 3, 43)]
    ref = _alone(hs, reqs, torch.float32)
    works = [hs[h][2].fine.n_dofs * nr for h, nr, _ in reqs]
    large = sorted(works)[-3]  # the three largest requests are large
    srv = nn.Server(ctx, max_active=4, policy="smallest", aging_ms=1e6, large_work=large, max_large=1)
    t0 = time.perf_counter()
    tickets = [(time.perf_counter() - t0, srv.submit(hs[h][2], b)) for (h, nr, seed), (b, _, _) in zip(reqs, ref)]
    spans = []
    for (ts, t), (b, x_ref, info_ref), w in zip(tickets, ref, works):
        x, info, tm = t.wait()
        assert torch.equal(x, x_ref) and _iters(info) == _iters(info_ref)
        start = ts * 1e3 + tm["queued_ms"]
        spans.append((w >= large, start, start + tm["run_ms"]))
    big = sorted((a, b) for is_large, a, b in spans if is_large)
    assert len(big) == 3
    for (a0, b0), (a1, b1) in zip(big, big[1:]):
        assert a1 >= b0 - 1.0, big  # the next large one starts after the previous ended (1 ms clock slack)
    st = srv.stats()
    assert st["completed"] == len(reqs) and 2 <= st["max_running"] <= 4
    srv.close()
    with pytest.raises(ValueError):
        nn.Server(ctx, policy="random")
