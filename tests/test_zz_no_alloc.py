"""nnmg_vmult_noalloc: the operator application whose contribution slots live in
the library's static per-GPU array, called through the C ABI and compared
with nnmg_vmult on the same inputs.

Both run the same kernels in the same order on the same data, so the bar is
bitwise equality (stricter than the 1e-12 / 2e-5 parity bar of the operator
against the oracle).  Two calls in a row share the array: the second, on a
smaller level, must not see anything the first left behind.
"""

import ctypes as C

import pytest
import torch

from workloads import config_levels, random_vector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2412_10910_amd as nn
    return nn.Context(0)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _both(level, x):
    from paper_2412_10910_amd import _lib
    lib = _lib.load()
    prec = _lib.FP64 if x.dtype == torch.float64 else _lib.FP32
    ref = torch.full_like(x, float("nan"))
    out = torch.full_like(x, float("nan"))
    assert lib.nnmg_vmult(level.handle, prec, _ptr(x), _ptr(ref), _stream()) == 0, lib.nnmg_last_error()
    code = lib.nnmg_vmult_noalloc(level.handle, prec, _ptr(x), _ptr(out), _stream())
    assert code == 0, lib.nnmg_last_error()
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_vmult_on_two_calls_in_a_row(ctx, dtype):
    import paper_2412_10910_amd as nn
    big = nn.Level.from_mesh(ctx, config_levels(2, cells=[10])[0], 3)
    small = nn.Level.from_mesh(ctx, config_levels(1, cells=[4])[0], 2)
    assert small.n_dofs < big.n_dofs
    for lv, seed in ((big, 11), (small, 12)):
        x = torch.tensor(random_vector(lv.n_dofs, seed), dtype=dtype, device="cuda:0")
        ref, out = _both(lv, x)
        assert torch.isfinite(ref).all()
        assert torch.equal(out, ref), float((out - ref).abs().max())
    # the larger level again after the smaller one: every slot is rewritten
    x = torch.tensor(random_vector(big.n_dofs, 13), dtype=dtype, device="cuda:0")
    ref, out = _both(big, x)
    assert torch.equal(out, ref)


def test_noalloc_rejects_a_level_beyond_the_static_array(ctx):
    """Q4 on 44^3 cells has about 8.9M contribution slots: 71 MB in float64
    (over the 64 MiB array, rejected before any launch), 36 MB in float32 (run)."""
    import paper_2412_10910_amd as nn
    from paper_2412_10910_amd import _lib
    lib = _lib.load()
    lv = nn.Level.from_mesh(ctx, config_levels(1, cells=[44])[0], 4)
    x64 = torch.tensor(random_vector(lv.n_dofs, 5), dtype=torch.float64, device="cuda:0")
    dst = torch.zeros_like(x64)
    code = lib.nnmg_vmult_noalloc(lv.handle, _lib.FP64, _ptr(x64), _ptr(dst), _stream())
    assert code == -2, (code, lib.nnmg_last_error())  # NNMG_ERR_UNSUPPORTED
    assert b"static scratch" in lib.nnmg_last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(dst) == 0  # nothing ran
    ref, out = _both(lv, x64.float())
    assert torch.equal(out, ref)


@pytest.mark.parametrize("variant", [4, 10, 6])
def test_noalloc_follows_the_level_variant(ctx, variant):
    """The static-scratch call runs the level's tuned slot variant (entity
    records, transposed sweeps) with the same bits as nnmg_vmult, and an
    elasticity level (three values per slot) after it."""
    import paper_2412_10910_amd as nn
    lv = nn.Level.from_mesh(ctx, config_levels(2, cells=[6])[0], 4)
    lv.set_variant(variant)
    for dtype, seed in ((torch.float64, 21), (torch.float32, 22)):
        x = torch.tensor(random_vector(lv.n_dofs, seed), dtype=dtype, device="cuda:0")
        ref, out = _both(lv, x)
        assert torch.equal(out, ref)
    el = nn.Level.from_mesh(ctx, config_levels(3, cells=[(7, 2, 2)])[0], 2, "elasticity")
    x = torch.tensor(random_vector(el.n_dofs, 23), dtype=torch.float64, device="cuda:0")
    ref, out = _both(el, x)
    assert torch.equal(out, ref)
