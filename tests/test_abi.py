"""CPU checks of the C ABI: the library loads and exports every declared symbol."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnmg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nnmg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for required in ("nnmg_level_create", "nnmg_transfer_create", "nnmg_vmult", "nnmg_vcycle", "nnmg_pcg_solve",
                     "nnmg_prolongate", "nnmg_restrict", "nnmg_hierarchy_create"):
        assert required in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2412_10910_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libnnmg.so is not built (run __graft_entry__.build())")
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES), "binding and header disagree"


def test_defaults_without_a_gpu():
    import ctypes as C

    from paper_2412_10910_amd import _lib
    lib = _lib.load()
    o = _lib.CgOpts()
    lib.nnmg_default_cg_opts(C.byref(o))
    assert o.rtol == 1e-8 and o.max_it == 200 and o.vcycle_prec == _lib.FP32
    m = _lib.MgOpts()
    lib.nnmg_default_mg_opts(C.byref(m))
    assert (m.cheb_degree, m.smoothing_range, m.eig_safety, m.eig_iters) == (3, 20.0, 1.2, 12)
    lo = _lib.LevelOpts()
    lib.nnmg_default_level_opts(C.byref(lo))
    assert (lo.op, lo.lam, lo.mu) == (_lib.OP_LAPLACE, 1.0, 1.0)
    t = _lib.TransferOpts()
    lib.nnmg_default_transfer_opts(C.byref(t))
    assert (t.bbox_expand, t.inside_tol, t.newton_tol, t.newton_max_it, t.allow_projection) == \
        (0.25, 1e-10, 1e-12, 50, 1)
    # a failing call without a device reports through the error channel
    h = C.c_void_p()
    code = lib.nnmg_level_create(None, None, 1, C.byref(h))
    assert code == -1 and lib.nnmg_last_error()


def test_library_binds_to_torchs_hip_runtime():
    """Exactly one HIP runtime in the process: the library reuses torch's."""
    import subprocess
    import sys
    code = ("import paper_2412_10910_amd\n"
            "maps = open('/proc/self/maps').read()\n"
            "paths = {l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}\n"
            "print(len(paths))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
