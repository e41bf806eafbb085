"""Python binding of libnnmg: argument marshalling only.

Every computation runs in the HIP library.  PyTorch supplies device memory
(vectors are CUDA/HIP tensors passed as raw pointers) and streams (the current
torch stream is passed to every asynchronous call).
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import FP32, FP64, check, lib

_DTYPE_PREC = {torch.float64: FP64, torch.float32: FP32}


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _vec(t: torch.Tensor, n: int, device: int, dtype=None, name="vector") -> C.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must live on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if t.dtype not in _DTYPE_PREC:
        raise ValueError(f"{name} must be float32 or float64")
    return C.c_void_p(t.data_ptr())


def _nrhs(t: torch.Tensor, n: int, name="vector") -> int:
    """Right-hand sides of a vector argument: 1 for shape [n], r for [n, r]
    (a contiguous [n][r] tensor is the library's interleaved layout)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dim() == 1:
        return 1
    if t.dim() == 2 and t.shape[0] == n:
        return int(t.shape[1])
    raise ValueError(f"{name} must have shape [{n}] or [{n}, nrhs], got {tuple(t.shape)}")


class Context:
    """Binds the library to one GPU.

    With ``torch_allocator=True`` the library's persistent buffers come from
    PyTorch's caching allocator; otherwise the library calls hipMalloc.
    """

    def __init__(self, device: int = 0, torch_allocator: bool = False):
        self.device = int(device)
        self._keep = []
        alloc = None
        if torch_allocator:
            dev = self.device

            def _alloc(user, nbytes, stream):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev)
                except Exception:  # out of memory -> NULL -> NNMG_ERR_OOM
                    return None

            def _free(user, ptr, stream):
                torch.cuda.caching_allocator_delete(int(ptr))

            af, ff = _lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free)
            alloc = _lib.Allocator(None, af, ff)
            self._keep = [af, ff, alloc]
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().nnmg_ctx_create(self.device, C.byref(alloc) if alloc is not None else None, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().nnmg_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Level:
    """One mesh level and its Q_k space (nnmg_level_create)."""

    OPERATORS = {"laplace": _lib.OP_LAPLACE, "elasticity": _lib.OP_ELASTICITY}

    def __init__(self, ctx: Context, vertices, cells, dirichlet=None, degree: int = 1, operator: str = "laplace",
                 lam: float = 1.0, mu: float = 1.0):
        """operator: "laplace" (scalar) or "elasticity" (vector Q_k, dim components
        interleaved by node; lam, mu are the Lame coefficients)."""
        self.ctx = ctx
        if operator not in self.OPERATORS:
            raise ValueError(f"operator must be one of {sorted(self.OPERATORS)}")
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
        if v.ndim != 2 or c.ndim != 2 or c.shape[1] != 2 ** v.shape[1]:
            raise ValueError("vertices must be [V, dim] and cells [C, 2^dim]")
        if d is not None and d.shape != (v.shape[0],):
            raise ValueError("dirichlet must have one flag per vertex")
        mesh = _lib.Mesh(
            v.shape[1], v.shape[0], v.ctypes.data_as(C.POINTER(C.c_double)), c.shape[0],
            c.ctypes.data_as(C.POINTER(C.c_int32)),
            d.ctypes.data_as(C.POINTER(C.c_uint8)) if d is not None else None)
        h = C.c_void_p()
        opts = _lib.LevelOpts()
        lib().nnmg_default_level_opts(C.byref(opts))
        opts.op = self.OPERATORS[operator]
        opts.lam, opts.mu = float(lam), float(mu)
        with torch.cuda.device(ctx.device):
            check(lib().nnmg_level_create_ex(ctx.handle, C.byref(mesh), int(degree), C.byref(opts), C.byref(h)))
        self.handle = h
        self.dim = int(v.shape[1])
        self.degree = int(degree)
        self.operator = operator
        nco = C.c_int()
        check(lib().nnmg_level_components(h, C.byref(nco)))
        self.ncomp = nco.value
        nd, nf, nc = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().nnmg_level_info(h, C.byref(nd), C.byref(nf), C.byref(nc)))
        self.n_dofs, self.n_free, self.n_cells = nd.value, nf.value, nc.value

    @classmethod
    def from_mesh(cls, ctx: Context, mesh, degree: int, operator: str = "laplace", lam: float = 1.0,
                  mu: float = 1.0):
        return cls(ctx, mesh.vertices, mesh.cells, mesh.dirichlet, degree, operator, lam, mu)

    def close(self):
        if getattr(self, "handle", None):
            lib().nnmg_level_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- host queries ---------------------------------------------------------
    def support_points(self) -> np.ndarray:
        out = np.empty((self.n_dofs, self.dim), dtype=np.float64)
        check(lib().nnmg_level_support_points(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def constrained(self) -> np.ndarray:
        out = np.empty(self.n_dofs, dtype=np.uint8)
        check(lib().nnmg_level_constrained(self.handle, out.ctypes.data_as(C.POINTER(C.c_uint8))))
        return out.astype(bool)

    def quadrature_points(self) -> np.ndarray:
        q = (self.degree + 1) ** self.dim
        out = np.empty((self.n_cells, q, self.dim), dtype=np.float64)
        check(lib().nnmg_level_quadrature_points(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    # -- device operations ----------------------------------------------------
    def empty(self, dtype=torch.float64) -> torch.Tensor:
        return torch.zeros(self.n_dofs, dtype=dtype, device=f"cuda:{self.ctx.device}")

    def assemble_rhs(self, f_qp: torch.Tensor, b: torch.Tensor | None = None) -> torch.Tensor:
        """f_qp: [n_cells][(k+1)^dim][ncomp] source values at quadrature_points()."""
        q = (self.degree + 1) ** self.dim
        fq = _vec(f_qp, self.n_cells * q * self.ncomp, self.ctx.device, torch.float64, "f_qp")
        b = self.empty(torch.float64) if b is None else b
        check(lib().nnmg_level_assemble_rhs(self.handle, fq, _vec(b, self.n_dofs, self.ctx.device,
                                                                   torch.float64, "b"), _stream()))
        return b

    def vmult(self, src: torch.Tensor, dst: torch.Tensor | None = None) -> torch.Tensor:
        """dst = A src; src of shape [n_dofs] or [n_dofs, nrhs] (several right-hand sides)."""
        dst = torch.empty_like(src) if dst is None else dst
        if dst.dtype != src.dtype or dst.shape != src.shape:
            raise ValueError("src and dst must have the same dtype and shape")
        nr = _nrhs(src, self.n_dofs, "src")
        s = _vec(src, self.n_dofs * nr, self.ctx.device, name="src")
        d = _vec(dst, self.n_dofs * nr, self.ctx.device, name="dst")
        if src.dim() == 1:
            check(lib().nnmg_vmult(self.handle, _DTYPE_PREC[src.dtype], s, d, _stream()))
        else:
            check(lib().nnmg_vmult_multi(self.handle, _DTYPE_PREC[src.dtype], nr, s, d, _stream()))
        return dst

    def vmult_noalloc(self, src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
        """dst = A src (one right-hand side) with the contribution slots in the library's
        static per-GPU array: the call allocates no device memory (nnmg_vmult_noalloc)."""
        if dst.dtype != src.dtype or dst.shape != src.shape or src.dim() != 1:
            raise ValueError("src and dst must be vectors of the same dtype and shape")
        s = _vec(src, self.n_dofs, self.ctx.device, name="src")
        d = _vec(dst, self.n_dofs, self.ctx.device, name="dst")
        check(lib().nnmg_vmult_noalloc(self.handle, _DTYPE_PREC[src.dtype], s, d, _stream()))
        return dst

    def vmult_add(self, src: torch.Tensor, dst: torch.Tensor) -> torch.Tensor:
        """dst += A src over the unconstrained rows and columns (one kernel launch)."""
        if dst.dtype != src.dtype or dst.shape != src.shape:
            raise ValueError("src and dst must have the same dtype and shape")
        nr = _nrhs(src, self.n_dofs, "src")
        s = _vec(src, self.n_dofs * nr, self.ctx.device, name="src")
        d = _vec(dst, self.n_dofs * nr, self.ctx.device, name="dst")
        if src.dim() == 1:
            check(lib().nnmg_vmult_add(self.handle, _DTYPE_PREC[src.dtype], s, d, _stream()))
        else:
            check(lib().nnmg_vmult_add_multi(self.handle, _DTYPE_PREC[src.dtype], nr, s, d, _stream()))
        return dst

    VARIANTS = ("trilinear+slots", "trilinear+atomic", "metric+slots", "metric+atomic",
                "trilinear+entity", "metric+entity",
                "trilinear+slots+transposed", None, "metric+slots+transposed", None,
                "trilinear+entity+transposed", "metric+entity+transposed")

    def tune(self, dtype=torch.float32, reps: int = 10) -> dict:
        """Time the operator variants in `dtype` on this GPU and keep the fastest for
        that precision (nnmg_level_tune; each precision has its own variant)."""
        res = _lib.TuneResult()
        check(lib().nnmg_level_tune(self.handle, _DTYPE_PREC[dtype], int(reps), C.byref(res)))
        return dict(ms={self.VARIANTS[v]: res.ms[v] for v in range(res.n_variants) if res.ms[v] >= 0},
                    chosen=self.VARIANTS[res.chosen], rhs_split=bool(res.rhs_split),
                    ms_rhs4={"loop": res.ms_rhs[0], "split": res.ms_rhs[1]} if res.ms_rhs[0] >= 0 else None,
                    cells_per_block=res.cells_per_block,
                    ms_cells={"one block": res.ms_cpb[0], "two blocks": res.ms_cpb[1]}
                    if res.ms_cpb[0] >= 0 else None)

    def set_cells_per_block(self, cells: int, dtype=None):
        """Cells per workgroup of the operator: one layout block or two
        (nnmg_level_set_cells_per_block), for one precision or both (dtype None)."""
        for dt in ((torch.float64, torch.float32) if dtype is None else (dtype,)):
            check(lib().nnmg_level_set_cells_per_block(self.handle, _DTYPE_PREC[dt], int(cells)))

    def cells_per_block(self, dtype=torch.float64) -> tuple:
        """(cells per workgroup in use, cells per layout block, layout blocks) of
        the `dtype` kernels."""
        c, base, nb = C.c_int(), C.c_int(), C.c_int64()
        check(lib().nnmg_level_cells_per_block(self.handle, _DTYPE_PREC[dtype], C.byref(c), C.byref(base),
                                               C.byref(nb)))
        return c.value, base.value, nb.value

    def set_rhs_split(self, split: bool, dtype=torch.float64):
        """Several right-hand sides: one row of workgroups each (True) or every
        workgroup looping over them (False), for the `dtype` kernels."""
        check(lib().nnmg_level_set_rhs_split(self.handle, _DTYPE_PREC[dtype], int(bool(split))))

    def variant_of(self, dtype) -> int:
        """The operator variant the `dtype` kernels use (index into VARIANTS)."""
        v = C.c_int()
        check(lib().nnmg_level_variant(self.handle, _DTYPE_PREC[dtype], C.byref(v)))
        return v.value

    @property
    def variant(self) -> int:
        """The float64 operator variant (see variant_of)."""
        return self.variant_of(torch.float64)

    def set_variant(self, variant: int, dtype=None):
        """Force an operator variant for one precision, or for both (dtype None)."""
        if dtype is None:
            check(lib().nnmg_level_set_variant(self.handle, int(variant)))
        else:
            check(lib().nnmg_level_set_variant_prec(self.handle, _DTYPE_PREC[dtype], int(variant)))

    def diagonal(self, dtype=torch.float64) -> torch.Tensor:
        out = self.empty(dtype)
        check(lib().nnmg_level_diagonal(self.handle, _DTYPE_PREC[dtype], _vec(out, self.n_dofs, self.ctx.device),
                                        _stream()))
        return out


class Transfer:
    """Non-nested transfer between a fine and a coarse level (nnmg_transfer_create)."""

    def __init__(self, ctx: Context, fine: Level, coarse: Level, bbox_expand=None, inside_tol=None,
                 newton_tol=None, newton_max_it=None, allow_projection=None, nested_p=None):
        self.ctx, self.fine, self.coarse = ctx, fine, coarse
        o = _lib.TransferOpts()
        lib().nnmg_default_transfer_opts(C.byref(o))
        for name, val in (("bbox_expand", bbox_expand), ("inside_tol", inside_tol), ("newton_tol", newton_tol),
                          ("newton_max_it", newton_max_it), ("allow_projection", allow_projection),
                          ("nested_p", nested_p)):
            if val is not None:
                setattr(o, name, type(getattr(o, name))(val))
        h = C.c_void_p()
        with torch.cuda.device(ctx.device):
            check(lib().nnmg_transfer_create(ctx.handle, fine.handle, coarse.handle, C.byref(o), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().nnmg_transfer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_points(self) -> int:
        """Number of fine support points carried by P (the unconstrained fine DoFs)."""
        n, npj = C.c_int64(), C.c_int64()
        check(lib().nnmg_transfer_points(self.handle, C.byref(n), None, None, None, C.byref(npj)))
        return n.value

    def tune(self, dtype=torch.float32, reps: int = 10) -> dict:
        """Time the restriction with 4..64 lanes per coarse cell and keep the fastest."""
        res = _lib.TuneResult()
        check(lib().nnmg_transfer_tune(self.handle, _DTYPE_PREC[dtype], int(reps), C.byref(res)))
        return dict(ms={4 << v: res.ms[v] for v in range(res.n_variants)}, chosen=4 << res.chosen)

    @property
    def team(self) -> int:
        v = C.c_int()
        check(lib().nnmg_transfer_team(self.handle, C.byref(v)))
        return v.value

    def set_team(self, team: int):
        check(lib().nnmg_transfer_set_team(self.handle, int(team)))

    def points(self) -> dict:
        n, npj = C.c_int64(), C.c_int64()
        check(lib().nnmg_transfer_points(self.handle, C.byref(n), None, None, None, C.byref(npj)))
        dof = np.empty(n.value, dtype=np.int32)
        own = np.empty(n.value, dtype=np.int32)
        xi = np.empty((n.value, self.fine.dim), dtype=np.float64)
        check(lib().nnmg_transfer_points(self.handle, None, dof.ctypes.data_as(C.POINTER(C.c_int32)),
                                         own.ctypes.data_as(C.POINTER(C.c_int32)),
                                         xi.ctypes.data_as(C.POINTER(C.c_double)), None))
        return dict(fine_dof=dof, owner=own, xi=xi, n_projected=npj.value)

    def _pair(self, coarse_vec, fine_vec):
        if coarse_vec.dtype != fine_vec.dtype:
            raise ValueError("dtype mismatch")
        nr = _nrhs(coarse_vec, self.coarse.n_dofs, "coarse")
        if _nrhs(fine_vec, self.fine.n_dofs, "fine") != nr or coarse_vec.dim() != fine_vec.dim():
            raise ValueError("coarse and fine carry different numbers of right-hand sides")
        c = _vec(coarse_vec, self.coarse.n_dofs * nr, self.ctx.device, name="coarse")
        f = _vec(fine_vec, self.fine.n_dofs * nr, self.ctx.device, name="fine")
        return nr, c, f

    def prolongate(self, coarse_vec: torch.Tensor, fine_vec: torch.Tensor) -> torch.Tensor:
        """fine_vec += P coarse_vec (shapes [n] or [n, nrhs])."""
        nr, c, f = self._pair(coarse_vec, fine_vec)
        prec = _DTYPE_PREC[coarse_vec.dtype]
        if coarse_vec.dim() == 1:
            check(lib().nnmg_prolongate(self.handle, prec, c, f, _stream()))
        else:
            check(lib().nnmg_prolongate_multi(self.handle, prec, nr, c, f, _stream()))
        return fine_vec

    def restrict(self, fine_vec: torch.Tensor, coarse_vec: torch.Tensor) -> torch.Tensor:
        """coarse_vec += P^T fine_vec (shapes [n] or [n, nrhs])."""
        nr, c, f = self._pair(coarse_vec, fine_vec)
        prec = _DTYPE_PREC[fine_vec.dtype]
        if fine_vec.dim() == 1:
            check(lib().nnmg_restrict(self.handle, prec, f, c, _stream()))
        else:
            check(lib().nnmg_restrict_multi(self.handle, prec, nr, f, c, _stream()))
        return coarse_vec


class Hierarchy:
    """Levels coarse -> fine and the transfers between them (nnmg_hierarchy_create)."""

    COMPONENTS = ("pre_smoother", "residual", "restriction", "coarse_solve", "prolongation", "post_smoother")

    def __init__(self, ctx: Context, levels, transfers, eig_start=None, cheb_degree=None, smoothing_range=None,
                 eig_safety=None, eig_iters=None):
        self.ctx = ctx
        self.levels = list(levels)
        self.transfers = list(transfers)
        L = len(self.levels)
        o = _lib.MgOpts()
        lib().nnmg_default_mg_opts(C.byref(o))
        for name, val in (("cheb_degree", cheb_degree), ("smoothing_range", smoothing_range),
                          ("eig_safety", eig_safety), ("eig_iters", eig_iters)):
            if val is not None:
                setattr(o, name, type(getattr(o, name))(val))
        starts = None
        if eig_start is not None:
            if len(eig_start) != L:
                raise ValueError("eig_start needs one entry per level")
            ptrs = []
            for lv, v in zip(self.levels, eig_start):
                ptrs.append(None if v is None else _vec(v, lv.n_dofs, ctx.device, torch.float64, "eig_start").value)
            starts = (C.c_void_p * L)(*ptrs)
            o.eig_start = C.cast(starts, C.POINTER(C.c_void_p))
        lv = (C.c_void_p * L)(*[l.handle.value for l in self.levels])
        tr = (C.c_void_p * max(L - 1, 1))(*[t.handle.value for t in self.transfers])
        h = C.c_void_p()
        with torch.cuda.device(ctx.device):
            torch.cuda.synchronize(ctx.device)
            check(lib().nnmg_hierarchy_create(ctx.handle, lv, L, tr, C.byref(o), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().nnmg_hierarchy_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def fine(self) -> Level:
        return self.levels[-1]

    def cheb_bounds(self, level: int):
        lo, hi = C.c_double(), C.c_double()
        check(lib().nnmg_get_cheb_bounds(self.handle, int(level), C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def set_cheb_bounds(self, level: int, lo: float, hi: float):
        check(lib().nnmg_set_cheb_bounds(self.handle, int(level), float(lo), float(hi)))

    def vcycle(self, r: torch.Tensor, z: torch.Tensor | None = None) -> torch.Tensor:
        """z = V(r); r of shape [n_dofs] or [n_dofs, nrhs]."""
        z = torch.empty_like(r) if z is None else z
        if z.dtype != r.dtype or z.shape != r.shape:
            raise ValueError("r and z must have the same dtype and shape")
        n = self.fine.n_dofs
        nr = _nrhs(r, n, "r")
        rp = _vec(r, n * nr, self.ctx.device, name="r")
        zp = _vec(z, n * nr, self.ctx.device, name="z")
        if r.dim() == 1:
            check(lib().nnmg_vcycle(self.handle, _DTYPE_PREC[r.dtype], rp, zp, _stream()))
        else:
            check(lib().nnmg_vcycle_multi(self.handle, _DTYPE_PREC[r.dtype], nr, rp, zp, _stream()))
        return z

    def pcg_solve(self, b: torch.Tensor, x: torch.Tensor | None = None, rtol: float = 1e-8, max_it: int = 200,
                  vcycle_dtype=torch.float32, history: bool = True, raise_on_failure: bool = True,
                  use_graph: bool = True):
        """Float64 PCG preconditioned by one V-cycle in vcycle_dtype.  b of shape
        [n_dofs] gives info as a dict; b of shape [n_dofs, nrhs] runs the nrhs
        solves in lockstep (nnmg_pcg_solve_multi) and gives a list of dicts."""
        n = self.fine.n_dofs
        nr = _nrhs(b, n, "b")
        x = torch.empty_like(b) if x is None else x
        if x.shape != b.shape:
            raise ValueError("b and x must have the same shape")
        o = _lib.CgOpts()
        lib().nnmg_default_cg_opts(C.byref(o))
        o.rtol = float(rtol)
        o.max_it = int(max_it)
        o.vcycle_prec = _DTYPE_PREC[vcycle_dtype]
        o.use_graph = int(bool(use_graph))
        hist = np.full((nr, max_it + 1), np.nan) if history else None
        o.history = hist.ctypes.data_as(C.POINTER(C.c_double)) if history else None
        res = (_lib.CgResult * nr)()
        bp = _vec(b, n * nr, self.ctx.device, torch.float64, "b")
        xp = _vec(x, n * nr, self.ctx.device, torch.float64, "x")
        if b.dim() == 1:
            code = lib().nnmg_pcg_solve(self.handle, bp, xp, C.byref(o), res, _stream())
        else:
            code = lib().nnmg_pcg_solve_multi(self.handle, nr, bp, xp, C.byref(o), res, _stream())
        infos = []
        for k in range(nr):
            info = dict(iterations=res[k].iterations, relres=res[k].relres,
                        status=_lib.ERRORS.get(res[k].status, "OK") if res[k].status else "OK")
            if history:
                info["history"] = hist[k, : res[k].iterations + 1].copy()
            infos.append(info)
        if code != 0 and raise_on_failure:
            check(code)
        return x, (infos[0] if b.dim() == 1 else infos)

    def tune(self, dtype=torch.float32, reps: int = 10) -> dict:
        """Tune every level's operator and every transfer's restriction (the
        V-cycle's precision is the one to tune for)."""
        return dict(levels=[lv.tune(dtype, reps) for lv in self.levels],
                    transfers=[tr.tune(dtype, reps) for tr in self.transfers])

    @property
    def coarse_free_dofs(self) -> int:
        """Unconstrained DoFs of the coarsest level: the order of the dense inverse."""
        return self.levels[0].n_free

    def footprint(self, nrhs: int = 1) -> int:
        """Device bytes a solve of nrhs right-hand sides needs beyond the hierarchy's fixed data."""
        v = C.c_size_t()
        check(lib().nnmg_hierarchy_footprint(self.handle, int(nrhs), C.byref(v)))
        return v.value

    def set_profiling(self, enabled: bool):
        check(lib().nnmg_hierarchy_set_profiling(self.handle, int(bool(enabled))))

    def profile(self) -> np.ndarray:
        out = np.zeros((len(self.levels), 6), dtype=np.float64)
        check(lib().nnmg_hierarchy_profile(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out


class Ticket:
    """A queued serving request; keeps its vectors alive until waited for."""

    def __init__(self, server, ident, b, x, nr, hist, multi):
        self.server, self.id, self.b, self.x, self.nr, self.hist, self.multi = server, ident, b, x, nr, hist, multi

    def done(self) -> bool:
        flag = C.c_int()
        check(lib().nnmg_server_poll(self.server.handle, C.c_int64(self.id), C.byref(flag)))
        return bool(flag.value)

    def wait(self, raise_on_failure: bool = True):
        """Block until the request has finished: (x, info or list of infos, times dict)."""
        res = (_lib.CgResult * self.nr)()
        times = _lib.RequestTimes()
        code = lib().nnmg_server_wait(self.server.handle, C.c_int64(self.id), res, C.byref(times))
        self.server._live.pop(self.id, None)  # finished: the server no longer touches its data
        infos = []
        for k in range(self.nr):
            info = dict(iterations=res[k].iterations, relres=res[k].relres,
                        status=_lib.ERRORS.get(res[k].status, "OK") if res[k].status else "OK")
            if self.hist is not None:
                info["history"] = self.hist[k, : res[k].iterations + 1].copy()
            infos.append(info)
        if code != 0 and raise_on_failure:
            check(code)
        t = dict(queued_ms=times.queued_ms, run_ms=times.run_ms, total_ms=times.total_ms)
        return self.x, (infos if self.multi else infos[0]), t


class Server:
    """Serving loop with continuous batching (nnmg_server_*): requests on
    resident hierarchies are admitted as slots and memory free up and run
    overlapped on their own streams."""

    POLICIES = {"arrival": 0, "smallest": 1}

    def __init__(self, ctx: Context, max_active: int = 4, memory_budget: int = 64 << 30, policy: str = "arrival",
                 aging_ms: float = 250.0, large_work: float = 0.0, max_large: int = 64):
        """policy "smallest": smallest expected work (fine DoFs x nrhs) first, a
        request queued for aging_ms taken in arrival order; at most max_large
        requests of expected work >= large_work run at once."""
        self.ctx = ctx
        if policy not in self.POLICIES:
            raise ValueError(f"policy must be one of {sorted(self.POLICIES)}")
        o = _lib.ServerOpts()
        lib().nnmg_default_server_opts(C.byref(o))
        o.max_active = int(max_active)
        o.memory_budget = int(memory_budget)
        o.policy = self.POLICIES[policy]
        o.aging_ms, o.large_work, o.max_large = float(aging_ms), float(large_work), int(max_large)
        h = C.c_void_p()
        check(lib().nnmg_server_create(ctx.handle, C.byref(o), C.byref(h)))
        self.handle = h
        # everything a queued or running request reads or writes (its
        # hierarchies, b, x, the history array), by ticket id: the server's
        # thread uses them until the request has finished, whether or not the
        # caller keeps the ticket; released by Ticket.wait and by close()
        self._live = {}

    def submit(self, hierarchy, b: torch.Tensor, x: torch.Tensor | None = None, rtol: float = 1e-8,
               max_it: int = 200, vcycle_dtype=torch.float32, history: bool = False, use_graph: bool = True) -> Ticket:
        """Queue a solve on `hierarchy`, or on whichever of a list of equivalent
        replicas is idle first (nnmg_server_submit_any)."""
        replicas = list(hierarchy) if isinstance(hierarchy, (list, tuple)) else [hierarchy]
        n = replicas[0].fine.n_dofs
        nr = _nrhs(b, n, "b")
        x = torch.empty_like(b) if x is None else x
        if x.shape != b.shape:
            raise ValueError("b and x must have the same shape")
        bp = _vec(b, n * nr, self.ctx.device, torch.float64, "b")
        xp = _vec(x, n * nr, self.ctx.device, torch.float64, "x")
        o = _lib.CgOpts()
        lib().nnmg_default_cg_opts(C.byref(o))
        o.rtol, o.max_it = float(rtol), int(max_it)
        o.vcycle_prec = _DTYPE_PREC[vcycle_dtype]
        o.use_graph = int(bool(use_graph))
        hist = np.full((nr, max_it + 1), np.nan) if history else None
        o.history = hist.ctypes.data_as(C.POINTER(C.c_double)) if history else None
        torch.cuda.current_stream().synchronize()  # b complete before the server's streams read it
        t = C.c_int64()
        hs = (C.c_void_p * len(replicas))(*[h.handle.value for h in replicas])
        check(lib().nnmg_server_submit_any(self.handle, hs, len(replicas), nr, bp, xp, C.byref(o), C.byref(t)))
        self._live[t.value] = (replicas, b, x, hist)
        return Ticket(self, t.value, b, x, nr, hist, b.dim() == 2)

    def stats(self) -> dict:
        st = _lib.ServerStats()
        check(lib().nnmg_server_get_stats(self.handle, C.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        """Finish every queued and running request, then stop the loop."""
        if getattr(self, "handle", None):
            lib().nnmg_server_destroy(self.handle)
            self.handle = None
        self._live = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, hierarchy: "Hierarchy", nrhs: int) -> int:
        return hierarchy.footprint(nrhs)


def build_levels(ctx: Context, meshes, degree: int, operator: str = "laplace", lam: float = 1.0, mu: float = 1.0,
                 p_coarsening: bool = False):
    """Levels (coarse -> fine) and transfers of a hierarchy over independent
    meshes.  With p_coarsening the coarsest mesh carries degrees 1, 2, ...,
    degree below the first mesh level (paper §2, Coarse grid solvers: polynomial
    multigrid on the coarsest triangulation), joined by nested polynomial
    transfers; the exact coarse solve then acts on the Q1 level."""
    specs = ([(meshes[0], d) for d in range(1, degree)] if p_coarsening else []) + [(m, degree) for m in meshes]
    levels = [Level.from_mesh(ctx, m, d, operator, lam, mu) for m, d in specs]
    transfers = [Transfer(ctx, levels[i + 1], levels[i]) for i in range(len(levels) - 1)]
    return levels, transfers

