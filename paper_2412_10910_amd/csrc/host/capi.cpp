// The extern "C" boundary: argument checks, error codes and the thread-local
// error message.  No C++ exception crosses this file.
#include <cstring>
#include <new>

#include "../internal.hpp"

namespace nnmg {

Level* level_create(Ctx* ctx, const nnmg_mesh* mesh, int degree, const nnmg_level_opts& opts);
void level_diagonal(const Level& L, int prec, void* out, hipStream_t s);
void level_quadrature_points(const Level& L, double* out);
Transfer* transfer_create(Ctx* ctx, Level* fine, Level* coarse, const nnmg_transfer_opts& o);
struct Hierarchy;
Hierarchy* hierarchy_create(Ctx* ctx, nnmg_level* const* levels, int nl, nnmg_transfer* const* transfers,
                            const nnmg_mg_opts& o);
void hierarchy_destroy(Hierarchy* h);
void get_bounds(const Hierarchy& H, int l, double* lo, double* hi);
void set_bounds(Hierarchy& H, int l, double lo, double hi);
void vcycle(Hierarchy& H, int prec, const void* r, void* z, int nr, hipStream_t s);
int pcg(Hierarchy& H, const double* b, double* x, const nnmg_cg_opts& o, nnmg_cg_result* res, int nr,
        hipStream_t s);
void set_profiling(Hierarchy& H, bool on);
size_t hierarchy_footprint(const Hierarchy& H, int nr);
struct Server;
Server* server_create(Ctx* ctx, const nnmg_server_opts& o);
void server_destroy(Server* S);
int64_t server_submit(Server* S, Hierarchy* const* replicas, int n_replicas, int nr, const double* b, double* x,
                      const nnmg_cg_opts& o);
int server_wait(Server* S, int64_t id, nnmg_cg_result* res, nnmg_request_times* times, std::string* err);
bool server_poll(Server* S, int64_t id);
void server_stats(Server* S, nnmg_server_stats* out);
void profile(Hierarchy& H, double* ms);

namespace {
thread_local std::string g_last_error;

int report(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

template <class F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error& e) {
        return report(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return report(NNMG_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return report(NNMG_ERR_INVALID_ARG, e.what());
    } catch (...) {
        return report(NNMG_ERR_INVALID_ARG, "unknown error");
    }
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void* Ctx::allocate(size_t bytes) {
    if (bytes == 0) return nullptr;
    void* p = nullptr;
    if (custom) {
        p = alloc.alloc(alloc.user, bytes, nullptr);
        if (!p) fail(NNMG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(NNMG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
    return p;
}

void Ctx::release(void* p) {
    if (!p) return;
    if (custom)
        alloc.free(alloc.user, p, nullptr);
    else
        (void)hipFree(p);
}

}  // namespace nnmg

using namespace nnmg;

struct nnmg_hierarchy;

extern "C" {

const char* nnmg_last_error(void) { return g_last_error.c_str(); }

void nnmg_default_transfer_opts(nnmg_transfer_opts* o) {
    if (!o) return;
    o->bbox_expand = 0.25;
    o->inside_tol = 1e-10;
    o->newton_tol = 1e-12;
    o->newton_max_it = 50;
    o->allow_projection = 1;
    o->nested_p = 1;
}

void nnmg_default_mg_opts(nnmg_mg_opts* o) {
    if (!o) return;
    o->cheb_degree = 3;
    o->smoothing_range = 20.0;
    o->eig_safety = 1.2;
    o->eig_iters = 12;
    o->eig_start = nullptr;
}

void nnmg_default_level_opts(nnmg_level_opts* o) {
    if (!o) return;
    o->op = NNMG_OP_LAPLACE;
    o->lambda = 1.0;
    o->mu = 1.0;
}

void nnmg_default_cg_opts(nnmg_cg_opts* o) {
    if (!o) return;
    o->rtol = 1e-8;
    o->max_it = 200;
    o->vcycle_prec = NNMG_FP32;
    o->history = nullptr;
    o->use_graph = 1;
}

int nnmg_ctx_create(int device, const nnmg_allocator* allocator, nnmg_ctx** out) {
    return guarded([&] {
        if (!out) fail(NNMG_ERR_INVALID_ARG, "out is NULL");
        int count = 0;
        NNMG_HIP(hipGetDeviceCount(&count));
        if (device < 0 || device >= count) fail(NNMG_ERR_INVALID_ARG, "no such device");
        if (allocator && (!allocator->alloc || !allocator->free))
            fail(NNMG_ERR_INVALID_ARG, "allocator needs both alloc and free");
        NNMG_HIP(hipSetDevice(device));
        // the static scratch array's device address, taken once per device
        // with the device current (nnmg_vmult_noalloc uses it)
        void* scratch = noalloc_scratch_init(device);
        auto* c = new nnmg_ctx();
        c->device = device;
        c->noalloc_scratch = scratch;
        if (allocator) {
            c->alloc = *allocator;
            c->custom = true;
        }
        *out = c;
        return NNMG_OK;
    });
}

void nnmg_ctx_destroy(nnmg_ctx* ctx) { delete ctx; }

int nnmg_level_create_ex(nnmg_ctx* ctx, const nnmg_mesh* mesh, int degree, const nnmg_level_opts* opts,
                         nnmg_level** out) {
    return guarded([&] {
        if (!ctx || !out) fail(NNMG_ERR_INVALID_ARG, "ctx or out is NULL");
        NNMG_HIP(hipSetDevice(ctx->device));
        nnmg_level_opts o;
        nnmg_default_level_opts(&o);
        if (opts) o = *opts;
        *out = static_cast<nnmg_level*>(level_create(ctx, mesh, degree, o));
        return NNMG_OK;
    });
}

int nnmg_level_create(nnmg_ctx* ctx, const nnmg_mesh* mesh, int degree, nnmg_level** out) {
    return nnmg_level_create_ex(ctx, mesh, degree, nullptr, out);
}

int nnmg_level_components(const nnmg_level* l, int* ncomp) {
    return guarded([&] {
        if (!l || !ncomp) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        *ncomp = l->ncomp;
        return NNMG_OK;
    });
}

void nnmg_level_destroy(nnmg_level* level) {
    if (level) level_release(level);
}

int nnmg_level_info(const nnmg_level* l, int64_t* n_dofs, int64_t* n_free, int64_t* n_cells) {
    return guarded([&] {
        if (!l) fail(NNMG_ERR_INVALID_ARG, "level is NULL");
        if (n_dofs) *n_dofs = l->n_dofs;
        if (n_free) *n_free = l->n_free;
        if (n_cells) *n_cells = l->n_cells;
        return NNMG_OK;
    });
}

int nnmg_level_support_points(const nnmg_level* l, double* xyz) {
    return guarded([&] {
        if (!l || !xyz) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        const int d = l->dim, nc = l->ncomp;
        for (int64_t i = 0; i < l->n_nodes; ++i)
            for (int c = 0; c < nc; ++c)
                std::memcpy(xyz + (i * nc + c) * d, l->support.data() + i * d, (size_t)d * sizeof(double));
        return NNMG_OK;
    });
}

int nnmg_level_constrained(const nnmg_level* l, uint8_t* mask) {
    return guarded([&] {
        if (!l || !mask) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        for (int64_t i = 0; i < l->n_nodes; ++i)
            for (int c = 0; c < l->ncomp; ++c) mask[i * l->ncomp + c] = l->constrained[(size_t)i];
        return NNMG_OK;
    });
}

int nnmg_level_quadrature_points(const nnmg_level* l, double* xyz) {
    return guarded([&] {
        if (!l || !xyz) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        level_quadrature_points(*l, xyz);
        return NNMG_OK;
    });
}

int nnmg_level_assemble_rhs(nnmg_level* l, const double* fq, double* b, void* stream) {
    return guarded([&] {
        if (!l || !fq || !b) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        NNMG_HIP(hipSetDevice(l->ctx->device));
        launch_fill(b, (size_t)l->n_dofs, NNMG_FP64, as_stream(stream));
        launch_assemble_rhs(*l, fq, b, as_stream(stream));
        return NNMG_OK;
    });
}

static void check_rhs(int nrhs) {
    if (nrhs < 1 || nrhs > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "nrhs must be in 1..8");
}

static void vmult_impl(const nnmg_level* l, int prec, int nr, const void* src, void* dst, bool add, void* stream) {
    if (!l || !src || !dst) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
    if (src == dst) fail(NNMG_ERR_INVALID_ARG, "src and dst alias");
    if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
    check_rhs(nr);
    NNMG_HIP(hipSetDevice(l->ctx->device));
    Level& L = const_cast<nnmg_level&>(*l);
    level_reserve_rhs(L, nr);
    const hipStream_t s = as_stream(stream);
    if (add) {
        launch_vmult_cells(L, prec, src, dst, s, nr, L.d_contrib.ptr);
    } else if (L.var[prec].atomic && L.op == NNMG_OP_LAPLACE) {
        launch_fill(dst, (size_t)L.n_dofs * (size_t)nr, prec, s);  // the atomics add into dst
        launch_vmult_cells(L, prec, src, dst, s, nr, L.d_contrib.ptr);
    } else {
        // every unconstrained value has contribution slots, so the gather
        // writes all of them: no fill and no read of dst
        launch_vmult_contrib(L, prec, src, L.d_contrib.ptr, s, nr);
        launch_gather(L, prec, L.d_contrib.ptr, dst, false, s, nr);
    }
    if (!add)
        launch_copy_constrained(L.d_constrained.ptr, L.constrained_idx.size(), src, dst, prec, s, nr);
}

int nnmg_vmult(const nnmg_level* l, nnmg_prec prec, const void* src, void* dst, void* stream) {
    return guarded([&] {
        vmult_impl(l, prec, 1, src, dst, false, stream);
        return NNMG_OK;
    });
}

int nnmg_vmult_noalloc(const nnmg_level* l, nnmg_prec prec, const void* src, void* dst, void* stream) {
    return guarded([&] {
        if (!l || !src || !dst) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (src == dst) fail(NNMG_ERR_INVALID_ARG, "src and dst alias");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        NNMG_HIP(hipSetDevice(l->ctx->device));
        vmult_noalloc(*l, prec, src, dst, l->ctx->noalloc_scratch, as_stream(stream));
        return NNMG_OK;
    });
}

int nnmg_vmult_add(const nnmg_level* l, nnmg_prec prec, const void* src, void* dst, void* stream) {
    return guarded([&] {
        vmult_impl(l, prec, 1, src, dst, true, stream);
        return NNMG_OK;
    });
}

int nnmg_vmult_multi(const nnmg_level* l, nnmg_prec prec, int nrhs, const void* src, void* dst, void* stream) {
    return guarded([&] {
        vmult_impl(l, prec, nrhs, src, dst, false, stream);
        return NNMG_OK;
    });
}

int nnmg_vmult_add_multi(const nnmg_level* l, nnmg_prec prec, int nrhs, const void* src, void* dst,
                         void* stream) {
    return guarded([&] {
        vmult_impl(l, prec, nrhs, src, dst, true, stream);
        return NNMG_OK;
    });
}

int nnmg_level_diagonal(const nnmg_level* l, nnmg_prec prec, void* diag, void* stream) {
    return guarded([&] {
        if (!l || !diag) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        NNMG_HIP(hipSetDevice(l->ctx->device));
        level_diagonal(*l, prec, diag, as_stream(stream));
        return NNMG_OK;
    });
}

int nnmg_transfer_create(nnmg_ctx* ctx, const nnmg_level* fine, const nnmg_level* coarse,
                         const nnmg_transfer_opts* opts, nnmg_transfer** out) {
    return guarded([&] {
        if (!ctx || !out) fail(NNMG_ERR_INVALID_ARG, "ctx or out is NULL");
        nnmg_transfer_opts o;
        nnmg_default_transfer_opts(&o);
        if (opts) o = *opts;
        NNMG_HIP(hipSetDevice(ctx->device));
        *out = static_cast<nnmg_transfer*>(
            transfer_create(ctx, const_cast<nnmg_level*>(fine), const_cast<nnmg_level*>(coarse), o));
        return NNMG_OK;
    });
}

void nnmg_transfer_destroy(nnmg_transfer* t) {
    if (t) transfer_release(t);
}

int nnmg_transfer_points(const nnmg_transfer* t, int64_t* n_points, int32_t* fine_dof, int32_t* owner, double* xi,
                         int64_t* n_projected) {
    return guarded([&] {
        if (!t) fail(NNMG_ERR_INVALID_ARG, "transfer is NULL");
        if (n_points) *n_points = t->n_points;
        if (n_projected) *n_projected = t->n_projected;
        if (fine_dof) std::memcpy(fine_dof, t->h_point_dof.data(), t->h_point_dof.size() * sizeof(int32_t));
        if (owner) std::memcpy(owner, t->h_point_owner.data(), t->h_point_owner.size() * sizeof(int32_t));
        if (xi) std::memcpy(xi, t->h_point_xi.data(), t->h_point_xi.size() * sizeof(double));
        return NNMG_OK;
    });
}

static void transfer_impl(const nnmg_transfer* t, int prec, int nr, const void* in, void* out, bool prolong,
                          void* stream) {
    if (!t || !in || !out) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
    if (in == out) fail(NNMG_ERR_INVALID_ARG, "vectors alias");
    if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
    check_rhs(nr);
    NNMG_HIP(hipSetDevice(t->ctx->device));
    Transfer& T = const_cast<nnmg_transfer&>(*t);
    if (prolong) {
        launch_prolongate(T, prec, in, out, as_stream(stream), nr);
    } else {
        transfer_reserve_rhs(T, nr);
        launch_restrict(T, prec, in, out, true, as_stream(stream), nr);
    }
}

int nnmg_prolongate(const nnmg_transfer* t, nnmg_prec prec, const void* coarse, void* fine, void* stream) {
    return guarded([&] {
        transfer_impl(t, prec, 1, coarse, fine, true, stream);
        return NNMG_OK;
    });
}

int nnmg_restrict(const nnmg_transfer* t, nnmg_prec prec, const void* fine, void* coarse, void* stream) {
    return guarded([&] {
        transfer_impl(t, prec, 1, fine, coarse, false, stream);
        return NNMG_OK;
    });
}

int nnmg_prolongate_multi(const nnmg_transfer* t, nnmg_prec prec, int nrhs, const void* coarse, void* fine,
                          void* stream) {
    return guarded([&] {
        transfer_impl(t, prec, nrhs, coarse, fine, true, stream);
        return NNMG_OK;
    });
}

int nnmg_restrict_multi(const nnmg_transfer* t, nnmg_prec prec, int nrhs, const void* fine, void* coarse,
                        void* stream) {
    return guarded([&] {
        transfer_impl(t, prec, nrhs, fine, coarse, false, stream);
        return NNMG_OK;
    });
}

int nnmg_hierarchy_create(nnmg_ctx* ctx, nnmg_level* const* levels, int n_levels, nnmg_transfer* const* transfers,
                          const nnmg_mg_opts* opts, nnmg_hierarchy** out) {
    return guarded([&] {
        if (!ctx || !out) fail(NNMG_ERR_INVALID_ARG, "ctx or out is NULL");
        nnmg_mg_opts o;
        nnmg_default_mg_opts(&o);
        if (opts) o = *opts;
        NNMG_HIP(hipSetDevice(ctx->device));
        *out = reinterpret_cast<nnmg_hierarchy*>(hierarchy_create(ctx, levels, n_levels, transfers, o));
        return NNMG_OK;
    });
}

void nnmg_hierarchy_destroy(nnmg_hierarchy* h) {
    if (h) hierarchy_destroy(reinterpret_cast<Hierarchy*>(h));
}

int nnmg_get_cheb_bounds(const nnmg_hierarchy* h, int level, double* lo, double* hi) {
    return guarded([&] {
        if (!h) fail(NNMG_ERR_INVALID_ARG, "hierarchy is NULL");
        get_bounds(*reinterpret_cast<const Hierarchy*>(h), level, lo, hi);
        return NNMG_OK;
    });
}

int nnmg_set_cheb_bounds(nnmg_hierarchy* h, int level, double lo, double hi) {
    return guarded([&] {
        if (!h) fail(NNMG_ERR_INVALID_ARG, "hierarchy is NULL");
        set_bounds(*reinterpret_cast<Hierarchy*>(h), level, lo, hi);
        return NNMG_OK;
    });
}

static void vcycle_impl(nnmg_hierarchy* h, int prec, int nr, const void* r, void* z, void* stream) {
    if (!h || !r || !z) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
    if (r == z) fail(NNMG_ERR_INVALID_ARG, "vectors alias");
    if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
    check_rhs(nr);
    vcycle(*reinterpret_cast<Hierarchy*>(h), prec, r, z, nr, as_stream(stream));
}

int nnmg_vcycle(nnmg_hierarchy* h, nnmg_prec prec, const void* r, void* z, void* stream) {
    return guarded([&] {
        vcycle_impl(h, prec, 1, r, z, stream);
        return NNMG_OK;
    });
}

int nnmg_vcycle_multi(nnmg_hierarchy* h, nnmg_prec prec, int nrhs, const void* r, void* z, void* stream) {
    return guarded([&] {
        vcycle_impl(h, prec, nrhs, r, z, stream);
        return NNMG_OK;
    });
}

static int pcg_impl(nnmg_hierarchy* h, int nr, const double* b, double* x, const nnmg_cg_opts* opts,
                    nnmg_cg_result* res, void* stream) {
    if (!h || !b || !x || !res) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
    if (b == x) fail(NNMG_ERR_INVALID_ARG, "vectors alias");
    check_rhs(nr);
    nnmg_cg_opts o;
    nnmg_default_cg_opts(&o);
    if (opts) o = *opts;
    const int st = pcg(*reinterpret_cast<Hierarchy*>(h), b, x, o, res, nr, as_stream(stream));
    if (st == NNMG_ERR_NOT_CONVERGED) report(st, "CG reached max_it before the tolerance");
    if (st == NNMG_ERR_BREAKDOWN) report(st, "CG breakdown (non-positive curvature or NaN)");
    return st;
}

int nnmg_pcg_solve(nnmg_hierarchy* h, const double* b, double* x, const nnmg_cg_opts* opts, nnmg_cg_result* res,
                   void* stream) {
    return guarded([&] { return pcg_impl(h, 1, b, x, opts, res, stream); });
}

int nnmg_pcg_solve_multi(nnmg_hierarchy* h, int nrhs, const double* b, double* x, const nnmg_cg_opts* opts,
                         nnmg_cg_result* res, void* stream) {
    return guarded([&] { return pcg_impl(h, nrhs, b, x, opts, res, stream); });
}

int nnmg_level_tune(nnmg_level* level, nnmg_prec prec, int reps, nnmg_tune_result* res) {
    return guarded([&] {
        if (!level || !res) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        level_tune(*level, prec, reps, res);
        return NNMG_OK;
    });
}

int nnmg_level_set_variant(nnmg_level* level, int variant) {
    return guarded([&] {
        if (!level) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        level_set_variant(*level, -1, variant);
        return NNMG_OK;
    });
}

int nnmg_level_set_variant_prec(nnmg_level* level, nnmg_prec prec, int variant) {
    return guarded([&] {
        if (!level) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        level_set_variant(*level, prec, variant);
        return NNMG_OK;
    });
}

int nnmg_level_set_rhs_split(nnmg_level* level, nnmg_prec prec, int split) {
    return guarded([&] {
        if (!level) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        level_set_rhs_split(*level, prec, split);
        return NNMG_OK;
    });
}

int nnmg_level_set_cells_per_block(nnmg_level* level, nnmg_prec prec, int cells) {
    return guarded([&] {
        if (!level) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        level_set_cells_per_block(*level, prec, cells);
        return NNMG_OK;
    });
}

int nnmg_level_cells_per_block(const nnmg_level* level, nnmg_prec prec, int* cells, int* layout_cells,
                               int64_t* layout_blocks) {
    return guarded([&] {
        if (!level || !cells || !layout_cells || !layout_blocks) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        *cells = level_cells_per_block(*level, prec);
        *layout_cells = level->cpb;
        *layout_blocks = level->nblocks;
        return NNMG_OK;
    });
}

int nnmg_level_variant(const nnmg_level* level, nnmg_prec prec, int* variant) {
    return guarded([&] {
        if (!level || !variant) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        *variant = level_variant(*level, prec);
        return NNMG_OK;
    });
}

int nnmg_transfer_tune(nnmg_transfer* transfer, nnmg_prec prec, int reps, nnmg_tune_result* res) {
    return guarded([&] {
        if (!transfer || !res) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (prec != NNMG_FP64 && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "precision");
        transfer_tune(*transfer, prec, reps, res);
        return NNMG_OK;
    });
}

int nnmg_transfer_set_team(nnmg_transfer* transfer, int team) {
    return guarded([&] {
        if (!transfer) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        transfer_set_team(*transfer, team);
        return NNMG_OK;
    });
}

int nnmg_transfer_team(const nnmg_transfer* transfer, int* team) {
    return guarded([&] {
        if (!transfer || !team) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        *team = transfer->team;
        return NNMG_OK;
    });
}

int nnmg_hierarchy_footprint(const nnmg_hierarchy* h, int nrhs, size_t* bytes) {
    return guarded([&] {
        if (!h || !bytes) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        check_rhs(nrhs);
        *bytes = hierarchy_footprint(*reinterpret_cast<const Hierarchy*>(h), nrhs);
        return NNMG_OK;
    });
}

void nnmg_default_server_opts(nnmg_server_opts* o) {
    if (!o) return;
    o->max_active = 4;
    o->memory_budget = (size_t)64 << 30;
    o->policy = NNMG_ADMIT_ARRIVAL;
    o->aging_ms = 250.0;
    o->large_work = 0.0;
    o->max_large = 64;
}

int nnmg_server_create(nnmg_ctx* ctx, const nnmg_server_opts* opts, nnmg_server** out) {
    return guarded([&] {
        if (!ctx || !out) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        nnmg_server_opts o;
        nnmg_default_server_opts(&o);
        if (opts) o = *opts;
        *out = reinterpret_cast<nnmg_server*>(server_create(ctx, o));
        return NNMG_OK;
    });
}

void nnmg_server_destroy(nnmg_server* server) {
    try {
        server_destroy(reinterpret_cast<Server*>(server));
    } catch (...) {
    }
}

int nnmg_server_submit_any(nnmg_server* server, nnmg_hierarchy* const* replicas, int n_replicas, int nrhs,
                           const double* b, double* x, const nnmg_cg_opts* opts, int64_t* ticket) {
    return guarded([&] {
        if (!server || !replicas || !b || !x || !ticket) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        if (b == x) fail(NNMG_ERR_INVALID_ARG, "vectors alias");
        check_rhs(nrhs);
        nnmg_cg_opts o;
        nnmg_default_cg_opts(&o);
        if (opts) o = *opts;
        *ticket = server_submit(reinterpret_cast<Server*>(server), reinterpret_cast<Hierarchy* const*>(replicas),
                                n_replicas, nrhs, b, x, o);
        return NNMG_OK;
    });
}

int nnmg_server_submit(nnmg_server* server, nnmg_hierarchy* h, int nrhs, const double* b, double* x,
                       const nnmg_cg_opts* opts, int64_t* ticket) {
    return nnmg_server_submit_any(server, &h, 1, nrhs, b, x, opts, ticket);
}

int nnmg_server_poll(nnmg_server* server, int64_t ticket, int* done) {
    return guarded([&] {
        if (!server || !done) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        *done = server_poll(reinterpret_cast<Server*>(server), ticket) ? 1 : 0;
        return NNMG_OK;
    });
}

int nnmg_server_wait(nnmg_server* server, int64_t ticket, nnmg_cg_result* res, nnmg_request_times* times) {
    return guarded([&] {
        if (!server) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        std::string err;
        const int st = server_wait(reinterpret_cast<Server*>(server), ticket, res, times, &err);
        if (st != NNMG_OK)
            report(st, err.empty() ? (st == NNMG_ERR_NOT_CONVERGED ? "CG reached max_it before the tolerance"
                                                                     : "request failed")
                                   : err);
        return st;
    });
}

int nnmg_server_get_stats(nnmg_server* server, nnmg_server_stats* stats) {
    return guarded([&] {
        if (!server || !stats) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        server_stats(reinterpret_cast<Server*>(server), stats);
        return NNMG_OK;
    });
}

int nnmg_hierarchy_set_profiling(nnmg_hierarchy* h, int enabled) {
    return guarded([&] {
        if (!h) fail(NNMG_ERR_INVALID_ARG, "hierarchy is NULL");
        set_profiling(*reinterpret_cast<Hierarchy*>(h), enabled != 0);
        return NNMG_OK;
    });
}

int nnmg_hierarchy_profile(nnmg_hierarchy* h, double* ms) {
    return guarded([&] {
        if (!h || !ms) fail(NNMG_ERR_INVALID_ARG, "NULL argument");
        profile(*reinterpret_cast<Hierarchy*>(h), ms);
        return NNMG_OK;
    });
}

}  // extern "C"
