// Multigrid hierarchy: Chebyshev-Jacobi smoothing, the non-nested V-cycle of
// Algorithm V_cycle (paper §2), the exact float64 coarse solve and the float64
// preconditioned CG of the paper's solver recipe (§4).
//
// V-cycle on level l >= 1 with right-hand side f and zero initial guess:
//   x   <- Chebyshev sweep from 0          (degree-1 operator products)
//   r   <- f - A x
//   f_c <- P^T r                           (restriction, paper eq. residual2)
//   x_c <- V-cycle(l-1, f_c)
//   x   <- x + P x_c                       (prolongation)
//   x   <- Chebyshev sweep from x          (degree operator products)
// The post-smoother starts from the current iterate (Algorithm V_cycle writes
// a zero initial guess there, which would discard the correction).  On level 0
// the coarse problem is solved with the explicit inverse of the unconstrained
// block plus one step of iterative refinement, always in float64.
//
// Several right-hand sides (nr <= kMaxRhs, vectors interleaved as [DoF][nr])
// run through one V-cycle or one CG together: every launch carries all of
// them, and each is computed exactly as it would be on its own.
//
// The Chebyshev sweep is the three-term recurrence on D^{-1} A over
// [lambda_max / range, lambda_max] (Saad, Alg. 12.1), with the residual
// recomputed as f - A x at every step; lambda_max is eig_safety times the
// largest Ritz value of eig_iters steps of Jacobi-preconditioned CG (Lanczos).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "../internal.hpp"

namespace nnmg {


enum { kPre = 0, kRes = 1, kRestrict = 2, kCoarse = 3, kProlong = 4, kPost = 5, kComponents = 6 };

struct WorkVectors {
    DeviceArray<char> f, x, d, ax, r;  // ax: operator output of atomic-scatter levels, kept zero between uses
    DeviceArray<char> contrib;         // operator contribution slots of this level
    DeviceArray<char> rbuf;            // restriction sums into this level (its transfer's slots): the
                                       // hierarchy's own, so hierarchies sharing a transfer can run at once
};

struct ProfileRecord {
    int level, comp;
    hipEvent_t a, b;
};

struct Hierarchy {
    Ctx* ctx = nullptr;
    std::vector<Level*> levels;
    std::vector<Transfer*> transfers;
    nnmg_mg_opts opts{};
    std::vector<double> lo, hi;

    // coarse solve
    int64_t m = 0;
    DeviceArray<int32_t> free_idx;
    DeviceArray<double> inv;        // m x m: A^{-1} on the unconstrained block
    DeviceArray<double> cx, cax;    // [N] unit vectors and operator columns at setup; [N][nr] y and r of the solve

    WorkVectors work[2][16];  // [prec][level], vectors of rhs_cap right-hand sides
    int rhs_cap = 0;          // right-hand sides the work and CG vectors hold

    // CG: vectors [N][rhs_cap]; scalars kScal per right-hand side, then a scratch word
    DeviceArray<double> r, p, qv, z, partial, scal;
    double* hscal = nullptr;  // pinned

    bool profiling = false;
    std::vector<ProfileRecord> records;
    std::vector<hipEvent_t> pool;
    std::vector<double> acc;
    hipStream_t last = nullptr;

    // the CG preconditioner (cast, V-cycle, cast back on the fixed CG vectors)
    // captured as a HIP graph per V-cycle precision
    // and number of right-hand sides
    hipStream_t capture = nullptr;
    hipGraphExec_t precond_graph[2][kMaxRhs + 1] = {};
    long graph_sig = 0;  // config_sig() when the graphs were captured

    std::atomic<bool> in_use{false};  // held by a serving request

    // changes whenever the autotuner switches a kernel variant of a level or transfer
    long config_sig() const {
        long v = 0;
        for (auto* l : levels) v += l->config_version;
        for (auto* t : transfers) v += t->config_version;
        return v;
    }

    void drop_graphs() {
        for (auto& row : precond_graph)
            for (auto& g : row)
                if (g) {
                    (void)hipGraphExecDestroy(g);
                    g = nullptr;
                }
    }

    ~Hierarchy() {
        drop_graphs();
        if (capture) (void)hipStreamDestroy(capture);
        for (auto& rec : records) {
            (void)hipEventDestroy(rec.a);
            (void)hipEventDestroy(rec.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
        if (hscal) (void)hipHostFree(hscal);
        for (auto* t : transfers) transfer_release(t);
        for (auto* l : levels) level_release(l);
    }
};

}  // namespace nnmg

struct nnmg_hierarchy : nnmg::Hierarchy {};

namespace nnmg {

static size_t wsize(int prec) { return prec == NNMG_FP64 ? 8 : 4; }

// (re)allocate the work vectors of both precisions, the CG vectors and the
// coarse-solve vectors for nr right-hand sides, and grow the transfers'
// restriction buffers; drops the captured preconditioners, which hold the
// previous addresses
static void ensure_rhs(Hierarchy& H, int nr) {
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides must be in 1..8");
    if (nr <= H.rhs_cap) return;
    NNMG_HIP(hipDeviceSynchronize());  // earlier launches may still use the vectors
    H.drop_graphs();
    for (int prec : {NNMG_FP64, NNMG_FP32})
        for (size_t l = 0; l < H.levels.size(); ++l) {
            WorkVectors& w = H.work[prec][l];
            const Level& L = *H.levels[l];
            const size_t b = std::max<size_t>((size_t)L.n_dofs * (size_t)nr, 1) * wsize(prec);
            for (auto* a : {&w.f, &w.x, &w.d, &w.r, &w.ax}) {
                a->alloc(H.ctx, b);
                NNMG_HIP(hipMemset(a->ptr, 0, b));
            }
            w.contrib.alloc(H.ctx, std::max<size_t>(L.contrib_len * L.ncomp * (size_t)nr, 1) * wsize(prec));
            if (l + 1 < H.levels.size()) w.rbuf.alloc(H.ctx, restriction_scratch_bytes(*H.transfers[l], nr));
        }
    const size_t n = std::max<size_t>((size_t)H.levels.back()->n_dofs * (size_t)nr, 1);
    for (auto* a : {&H.r, &H.p, &H.qv, &H.z}) a->alloc(H.ctx, n);
    const size_t nc = std::max<size_t>((size_t)H.levels[0]->n_dofs * (size_t)nr, 1);
    for (auto* a : {&H.cx, &H.cax}) {
        a->alloc(H.ctx, nc);
        NNMG_HIP(hipMemset(a->ptr, 0, a->bytes()));
    }
    H.rhs_cap = nr;
}

static hipEvent_t take_event(Hierarchy& H) {
    if (!H.pool.empty()) {
        hipEvent_t e = H.pool.back();
        H.pool.pop_back();
        return e;
    }
    hipEvent_t e;
    NNMG_HIP(hipEventCreate(&e));
    return e;
}

struct Scope {
    Hierarchy& H;
    int level, comp;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Scope(Hierarchy& h, int l, int c, hipStream_t st) : H(h), level(l), comp(c), s(st) {
        if (H.profiling) {
            a = take_event(H);
            NNMG_HIP(hipEventRecord(a, s));
        }
    }
    ~Scope() noexcept(false) {
        if (H.profiling && a) {
            hipEvent_t b = take_event(H);
            NNMG_HIP(hipEventRecord(b, s));
            H.records.push_back({level, comp, a, b});
        }
    }
};

// ---------------------------------------------------------------------------
// coarse solve
// ---------------------------------------------------------------------------
static void setup_coarse(Hierarchy& H) {
    Level& C = *H.levels[0];
    Ctx* ctx = H.ctx;
    std::vector<int32_t> idx;
    for (int64_t i = 0; i < C.n_dofs; ++i)
        if (!C.constrained[(size_t)(i / C.ncomp)]) idx.push_back((int32_t)i);
    H.m = (int64_t)idx.size();
    const size_t N = (size_t)C.n_dofs, m = (size_t)H.m;
    H.cx.alloc(ctx, N);
    H.cax.alloc(ctx, N);
    for (auto* a : {&H.cx, &H.cax}) NNMG_HIP(hipMemset(a->ptr, 0, a->bytes()));
    if (m == 0) return;
    H.free_idx.upload(ctx, idx);
    H.inv.alloc(ctx, m * m);
    // columns of A on the unconstrained block: A e_j by the operator kernel
    for (size_t j = 0; j < m; ++j) {
        launch_set_unit(H.cx.ptr, N, idx[j], 1.0, nullptr);
        launch_vmult_cells(C, NNMG_FP64, H.cx.ptr, H.cax.ptr, nullptr);
        launch_column_from_unit(H.free_idx.ptr, m, H.cax.ptr, H.inv.ptr, j, nullptr);
        launch_fill(H.cax.ptr, N, NNMG_FP64, nullptr);
        launch_set_unit(H.cx.ptr, N, idx[j], 0.0, nullptr);
    }
    DeviceArray<double> rowbuf, colbuf;
    rowbuf.alloc(ctx, m);
    colbuf.alloc(ctx, m);
    launch_gauss_jordan(H.inv.ptr, m, rowbuf.ptr, colbuf.ptr, nullptr);
    NNMG_HIP(hipDeviceSynchronize());
}

static void op_residual(Hierarchy& H, int l, int prec, const void* f, const void* x, void* r, int nr, hipStream_t s);

// x = A_0^{-1} f on the unconstrained block with the dense float64 inverse
// (row-parallel kernels that gather f and scatter x through the free-DoF list
// themselves).  In float64, one refinement step:
//   y = A^{-1} f,  r = f - A y (the level's own operator),  x = y + A^{-1} r.
// In float32 the single product suffices: its error, cond(A) times the
// float64 rounding, lies far below the float32 rounding of x.
static void coarse_solve(Hierarchy& H, int prec, const void* f, void* x, int nr, hipStream_t s) {
    Level& C = *H.levels[0];
    const size_t N = (size_t)C.n_dofs, m = (size_t)H.m;
    launch_fill(x, N * (size_t)nr, prec, s);  // constrained entries
    if (m == 0) return;
    const int32_t* fi = H.free_idx.ptr;
    if (prec == NNMG_FP32) {
        launch_coarse_gemv(H.inv.ptr, m, f, prec, fi, nullptr, NNMG_FP64, nullptr, 1.0, x, prec, fi, s, nr);
        return;
    }
    // y into the unconstrained entries of cx, whose constrained entries stay zero
    launch_coarse_gemv(H.inv.ptr, m, f, prec, fi, nullptr, NNMG_FP64, nullptr, 1.0, H.cx.ptr, NNMG_FP64, fi, s, nr);
    op_residual(H, 0, NNMG_FP64, f, H.cx.ptr, H.cax.ptr, nr, s);
    launch_coarse_gemv(H.inv.ptr, m, H.cax.ptr, NNMG_FP64, fi, H.cx.ptr, NNMG_FP64, fi, 1.0, x, prec, fi, s, nr);
}

// ---------------------------------------------------------------------------
// smoother and V-cycle
// ---------------------------------------------------------------------------
// x <- x + d with d <- c1 d + c2 D^{-1} (f - A x); mode (kCheb*): the old d
// is 0 (c1 unused) or x, and the new d is dropped after the last step
static void op_cheb_step(Hierarchy& H, int l, int prec, const void* f, const void* dinv, void* x, double c1,
                         double c2, int mode, int nr, hipStream_t s) {
    Level& L = *H.levels[l];
    WorkVectors& w = H.work[prec][l];
    if (L.var[prec].atomic) {
        launch_vmult_cells(L, prec, x, w.ax.ptr, s, nr, w.contrib.ptr);
        launch_cheb_step(prec, (size_t)L.n_dofs, f, w.ax.ptr, dinv, x, w.d.ptr, c1, c2, mode, s, nr);
    } else {
        launch_vmult_contrib(L, prec, x, w.contrib.ptr, s, nr);
        launch_cheb_step_gather(L, prec, w.contrib.ptr, f, dinv, x, w.d.ptr, c1, c2, mode, s, nr);
    }
}

// r = f - A x
static void op_residual(Hierarchy& H, int l, int prec, const void* f, const void* x, void* r, int nr, hipStream_t s) {
    Level& L = *H.levels[l];
    WorkVectors& w = H.work[prec][l];
    if (L.var[prec].atomic) {
        launch_vmult_cells(L, prec, x, w.ax.ptr, s, nr, w.contrib.ptr);
        launch_residual(prec, (size_t)L.n_dofs * (size_t)nr, f, w.ax.ptr, r, s);
    } else {
        launch_vmult_contrib(L, prec, x, w.contrib.ptr, s, nr);
        launch_residual_gather(L, prec, w.contrib.ptr, f, r, s, nr);
    }
}

// cast_from (float32 cycle, zero start): the right-hand side arrives in
// float64 and the first step also writes its float32 copy into f
// first_done (zero start): the first step, x = D^-1 f / theta, was fused
// into the restriction that formed f.  A first step from zero leaves d = x and
// stores only x; the second step reads x as d.  The last step does not store d.
static void chebyshev(Hierarchy& H, int l, int prec, const void* f, void* x, bool zero_start, int nr,
                      hipStream_t s, const double* cast_from = nullptr, bool first_done = false) {
    Level& L = *H.levels[l];
    const void* dinv = prec == NNMG_FP64 ? (const void*)L.d_dinv64.ptr : (const void*)L.d_dinv32.ptr;
    const double lo = H.lo[l], hi = H.hi[l];
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    const int deg = H.opts.cheb_degree;
    if (zero_start && first_done) {
        // x holds the first step already
    } else if (zero_start && cast_from)
        launch_cast_cheb_first_zero((size_t)L.n_dofs, cast_from, (float*)const_cast<void*>(f), (const float*)dinv,
                                    (float*)x, 1.0 / theta, s, nr);
    else if (zero_start)
        launch_cheb_first_zero(prec, (size_t)L.n_dofs, f, dinv, x, 1.0 / theta, s, nr);
    else
        op_cheb_step(H, l, prec, f, dinv, x, 0.0, 1.0 / theta, kChebFirst | (deg == 1 ? kChebLast : 0), nr, s);
    for (int j = 1; j < deg; ++j) {
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        const int mode = (j == 1 && zero_start ? kChebDIsX : 0) | (j == deg - 1 ? kChebLast : 0);
        op_cheb_step(H, l, prec, f, dinv, x, rho_new * rho, 2.0 * rho_new / delta, mode, nr, s);
        rho = rho_new;
    }
}

// cast_from: a float32 cycle whose right-hand side f is first cast from these
// float64 values (the cast is fused into the first smoothing step)
static void vcycle_level(Hierarchy& H, int l, int prec, const void* f, void* x, int nr, hipStream_t s,
                         const double* cast_from = nullptr, bool first_done = false) {
    if (cast_from && prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "cast into a float64 cycle");
    if (l == 0) {
        Scope sc(H, 0, kCoarse, s);
        if (cast_from)
            launch_cast_64_to_32(cast_from, (float*)const_cast<void*>(f),
                                 (size_t)H.levels[0]->n_dofs * (size_t)nr, s);
        coarse_solve(H, prec, f, x, nr, s);
        return;
    }
    WorkVectors& w = H.work[prec][l];
    WorkVectors& wc = H.work[prec][l - 1];
    const Transfer& T = *H.transfers[l - 1];
    {
        Scope sc(H, l, kPre, s);
        chebyshev(H, l, prec, f, x, true, nr, s, cast_from, first_done);
    }
    {
        Scope sc(H, l, kRes, s);
        op_residual(H, l, prec, f, x, w.r.ptr, nr, s);
    }
    {
        Scope sc(H, l, kRestrict, s);
        // every unconstrained coarse DoF has restriction slots; the constrained
        // entries of f_c are never written and stay zero.  Above the coarsest
        // level the coarse pre-smoothing's first step is fused in.
        if (l - 1 >= 1) {
            const Level& C = *H.levels[l - 1];
            const void* dinv = prec == NNMG_FP64 ? (const void*)C.d_dinv64.ptr : (const void*)C.d_dinv32.ptr;
            const double theta = 0.5 * (H.hi[l - 1] + H.lo[l - 1]);
            launch_restrict_first_zero(T, prec, w.r.ptr, wc.f.ptr, dinv, wc.x.ptr, 1.0 / theta, s, nr,
                                       wc.rbuf.ptr);
        } else {
            launch_restrict(T, prec, w.r.ptr, wc.f.ptr, false, s, nr, wc.rbuf.ptr);
        }
    }
    vcycle_level(H, l - 1, prec, wc.f.ptr, wc.x.ptr, nr, s, nullptr, l - 1 >= 1);
    {
        Scope sc(H, l, kProlong, s);
        launch_prolongate(T, prec, wc.x.ptr, x, s, nr);
    }
    {
        Scope sc(H, l, kPost, s);
        chebyshev(H, l, prec, f, x, false, nr, s);
    }
}

// ---------------------------------------------------------------------------
// Lanczos estimate of lambda_max(D^{-1} A)
// ---------------------------------------------------------------------------
static double tridiagonal_max_eig(const std::vector<double>& d, const std::vector<double>& e) {
    // Sturm-sequence bisection for the largest eigenvalue of a symmetric tridiagonal matrix
    const int m = (int)d.size();
    if (m == 0) return 0.0;
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(e[(size_t)i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[(size_t)i]) : 0.0);
        lo = std::min(lo, d[(size_t)i] - r);
        hi = std::max(hi, d[(size_t)i] + r);
    }
    auto count_below = [&](double x) {  // eigenvalues < x
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < m; ++i) {
            const double off = i > 0 ? e[(size_t)i - 1] * e[(size_t)i - 1] : 0.0;
            q = d[(size_t)i] - x - (i > 0 ? off / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (count_below(mid) >= m)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

static double host_dot(Hierarchy& H, const double* a, const double* b, size_t n) {
    double* scratch = H.scal.ptr + kScal * kMaxRhs;
    launch_dot(a, b, n, H.partial.ptr, scratch, nullptr);
    double v = 0.0;
    NNMG_HIP(hipMemcpy(&v, scratch, sizeof(double), hipMemcpyDeviceToHost));
    return v;
}

static double estimate_lambda_max(Hierarchy& H, int l) {
    Level& L = *H.levels[l];
    const size_t n = (size_t)L.n_dofs;
    DeviceArray<double> r, z, p, q;
    r.alloc(H.ctx, n);
    z.alloc(H.ctx, n);
    p.alloc(H.ctx, n);
    q.alloc(H.ctx, n);
    const void* start = H.opts.eig_start ? H.opts.eig_start[l] : nullptr;
    if (start)
        NNMG_HIP(hipMemcpy(r.ptr, start, n * sizeof(double), hipMemcpyDeviceToDevice));
    else
        launch_splitmix_vector(r.ptr, nullptr, n, 0x5EEDull + (uint64_t)l, nullptr);
    launch_set_constrained(L.d_constrained.ptr, L.constrained_idx.size(), 0.0, r.ptr, NNMG_FP64, nullptr);
    launch_jacobi(n, L.d_dinv64.ptr, r.ptr, z.ptr, nullptr);
    NNMG_HIP(hipMemcpy(p.ptr, z.ptr, n * sizeof(double), hipMemcpyDeviceToDevice));
    double rz = host_dot(H, r.ptr, z.ptr, n);
    const double r0 = std::sqrt(host_dot(H, r.ptr, r.ptr, n));
    std::vector<double> alphas, betas;
    for (int it = 0; it < H.opts.eig_iters; ++it) {
        launch_fill(q.ptr, n, NNMG_FP64, nullptr);
        launch_vmult_cells(L, NNMG_FP64, p.ptr, q.ptr, nullptr);
        const double pq = host_dot(H, p.ptr, q.ptr, n);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        alphas.push_back(alpha);
        launch_lincomb(n, -alpha, q.ptr, 1.0, r.ptr, nullptr);
        if (std::sqrt(host_dot(H, r.ptr, r.ptr, n)) <= 1e-14 * r0) break;
        launch_jacobi(n, L.d_dinv64.ptr, r.ptr, z.ptr, nullptr);
        const double rz_new = host_dot(H, r.ptr, z.ptr, n);
        const double beta = rz_new / rz;
        betas.push_back(beta);
        launch_lincomb(n, 1.0, z.ptr, beta, p.ptr, nullptr);
        rz = rz_new;
    }
    const size_t k = alphas.size();
    std::vector<double> d(k), e(k > 0 ? k - 1 : 0);
    for (size_t j = 0; j < k; ++j) {
        d[j] = 1.0 / alphas[j] + (j > 0 ? betas[j - 1] / alphas[j - 1] : 0.0);
        if (j + 1 < k) e[j] = std::sqrt(betas[j]) / alphas[j];
    }
    return tridiagonal_max_eig(d, e);
}

// ---------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------
Hierarchy* hierarchy_create(Ctx* ctx, nnmg_level* const* levels, int nl, nnmg_transfer* const* transfers,
                            const nnmg_mg_opts& o) {
    if (nl < 1 || nl > 16 || !levels) fail(NNMG_ERR_INVALID_ARG, "n_levels must be in 1..16");
    if (nl > 1 && !transfers) fail(NNMG_ERR_INVALID_ARG, "transfers is NULL");
    if (o.cheb_degree < 1 || !(o.smoothing_range > 1.0) || !(o.eig_safety > 0.0) || o.eig_iters < 1)
        fail(NNMG_ERR_INVALID_ARG, "multigrid options");
    for (int i = 0; i < nl; ++i) {
        if (!levels[i]) fail(NNMG_ERR_INVALID_ARG, "level is NULL");
        if (levels[i]->op != levels[0]->op || levels[i]->lam != levels[0]->lam || levels[i]->mu != levels[0]->mu)
            fail(NNMG_ERR_INVALID_ARG, "all levels must carry the same operator");
    }
    for (int i = 0; i + 1 < nl; ++i) {
        const Transfer* t = transfers[i];
        if (!t || t->fine != levels[i + 1] || t->coarse != levels[i])
            fail(NNMG_ERR_INVALID_ARG, "transfers[i] must connect levels[i+1] (fine) to levels[i] (coarse)");
    }
    NNMG_HIP(hipSetDevice(ctx->device));
    auto* H = new nnmg_hierarchy();
    try {
        H->ctx = ctx;
        H->opts = o;
        for (int i = 0; i < nl; ++i) {
            level_retain(levels[i]);
            H->levels.push_back(levels[i]);
        }
        for (int i = 0; i + 1 < nl; ++i) {
            transfer_retain(transfers[i]);
            H->transfers.push_back(transfers[i]);
        }
        H->opts.eig_start = nullptr;
        const size_t nmax = (size_t)H->levels.back()->n_dofs;
        H->partial.alloc(ctx, dot_partials(nmax > 0 ? nmax : 1) * kMaxRhs + 8);
        H->scal.alloc(ctx, kScal * kMaxRhs + 8);
        NNMG_HIP(hipMemset(H->scal.ptr, 0, H->scal.bytes()));
        NNMG_HIP(hipHostMalloc((void**)&H->hscal, (kScal * kMaxRhs + 8) * sizeof(double), hipHostMallocDefault));
        H->lo.assign((size_t)nl, 0.0);
        H->hi.assign((size_t)nl, 0.0);
        H->opts.eig_start = o.eig_start;
        for (int l = 1; l < nl; ++l) {
            const double lam = estimate_lambda_max(*H, l);
            H->hi[(size_t)l] = o.eig_safety * lam;
            H->lo[(size_t)l] = H->hi[(size_t)l] / o.smoothing_range;
        }
        H->opts.eig_start = nullptr;  // the caller's vectors are not kept
        setup_coarse(*H);
        ensure_rhs(*H, 1);
        H->acc.assign((size_t)nl * kComponents, 0.0);
        NNMG_HIP(hipDeviceSynchronize());
    } catch (...) {
        delete H;
        throw;
    }
    return H;
}

void hierarchy_destroy(Hierarchy* h) { delete static_cast<nnmg_hierarchy*>(h); }

void get_bounds(const Hierarchy& H, int l, double* lo, double* hi) {
    if (l < 0 || l >= (int)H.levels.size()) fail(NNMG_ERR_INVALID_ARG, "level index");
    if (lo) *lo = H.lo[(size_t)l];
    if (hi) *hi = H.hi[(size_t)l];
}

void set_bounds(Hierarchy& H, int l, double lo, double hi) {
    if (l < 1 || l >= (int)H.levels.size()) fail(NNMG_ERR_INVALID_ARG, "level index (the coarsest has no smoother)");
    if (!(lo > 0.0) || !(hi > lo)) fail(NNMG_ERR_INVALID_ARG, "bounds must satisfy 0 < lo < hi");
    H.lo[(size_t)l] = lo;
    H.hi[(size_t)l] = hi;
    H.drop_graphs();  // the captured V-cycles hold the previous coefficients
}

void vcycle(Hierarchy& H, int prec, const void* r, void* z, int nr, hipStream_t s) {
    ensure_rhs(H, nr);
    H.last = s;
    vcycle_level(H, (int)H.levels.size() - 1, prec, r, z, nr, s);
}

// ---------------------------------------------------------------------------
// PCG (float64), Saad Alg. 9.1 with x0 = 0, for nr right-hand sides at once
// ---------------------------------------------------------------------------
// Each right-hand side has its own scalars (scal + r * kScal) and its own
// stopping test.  One that has converged (or broken down) is frozen: its
// active flag is cleared, so alpha = beta = 0 from then on and its iterate and
// residual stay exactly as they were, while the others go on.  An iteration
// updates r at once and x with the next direction (both read the old p there),
// the last x update being launched when the solve ends: the same operations
// in another kernel, so the iterates are those of the textbook order.
//
// The solve is a resumable task: every stage ends with an asynchronous copy
// of the scalars to pinned host memory and an event; step() runs when that
// event has completed, takes the decisions the scalars call for and launches
// the next stage.  The blocking solve waits for each event in turn; the
// serving loop (host/server.cpp) advances many tasks on their own streams.
struct PcgTask {
    Hierarchy& H;
    const double* b;
    double* x;
    nnmg_cg_opts o;
    nnmg_cg_result* res;
    int nr;
    hipStream_t s;
    hipEvent_t ev = nullptr;
    int it = 0;
    bool started = false;  // the b.b stage is done once started
    bool done = false;
    std::vector<double> bnorm;
    std::vector<char> active;
    int n_active = 0;
    bool graph = false;
    int prec = NNMG_FP64;
    size_t n = 0, nv = 0, nsc = 0, hlen = 0;

    PcgTask(Hierarchy& h, const double* b_, double* x_, const nnmg_cg_opts& o_, nnmg_cg_result* r_, int nr_,
            hipStream_t s_)
        : H(h), b(b_), x(x_), o(o_), res(r_), nr(nr_), s(s_) {}
    ~PcgTask() {
        if (ev) (void)hipEventDestroy(ev);
    }

    Level& L() { return *H.levels.back(); }
    int top() const { return (int)H.levels.size() - 1; }

    // z = V(r) on the hierarchy's own vectors, so the launches can be captured
    // once.  A float32 cycle reads r through its first smoothing step and
    // leaves its result in float32, which r.z and the direction update read.
    void launches(hipStream_t st) {
        WorkVectors& w32 = H.work[NNMG_FP32][top()];
        if (prec == NNMG_FP64)
            vcycle_level(H, top(), NNMG_FP64, H.r.ptr, H.z.ptr, nr, st);
        else
            vcycle_level(H, top(), NNMG_FP32, w32.f.ptr, w32.x.ptr, nr, st, H.r.ptr);
    }

    // z = V(r), then r.z into out (and the CG scalar op on it, op >= 0).  The
    // float32 cycle leaves z in float32; its float64 value goes to z64 if that
    // is given (the first direction), else the direction update widens it.
    void precondition_dot(double* out, int op, double* z64 = nullptr) {
        if (graph)
            NNMG_HIP(hipGraphLaunch(H.precond_graph[prec][nr], s));
        else
            launches(s);
        double* sc = op >= 0 ? H.scal.ptr : nullptr;
        if (prec == NNMG_FP64)
            launch_dot(H.r.ptr, H.z.ptr, n, H.partial.ptr, out, s, nr, kScal, sc, op);
        else
            launch_cast_dot(H.r.ptr, z32(), z64, n, H.partial.ptr, out, s, nr, kScal, sc, op);
    }

    const float* z32() { return (const float*)H.work[NNMG_FP32][top()].x.ptr; }

    // scalars to the host, then the event step() waits for
    void fetch_async() {
        NNMG_HIP(hipMemcpyAsync(H.hscal, H.scal.ptr, nsc * sizeof(double), hipMemcpyDeviceToHost, s));
        NNMG_HIP(hipEventRecord(ev, s));
    }

    // the host copy is current (fetched with nothing launched since), so it can go back whole
    void push_flags() {
        NNMG_HIP(hipMemcpyAsync(H.scal.ptr, H.hscal, nsc * sizeof(double), hipMemcpyHostToDevice, s));
    }

    // operator product, alpha, update of r, and the fetch of the new scalars
    void iteration_body() {
        double* sc = H.scal.ptr;
        Level& lv = L();
        if (lv.var[NNMG_FP64].atomic) {
            launch_fill(H.qv.ptr, nv, NNMG_FP64, s);
            launch_vmult_cells(lv, NNMG_FP64, H.p.ptr, H.qv.ptr, s, nr, H.work[NNMG_FP64][top()].contrib.ptr);
            launch_dot(H.p.ptr, H.qv.ptr, n, H.partial.ptr, sc + 1, s, nr, kScal, sc, 0);
        } else {
            double* cb = (double*)H.work[NNMG_FP64][top()].contrib.ptr;
            launch_vmult_contrib(lv, NNMG_FP64, H.p.ptr, cb, s, nr);
            launch_gather_dot(lv, cb, H.p.ptr, H.qv.ptr, H.partial.ptr, sc + 1, s, nr, sc, 0);
        }
        // (alpha is formed by the reduction of p.q; x += alpha p follows with
        // the next direction, or at the end of the solve)
        launch_cg_update(n, H.r.ptr, H.qv.ptr, sc, H.partial.ptr, sc + 3, s, nr);
        fetch_async();
    }

    // first stage: r = b, x = 0, b.b
    void start() {
        if (o.max_it < 0 || !(o.rtol >= 0.0)) fail(NNMG_ERR_INVALID_ARG, "CG options");
        if (o.vcycle_prec != NNMG_FP64 && o.vcycle_prec != NNMG_FP32) fail(NNMG_ERR_INVALID_ARG, "vcycle_prec");
        ensure_rhs(H, nr);
        H.last = s;
        n = (size_t)L().n_dofs;
        nv = n * (size_t)nr;
        nsc = (size_t)kScal * (size_t)nr;
        hlen = (size_t)o.max_it + 1;
        prec = o.vcycle_prec;
        graph = o.use_graph && !H.profiling;
        if (H.graph_sig != H.config_sig()) {  // captured with other kernel variants
            H.drop_graphs();
            H.graph_sig = H.config_sig();
        }
        hipGraphExec_t& exec = H.precond_graph[prec][nr];
        if (graph && !exec) {
            if (!H.capture) NNMG_HIP(hipStreamCreateWithFlags(&H.capture, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            NNMG_HIP(hipStreamBeginCapture(H.capture, hipStreamCaptureModeThreadLocal));
            try {
                launches(H.capture);
            } catch (...) {
                (void)hipStreamEndCapture(H.capture, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            NNMG_HIP(hipStreamEndCapture(H.capture, &g));
            const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                exec = nullptr;
                fail(NNMG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
        }
        NNMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        NNMG_HIP(hipMemcpyAsync(H.r.ptr, b, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_fill(x, nv, NNMG_FP64, s);
        launch_dot(b, b, n, H.partial.ptr, H.scal.ptr + 6, s, nr, kScal);
        fetch_async();
    }

    int overall() const {
        int st = NNMG_OK;
        for (int k = 0; k < nr; ++k)
            if (res[k].status == NNMG_ERR_BREAKDOWN) st = NNMG_ERR_BREAKDOWN;
            else if (res[k].status != NNMG_OK && st == NNMG_OK) st = res[k].status;
        return st;
    }

    bool ready() const { return hipEventQuery(ev) == hipSuccess; }

    // the scalars of the last stage are on the host: decide and launch the
    // next stage; true when the solve has finished
    bool step() {
        double* hs = H.hscal;
        double* sc = H.scal.ptr;
        if (!started) {
            started = true;
            bnorm.assign((size_t)nr, 0.0);
            active.assign((size_t)nr, 0);
            for (int k = 0; k < nr; ++k) {
                const double bn = std::sqrt(hs[k * kScal + 6]);
                bnorm[(size_t)k] = bn;
                if (o.history) o.history[(size_t)k * hlen] = 1.0;
                res[k].iterations = 0;
                res[k].relres = bn > 0 ? 1.0 : 0.0;
                res[k].status = NNMG_OK;
                if (std::isnan(bn)) {
                    res[k].status = NNMG_ERR_BREAKDOWN;
                } else if (bn > 0.0) {
                    res[k].status = NNMG_ERR_NOT_CONVERGED;
                    active[(size_t)k] = 1;
                    ++n_active;
                }
                hs[k * kScal + 7] = active[(size_t)k] ? 1.0 : 0.0;
            }
            if (n_active == 0 || o.max_it == 0) return done = true;
            push_flags();
            // the first direction is z
            if (prec == NNMG_FP64) {
                precondition_dot(sc + 0, -1);
                NNMG_HIP(hipMemcpyAsync(H.p.ptr, H.z.ptr, nv * sizeof(double), hipMemcpyDeviceToDevice, s));
            } else {
                precondition_dot(sc + 0, -1, H.p.ptr);
            }
            it = 1;
            iteration_body();
            return false;
        }
        bool changed = false;
        for (int k = 0; k < nr; ++k) {
            if (!active[(size_t)k]) continue;
            const double pq = hs[k * kScal + 1], rr = hs[k * kScal + 3];
            res[k].iterations = it;
            bool stop = false;
            if (!(pq > 0.0) || !std::isfinite(rr)) {
                res[k].status = NNMG_ERR_BREAKDOWN;
                stop = true;
            } else {
                const double rel = std::sqrt(rr) / bnorm[(size_t)k];
                res[k].relres = rel;
                if (o.history) o.history[(size_t)k * hlen + (size_t)it] = rel;
                if (rel <= o.rtol) {
                    res[k].status = NNMG_OK;
                    stop = true;
                }
            }
            if (stop) {
                active[(size_t)k] = 0;
                hs[k * kScal + 7] = 0.0;
                --n_active;
                changed = true;
            }
        }
        if (n_active == 0 || it == o.max_it) {
            // the last iteration's x += alpha p (alpha as the iteration formed
            // it: the scalars on the device are unchanged since)
            launch_cg_direction(n, nullptr, H.p.ptr, x, sc, s, nr);
            return done = true;
        }
        if (changed) push_flags();
        precondition_dot(sc + 4, 1);  // and beta
        if (prec == NNMG_FP64)
            launch_cg_direction(n, H.z.ptr, H.p.ptr, x, sc, s, nr);
        else
            launch_cg_direction32(n, z32(), H.p.ptr, x, sc, s, nr);
        ++it;
        iteration_body();
        return false;
    }
};

PcgTask* pcg_task_create(Hierarchy& H, const double* b, double* x, const nnmg_cg_opts& o, nnmg_cg_result* res,
                         int nr, hipStream_t s) {
    auto* t = new PcgTask(H, b, x, o, res, nr, s);
    try {
        t->start();
    } catch (...) {
        delete t;
        throw;
    }
    return t;
}

bool pcg_task_ready(const PcgTask* t) { return t->ready(); }
bool pcg_task_step(PcgTask* t) { return t->step(); }
int pcg_task_status(const PcgTask* t) { return t->overall(); }
void pcg_task_destroy(PcgTask* t) { delete t; }

int pcg(Hierarchy& H, const double* b, double* x, const nnmg_cg_opts& o, nnmg_cg_result* res, int nr,
        hipStream_t s) {
    PcgTask t(H, b, x, o, res, nr, s);
    t.start();
    do {
        NNMG_HIP(hipEventSynchronize(t.ev));
    } while (!t.step());
    NNMG_HIP(hipStreamSynchronize(s));  // the final update of x
    return t.overall();
}

// device memory a solve of nr right-hand sides needs beyond the hierarchy's
// fixed data: work vectors of both precisions, CG vectors, coarse-solve
// vectors, contribution and restriction buffers
size_t hierarchy_footprint(const Hierarchy& H, int nr) {
    size_t bytes = 0;
    for (int prec : {NNMG_FP64, NNMG_FP32}) {
        const size_t w = prec == NNMG_FP64 ? 8 : 4;
        for (const Level* L : H.levels)
            bytes += (5 * (size_t)L->n_dofs + L->contrib_len * L->ncomp) * (size_t)nr * w;
    }
    bytes += 4 * (size_t)H.levels.back()->n_dofs * (size_t)nr * 8;
    bytes += 2 * (size_t)H.levels[0]->n_dofs * (size_t)nr * 8;
    for (const Transfer* t : H.transfers) bytes += 2 * restriction_scratch_bytes(*t, nr);
    return bytes;
}

int64_t hierarchy_fine_dofs(const Hierarchy& H) { return H.levels.back()->n_dofs; }

// the hierarchy's own work memory must not be shared by two solves at a time
bool hierarchy_try_acquire(Hierarchy& H) {
    bool expect = false;
    return H.in_use.compare_exchange_strong(expect, true);
}
void hierarchy_release(Hierarchy& H) { H.in_use.store(false); }

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
void set_profiling(Hierarchy& H, bool on) { H.profiling = on; }

void profile(Hierarchy& H, double* ms) {
    if (H.last) NNMG_HIP(hipStreamSynchronize(H.last));
    NNMG_HIP(hipDeviceSynchronize());
    for (auto& rec : H.records) {
        float t = 0.f;
        NNMG_HIP(hipEventElapsedTime(&t, rec.a, rec.b));
        H.acc[(size_t)(rec.level * kComponents + rec.comp)] += t;
        H.pool.push_back(rec.a);
        H.pool.push_back(rec.b);
    }
    H.records.clear();
    std::memcpy(ms, H.acc.data(), H.acc.size() * sizeof(double));
    std::fill(H.acc.begin(), H.acc.end(), 0.0);
}

}  // namespace nnmg
