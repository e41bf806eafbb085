// Transfer setup (timed setup of the non-nested transfer, paper §3.1 and §3.3).
//
// 1. The unconstrained fine support points are the query points.
// 2. Every coarse cell's vertex bounding box is grown on every side by
//    bbox_expand times its diagonal; a uniform bucket grid over the grown
//    boxes lists, per bucket, the cells whose grown box overlaps it, in
//    increasing cell number (the GPU replacement of a bounding-box tree).
// 3. On the GPU, each point visits the cells of its bucket in increasing
//    number, keeps those whose grown box contains it, inverts their Q1 maps by
//    Newton's method and stops at the first cell that contains the pre-image;
//    otherwise it keeps the candidate with the nearest clamped pre-image
//    (eq. closest_point).
// 4. The points are counting-sorted by owner cell (stable, so fine DoF order
//    within a cell), and the reference coordinates are stored per coordinate
//    in float64 and float32.
// Two levels on one mesh with a lower coarse degree get the nested polynomial
// transfer instead (setup_nested_p, kernels/pmg.hip).
#include <algorithm>
#include <cmath>
#include <memory>
#include <thread>

#include "../internal.hpp"

#ifndef NNMG_RESTRICT_PTS_PER_LANE
#define NNMG_RESTRICT_PTS_PER_LANE 4
#endif

namespace nnmg {

// host threads for the setup's passes over all fine points
static int sort_threads() {
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::min(8u, std::max(1u, h));
}

// fn(0) .. fn(n - 1), each on its own thread (fn(0) on the caller's)
template <class F>
static void run_threads(int n, F&& fn) {
    std::vector<std::thread> th;
    for (int t = 1; t < n; ++t) th.emplace_back([&fn, t] { fn(t); });
    fn(0);
    for (auto& x : th) x.join();
}

// host storage that is written in full before it is read, left uninitialised
template <class V>
static std::unique_ptr<V[]> host_buffer(size_t n) {
    return std::unique_ptr<V[]>(new V[n]);
}

// restriction slots: the sum of coarse cell K for node a goes to
// rslot[K q + a], the slots of coarse node j being [roff[j], roff[j+1])
static void build_restriction_slots(Transfer* T, Ctx* ctx) {
    const Level* coarse = T->coarse;
    const std::vector<int32_t>& cdm = coarse->dofmap;
    std::vector<int32_t> roff((size_t)coarse->n_nodes + 1, 0);
    for (size_t k = 0; k < cdm.size(); ++k)
        if (!coarse->constrained[(size_t)cdm[k]]) roff[(size_t)cdm[k] + 1]++;
    for (int64_t j = 0; j < coarse->n_nodes; ++j) roff[(size_t)j + 1] += roff[(size_t)j];
    std::vector<int32_t> cur(roff.begin(), roff.end() - 1);
    std::vector<int32_t> rslot(cdm.size(), -1);
    for (size_t k = 0; k < cdm.size(); ++k)
        if (!coarse->constrained[(size_t)cdm[k]]) rslot[k] = cur[(size_t)cdm[k]]++;
    T->d_rslot.upload(ctx, rslot);
    T->d_roff.upload(ctx, roff);
    // ncomp values per slot: component c of slot k at ncomp * k + c
    T->n_rslots = (size_t)roff.back();
    T->d_rbuf.alloc(ctx, std::max<size_t>(T->n_rslots * coarse->ncomp, 1));
}

// Nested polynomial transfer (paper §2, Coarse grid solvers): both levels on
// one mesh, coarse degree below the fine one.  Every unconstrained fine node
// is owned by the first cell (in cell order) that holds it; P on a cell is the
// tensor product of the 1D interpolation matrix E from the coarse Gauss-Lobatto
// basis to the fine nodes.  The location results (owner, reference position)
// are recorded as for the located transfer.
static void setup_nested_p(Transfer* T, Ctx* ctx) {
    const Level* fine = T->fine;
    const Level* coarse = T->coarse;
    const int dim = fine->dim, nf = fine->n, nc = coarse->n, qf = fine->q;
    const int64_t C = fine->n_cells;
    T->nested_p = true;
    for (int i = 0; i < nf; ++i)
        for (int a = 0; a < nc; ++a) {
            double v = 1.0;
            for (int m = 0; m < nc; ++m)
                if (m != a) v *= (fine->basis.node[i] - coarse->basis.node[m]) / (coarse->basis.node[a] - coarse->basis.node[m]);
            T->pmat[i * kMaxN + a] = v;
        }
    std::vector<int32_t> pfdm((size_t)(C * qf), -1), owner((size_t)fine->n_nodes, -1), local((size_t)fine->n_nodes, -1);
    for (int64_t c = 0; c < C; ++c)
        for (int a = 0; a < qf; ++a) {
            const int32_t node = fine->dofmap[(size_t)(c * qf + a)];
            if (fine->constrained[(size_t)node] || owner[(size_t)node] >= 0) continue;
            owner[(size_t)node] = (int32_t)c;
            local[(size_t)node] = a;
            pfdm[(size_t)(c * qf + a)] = node;
        }
    T->d_pfdm.upload(ctx, pfdm);
    for (int64_t i = 0; i < fine->n_nodes; ++i) {
        if (fine->constrained[(size_t)i]) continue;
        T->h_point_dof.push_back((int32_t)i);
        T->h_point_owner.push_back(owner[(size_t)i]);
        const int a = local[(size_t)i];
        const int ax = a % nf, ay = (a / nf) % nf, az = a / (nf * nf);
        T->h_point_xi.push_back(fine->basis.node[ax]);
        T->h_point_xi.push_back(fine->basis.node[ay]);
        if (dim == 3) T->h_point_xi.push_back(fine->basis.node[az]);
    }
    T->n_points = (int64_t)T->h_point_dof.size();
    T->n_projected = 0;
    build_restriction_slots(T, ctx);
}

static bool same_mesh(const Level* a, const Level* b) {
    return a->dim == b->dim && a->vertices == b->vertices && a->cells == b->cells;
}

Transfer* transfer_create(Ctx* ctx, Level* fine, Level* coarse, const nnmg_transfer_opts& o) {
    if (!fine || !coarse) fail(NNMG_ERR_INVALID_ARG, "level is NULL");
    if (fine->dim != coarse->dim) fail(NNMG_ERR_INVALID_ARG, "levels of different dimension");
    if (fine->ncomp != coarse->ncomp) fail(NNMG_ERR_INVALID_ARG, "levels with different numbers of components");
    if (fine->ctx->device != ctx->device || coarse->ctx->device != ctx->device)
        fail(NNMG_ERR_INVALID_ARG, "levels on another device");
    if (!(o.bbox_expand >= 0.0) || !(o.inside_tol >= 0.0) || !(o.newton_tol > 0.0) || o.newton_max_it < 1)
        fail(NNMG_ERR_INVALID_ARG, "transfer options");
    const int dim = fine->dim, nv = 1 << dim;
    NNMG_HIP(hipSetDevice(ctx->device));

    auto* T = new nnmg_transfer();
    try {
        T->ctx = ctx;
        T->fine = fine;
        T->coarse = coarse;
        level_retain(fine);
        level_retain(coarse);
        if (o.nested_p && coarse->degree < fine->degree && same_mesh(fine, coarse)) {
            setup_nested_p(T, ctx);
            return T;
        }

        // query points: the unconstrained fine nodes (P acts on every component alike),
        // and their bounds, which the bucket grid covers with the grown boxes
        int64_t np = 0;
        for (int64_t i = 0; i < fine->n_nodes; ++i) np += fine->constrained[(size_t)i] ? 0 : 1;
        if (np > INT32_MAX) fail(NNMG_ERR_UNSUPPORTED, "too many points");
        T->n_points = np;
        T->h_point_dof.resize((size_t)np);
        std::unique_ptr<double[]> pts = host_buffer<double>((size_t)(np * dim));
        double glo[3] = {1e300, 1e300, 1e300}, ghi[3] = {-1e300, -1e300, -1e300};
        for (int64_t i = 0, p = 0; i < fine->n_nodes; ++i) {
            if (fine->constrained[(size_t)i]) continue;
            T->h_point_dof[(size_t)p] = (int32_t)i;
            for (int a = 0; a < dim; ++a) {
                const double x = fine->support[(size_t)(i * dim + a)];
                pts[(size_t)(p * dim + a)] = x;
                glo[a] = std::min(glo[a], x);
                ghi[a] = std::max(ghi[a], x);
            }
            ++p;
        }

        // grown boxes of the coarse cells
        const int64_t C = coarse->n_cells;
        std::vector<double> boxes((size_t)(C * 2 * dim));
        std::vector<double> ext[3];
        for (int a = 0; a < dim; ++a) ext[a].resize((size_t)C);
        for (int64_t c = 0; c < C; ++c) {
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (int b = 0; b < nv; ++b) {
                const int32_t v = coarse->cells[(size_t)(c * nv + b)];
                for (int a = 0; a < dim; ++a) {
                    const double x = coarse->vertices[(size_t)(v * dim + a)];
                    lo[a] = std::min(lo[a], x);
                    hi[a] = std::max(hi[a], x);
                }
            }
            double d2 = 0.0;
            for (int a = 0; a < dim; ++a) d2 = d2 + (hi[a] - lo[a]) * (hi[a] - lo[a]);
            const double diag = std::sqrt(d2);
            for (int a = 0; a < dim; ++a) {
                const double l = lo[a] - o.bbox_expand * diag, h = hi[a] + o.bbox_expand * diag;
                boxes[(size_t)((c * 2 + 0) * dim + a)] = l;
                boxes[(size_t)((c * 2 + 1) * dim + a)] = h;
                glo[a] = std::min(glo[a], l);
                ghi[a] = std::max(ghi[a], h);
                ext[a][(size_t)c] = h - l;
            }
        }
        // bucket size: half the median grown-box extent per axis
        double step[3];
        int nb[3] = {1, 1, 1};
        for (int a = 0; a < dim; ++a) {
            std::vector<double> e = ext[a];
            std::nth_element(e.begin(), e.begin() + e.size() / 2, e.end());
            const double size = std::max(0.5 * e[e.size() / 2], 1e-300);
            const double span = std::max(ghi[a] - glo[a], 1e-300);
            nb[a] = (int)std::min(1024.0, std::max(1.0, std::ceil(span / size)));
            step[a] = span / nb[a];
        }
        int64_t nbt = 1;
        for (int a = 0; a < dim; ++a) nbt *= nb[a];
        auto bidx = [&](double x, int a) {
            int k = (int)std::floor((x - glo[a]) / step[a]);
            return std::min(std::max(k, 0), nb[a] - 1);
        };
        std::vector<int32_t> boff((size_t)(nbt + 1), 0);
        std::vector<int> lo_b((size_t)(C * dim)), hi_b((size_t)(C * dim));
        for (int64_t c = 0; c < C; ++c)
            for (int a = 0; a < dim; ++a) {
                lo_b[(size_t)(c * dim + a)] = bidx(boxes[(size_t)((c * 2 + 0) * dim + a)], a);
                hi_b[(size_t)(c * dim + a)] = bidx(boxes[(size_t)((c * 2 + 1) * dim + a)], a);
            }
        auto for_buckets = [&](int64_t c, auto&& fn) {
            const int* l = &lo_b[(size_t)(c * dim)];
            const int* h = &hi_b[(size_t)(c * dim)];
            for (int z = (dim == 3 ? l[2] : 0); z <= (dim == 3 ? h[2] : 0); ++z)
                for (int y = l[1]; y <= h[1]; ++y)
                    for (int x = l[0]; x <= h[0]; ++x) fn((int64_t)x + (int64_t)nb[0] * (y + (int64_t)nb[1] * z));
        };
        for (int64_t c = 0; c < C; ++c) for_buckets(c, [&](int64_t b) { boff[(size_t)(b + 1)]++; });
        for (int64_t b = 0; b < nbt; ++b) boff[(size_t)(b + 1)] += boff[(size_t)b];
        std::vector<int32_t> bcells((size_t)boff[(size_t)nbt]);
        {
            std::vector<int32_t> cur(boff.begin(), boff.end() - 1);
            for (int64_t c = 0; c < C; ++c) for_buckets(c, [&](int64_t b) { bcells[(size_t)cur[(size_t)b]++] = (int32_t)c; });
        }

        // locate on the GPU
        DeviceArray<double> d_pts, d_boxes, d_xi;
        DeviceArray<int32_t> d_boff, d_bcells, d_owner, d_flags;
        d_pts.upload(ctx, pts.get(), (size_t)(np * dim));
        d_boxes.upload(ctx, boxes);
        d_boff.upload(ctx, boff);
        d_bcells.upload(ctx, bcells);
        d_owner.alloc(ctx, (size_t)np);
        d_flags.alloc(ctx, (size_t)np);
        d_xi.alloc(ctx, (size_t)(np * dim));
        launch_locate(dim, d_pts.ptr, (int)np, coarse->d_cellverts.ptr, d_boxes.ptr, d_boff.ptr, d_bcells.ptr, glo,
                      step, nb, o.inside_tol, o.newton_tol, o.newton_max_it, d_owner.ptr, d_xi.ptr, d_flags.ptr,
                      nullptr);
        NNMG_HIP(hipDeviceSynchronize());
        T->h_point_owner = d_owner.download();
        T->h_point_xi = d_xi.download();
        const std::vector<int32_t> flags = d_flags.download();
        int64_t missing = 0, projected = 0;
        for (int64_t i = 0; i < np; ++i) {
            if (T->h_point_owner[(size_t)i] < 0) ++missing;
            if (flags[(size_t)i]) ++projected;
        }
        if (missing) fail(NNMG_ERR_POINT_NOT_FOUND, std::to_string(missing) + " fine points have no candidate coarse cell");
        if (projected && !o.allow_projection)
            fail(NNMG_ERR_POINT_NOT_FOUND, std::to_string(projected) + " fine points lie outside the coarse mesh");
        T->n_projected = projected;

        // group by owner: a stable counting sort, split into contiguous ranges of
        // points, one per thread; range t places its points of cell c after those
        // of cell c in the ranges before it, so the result is that of one pass
        std::vector<int32_t> off((size_t)(C + 1), 0);
        std::unique_ptr<int32_t[]> fidx = host_buffer<int32_t>((size_t)np);
        std::unique_ptr<double[]> xi64 = host_buffer<double>((size_t)(np * dim));
        std::unique_ptr<float[]> xi32 = host_buffer<float>((size_t)(np * dim));
        {
            const int64_t per = 1 << 20;
            const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(sort_threads(), (np + per - 1) / per));
            const int32_t* own = T->h_point_owner.data();
            auto range = [&](int t, int64_t& i0, int64_t& i1) {
                i0 = np * t / nt;
                i1 = np * (t + 1) / nt;
            };
            std::vector<std::vector<int32_t>> cur((size_t)nt, std::vector<int32_t>((size_t)C, 0));
            run_threads(nt, [&](int t) {
                int64_t i0, i1;
                range(t, i0, i1);
                int32_t* cnt = cur[(size_t)t].data();
                for (int64_t i = i0; i < i1; ++i) cnt[own[i]]++;
            });
            // cur[t][c] becomes the first position of range t's points of cell c
            int32_t pos = 0;
            for (int64_t c = 0; c < C; ++c) {
                off[(size_t)c] = pos;
                for (int t = 0; t < nt; ++t) {
                    const int32_t k = cur[(size_t)t][(size_t)c];
                    cur[(size_t)t][(size_t)c] = pos;
                    pos += k;
                }
            }
            off[(size_t)C] = pos;
            run_threads(nt, [&](int t) {
                int64_t i0, i1;
                range(t, i0, i1);
                int32_t* next = cur[(size_t)t].data();
                for (int64_t i = i0; i < i1; ++i) {
                    const int32_t p = next[own[i]]++;
                    fidx[(size_t)p] = T->h_point_dof[(size_t)i];
                    for (int a = 0; a < dim; ++a) {
                        const double x = T->h_point_xi[(size_t)(i * dim + a)];
                        xi64[(size_t)(a * np + p)] = x;
                        xi32[(size_t)(a * np + p)] = (float)x;
                    }
                }
            });
        }
        // owner of sorted point p: the last cell whose run starts at or before p
        auto owner_of = [&](int64_t p) {
            return (int32_t)(std::upper_bound(off.begin(), off.begin() + C, (int32_t)p) - off.begin() - 1);
        };
        // owner cells of the first and last point of every block of kPointBlock points
        const int64_t nblk = (np + kPointBlock - 1) / kPointBlock;
        std::vector<int32_t> bc((size_t)(2 * nblk));
        for (int64_t b = 0; b < nblk; ++b) {
            bc[(size_t)(2 * b)] = owner_of(b * kPointBlock);
            bc[(size_t)(2 * b + 1)] = owner_of(std::min<int64_t>(np, (b + 1) * kPointBlock) - 1);
        }
        T->d_blk_cells.upload(ctx, bc);
        build_restriction_slots(T, ctx);
        T->d_off.upload(ctx, off);
        T->d_fine.upload(ctx, fidx.get(), (size_t)np);
        T->d_xi64.upload(ctx, xi64.get(), (size_t)(np * dim));
        T->d_xi32.upload(ctx, xi32.get(), (size_t)(np * dim));
        // lanes per coarse cell and component of the restriction: about
        // avg / NNMG_RESTRICT_PTS_PER_LANE, 4..64 (the kernel multiplies by the
        // lanes that share a point)
        const double avg = C ? (double)np / (double)C : 0.0;
        const double per_lane = coarse->n <= 3 ? NNMG_RESTRICT_PTS_PER_LANE : 2 * NNMG_RESTRICT_PTS_PER_LANE;
        int team = 4;
        while (team < 64 && per_lane * (2 * team) <= avg) team *= 2;
        // small coarse levels: more lanes per cell, so that the launch still
        // has enough wavefronts in flight to hide the memory latency (about
        // 1k; larger teams cost more in the cross-lane reduction)
        const double teams = (double)C * coarse->ncomp;
        while (team < 64 && teams * team < 65536.0 && 2 * team <= avg) team *= 2;
        T->team = team;
    } catch (...) {
        level_release(T->fine);
        level_release(T->coarse);
        delete T;
        throw;
    }
    return T;
}

void transfer_retain(Transfer* t) { t->refs.fetch_add(1); }

void transfer_reserve_rhs(Transfer& t, int nr) {
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides must be in 1..8");
    if (nr <= t.rbuf_rhs) return;
    NNMG_HIP(hipSetDevice(t.ctx->device));
    NNMG_HIP(hipDeviceSynchronize());  // earlier launches may still use the buffer
    t.d_rbuf.alloc(t.ctx, std::max<size_t>(t.n_rslots * t.coarse->ncomp * (size_t)nr, 1));
    t.rbuf_rhs = nr;
}

void transfer_release(Transfer* t) {
    if (!t || t->refs.fetch_sub(1) != 1) return;
    Level* f = t->fine;
    Level* c = t->coarse;
    delete static_cast<nnmg_transfer*>(t);
    level_release(f);
    level_release(c);
}

}  // namespace nnmg
