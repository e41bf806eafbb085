// Autotuner: times the variants of a level's operator application and of a
// transfer's restriction on the GPU at hand and keeps the fastest.
//
// Level variants (the operator as the V-cycle uses it, product plus the
// residual that consumes it):
//   0  geometry rebuilt from the trilinear map, contributions in slots + gather
//   1  geometry rebuilt from the trilinear map, float atomics into the output
//   2  stored merged metric per Gauss point,    contributions in slots + gather
//   3  stored merged metric per Gauss point,    float atomics into the output
//   4  as 0, with the entity-compressed indices (one record per cell)
//   5  as 2, with the entity-compressed indices
//   6..11  as 0..5 with the transposed sweeps: the lanes of a cell swap the
//          line they own through LDS between the contraction stages, so
//          every contraction runs in registers (7 and 9, atomics, do not exist)
// Variants 4, 5, 10 and 11 exist for 3D Laplace levels of degree >= 3 (where
// the records were built).  The elasticity operator has variant 0 only.
// Each variant is timed with one and with two layout blocks of cpb cells per
// workgroup (Laplace slot variants), in two passes over the candidates (the
// second in reverse order, the two times averaged), and the fastest pair is
// kept.  On a small level (a grid of few wavefronts) the variant kept is then
// timed with four right-hand sides as one grid row per right-hand side
// against every block looping over them.  Transfer variants: the lanes per
// coarse cell of the restriction, 4 << v for v = 0..4.
//
// Each precision has its own variant: the float64 and float32 kernels of one
// level are timed and chosen separately.
//
// Every choice changes only the order in which floating-point sums are formed
// (atomics: an order that varies from run to run), never what is summed.  The
// tuner times the deterministic variants only (0, 2, 4, 5, 6, 8, 10, 11), so that a tuned
// hierarchy stays bitwise reproducible; the atomic ones are an explicit opt-in
// through level_set_variant.
#include <algorithm>
#include <functional>
#include <utility>
#include <vector>

#include "../internal.hpp"

namespace nnmg {

namespace {

double time_ms(const std::function<void(hipStream_t)>& fn, int reps, hipStream_t s) {
    for (int i = 0; i < 2; ++i) fn(s);
    hipEvent_t a, b;
    NNMG_HIP(hipEventCreate(&a));
    NNMG_HIP(hipEventCreate(&b));
    NNMG_HIP(hipEventRecord(a, s));
    for (int i = 0; i < reps; ++i) fn(s);
    NNMG_HIP(hipEventRecord(b, s));
    NNMG_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    NNMG_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return (double)ms / reps;
}

// a scratch vector of n values with entries in [-1, 1) in `prec`
DeviceArray<char> scratch_vector(Ctx* ctx, size_t n, int prec, uint64_t seed, hipStream_t s) {
    DeviceArray<double> v64;
    v64.alloc(ctx, std::max<size_t>(n, 1));
    launch_splitmix_vector(v64.ptr, nullptr, n, seed, s);
    DeviceArray<char> out;
    out.alloc(ctx, std::max<size_t>(n, 1) * (prec == NNMG_FP64 ? 8 : 4));
    if (prec == NNMG_FP64)
        NNMG_HIP(hipMemcpyAsync(out.ptr, v64.ptr, n * 8, hipMemcpyDeviceToDevice, s));
    else
        launch_cast_64_to_32(v64.ptr, (float*)out.ptr, n, s);
    NNMG_HIP(hipStreamSynchronize(s));
    return out;
}

void ensure_metric(Level& L) {
    if (L.d_metric64.ptr) return;
    const int M = L.dim * (L.dim + 1) / 2;
    const size_t mlen = (size_t)(L.nblocks * M * L.n * L.wg);
    L.d_metric64.alloc(L.ctx, mlen);
    L.d_metric32.alloc(L.ctx, mlen);
    NNMG_HIP(hipMemset(L.d_metric64.ptr, 0, L.d_metric64.bytes()));
    NNMG_HIP(hipMemset(L.d_metric32.ptr, 0, L.d_metric32.bytes()));
    DeviceArray<int> bad;
    bad.alloc(L.ctx, 1);
    NNMG_HIP(hipMemset(bad.ptr, 0, sizeof(int)));
    launch_geometry(L, bad.ptr, nullptr);
    NNMG_HIP(hipDeviceSynchronize());
}

bool has_entity_variants(const Level& L) { return L.d_ent_rec.ptr != nullptr; }

Level::OpVariant variant_state(int v) {
    const int b = v % 6;
    Level::OpVariant s;
    s.geometry_mode = (b == 2 || b == 3 || b == 5) ? 0 : 1;
    s.atomic = b == 1 || b == 3;
    s.index_layout = b >= 4 ? 1 : 0;
    s.sweep = v / 6;
    return s;
}

bool atomic_variant(int v) { return v % 6 == 1 || v % 6 == 3; }

// levels whose operator grid has fewer wavefronts than this (a few per SIMD)
// also time the several-right-hand-side launch with one grid row per
// right-hand side
constexpr int64_t kSmallLevelWaves = 16384;

// prec: NNMG_FP64, NNMG_FP32, or -1 for both
void apply_variant(Level& L, int prec, int v) {
    if (L.op != NNMG_OP_LAPLACE && v != 0) fail(NNMG_ERR_UNSUPPORTED, "the elasticity operator has variant 0 only");
    if (v < 0 || v > 11) fail(NNMG_ERR_INVALID_ARG, "operator variant must be in 0..11");
    if (v == 7 || v == 9) fail(NNMG_ERR_INVALID_ARG, "the atomic variants have no transposed-sweep form");
    if (v % 6 >= 4 && !has_entity_variants(L))
        fail(NNMG_ERR_UNSUPPORTED, "variants 4, 5, 10, 11 (entity-compressed indices) need a 3D Laplace level of degree >= 3");
    NNMG_HIP(hipDeviceSynchronize());  // launches of the previous variant may be in flight
    const Level::OpVariant st = variant_state(v);
    if (st.geometry_mode == 0) ensure_metric(L);
    for (int p = 0; p < 2; ++p)
        if (prec < 0 || prec == p) {
            // separate choices (level_tune): kept across variant changes
            const int split = L.var[p].rhs_split, group = L.var[p].group;
            L.var[p] = st;
            L.var[p].rhs_split = split;
            L.var[p].group = group;
        }
    if (L.var[0].geometry_mode == 1 && L.var[1].geometry_mode == 1) {
        // no precision reads the stored metric any more
        L.d_metric64.reset();
        L.d_metric32.reset();
    }
    ++L.config_version;
}

}  // namespace

int level_variant(const Level& L, int prec) {
    const Level::OpVariant& s = L.var[prec];
    const int b = s.index_layout == 1 ? (s.geometry_mode == 0 ? 5 : 4)
                                      : (s.geometry_mode == 0 ? 2 : 0) + (s.atomic ? 1 : 0);
    return b + 6 * s.sweep;
}

void level_set_variant(Level& L, int prec, int v) {
    NNMG_HIP(hipSetDevice(L.ctx->device));
    apply_variant(L, prec, v);
}

void level_set_rhs_split(Level& L, int prec, int split) {
    if (split != 0 && split != 1) fail(NNMG_ERR_INVALID_ARG, "rhs split must be 0 or 1");
    NNMG_HIP(hipSetDevice(L.ctx->device));
    NNMG_HIP(hipDeviceSynchronize());
    for (int p = 0; p < 2; ++p)
        if (prec < 0 || prec == p) L.var[p].rhs_split = split;
    ++L.config_version;
}

void level_set_cells_per_block(Level& L, int prec, int cells) {
    int group = 0;
    if (cells == L.cpb) group = 1;
    else if (cells == 2 * L.cpb) group = 2;
    else fail(NNMG_ERR_INVALID_ARG, "cells per block must be " + std::to_string(L.cpb) + " or " +
                                        std::to_string(2 * L.cpb) + " on this level");
    if (group == 2 && L.op != NNMG_OP_LAPLACE)
        fail(NNMG_ERR_UNSUPPORTED, "the elasticity operator runs one layout block per workgroup");
    NNMG_HIP(hipSetDevice(L.ctx->device));
    NNMG_HIP(hipDeviceSynchronize());
    for (int p = 0; p < 2; ++p)
        if (prec < 0 || prec == p) L.var[p].group = group;
    ++L.config_version;
}

int level_cells_per_block(const Level& L, int prec) { return L.var[prec].atomic ? L.cpb : L.var[prec].group * L.cpb; }

void level_tune(Level& L, int prec, int reps, nnmg_tune_result* res) {
    if (reps < 1) fail(NNMG_ERR_INVALID_ARG, "reps must be positive");
    NNMG_HIP(hipSetDevice(L.ctx->device));
    const size_t n = (size_t)L.n_dofs;
    const int nvar = L.op != NNMG_OP_LAPLACE ? 1 : 12;
    hipStream_t s;
    NNMG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
        DeviceArray<char> x = scratch_vector(L.ctx, n, prec, 0x7E57ull, s);
        DeviceArray<char> f = scratch_vector(L.ctx, n, prec, 0x7E58ull, s);
        DeviceArray<char> r, ax;
        const size_t bytes = std::max<size_t>(n, 1) * (prec == NNMG_FP64 ? 8 : 4);
        r.alloc(L.ctx, bytes / sizeof(char));
        ax.alloc(L.ctx, bytes / sizeof(char));
        NNMG_HIP(hipMemset(ax.ptr, 0, bytes));
        level_reserve_rhs(L, 1);
        res->n_variants = nvar;
        for (double& t : res->ms) t = -1.0;
        // every variant with one and with two layout blocks per workgroup (the
        // Laplace slot variants; same sums either way), timed in two passes,
        // the second in reverse order, and averaged, so that a drift of the
        // clocks over the tuning does not favour the candidates timed first:
        // ms[v] is the faster of the variant's two sizes, ms_cpb the pair of
        // the variant kept
        const bool grouped = L.op == NNMG_OP_LAPLACE && L.nblocks > 0;
        std::vector<std::pair<int, int>> cand;  // (variant, layout blocks per workgroup)
        for (int v = 0; v < nvar; ++v) {
            if (atomic_variant(v)) continue;  // float atomics: not reproducible, never picked by the tuner
            if (v % 6 >= 4 && !has_entity_variants(L)) continue;
            for (int g = 1; g <= (grouped ? 2 : 1); ++g) cand.emplace_back(v, g);
        }
        std::vector<double> t(cand.size(), 0.0);
        for (int pass = 0; pass < 2; ++pass)
            for (size_t k = 0; k < cand.size(); ++k) {
                const size_t c = pass == 0 ? k : cand.size() - 1 - k;
                apply_variant(L, prec, cand[c].first);
                L.var[prec].group = cand[c].second;
                t[c] += 0.5 * time_ms(
                    [&](hipStream_t st) {
                        launch_vmult_contrib(L, prec, x.ptr, L.d_contrib.ptr, st);
                        launch_residual_gather(L, prec, L.d_contrib.ptr, f.ptr, r.ptr, st);
                    },
                    reps, s);
            }
        double ms_g[16][2];
        for (auto& m : ms_g) m[0] = m[1] = -1.0;
        double best_ms = -1.0;
        int best = 0, best_g = 1;
        for (size_t c = 0; c < cand.size(); ++c) {
            const int v = cand[c].first, g = cand[c].second;
            ms_g[v][g - 1] = t[c];
            if (res->ms[v] < 0 || t[c] < res->ms[v]) res->ms[v] = t[c];
            if (best_ms < 0 || t[c] < best_ms) {
                best_ms = t[c];
                best = v;
                best_g = g;
            }
        }
        apply_variant(L, prec, best);
        L.var[prec].group = best_g;
        ++L.config_version;
        res->chosen = best;
        res->cells_per_block = level_cells_per_block(L, prec);
        res->ms_cpb[0] = ms_g[best][0];
        res->ms_cpb[1] = grouped ? ms_g[best][1] : -1.0;
        // several right-hand sides on a small level (a grid of few wavefronts):
        // one grid row per right-hand side, or every block looping over them
        res->rhs_split = L.var[prec].rhs_split;
        res->ms_rhs[0] = res->ms_rhs[1] = -1.0;
        const int64_t waves = L.nblocks * (L.wg / 64);
        if (waves < kSmallLevelWaves) {
            constexpr int nr = 4;
            level_reserve_rhs(L, nr);
            DeviceArray<char> x4 = scratch_vector(L.ctx, n * nr, prec, 0x7E5Aull, s);
            DeviceArray<char> f4 = scratch_vector(L.ctx, n * nr, prec, 0x7E5Bull, s);
            DeviceArray<char> r4;
            r4.alloc(L.ctx, std::max<size_t>(n * nr, 1) * (prec == NNMG_FP64 ? 8 : 4));
            for (int split = 0; split < 2; ++split) {
                L.var[prec].rhs_split = split;
                res->ms_rhs[split] = time_ms(
                    [&](hipStream_t st) {
                        launch_vmult_contrib(L, prec, x4.ptr, L.d_contrib.ptr, st, nr);
                        launch_residual_gather(L, prec, L.d_contrib.ptr, f4.ptr, r4.ptr, st, nr);
                    },
                    reps, s);
            }
            L.var[prec].rhs_split = res->ms_rhs[1] < res->ms_rhs[0] ? 1 : 0;
            res->rhs_split = L.var[prec].rhs_split;
            ++L.config_version;
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        throw;
    }
    NNMG_HIP(hipStreamSynchronize(s));
    NNMG_HIP(hipStreamDestroy(s));
}

void transfer_set_team(Transfer& T, int team) {
    if (team != 4 && team != 8 && team != 16 && team != 32 && team != 64)
        fail(NNMG_ERR_INVALID_ARG, "restriction team must be 4, 8, 16, 32 or 64 lanes");
    NNMG_HIP(hipSetDevice(T.ctx->device));
    NNMG_HIP(hipDeviceSynchronize());
    T.team = team;
    ++T.config_version;
}

void transfer_tune(Transfer& T, int prec, int reps, nnmg_tune_result* res) {
    if (reps < 1) fail(NNMG_ERR_INVALID_ARG, "reps must be positive");
    NNMG_HIP(hipSetDevice(T.ctx->device));
    hipStream_t s;
    NNMG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
        DeviceArray<char> fine = scratch_vector(T.ctx, (size_t)T.fine->n_dofs, prec, 0x7E59ull, s);
        DeviceArray<char> coarse;
        coarse.alloc(T.ctx, std::max<size_t>((size_t)T.coarse->n_dofs, 1) * (prec == NNMG_FP64 ? 8 : 4));
        NNMG_HIP(hipMemset(coarse.ptr, 0, coarse.bytes()));
        // 3D cells of degree 3 and 4 take one wavefront per cell and value
        // whatever the team: one timing
        const bool teamless = !T.nested_p && T.coarse->dim == 3 && T.coarse->n >= 4;
        res->n_variants = teamless ? 1 : 5;
        for (double& t : res->ms) t = -1.0;
        int best = 0;
        for (int v = 0; v < res->n_variants; ++v) {
            transfer_set_team(T, 4 << v);
            res->ms[v] = time_ms([&](hipStream_t st) { launch_restrict(T, prec, fine.ptr, coarse.ptr, false, st); },
                                 reps, s);
            if (res->ms[v] < res->ms[best]) best = v;
        }
        transfer_set_team(T, 4 << best);
        res->chosen = best;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        throw;
    }
    NNMG_HIP(hipStreamSynchronize(s));
    NNMG_HIP(hipStreamDestroy(s));
}

}  // namespace nnmg
