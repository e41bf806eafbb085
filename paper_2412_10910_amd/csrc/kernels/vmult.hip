// Matrix-free operator apply by sum factorisation (paper §3.2: tensor-product
// evaluation; the operator A_l of §2, eq. linear_system, for the Poisson
// bilinear form with the (k+1)^d Gauss rule of §4).
//
// Work decomposition (gfx950).  A team of L = N^(d-1) lanes (N = k+1) handles
// one cell; each lane owns one x-line of N nodal values / Gauss points, held
// in registers.  Contractions along x run in registers, those along y and z
// (3D) or y (2D) go through LDS, with per-cell tiles of N^d values.  A block
// of WG lanes holds CPB = WG / L cells; WG is 64, or 128 for 3D Q4 so that
// five 25-lane teams fill two wavefronts.  Every per-cell array is stored in
// the block layout of the lanes that read it, so each load is coalesced:
//
//   dofmap_blk[(blk * N + i) * WG + lane]          node i of the lane's x-line
//
// Forward: nodal values -> Gauss points (S in each direction), reference
// gradient by collocation (D on the Gauss points; along z in 3D / y in 2D the
// derivative DS = D S is fused with the interpolation).  At each Gauss point
// the flux is G grad_ref(u), G = w det(J) J^{-1} J^{-T} the merged metric.
// Backward: the transposes.  The cell results are not added with float
// atomics: each (cell, node) contribution is written to its own slot of a
// buffer sorted by DoF,
//
//   contrib[pos_blk[(blk * N + i) * WG + lane]],
//
// and the consumers (gather, Chebyshev step, residual, CG product) sum every
// DoF's contiguous run of slots in a fixed order: one launch, no atomics, and
// a deterministic operator.  (A float-atomic variant is kept for comparison.)
//
// Two geometry sources:
//  * kStoredMetric: G read per Gauss point from
//      metric_blk[((blk * M + m) * N + i) * WG + lane],  M = d(d+1)/2
//    (components 00,11,22,01,02,12 in 3D; 00,11,01 in 2D);
//  * kTrilinear: the Q1 map x(xi) = a + b xi + c eta + d zeta + e xi eta
//    + f xi zeta + g eta zeta + h xi eta zeta kept as its 7 (2D: 3) vector
//    coefficients per cell, coef_blk[(blk * NC + m) * CPB + cell_in_block],
//    and J rebuilt at every Gauss point.  The rows of det(J) J^{-1} are the
//    cross products of the columns of J, so G grad = (w / det J) R^T (R grad)
//    with R the matrix of those rows.  This moves 21 words per cell instead
//    of 6 per Gauss point, for about 60 flops per Gauss point.
#include <cmath>
#include <cstdlib>
#include <string>

#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

template <int N, class T>
struct OpTables {
    T S[N][N];   // S[q][a]  = phi_a(g_q)
    T DS[N][N];  // DS[q][a] = phi_a'(g_q)
    T D[N][N];   // D[q][p]  = psi_p'(g_q)
    T g[N];      // Gauss points on [0,1]
    T w[N];      // Gauss weights
};

__device__ __forceinline__ double recip(double x) {
    // hardware estimate refined by two Newton steps
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

__device__ __forceinline__ float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// out[i] = sum_a M[i][a] in[a]  (or M^T)
template <int N, class T, bool TRANS>
__device__ __forceinline__ void line_apply(const T (&M)[N][N], const T* in, T* out) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = (TRANS ? M[0][i] : M[i][0]) * in[0];
#pragma unroll
        for (int a = 1; a < N; ++a) s += (TRANS ? M[a][i] : M[i][a]) * in[a];
        out[i] = s;
    }
}

// Even-odd form of an N x N matrix M with M[N-1-i][N-1-j] = sig M[i][j]
// (sig = +1: the values of the nodal basis at the Gauss points, S; sig = -1:
// the derivative matrices DS and D, as the node and point sets are symmetric
// about 1/2).  With e_j = u_j + u_{N-1-j}, o_j = u_j - u_{N-1-j} (j < N/2) and
// the middle value m = u_{N/2} (odd N), row i < N/2 and its mirror are
//   (M u)_i = E_i + O_i,   (M u)_{N-1-i} = sig (E_i - O_i),
//   E_i = sum_j P_ij e_j + c_i m,   O_i = sum_j Q_ij o_j,
//   P_ij = (M_ij + M_i,N-1-j) / 2,  Q_ij = (M_ij - M_i,N-1-j) / 2,  c_i = M_i,N/2,
// and the middle row (odd N) is E (sig = +1) or O (sig = -1) alone: at N = 5
// 21 (sig = +1) or 20 (sig = -1) operations instead of 25.  Below N = 5 the
// split costs as much as it saves, and the plain product is used.
template <int N, class T>
struct EOMat {
    T P[(N + 1) / 2][N / 2];
    T Q[(N + 1) / 2][N / 2];
    T c[(N + 1) / 2];
};

template <int N, class T>
struct OpEO {  // even-odd forms of S, DS, D and their transposes (N >= 5)
    EOMat<N, T> S, St, DS, DSt, D, Dt;
};

template <int N, class T, int SIG>
__device__ __forceinline__ void line_apply_eo(const EOMat<N, T>& M, const T* in, T* out) {
    constexpr int H = N / 2;
    T e[H], o[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        e[j] = in[j] + in[N - 1 - j];
        o[j] = in[j] - in[N - 1 - j];
    }
#pragma unroll
    for (int i = 0; i < H; ++i) {
        T E = M.P[i][0] * e[0];
#pragma unroll
        for (int j = 1; j < H; ++j) E += M.P[i][j] * e[j];
        if constexpr (N % 2 == 1) E += M.c[i] * in[H];
        T O = M.Q[i][0] * o[0];
#pragma unroll
        for (int j = 1; j < H; ++j) O += M.Q[i][j] * o[j];
        out[i] = E + O;
        out[N - 1 - i] = SIG > 0 ? E - O : O - E;
    }
    if constexpr (N % 2 == 1) {
        if constexpr (SIG > 0) {
            T E = M.P[H][0] * e[0];
#pragma unroll
            for (int j = 1; j < H; ++j) E += M.P[H][j] * e[j];
            out[H] = E + M.c[H] * in[H];
        } else {
            T O = M.Q[H][0] * o[0];
#pragma unroll
            for (int j = 1; j < H; ++j) O += M.Q[H][j] * o[j];
            out[H] = O;
        }
    }
}

// the 1D contractions of the Laplace kernel: the even-odd form from N = 5 on
template <int N, class T, bool TRANS, int SIG>
__device__ __forceinline__ void line_apply_sym(const T (&M)[N][N], const EOMat<N, T>& E, const T* in, T* out) {
    if constexpr (N >= 5)
        line_apply_eo<N, T, SIG>(E, in, out);
    else
        line_apply<N, T, TRANS>(M, in, out);
}

template <int DIM, int N>
struct OpShape {
    static constexpr int L = DIM == 3 ? N * N : N;   // lanes per cell
    static constexpr int WG = (DIM == 3 && N == 5) ? 128 : 64;
    static constexpr int CPB = WG / L;               // cells per block
    static constexpr int TILE = DIM == 3 ? N * N * N : N * N;
};

constexpr int kStoredMetric = 0;
constexpr int kTrilinear = 1;
constexpr int kSlots = 0;
constexpr int kAtomic = 1;
constexpr int kIdxNodes = 0;   // per-node DoF indices and slots, dofmap_blk / pos_blk
constexpr int kIdxEntity = 1;  // one record of entity bases and slot bases per cell

#ifndef NNMG_VMULT_MINWAVES
#define NNMG_VMULT_MINWAVES 1
#endif
// nr right-hand sides (vectors interleaved as [DoF][nr]) are applied one
// after the other by each block: the indices, slots, map coefficients and
// tables are loaded once per cell for all of them.  The contributions of
// right-hand side r go to their own plane, dst + r * plane, so that each
// pass stores exactly what a single-vector call stores (interleaved stores
// would write partial cache lines); the atomic variant adds into the
// interleaved output vector.  NRT = 1 fixes nr = 1 at
// compile time (the loop disappears); NRT = 0 takes nr_in.
//
// Index layouts (IDX).  kIdxNodes reads each lane's N DoF indices and N slots
// from dofmap_blk / slots.  kIdxEntity reads one record per cell, in the block
// layout rec[(blk * kEntWords + word) * CPB + cell]: the first DoF D_e and the
// first slot (plus the cell's rank) SR_e of each of the cell's 27 mesh
// entities, 8 bits of writer count and orientation per entity, and the x-face
// merge flags.  The block's records go through LDS, and each lane derives its
// nodes' DoFs D_e + m and slots SR_e + m c_e from the canonical index m of the
// node on its entity: a record of 62 words per cell instead of 2 q words
// (q = 64 at Q3, 125 at Q4).
// waves per SIMD the register allocation must allow: 4 for the float64 Q3
// single-vector kernels with entity records or transposed sweeps (they would
// otherwise take 132-150 VGPRs, 3 waves; at 128 they spill a few)
// The float64 degree-4 transposed kernel keeps its per-point state in LDS:
// three tiles instead of five (the z stages wait for every lane's reads before
// overwriting their inputs), the z-stage outputs computed and stored one at a
// time, and the geometry step run one point at a time on the lane's own tile
// positions.  Holding the whole line's gradient and geometry in registers took
// 148 VGPRs and 26.5 KB of LDS per workgroup (three waves per SIMD); this form
// takes 83 VGPRs and 16.5 KB (four).  At lower degrees and in float32 the
// register form is as fast or faster.
template <int N, class T, int SW>
constexpr bool vmult_lds_geometry() {
    return SW == 1 && N == 5 && sizeof(T) == 8;
}

template <int N, class T, int NRT, int IDX, int SW, int G>
constexpr int vmult_min_waves() {
    // two layout blocks per workgroup double the LDS of a workgroup: three
    // waves per SIMD is what the LDS then holds
    return ((IDX == 1 || SW == 1) && N == 4 && sizeof(T) == 8 && NRT == 1) ? (G == 1 ? 4 : 3) : NNMG_VMULT_MINWAVES;
}

template <int DIM, int N, class T, int GEO, int SCATTER, int NRT, int IDX = kIdxNodes, int SW = 0, int G = 1>
__global__ __launch_bounds__((OpShape<DIM, N>::WG * G), (vmult_min_waves<N, T, NRT, IDX, SW, G>())) void vmult_kernel(const int32_t* __restrict__ dmap,
                                                                    const T* __restrict__ geo,
                                                                    const T* __restrict__ src,
                                                                    const int32_t* __restrict__ slots,
                                                                    T* __restrict__ dst, OpTables<N, T> tb,
                                                                    OpEO<N, T> eo, int nr_in, int64_t plane,
                                                                    int64_t nblk) {
    const int nr = NRT > 0 ? NRT : nr_in;
    // right-hand sides of this block: all of them one after the other, or,
    // when the grid has one row per right-hand side (small meshes, where a
    // loop would leave the device idle), the one of its row
    const int rhs0 = NRT == 0 ? (int)blockIdx.y : 0;
    const int rhs_end = (NRT == 0 && gridDim.y > 1) ? rhs0 + 1 : nr;
    using Sh = OpShape<DIM, N>;
    constexpr int L = Sh::L, WG = Sh::WG, CPB = Sh::CPB, TILE = Sh::TILE;
    constexpr int M = DIM * (DIM + 1) / 2;
    constexpr int NC = DIM == 3 ? 21 : 6;
    // G layout blocks of WG lanes per workgroup (G CPB cells): the lanes of
    // layout block `sub` own LDS regions of their own and synchronize among
    // themselves only.  In the last workgroup of an odd block count, the
    // block past the end repeats the loads of the last block and stores
    // nothing.
    static_assert(G == 1 || SCATTER == kSlots, "several layout blocks per workgroup: contribution slots only");
    constexpr bool kSeq = DIM == 3 && vmult_lds_geometry<N, T, SW>();
    __shared__ T lds[SW == 1 && !kSeq ? 5 : 3][G * CPB][TILE];
    const int sub = G == 1 ? 0 : (int)threadIdx.x / WG;
    const int64_t bg = G == 1 ? xcd_remap(blockIdx.x, gridDim.x) : xcd_remap(blockIdx.x, gridDim.x) * G + sub;
    const bool bok = G == 1 || bg < nblk;
    const int64_t b = bok ? bg : nblk - 1;
    const int lane = (int)threadIdx.x - sub * WG;
    const int cell = lane / L;
    const int line = lane - cell * L;
    const bool act = cell < CPB && bok;
    const int cbl = act ? cell : 0;  // cell within the layout block
    const int cb = sub * CPB + cbl;  // cell within the workgroup (LDS)
    // 3D: line = j + N t (y index j, z index t); 2D: line = t (y index)
    const int j = DIM == 3 ? line % N : 0;
    const int t = DIM == 3 ? line / N : line;
    const int row = line * N;  // offset of this lane's x-line in a cell tile

    // Prologue, in issue order: the DoF indices and output slots of the
    // lane's line, the cell's map coefficients and the 1D tables (both bound
    // for LDS), then the source gathers, which wait only for the indices; the
    // LDS stores come last so that no load waits behind them.
    static_assert(IDX == kIdxNodes || (DIM == 3 && SCATTER == kSlots && N >= 3),
                  "entity records: 3D, contribution slots");
    int32_t idx[N], slot[N];
    T u[N], v[N];
    constexpr int EW = kEntWords;
    constexpr int RE = IDX == kIdxEntity ? (EW * CPB + WG - 1) / WG : 1;  // record words per lane
    int32_t rv[RE];
    if constexpr (IDX == kIdxEntity) {
        const int32_t* gr = dmap + b * (EW * CPB);
#pragma unroll
        for (int r = 0; r < RE; ++r) rv[r] = lane + r * WG < EW * CPB ? gr[lane + r * WG] : 0;
    } else {
        const int32_t* dm = dmap + b * (N * WG) + lane;
#pragma unroll
        for (int i = 0; i < N; ++i) idx[i] = dm[i * WG];
        if constexpr (SCATTER == kSlots) {
            const int32_t* ps = slots + b * (N * WG) + lane;
#pragma unroll
            for (int i = 0; i < N; ++i) slot[i] = bok ? ps[i * WG] : -1;
        }
    }
    // the cell's map coefficients: each lane turns them into the constants of
    // its line just before the geometry step, so they hold no registers
    // during the sweeps
    __shared__ T lcf[G * CPB][GEO == kTrilinear ? NC : 1];
    constexpr int R = GEO == kTrilinear ? (NC + L - 1) / L : 1;
    T cv[R];
    if constexpr (GEO == kTrilinear) {
        const T* gc = geo + b * (NC * CPB) + cbl;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m = line + r * L;
            cv[r] = (act && m < NC) ? gc[m * CPB] : T(0);
        }
    }
    // the 1D tables: rows selected by the lane's y/z index are read from LDS
    // (indexing the by-value argument with a lane-dependent index would be a
    // global load on the critical path of every sweep)
    // (the transposed sweeps contract with the by-value tables alone and stage
    // only the Gauss points and weights)
    constexpr int NT = 3 * N * N + 2 * N;
    static_assert(sizeof(OpTables<N, T>) == NT * sizeof(T), "OpTables must be a flat array of T");
    constexpr int TOFF = SW == 1 ? 3 * N * N : 0;  // first table entry staged in LDS
    constexpr int NTL = NT - TOFF;                 // entries staged
    constexpr int TE = (NTL + WG - 1) / WG;        // table entries per lane
    __shared__ T ltab[G][NTL];
    T tv[TE];
#pragma unroll
    for (int e = 0; e < TE; ++e)
        tv[e] = lane + e * WG < NTL ? reinterpret_cast<const T*>(&tb)[TOFF + lane + e * WG] : T(0);
    // Entity records (IDX == kIdxEntity): node i of the lane's line has classes
    // (cx, cy, cz) in {0: first, 1: inside, 2: last} per direction, lies on
    // entity e = cx + 3 cy + 9 cz, and has local coordinates (u, v, w) = its
    // indices - 1 along the entity's own (inside) directions in x, y, z order;
    // the record's orientation code maps them to the canonical index m.  The
    // DoFs are decoded here and, where registers allow, the slots with them
    // (they then hold N registers through the sweeps; decoding them again at
    // the store costs instructions).  The float64 degree-3 kernels, capped at
    // four waves per SIMD, decode the slots at the store.
    constexpr bool kSlotsEarly = SCATTER == kSlots && !(N == 4 && sizeof(T) == 8);
    __shared__ int32_t lrec[IDX == kIdxEntity ? G * CPB : 1][IDX == kIdxEntity ? EW : 1];
    constexpr int K1 = N - 2;  // DoFs along an edge
    const int ecy = j == 0 ? 0 : (j == N - 1 ? 2 : 1);
    const int ecz = t == 0 ? 0 : (t == N - 1 ? 2 : 1);
    const int ea = ecy == 1 ? j - 1 : (ecz == 1 ? t - 1 : 0);
    const int eb = (ecy == 1 && ecz == 1) ? t - 1 : 0;
    auto ent_node = [&](int i, int& e, int& m, int& code) {
        const int cx = i == 0 ? 0 : (i == N - 1 ? 2 : 1);
        e = cx + 3 * ecy + 9 * ecz;
        const int eu = cx == 1 ? i - 1 : ea;
        const int ev = cx == 1 ? ea : eb;
        const int ew = cx == 1 ? eb : 0;
        code = (lrec[cb][54 + (e >> 2)] >> ((e & 3) * 8)) & 0xff;
        int u1 = (code & 16) ? K1 - 1 - eu : eu;
        int v1 = (code & 32) ? K1 - 1 - ev : ev;
        if (code & 64) {
            const int tmp = u1;
            u1 = v1;
            v1 = tmp;
        }
        m = u1 + K1 * (v1 + K1 * ew);
    };
    if constexpr (IDX == kIdxEntity) {
        // the block's records to LDS, transposed to [cell][word]
#pragma unroll
        for (int r = 0; r < RE; ++r) {
            const int wd = lane + r * WG;
            if (wd < EW * CPB) lrec[sub * CPB + wd % CPB][wd / CPB] = rv[r];
        }
        block_sync<WG>();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            int e, m, code;
            ent_node(i, e, m, code);
            const int32_t D = lrec[cb][e];
            idx[i] = (act && D >= 0) ? D + m : -1;
            if constexpr (kSlotsEarly) {
                const int32_t SR = lrec[cb][27 + e];
                slot[i] = (act && SR >= 0) ? SR + m * (code & 15) : -1;
            }
        }
        if constexpr (kSlotsEarly)
            if ((lrec[cb][EW - 1] & 2) && slot[N - 1] >= 0) slot[N - 1] |= kMergeNext;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = idx[i] >= 0 ? src[(int64_t)idx[i] * nr + rhs0] : T(0);
    if constexpr (GEO == kTrilinear) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m = line + r * L;
            if (act && m < NC) lcf[cb][m] = cv[r];
        }
    }
#pragma unroll
    for (int e = 0; e < TE; ++e)
        if (lane + e * WG < NTL) ltab[sub][lane + e * WG] = tv[e];
    [[maybe_unused]] const T* lS = SW == 1 ? nullptr : ltab[sub];
    [[maybe_unused]] const T* lDS = SW == 1 ? nullptr : ltab[sub] + N * N;
    [[maybe_unused]] const T* lD = SW == 1 ? nullptr : ltab[sub] + 2 * N * N;
    const T* lg = ltab[sub] + (3 * N * N - TOFF);
    const T* lw = lg + N;

    T* A = lds[0][cb];
    T* B = lds[1][cb];
    T* Cc = lds[2][cb];

    for (int rhs = rhs0;;) {
    // the next right-hand side's values are loaded while this one is swept
    T un[N];
    if (NRT != 1 && rhs + 1 < rhs_end) {
#pragma unroll
        for (int i = 0; i < N; ++i) un[i] = idx[i] >= 0 ? src[(int64_t)idx[i] * nr + rhs + 1] : T(0);
    }
    // ---- forward --------------------------------------------------------
    T gx[N], gy[N], gz[N];  // reference gradient at the Gauss points of the line (2D: x, gz = y)
    if constexpr (SW == 1) {
        // Transposed sweeps: between the stages the lanes of a cell swap the
        // line they own through LDS (x-line (j, t) = (a, b), y-line (i, t) =
        // (a, b), z-line (i, j) = (a, b) for a = line % N, b = line / N), so
        // every contraction runs in registers with the 1D tables as constants
        // and each stage moves N values per lane through LDS, instead of N^2
        // tile and N^2 table reads per lane for a contraction across lanes.
        // The y (2D) / y and z (3D) derivatives come from the DS table (the
        // derivative of the interpolant at the Gauss points) in the stage that
        // interpolates along that direction.
        T* T0 = lds[0][cb];
        T* T1 = lds[1][cb];
        T* T2 = lds[2][cb];
        line_apply_sym<N, T, false, 1>(tb.S, eo.S, u, v);  // x: nodes -> Gauss points
        if (act) {
#pragma unroll
            for (int i = 0; i < N; ++i) T0[row + i] = v[i];
        }
        block_sync<WG>();
        if constexpr (DIM == 3) {
            T* T3 = lds[kSeq ? 1 : 3][cb];
            T* T4 = lds[kSeq ? 2 : 4][cb];
            // y-line (i, t) = (j, t) of this lane's indices
            T a[N], w[N], wy[N];
#pragma unroll
            for (int c = 0; c < N; ++c) a[c] = T0[(t * N + c) * N + j];
            line_apply_sym<N, T, false, 1>(tb.S, eo.S, a, w);
            line_apply_sym<N, T, false, -1>(tb.DS, eo.DS, a, wy);
            if (act) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    T1[(t * N + c) * N + j] = w[c];
                    T2[(t * N + c) * N + j] = wy[c];
                }
            }
            block_sync<WG>();
            // z-line (i, j) = (j, t) of this lane's indices: values, z and y derivatives
#pragma unroll
            for (int c = 0; c < N; ++c) {
                a[c] = T1[(c * N + t) * N + j];
                w[c] = T2[(c * N + t) * N + j];
            }
            if constexpr (kSeq) {
                block_sync<WG>();  // T1 and T2 are overwritten below
                T o[N];
                line_apply_sym<N, T, false, 1>(tb.S, eo.S, a, o);
                if (act) {
#pragma unroll
                    for (int c = 0; c < N; ++c) T0[(c * N + t) * N + j] = o[c];
                }
                __builtin_amdgcn_sched_barrier(0);
                line_apply_sym<N, T, false, -1>(tb.DS, eo.DS, a, o);
                if (act) {
#pragma unroll
                    for (int c = 0; c < N; ++c) T3[(c * N + t) * N + j] = o[c];
                }
                __builtin_amdgcn_sched_barrier(0);
                line_apply_sym<N, T, false, 1>(tb.S, eo.S, w, o);
                if (act) {
#pragma unroll
                    for (int c = 0; c < N; ++c) T4[(c * N + t) * N + j] = o[c];
                }
            } else {
                T zv[N], zz[N], zy[N];
                line_apply_sym<N, T, false, 1>(tb.S, eo.S, a, zv);
                line_apply_sym<N, T, false, -1>(tb.DS, eo.DS, a, zz);
                line_apply_sym<N, T, false, 1>(tb.S, eo.S, w, zy);
                if (act) {
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        T0[(c * N + t) * N + j] = zv[c];
                        T3[(c * N + t) * N + j] = zz[c];
                        T4[(c * N + t) * N + j] = zy[c];
                    }
                }
            }
            block_sync<WG>();
            if constexpr (kSeq) {
                // back on the x-line: the x derivative replaces the values in
                // place; the y and z derivatives stay in their tiles for the
                // geometry step, which works on one point at a time
                T dx[N];
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = T0[row + i];
                line_apply_sym<N, T, false, -1>(tb.D, eo.D, v, dx);
                if (act) {
#pragma unroll
                    for (int i = 0; i < N; ++i) T0[row + i] = dx[i];
                }
            } else {
                // back on the x-line
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    v[i] = T0[row + i];
                    gy[i] = T4[row + i];
                    gz[i] = T3[row + i];
                }
            }
        } else {
            // y-line i = t of this lane's index
            T a[N], w[N], wy[N];
#pragma unroll
            for (int c = 0; c < N; ++c) a[c] = T0[c * N + t];
            line_apply_sym<N, T, false, 1>(tb.S, eo.S, a, w);
            line_apply_sym<N, T, false, -1>(tb.DS, eo.DS, a, wy);
            if (act) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    T1[c * N + t] = w[c];
                    T2[c * N + t] = wy[c];
                }
            }
            block_sync<WG>();
#pragma unroll
            for (int i = 0; i < N; ++i) {
                v[i] = T1[row + i];
                gz[i] = T2[row + i];
            }
        }
        if constexpr (!kSeq) line_apply_sym<N, T, false, -1>(tb.D, eo.D, v, gx);
    } else {
        line_apply_sym<N, T, false, 1>(tb.S, eo.S, u, v);  // x: nodes -> Gauss points
        if constexpr (DIM == 3) {
            // y: interpolate
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) A[row + i] = v[i];
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = lS[j * N + 0] * A[(t * N + 0) * N + i];
    #pragma unroll
                for (int c = 1; c < N; ++c) s += lS[j * N + c] * A[(t * N + c) * N + i];
                u[i] = s;
            }
            // z: interpolate and differentiate
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) B[row + i] = u[i];
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                const T w0 = B[(0 * N + j) * N + i];
                T s0 = lS[t * N + 0] * w0, s1 = lDS[t * N + 0] * w0;
    #pragma unroll
                for (int c = 1; c < N; ++c) {
                    const T w = B[(c * N + j) * N + i];
                    s0 += lS[t * N + c] * w;
                    s1 += lDS[t * N + c] * w;
                }
                v[i] = s0;
                gz[i] = s1;
            }
        } else {
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) A[row + i] = v[i];
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                const T w0 = A[0 * N + i];
                T s0 = lS[t * N + 0] * w0, s1 = lDS[t * N + 0] * w0;
    #pragma unroll
                for (int c = 1; c < N; ++c) {
                    const T w = A[c * N + i];
                    s0 += lS[t * N + c] * w;
                    s1 += lDS[t * N + c] * w;
                }
                v[i] = s0;
                gz[i] = s1;
            }
        }
        // v: values at the Gauss points of the line; x (and y) derivatives
        line_apply_sym<N, T, false, -1>(tb.D, eo.D, v, gx);
        if constexpr (DIM == 3) {
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) Cc[row + i] = v[i];
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = lD[j * N + 0] * Cc[(t * N + 0) * N + i];
    #pragma unroll
                for (int c = 1; c < N; ++c) s += lD[j * N + c] * Cc[(t * N + c) * N + i];
                gy[i] = s;
            }
        }

    }

    // ---- geometry at the Gauss points of the line ------------------------
    if constexpr (kSeq) {
        // one point at a time, the reference gradient read from and the
        // result written back to the lane's own positions of the tiles (x in
        // tile 0, z in tile 1, y in tile 2): the same arithmetic as below with
        // the registers of one point instead of the whole line
        T* Gx = lds[0][cb];
        T* Gz = lds[1][cb];
        T* Gy = lds[2][cb];
        if constexpr (GEO == kStoredMetric) {
            const T* mt = geo + b * (M * N * WG) + lane;
#pragma unroll 1
            for (int i = 0; i < N; ++i) {
                const T g00 = mt[(0 * N + i) * WG], g11 = mt[(1 * N + i) * WG], g22 = mt[(2 * N + i) * WG];
                const T g01 = mt[(3 * N + i) * WG], g02 = mt[(4 * N + i) * WG], g12 = mt[(5 * N + i) * WG];
                const T x = Gx[row + i], y = Gy[row + i], z = Gz[row + i];
                const T ox = g00 * x + g01 * y + g02 * z;
                const T oy = g01 * x + g11 * y + g12 * z;
                const T oz = g02 * x + g12 * y + g22 * z;
                if (act) {
                    Gx[row + i] = ox;
                    Gy[row + i] = oy;
                    Gz[row + i] = oz;
                }
            }
        } else {
            T c0[3], C1[3], E1[3], D2[3], F2[3];
            const T* cf = lcf[cb];
            const T eta = lg[j], zeta = lg[t];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                c0[k] = cf[0 + k] + cf[9 + k] * eta + (cf[12 + k] + cf[18 + k] * eta) * zeta;
                C1[k] = cf[3 + k] + cf[15 + k] * zeta;
                E1[k] = cf[9 + k] + cf[18 + k] * zeta;
                D2[k] = cf[6 + k] + cf[15 + k] * eta;
                F2[k] = cf[12 + k] + cf[18 + k] * eta;
            }
            const T wl = lw[j] * lw[t];
#pragma unroll 1
            for (int i = 0; i < N; ++i) {
                const T xi = lg[i];
                T c1[3], c2[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    c1[k] = C1[k] + E1[k] * xi;
                    c2[k] = D2[k] + F2[k] * xi;
                }
                const T r0[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2],
                                 c1[0] * c2[1] - c1[1] * c2[0]};
                const T r1[3] = {c2[1] * c0[2] - c2[2] * c0[1], c2[2] * c0[0] - c2[0] * c0[2],
                                 c2[0] * c0[1] - c2[1] * c0[0]};
                const T r2[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2],
                                 c0[0] * c1[1] - c0[1] * c1[0]};
                const T det = c0[0] * r0[0] + c0[1] * r0[1] + c0[2] * r0[2];
                const T s = lw[i] * wl * recip(det);
                const T x = Gx[row + i], y = Gy[row + i], z = Gz[row + i];
                T p[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) p[k] = (r0[k] * x + r1[k] * y + r2[k] * z) * s;
                if (act) {
                    Gx[row + i] = r0[0] * p[0] + r0[1] * p[1] + r0[2] * p[2];
                    Gy[row + i] = r1[0] * p[0] + r1[1] * p[1] + r1[2] * p[2];
                    Gz[row + i] = r2[0] * p[0] + r2[1] * p[1] + r2[2] * p[2];
                }
            }
        }
    } else if constexpr (GEO == kStoredMetric) {
        const T* mt = geo + b * (M * N * WG) + lane;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if constexpr (DIM == 3) {
                const T g00 = mt[(0 * N + i) * WG], g11 = mt[(1 * N + i) * WG], g22 = mt[(2 * N + i) * WG];
                const T g01 = mt[(3 * N + i) * WG], g02 = mt[(4 * N + i) * WG], g12 = mt[(5 * N + i) * WG];
                const T x = gx[i], y = gy[i], z = gz[i];
                gx[i] = g00 * x + g01 * y + g02 * z;
                gy[i] = g01 * x + g11 * y + g12 * z;
                gz[i] = g02 * x + g12 * y + g22 * z;
            } else {
                const T g00 = mt[(0 * N + i) * WG], g11 = mt[(1 * N + i) * WG], g01 = mt[(2 * N + i) * WG];
                const T x = gx[i], y = gz[i];
                gx[i] = g00 * x + g01 * y;
                gz[i] = g01 * x + g11 * y;
            }
        }
    } else {
        T c0[DIM], C1[DIM], E1[DIM], D2[DIM], F2[DIM];
        const T* cf = lcf[cb];
        if constexpr (DIM == 3) {
            const T eta = lg[j], zeta = lg[t];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                // d/dxi = b + e eta + f zeta + h eta zeta          (constant on the line)
                c0[k] = cf[0 + k] + cf[9 + k] * eta + (cf[12 + k] + cf[18 + k] * eta) * zeta;
                // d/deta = (c + g zeta) + (e + h zeta) xi
                C1[k] = cf[3 + k] + cf[15 + k] * zeta;
                E1[k] = cf[9 + k] + cf[18 + k] * zeta;
                // d/dzeta = (d + g eta) + (f + h eta) xi
                D2[k] = cf[6 + k] + cf[15 + k] * eta;
                F2[k] = cf[12 + k] + cf[18 + k] * eta;
            }
        } else {
            const T eta = lg[t];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                c0[k] = cf[0 + k] + cf[4 + k] * eta;  // d/dxi = b + d eta
                C1[k] = cf[2 + k];                    // d/deta = c + d xi
                E1[k] = cf[4 + k];
            }
        }
        const T wl = DIM == 3 ? lw[j] * lw[t] : lw[t];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const T xi = tb.g[i];
            if constexpr (DIM == 3) {
                T c1[3], c2[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    c1[k] = C1[k] + E1[k] * xi;
                    c2[k] = D2[k] + F2[k] * xi;
                }
                const T r0[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2],
                                 c1[0] * c2[1] - c1[1] * c2[0]};
                const T r1[3] = {c2[1] * c0[2] - c2[2] * c0[1], c2[2] * c0[0] - c2[0] * c0[2],
                                 c2[0] * c0[1] - c2[1] * c0[0]};
                const T r2[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2],
                                 c0[0] * c1[1] - c0[1] * c1[0]};
                const T det = c0[0] * r0[0] + c0[1] * r0[1] + c0[2] * r0[2];
                const T s = tb.w[i] * wl * recip(det);
                const T x = gx[i], y = gy[i], z = gz[i];
                T p[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) p[k] = (r0[k] * x + r1[k] * y + r2[k] * z) * s;
                gx[i] = r0[0] * p[0] + r0[1] * p[1] + r0[2] * p[2];
                gy[i] = r1[0] * p[0] + r1[1] * p[1] + r1[2] * p[2];
                gz[i] = r2[0] * p[0] + r2[1] * p[1] + r2[2] * p[2];
            } else {
                const T c1[2] = {C1[0] + E1[0] * xi, C1[1] + E1[1] * xi};
                const T det = c0[0] * c1[1] - c0[1] * c1[0];
                const T s = tb.w[i] * wl * recip(det);
                // rows of det(J) J^{-1}: (c1.y, -c1.x) and (-c0.y, c0.x)
                const T x = gx[i], y = gz[i];
                const T p0 = (c1[1] * x - c0[1] * y) * s;
                const T p1 = (-c1[0] * x + c0[0] * y) * s;
                gx[i] = c1[1] * p0 - c1[0] * p1;
                gz[i] = -c0[1] * p0 + c0[0] * p1;
            }
        }
    }

    // ---- backward -------------------------------------------------------
    if constexpr (SW == 1) {
        // out = Sx^T Sy^T Sz^T (Dx^T fx) + Sx^T DSy^T Sz^T fy + Sx^T Sy^T DSz^T fz
        // (2D: Sx^T Sy^T (Dx^T fx) + Sx^T DSy^T fy), the stages in reverse
        T* T0 = lds[0][cb];
        T* T1 = lds[1][cb];
        T* T2 = lds[2][cb];
        if constexpr (kSeq) {
            // the geometry step left f_x, f_z, f_y in the lane's positions of
            // tiles 0, 1, 2: Dx^T f_x replaces f_x in place
            T g0[N];
#pragma unroll
            for (int i = 0; i < N; ++i) g0[i] = T0[row + i];
            line_apply_sym<N, T, true, -1>(tb.D, eo.Dt, g0, u);  // Dx^T fx
        } else {
            line_apply_sym<N, T, true, -1>(tb.D, eo.Dt, gx, u);  // Dx^T fx
            block_sync<WG>();                     // every lane has read the forward tiles
        }
        if constexpr (DIM == 3) {
            // outputs of the z stage (T3, T4) and of the y stage (Ty)
            T* T3 = lds[kSeq ? 0 : 3][cb];
            T* T4 = lds[kSeq ? 1 : 4][cb];
            T* Ty = lds[kSeq ? 2 : 0][cb];
            if (act) {
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    T0[row + i] = u[i];
                    if constexpr (!kSeq) {
                        T1[row + i] = gy[i];
                        T2[row + i] = gz[i];
                    }
                }
            }
            block_sync<WG>();
            // z-line (i, j) = (j, t) of this lane's indices: Dx^T f_x, f_y, f_z
            T* Fy = kSeq ? T2 : T1;
            T* Fz = kSeq ? T1 : T2;
            T a[N], b2[N], c2[N], r0[N], r1[N];
#pragma unroll
            for (int c = 0; c < N; ++c) {
                a[c] = T0[(c * N + t) * N + j];
                b2[c] = Fy[(c * N + t) * N + j];
                c2[c] = Fz[(c * N + t) * N + j];
            }
            if constexpr (kSeq) {
                block_sync<WG>();  // T0 and T1 are overwritten below
                line_apply_sym<N, T, true, 1>(tb.S, eo.St, a, r0);
                line_apply_sym<N, T, true, -1>(tb.DS, eo.DSt, c2, r1);
                if (act) {
#pragma unroll
                    for (int c = 0; c < N; ++c) T3[(c * N + t) * N + j] = r0[c] + r1[c];
                }
                __builtin_amdgcn_sched_barrier(0);
                line_apply_sym<N, T, true, 1>(tb.S, eo.St, b2, a);
                if (act) {
#pragma unroll
                    for (int c = 0; c < N; ++c) T4[(c * N + t) * N + j] = a[c];
                }
            } else {
                line_apply_sym<N, T, true, 1>(tb.S, eo.St, a, r0);
                line_apply_sym<N, T, true, -1>(tb.DS, eo.DSt, c2, r1);
                line_apply_sym<N, T, true, 1>(tb.S, eo.St, b2, a);
                if (act) {
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        T3[(c * N + t) * N + j] = r0[c] + r1[c];
                        T4[(c * N + t) * N + j] = a[c];
                    }
                }
            }
            block_sync<WG>();
            // y-line (i, t) = (j, t) of this lane's indices
#pragma unroll
            for (int c = 0; c < N; ++c) {
                a[c] = T3[(t * N + c) * N + j];
                b2[c] = T4[(t * N + c) * N + j];
            }
            line_apply_sym<N, T, true, 1>(tb.S, eo.St, a, r0);
            line_apply_sym<N, T, true, -1>(tb.DS, eo.DSt, b2, r1);
            if (act) {
#pragma unroll
                for (int c = 0; c < N; ++c) Ty[(t * N + c) * N + j] = r0[c] + r1[c];
            }
            block_sync<WG>();
#pragma unroll
            for (int i = 0; i < N; ++i) u[i] = Ty[row + i];
        } else {
            if (act) {
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    T0[row + i] = u[i];
                    T1[row + i] = gz[i];
                }
            }
            block_sync<WG>();
            // y-line i = t of this lane's index
            T a[N], b2[N], r0[N], r1[N];
#pragma unroll
            for (int c = 0; c < N; ++c) {
                a[c] = T0[c * N + t];
                b2[c] = T1[c * N + t];
            }
            line_apply_sym<N, T, true, 1>(tb.S, eo.St, a, r0);
            line_apply_sym<N, T, true, -1>(tb.DS, eo.DSt, b2, r1);
            if (act) {
#pragma unroll
                for (int c = 0; c < N; ++c) T2[c * N + t] = r0[c] + r1[c];
            }
            block_sync<WG>();
#pragma unroll
            for (int i = 0; i < N; ++i) u[i] = T2[row + i];
        }
        line_apply_sym<N, T, true, 1>(tb.S, eo.St, u, v);  // x: S^T
    } else {
        line_apply_sym<N, T, true, -1>(tb.D, eo.Dt, gx, u);  // Dx^T fx
        if constexpr (DIM == 3) {
            // + Dy^T fy
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) A[row + i] = gy[i];
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = u[i];
    #pragma unroll
                for (int c = 0; c < N; ++c) s += lD[c * N + j] * A[(t * N + c) * N + i];
                u[i] = s;
            }
            // z: S^T (sum) + DS^T fz
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) {
                    B[row + i] = u[i];
                    Cc[row + i] = gz[i];
                }
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = lS[0 * N + t] * B[(0 * N + j) * N + i] + lDS[0 * N + t] * Cc[(0 * N + j) * N + i];
    #pragma unroll
                for (int q = 1; q < N; ++q)
                    s += lS[q * N + t] * B[(q * N + j) * N + i] + lDS[q * N + t] * Cc[(q * N + j) * N + i];
                v[i] = s;
            }
            // y: S^T
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) A[row + i] = v[i];
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = lS[0 * N + j] * A[(t * N + 0) * N + i];
    #pragma unroll
                for (int q = 1; q < N; ++q) s += lS[q * N + j] * A[(t * N + q) * N + i];
                u[i] = s;
            }
        } else {
            // y: S^T (sum) + DS^T fy
            if (act) {
    #pragma unroll
                for (int i = 0; i < N; ++i) {
                    B[row + i] = u[i];
                    Cc[row + i] = gz[i];
                }
            }
            block_sync<WG>();
    #pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = lS[0 * N + t] * B[0 * N + i] + lDS[0 * N + t] * Cc[0 * N + i];
    #pragma unroll
                for (int q = 1; q < N; ++q) s += lS[q * N + t] * B[q * N + i] + lDS[q * N + t] * Cc[q * N + i];
                u[i] = s;
            }
        }
        line_apply_sym<N, T, true, 1>(tb.S, eo.St, u, v);  // x: S^T
    }
    if constexpr (SCATTER == kSlots) {
        // the next cell's first node of this line, added here where setup found
        // it to be the same DoF as this line's last node (per-node layout: in
        // the same wavefront; entity records of blocks wider than a wavefront:
        // through LDS, for every pair of cells of the block)
        if constexpr (IDX == kIdxEntity && !kSlotsEarly) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                int e, m, code;
                ent_node(i, e, m, code);
                const int32_t SR = lrec[cb][27 + e];
                slot[i] = (act && SR >= 0) ? SR + m * (code & 15) : -1;
            }
            if ((lrec[cb][EW - 1] & 2) && slot[N - 1] >= 0) slot[N - 1] |= kMergeNext;
        }
        T nxt;
        if constexpr (IDX == kIdxEntity && WG > kWave) {
            __shared__ T lxm[G * CPB][L];
            if (act) lxm[cb][line] = v[0];
            block_sync<WG>();
            nxt = (act && cbl + 1 < CPB) ? lxm[cb + 1][line] : T(0);
        } else {
            nxt = __shfl_down(v[0], L, kWave);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            int32_t k = slot[i];
            if (k >= 0) {
                if (i == N - 1 && (k & kMergeNext)) {
                    v[i] += nxt;
                    k &= ~kMergeNext;
                }
                dst[(int64_t)rhs * plane + k] = v[i];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (idx[i] >= 0) atomic_add(dst + (int64_t)idx[i] * nr + rhs, v[i]);
    }
    if (++rhs >= rhs_end) break;
    // the tiles are rewritten by the next right-hand side
    block_sync<WG>();
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = un[i];
    }
}

// ---------------------------------------------------------------------------
// Linear elasticity (paper §4, Applications to FEA, eq. linear_elasticity):
// a(u, v) = (sigma(u), grad v), sigma = lam tr(grad u) I + mu (grad u + grad u^T),
// for dim = 3 displacement components interleaved by node (vector DoF 3 i + c).
//
// Same block shape, lane layout, geometry rebuild and contribution slots as
// the Laplace kernel; each lane keeps one x-line of a cell for all three
// components.  The forward sweeps run once per component and leave the
// reference gradient ghat_c,k = d u_c / d xi_k at the lane's Gauss points in
// lane-private LDS.  At each point, with R the rows of det(J) J^{-1} (cross
// products of the columns of J),
//   grad u = ghat R / det J,  sigma as above,  F = w sigma R^T,
// and F_c,k is integrated against d phi / d xi_k by the backward sweeps, one
// component at a time; component c of slot k is contrib[3 k + c] in the
// plane of its right-hand side.
// ---------------------------------------------------------------------------
template <int N, class T, int NRT>
__global__ __launch_bounds__((OpShape<3, N>::WG)) void elasticity_kernel(const int32_t* __restrict__ dmap,
                                                                         const T* __restrict__ geo,
                                                                         const T* __restrict__ src,
                                                                         const int32_t* __restrict__ slots,
                                                                         T* __restrict__ dst, OpTables<N, T> tb,
                                                                         T lam, T mu, int nr_in, int64_t plane) {
    const int nr = NRT > 0 ? NRT : nr_in;  // as in vmult_kernel
    const int rhs0 = NRT == 0 ? (int)blockIdx.y : 0;
    const int rhs_end = (NRT == 0 && gridDim.y > 1) ? rhs0 + 1 : nr;
    using Sh = OpShape<3, N>;
    constexpr int L = Sh::L, WG = Sh::WG, CPB = Sh::CPB, TILE = Sh::TILE;
    constexpr int NC = 21;
    __shared__ T lds[3][CPB][TILE];
    __shared__ T lg9[9 * N][WG];  // lane-private: ghat (then F) of [component][direction][point]
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const int cell = lane / L;
    const int line = lane - cell * L;
    const bool act = cell < CPB;
    const int cb = act ? cell : 0;
    const int j = line % N, t = line / N;
    const int row = line * N;

    const int32_t* dm = dmap + b * (N * WG) + lane;
    int32_t idx[N], slot[N];
#pragma unroll
    for (int i = 0; i < N; ++i) idx[i] = dm[i * WG];
    const int32_t* ps = slots + b * (N * WG) + lane;
#pragma unroll
    for (int i = 0; i < N; ++i) slot[i] = ps[i * WG];
    __shared__ T lcf[CPB][NC];
    constexpr int R = (NC + L - 1) / L;
    T cv[R];
    {
        const T* gc = geo + b * (NC * CPB) + cb;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m = line + r * L;
            cv[r] = (act && m < NC) ? gc[m * CPB] : T(0);
        }
    }
    constexpr int NT = 3 * N * N + 2 * N;
    static_assert(sizeof(OpTables<N, T>) == NT * sizeof(T), "OpTables must be a flat array of T");
    constexpr int TE = (NT + WG - 1) / WG;
    __shared__ T ltab[NT];
    T tv[TE];
#pragma unroll
    for (int e = 0; e < TE; ++e)
        tv[e] = lane + e * WG < NT ? reinterpret_cast<const T*>(&tb)[lane + e * WG] : T(0);
    T uc[3][N];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < N; ++i) uc[c][i] = idx[i] >= 0 ? src[((int64_t)idx[i] * 3 + c) * nr + rhs0] : T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = line + r * L;
        if (act && m < NC) lcf[cb][m] = cv[r];
    }
#pragma unroll
    for (int e = 0; e < TE; ++e)
        if (lane + e * WG < NT) ltab[lane + e * WG] = tv[e];
    const T* lS = ltab;
    const T* lDS = ltab + N * N;
    const T* lD = ltab + 2 * N * N;
    const T* lg = ltab + 3 * N * N;
    const T* lw = lg + N;
    T* A = lds[0][cb];
    T* B = lds[1][cb];
    T* Cc = lds[2][cb];
    auto G = [&](int c, int k, int i) -> T& { return lg9[(c * 3 + k) * N + i][lane]; };

    for (int rhs = rhs0;;) {
    // the next right-hand side's values are loaded while this one is swept
    T ucn[3][N];
    if (NRT != 1 && rhs + 1 < rhs_end) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < N; ++i)
                ucn[c][i] = idx[i] >= 0 ? src[((int64_t)idx[i] * 3 + c) * nr + rhs + 1] : T(0);
    }
    // ---- forward, one component at a time ---------------------------------
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        T u[N], v[N], gz[N], gx[N], gy[N];
#pragma unroll
        for (int i = 0; i < N; ++i) u[i] = uc[c][i];
        line_apply<N, T, false>(tb.S, u, v);
        if (act) {
#pragma unroll
            for (int i = 0; i < N; ++i) A[row + i] = v[i];
        }
        block_sync<WG>();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = lS[j * N + 0] * A[(t * N + 0) * N + i];
#pragma unroll
            for (int q = 1; q < N; ++q) s += lS[j * N + q] * A[(t * N + q) * N + i];
            u[i] = s;
        }
        if (act) {
#pragma unroll
            for (int i = 0; i < N; ++i) B[row + i] = u[i];
        }
        block_sync<WG>();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const T w0 = B[(0 * N + j) * N + i];
            T s0 = lS[t * N + 0] * w0, s1 = lDS[t * N + 0] * w0;
#pragma unroll
            for (int q = 1; q < N; ++q) {
                const T w = B[(q * N + j) * N + i];
                s0 += lS[t * N + q] * w;
                s1 += lDS[t * N + q] * w;
            }
            v[i] = s0;
            gz[i] = s1;
        }
        line_apply<N, T, false>(tb.D, v, gx);
        if (act) {
#pragma unroll
            for (int i = 0; i < N; ++i) Cc[row + i] = v[i];
        }
        block_sync<WG>();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = lD[j * N + 0] * Cc[(t * N + 0) * N + i];
#pragma unroll
            for (int q = 1; q < N; ++q) s += lD[j * N + q] * Cc[(t * N + q) * N + i];
            gy[i] = s;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            G(c, 0, i) = gx[i];
            G(c, 1, i) = gy[i];
            G(c, 2, i) = gz[i];
        }
        // the tiles are rewritten by the next component
        block_sync<WG>();
    }

    // ---- stress at the Gauss points of the line ---------------------------
    {
        T c0[3], C1[3], E1[3], D2[3], F2[3];
        const T* cf = lcf[cb];
        const T eta = lg[j], zeta = lg[t];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            c0[k] = cf[0 + k] + cf[9 + k] * eta + (cf[12 + k] + cf[18 + k] * eta) * zeta;
            C1[k] = cf[3 + k] + cf[15 + k] * zeta;
            E1[k] = cf[9 + k] + cf[18 + k] * zeta;
            D2[k] = cf[6 + k] + cf[15 + k] * eta;
            F2[k] = cf[12 + k] + cf[18 + k] * eta;
        }
        const T wl = lw[j] * lw[t];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const T xi = tb.g[i];
            T c1[3], c2[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                c1[k] = C1[k] + E1[k] * xi;
                c2[k] = D2[k] + F2[k] * xi;
            }
            // rows of det(J) J^{-1}
            const T Rm[3][3] = {{c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2], c1[0] * c2[1] - c1[1] * c2[0]},
                                {c2[1] * c0[2] - c2[2] * c0[1], c2[2] * c0[0] - c2[0] * c0[2], c2[0] * c0[1] - c2[1] * c0[0]},
                                {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2], c0[0] * c1[1] - c0[1] * c1[0]}};
            const T det = c0[0] * Rm[0][0] + c0[1] * Rm[0][1] + c0[2] * Rm[0][2];
            const T rdet = recip(det);
            T gp[3][3];  // physical gradient: gp[c][m] = d u_c / d x_m
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T h0 = G(c, 0, i), h1 = G(c, 1, i), h2 = G(c, 2, i);
#pragma unroll
                for (int m = 0; m < 3; ++m) gp[c][m] = (h0 * Rm[0][m] + h1 * Rm[1][m] + h2 * Rm[2][m]) * rdet;
            }
            const T tr = gp[0][0] + gp[1][1] + gp[2][2];
            const T w = tb.w[i] * wl;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T sg[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) sg[m] = mu * (gp[c][m] + gp[m][c]) + (m == c ? lam * tr : T(0));
#pragma unroll
                for (int k = 0; k < 3; ++k) G(c, k, i) = w * (sg[0] * Rm[k][0] + sg[1] * Rm[k][1] + sg[2] * Rm[k][2]);
            }
        }
    }

    // ---- backward, one component at a time --------------------------------
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        T u[N], v[N], gx[N], gy[N], gz[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            gx[i] = G(c, 0, i);
            gy[i] = G(c, 1, i);
            gz[i] = G(c, 2, i);
        }
        line_apply<N, T, true>(tb.D, gx, u);
        if (act) {
#pragma unroll
            for (int i = 0; i < N; ++i) A[row + i] = gy[i];
        }
        block_sync<WG>();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = u[i];
#pragma unroll
            for (int q = 0; q < N; ++q) s += lD[q * N + j] * A[(t * N + q) * N + i];
            u[i] = s;
        }
        if (act) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                B[row + i] = u[i];
                Cc[row + i] = gz[i];
            }
        }
        block_sync<WG>();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = lS[0 * N + t] * B[(0 * N + j) * N + i] + lDS[0 * N + t] * Cc[(0 * N + j) * N + i];
#pragma unroll
            for (int q = 1; q < N; ++q)
                s += lS[q * N + t] * B[(q * N + j) * N + i] + lDS[q * N + t] * Cc[(q * N + j) * N + i];
            v[i] = s;
        }
        if (act) {
#pragma unroll
            for (int i = 0; i < N; ++i) A[row + i] = v[i];
        }
        block_sync<WG>();
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = lS[0 * N + j] * A[(t * N + 0) * N + i];
#pragma unroll
            for (int q = 1; q < N; ++q) s += lS[q * N + j] * A[(t * N + q) * N + i];
            u[i] = s;
        }
        line_apply<N, T, true>(tb.S, u, v);
        const T nxt = __shfl_down(v[0], L, kWave);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            int32_t k = slot[i];
            if (k >= 0) {
                if (i == N - 1 && (k & kMergeNext)) {
                    v[i] += nxt;
                    k &= ~kMergeNext;
                }
                dst[(int64_t)rhs * plane + (int64_t)k * 3 + c] = v[i];
            }
        }
        block_sync<WG>();
    }
    if (++rhs >= rhs_end) break;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < N; ++i) uc[c][i] = ucn[c][i];
    }
}

// even-odd form of M (or of M^T): rows 0 .. (N-1)/2 of P, Q and c; the
// mirror rows are implied by M[N-1-i][N-1-j] = sig M[i][j], checked here
template <int N, class T>
static EOMat<N, T> make_eo(const double (&M)[kMaxN][kMaxN], bool trans, int sig) {
    auto m = [&](int i, int j) { return trans ? M[j][i] : M[i][j]; };
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            if (std::fabs(m(N - 1 - i, N - 1 - j) - sig * m(i, j)) > 1e-12 * (1.0 + std::fabs(m(i, j))))
                fail(NNMG_ERR_UNSUPPORTED, "1D basis matrix without the mirror symmetry of its node and point sets");
    EOMat<N, T> e{};
    for (int i = 0; i < (N + 1) / 2; ++i) {
        for (int j = 0; j < N / 2; ++j) {
            e.P[i][j] = (T)(0.5 * (m(i, j) + m(i, N - 1 - j)));
            e.Q[i][j] = (T)(0.5 * (m(i, j) - m(i, N - 1 - j)));
        }
        e.c[i] = (N % 2 == 1) ? (T)m(i, N / 2) : T(0);
    }
    return e;
}

template <int N, class T>
static OpEO<N, T> make_op_eo(const Basis1D& b) {
    OpEO<N, T> t;
    t.S = make_eo<N, T>(b.S, false, 1);
    t.St = make_eo<N, T>(b.S, true, 1);
    t.DS = make_eo<N, T>(b.DS, false, -1);
    t.DSt = make_eo<N, T>(b.DS, true, -1);
    t.D = make_eo<N, T>(b.D, false, -1);
    t.Dt = make_eo<N, T>(b.D, true, -1);
    return t;
}

template <int N, class T>
static OpTables<N, T> make_tables(const Basis1D& b) {
    OpTables<N, T> t;
    for (int i = 0; i < N; ++i) {
        t.g[i] = (T)b.gauss[i];
        t.w[i] = (T)b.weight[i];
        for (int j = 0; j < N; ++j) {
            t.S[i][j] = (T)b.S[i][j];
            t.DS[i][j] = (T)b.DS[i][j];
            t.D[i][j] = (T)b.D[i][j];
        }
    }
    return t;
}

// contribution-slot launches of one index layout, sweep form and number G
// of layout blocks per workgroup (several right-hand sides: one grid row per
// right-hand side when the precision's variant splits them, else every block
// loops over them)
template <int DIM, int N, class T, int GEO, int IDX, int SW, int G>
static void launch_slots_g(const Level& L, const T* geo, const int32_t* dmap, const int32_t* slots, const void* src,
                           void* dst, const OpTables<N, T>& tb, int nr, int64_t plane, hipStream_t s) {
    const dim3 block(OpShape<DIM, N>::WG * G);
    const unsigned gx = (unsigned)((L.nblocks + G - 1) / G);
    const OpEO<N, T> eo = make_op_eo<N, T>(L.basis);
    if (nr == 1) {
        hipLaunchKernelGGL((vmult_kernel<DIM, N, T, GEO, kSlots, 1, IDX, SW, G>), dim3(gx), block, 0, s, dmap, geo,
                           (const T*)src, slots, (T*)dst, tb, eo, nr, plane, (int64_t)L.nblocks);
    } else {
        const bool split = L.var[sizeof(T) == 8 ? NNMG_FP64 : NNMG_FP32].rhs_split != 0;
        hipLaunchKernelGGL((vmult_kernel<DIM, N, T, GEO, kSlots, 0, IDX, SW, G>), dim3(gx, split ? (unsigned)nr : 1u),
                           block, 0, s, dmap, geo, (const T*)src, slots, (T*)dst, tb, eo, nr, plane,
                           (int64_t)L.nblocks);
    }
}

template <int DIM, int N, class T, int GEO, int IDX, int SW>
static void launch_slots(const Level& L, const T* geo, const int32_t* dmap, const int32_t* slots, const void* src,
                         void* dst, const OpTables<N, T>& tb, int nr, int64_t plane, hipStream_t s) {
    if (L.var[sizeof(T) == 8 ? NNMG_FP64 : NNMG_FP32].group == 2)
        launch_slots_g<DIM, N, T, GEO, IDX, SW, 2>(L, geo, dmap, slots, src, dst, tb, nr, plane, s);
    else
        launch_slots_g<DIM, N, T, GEO, IDX, SW, 1>(L, geo, dmap, slots, src, dst, tb, nr, plane, s);
}

template <int DIM, int N, class T, int GEO>
static void vmult_launches(const Level& L, const T* geo, bool atomic, const void* src, void* dst, int nr,
                           hipStream_t s) {
    using Sh = OpShape<DIM, N>;
    const OpTables<N, T> tb = make_tables<N, T>(L.basis);
    const dim3 grid((unsigned)L.nblocks), block(Sh::WG);
    const int64_t plane = (int64_t)contrib_plane(L);
    const bool sw = L.var[sizeof(T) == 8 ? NNMG_FP64 : NNMG_FP32].sweep == 1;
    if (atomic) {
        const OpEO<N, T> eo = make_op_eo<N, T>(L.basis);
        if (nr == 1)
            hipLaunchKernelGGL((vmult_kernel<DIM, N, T, GEO, kAtomic, 1>), grid, block, 0, s, L.d_dofmap_blk.ptr, geo,
                               (const T*)src, L.d_pos_blk.ptr, (T*)dst, tb, eo, nr, plane, (int64_t)L.nblocks);
        else
            hipLaunchKernelGGL((vmult_kernel<DIM, N, T, GEO, kAtomic, 0>), grid, block, 0, s, L.d_dofmap_blk.ptr, geo,
                               (const T*)src, L.d_pos_blk.ptr, (T*)dst, tb, eo, nr, plane, (int64_t)L.nblocks);
    } else if (L.var[sizeof(T) == 8 ? NNMG_FP64 : NNMG_FP32].index_layout == 1) {
        if constexpr (DIM == 3 && N >= 4) {
            if (sw)
                launch_slots<DIM, N, T, GEO, kIdxEntity, 1>(L, geo, L.d_ent_rec.ptr, nullptr, src, dst, tb, nr, plane, s);
            else
                launch_slots<DIM, N, T, GEO, kIdxEntity, 0>(L, geo, L.d_ent_rec.ptr, nullptr, src, dst, tb, nr, plane, s);
        } else {
            fail(NNMG_ERR_UNSUPPORTED, "entity records: 3D, degree >= 3");
        }
    } else {
        if (sw)
            launch_slots<DIM, N, T, GEO, kIdxNodes, 1>(L, geo, L.d_dofmap_blk.ptr, L.d_pos_blk.ptr, src, dst, tb, nr,
                                                      plane, s);
        else
            launch_slots<DIM, N, T, GEO, kIdxNodes, 0>(L, geo, L.d_dofmap_blk.ptr, L.d_pos_blk.ptr, src, dst, tb, nr,
                                                      plane, s);
    }
    NNMG_HIP(hipGetLastError());
}

template <int DIM, int N, class T>
static void vmult_dispatch(const Level& L, const T* geo, int mode, bool atomic, const void* src, void* dst, int nr,
                           hipStream_t s) {
    if (L.nblocks == 0) return;
    if constexpr (DIM == 3) {
        if (L.op == NNMG_OP_ELASTICITY) {
            // contribution slots only (no atomic variant), trilinear geometry
            const OpTables<N, T> tb = make_tables<N, T>(L.basis);
            const int64_t plane = (int64_t)contrib_plane(L);
            if (nr == 1)
                hipLaunchKernelGGL((elasticity_kernel<N, T, 1>), dim3((unsigned)L.nblocks), dim3(OpShape<3, N>::WG), 0,
                                   s, L.d_dofmap_blk.ptr, geo, (const T*)src, L.d_pos_blk.ptr, (T*)dst, tb, (T)L.lam,
                                   (T)L.mu, nr, plane);
            else
                hipLaunchKernelGGL((elasticity_kernel<N, T, 0>),
                                   dim3((unsigned)L.nblocks,
                                        L.var[sizeof(T) == 8 ? NNMG_FP64 : NNMG_FP32].rhs_split ? (unsigned)nr : 1u),
                                   dim3(OpShape<3, N>::WG), 0,
                                   s, L.d_dofmap_blk.ptr, geo, (const T*)src, L.d_pos_blk.ptr, (T*)dst, tb, (T)L.lam,
                                   (T)L.mu, nr, plane);
            NNMG_HIP(hipGetLastError());
            return;
        }
    }
    if (mode == kTrilinear)
        vmult_launches<DIM, N, T, kTrilinear>(L, geo, atomic, src, dst, nr, s);
    else
        vmult_launches<DIM, N, T, kStoredMetric>(L, geo, atomic, src, dst, nr, s);
}

template <class T>
static void vmult_prec(const Level& L, const T* geo, int mode, bool atomic, const void* src, void* dst, int nr,
                       hipStream_t s) {
#define NNMG_CASE(D, NN) \
    if (L.dim == D && L.n == NN) return vmult_dispatch<D, NN, T>(L, geo, mode, atomic, src, dst, nr, s);
    NNMG_CASE(2, 2) NNMG_CASE(2, 3) NNMG_CASE(2, 4) NNMG_CASE(2, 5)
    NNMG_CASE(3, 2) NNMG_CASE(3, 3) NNMG_CASE(3, 4) NNMG_CASE(3, 5)
#undef NNMG_CASE
    fail(NNMG_ERR_UNSUPPORTED, "operator degree/dimension");
}

static void launch_op(const Level& L, int prec, bool atomic, const void* src, void* dst, int nr, hipStream_t s) {
    const int mode = L.var[prec].geometry_mode;
    const void* geo = mode == kTrilinear ? (prec == NNMG_FP64 ? (const void*)L.d_coef64.ptr : (const void*)L.d_coef32.ptr)
                                         : (prec == NNMG_FP64 ? (const void*)L.d_metric64.ptr
                                                              : (const void*)L.d_metric32.ptr);
    if (L.nblocks > 0 && (!geo || !L.d_dofmap_blk.ptr || !dst)) fail(NNMG_ERR_INVALID_ARG, "operator data missing");
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides");
    if (prec == NNMG_FP64)
        vmult_prec<double>(L, (const double*)geo, mode, atomic, src, dst, nr, s);
    else
        vmult_prec<float>(L, (const float*)geo, mode, atomic, src, dst, nr, s);
}

void launch_vmult_contrib(const Level& L, int prec, const void* src, void* contrib, hipStream_t s, int nr) {
    launch_op(L, prec, false, src, contrib, nr, s);
}

void launch_vmult_cells(const Level& L, int prec, const void* src, void* dst, hipStream_t s, int nr,
                        void* contrib) {
    if (L.var[prec].atomic && L.op == NNMG_OP_LAPLACE) {
        launch_op(L, prec, true, src, dst, nr, s);
    } else {
        void* cb = contrib ? contrib : (void*)L.d_contrib.ptr;
        if (!contrib && nr != 1) fail(NNMG_ERR_INVALID_ARG, "a contribution buffer is needed for several right-hand sides");
        launch_op(L, prec, false, src, cb, nr, s);
        launch_gather(L, prec, cb, dst, true, s, nr);
    }
}

// block shape of the operator kernel, shared with the layout code of the level setup
void vmult_shape(int dim, int n, int* wg, int* cells_per_block) {
    const int L = dim == 3 ? n * n : n;
    const int w = (dim == 3 && n == 5) ? 128 : 64;
    *wg = w;
    *cells_per_block = w / L;
}

}  // namespace nnmg
