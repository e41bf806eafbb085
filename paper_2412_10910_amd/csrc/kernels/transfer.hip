// Non-nested transfer kernels.
//
// locate:     owner coarse cell and reference position of every unconstrained
//             fine support point (paper §3.1: candidate search, then Newton
//             inversion of the cell map; §3.3 eq. closest_point for points
//             outside every candidate).
// prolongate: fine += P coarse with P_ij = phi_j(x_i) (paper §2 after eq.
//             residual2), evaluated per point by the tensor-product form of
//             §3.2 (eqs. local_evaluation, tensor_product_evaluation).
// restrict:   coarse += P^T fine (paper §2, eq. residual2).
//
// The points are stored grouped by owner coarse cell.
//
// Prolongation is point-parallel: one lane per point, blocks of kPointBlock
// consecutive points.  The few coarse cells a block's points belong to have
// their q coarse values staged in LDS once, and each lane evaluates its point
// against its cell's values and adds the result into its fine DoF (each fine
// DoF is the target of exactly one point, so there are no write conflicts).
// All point data are read with coalesced loads.
//
// Restriction is cell-parallel: a team of `team` lanes (a power of two
// dividing 64) handles one coarse cell.  Every lane accumulates the cell's
// local vector over its points, loading the data of several points before
// using any of them; the team reduces by cross-lane shuffles and writes the
// cell's q sums to their slots, which are sorted by coarse DoF; a gather then
// adds every coarse DoF's slots in a fixed order.  No float atomics, so the
// restriction (and the V-cycle) is deterministic.
#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

// ---------------------------------------------------------------------------
// point location
// ---------------------------------------------------------------------------
template <int DIM>
struct Grid {
    double lo[DIM];
    double step[DIM];
    int nb[DIM];
};

template <int DIM>
__device__ inline bool newton_q1(const double* __restrict__ cv, const double* x, double tol, int max_it,
                                 double* xi) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) xi[a] = 0.5;
    for (int it = 0; it < max_it; ++it) {
        double F[DIM], J[DIM][DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            F[i] = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) J[i][a] = 0.0;
        }
#pragma unroll
        for (int b = 0; b < (1 << DIM); ++b) {
            double N = 1.0, dN[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                N *= ((b >> a) & 1) ? xi[a] : 1.0 - xi[a];
                double v = ((b >> a) & 1) ? 1.0 : -1.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c)
                    if (c != a) v *= ((b >> c) & 1) ? xi[c] : 1.0 - xi[c];
                dN[a] = v;
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                const double X = cv[b * DIM + i];
                F[i] += X * N;
#pragma unroll
                for (int a = 0; a < DIM; ++a) J[i][a] += X * dN[a];
            }
        }
        double r[DIM], d[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) r[i] = F[i] - x[i];
        double det;
        if constexpr (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            if (det == 0.0) return false;
            d[0] = (J[1][1] * r[0] - J[0][1] * r[1]) / det;
            d[1] = (J[0][0] * r[1] - J[1][0] * r[0]) / det;
        } else {
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
            if (det == 0.0) return false;
            const double i10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
            const double i11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
            const double i12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
            const double i20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            const double i21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            const double i22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            d[0] = (c00 * r[0] + i10 * r[1] + i20 * r[2]) / det;
            d[1] = (c01 * r[0] + i11 * r[1] + i21 * r[2]) / det;
            d[2] = (c02 * r[0] + i12 * r[1] + i22 * r[2]) / det;
        }
        double dmax = 0.0, xmax = 0.0;
        bool finite = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            xi[a] -= d[a];
            finite = finite && isfinite(xi[a]);
            dmax = fmax(dmax, fabs(d[a]));
            xmax = fmax(xmax, fabs(xi[a]));
        }
        if (!finite || xmax > 1e6) return false;
        if (dmax <= tol) return true;
    }
    return false;
}

template <int DIM>
__global__ void locate_kernel(const double* __restrict__ pts, int np, const double* __restrict__ cverts,
                              const double* __restrict__ boxes, const int32_t* __restrict__ boff,
                              const int32_t* __restrict__ bcells, Grid<DIM> g, double inside_tol,
                              double newton_tol, int newton_max_it, int32_t* __restrict__ owner,
                              double* __restrict__ xi_out, int32_t* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double x[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) x[a] = pts[(int64_t)i * DIM + a];
    int64_t bucket = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int k = (int)floor((x[a] - g.lo[a]) / g.step[a]);
        k = k < 0 ? 0 : (k >= g.nb[a] ? g.nb[a] - 1 : k);
        bucket += k * stride;
        stride *= g.nb[a];
    }
    int best = -1;
    double best_d = 0.0;
    double best_xi[DIM];
    int found = -1;
    double found_xi[DIM];
    for (int k = boff[bucket]; k < boff[bucket + 1]; ++k) {
        const int c = bcells[k];
        bool in = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double lo = boxes[((int64_t)c * 2 + 0) * DIM + a];
            const double hi = boxes[((int64_t)c * 2 + 1) * DIM + a];
            in = in && x[a] >= lo && x[a] <= hi;
        }
        if (!in) continue;
        double xi[DIM];
        if (!newton_q1<DIM>(cverts + (int64_t)c * (1 << DIM) * DIM, x, newton_tol, newton_max_it, xi)) continue;
        double dinf = 0.0, d2 = 0.0, cl[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            cl[a] = fmin(fmax(xi[a], 0.0), 1.0);
            const double e = xi[a] - cl[a];
            dinf = fmax(dinf, fabs(e));
            d2 += e * e;
        }
        if (dinf <= inside_tol) {
            found = c;
#pragma unroll
            for (int a = 0; a < DIM; ++a) found_xi[a] = cl[a];
            break;  // candidates are visited in increasing cell number
        }
        d2 = sqrt(d2);
        if (best < 0 || d2 < best_d) {
            best = c;
            best_d = d2;
#pragma unroll
            for (int a = 0; a < DIM; ++a) best_xi[a] = cl[a];
        }
    }
    if (found >= 0) {
        owner[i] = found;
        flags[i] = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) xi_out[(int64_t)i * DIM + a] = found_xi[a];
    } else {
        owner[i] = best;
        flags[i] = best >= 0 ? 1 : 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) xi_out[(int64_t)i * DIM + a] = best >= 0 ? best_xi[a] : 0.0;
    }
}

void launch_locate(int dim, const double* pts, int np, const double* cverts, const double* boxes,
                   const int32_t* boff, const int32_t* bcells, const double* glo, const double* gstep,
                   const int* gnb, double inside_tol, double newton_tol, int newton_max_it, int32_t* owner,
                   double* xi, int32_t* flags, hipStream_t s) {
    if (np == 0) return;
    const int threads = 128;
    const dim3 grid((unsigned)((np + threads - 1) / threads));
    if (dim == 3) {
        Grid<3> g;
        for (int a = 0; a < 3; ++a) {
            g.lo[a] = glo[a];
            g.step[a] = gstep[a];
            g.nb[a] = gnb[a];
        }
        hipLaunchKernelGGL(locate_kernel<3>, grid, dim3(threads), 0, s, pts, np, cverts, boxes, boff, bcells, g,
                           inside_tol, newton_tol, newton_max_it, owner, xi, flags);
    } else {
        Grid<2> g;
        for (int a = 0; a < 2; ++a) {
            g.lo[a] = glo[a];
            g.step[a] = gstep[a];
            g.nb[a] = gnb[a];
        }
        hipLaunchKernelGGL(locate_kernel<2>, grid, dim3(threads), 0, s, pts, np, cverts, boxes, boff, bcells, g,
                           inside_tol, newton_tol, newton_max_it, owner, xi, flags);
    }
    NNMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// prolongation and restriction
// ---------------------------------------------------------------------------
template <int DIM, int N>
struct Pow {
    static constexpr int value = DIM == 2 ? N * N : N * N * N;
};

// values at PPL reference points of the Q_k function with nodal values
// get(a) on one cell, from the 1D basis values px[u], py[u] (, pz[u]) at the
// coordinates of point u: tensor-product evaluation, x direction innermost.
// Each nodal value is read once for all PPL points; every point's sums are
// formed in the same order whatever PPL is.
template <int DIM, int N, int PPL, class T, class Get>
__device__ __forceinline__ void contract_points(const T (&px)[PPL][N], const T (&py)[PPL][N],
                                                const T (&pz)[PPL][N], Get get, T (&val)[PPL]) {
#pragma unroll
    for (int u = 0; u < PPL; ++u) val[u] = T(0);
    if constexpr (DIM == 3) {
        // one z-slice of values in flight at a time for the larger cells
        constexpr int ZU = N <= 3 ? N : 1;
#pragma unroll ZU
        for (int c = 0; c < N; ++c) {
            T s1[PPL];
#pragma unroll
            for (int u = 0; u < PPL; ++u) s1[u] = T(0);
#pragma unroll
            for (int b = 0; b < N; ++b) {
                T s0[PPL];
#pragma unroll
                for (int u = 0; u < PPL; ++u) s0[u] = T(0);
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const T g = get((c * N + b) * N + a);
#pragma unroll
                    for (int u = 0; u < PPL; ++u) s0[u] += px[u][a] * g;
                }
#pragma unroll
                for (int u = 0; u < PPL; ++u) s1[u] += py[u][b] * s0[u];
            }
#pragma unroll
            for (int u = 0; u < PPL; ++u) val[u] += pz[u][c] * s1[u];
        }
    } else {
#pragma unroll
        for (int b = 0; b < N; ++b) {
            T s0[PPL];
#pragma unroll
            for (int u = 0; u < PPL; ++u) s0[u] = T(0);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const T g = get(b * N + a);
#pragma unroll
                for (int u = 0; u < PPL; ++u) s0[u] += px[u][a] * g;
            }
#pragma unroll
            for (int u = 0; u < PPL; ++u) val[u] += py[u][b] * s0[u];
        }
    }
}

// the point-parallel prolongation takes PPL consecutive points per lane at
// Q4 in 3D, where reading the staged q = 125 coarse values from LDS for every
// point would bound the kernel: the points of a lane almost always share
// their cell, and then each staged value is read once for all of them (at Q3
// the extra registers cost more than the LDS reads saved in float64)
template <int DIM, int N>
constexpr int prolong_ppl() {
    return DIM == 3 && N >= 5 ? 2 : 1;
}

// nv values per coarse node (nc components times nr interleaved right-hand
// sides, value c of node g at g nv + c): the staged values of a cell are
// [node][value], and the basis at a point is evaluated once for all values.
// NVT > 0 fixes nv at compile time; NVT = 0 takes nv_in.  A block takes PPL
// runs of kPointBlock points (blk_cells holds the first and last owner cell
// of every run), lane t the points PPL t .. PPL t + PPL - 1 of the block.
template <int DIM, int N, class T, int NVT, int PPL>
__global__ __launch_bounds__(kPointBlock) void prolongate_points_kernel(
    const int32_t* __restrict__ off, const int32_t* __restrict__ fine, const T* __restrict__ xi, int64_t npts,
    const int32_t* __restrict__ blk_cells, const int32_t* __restrict__ cdm, const T* __restrict__ uc,
    T* __restrict__ uf, NodeTable<N, T> nt, int nv_in) {
    const int nv = NVT > 0 ? NVT : nv_in;
    constexpr int Q = Pow<DIM, N>::value;
    // LDS for the coarse values of the block's first cells (16 KB in float64)
    constexpr int kStage = 2048;
    __shared__ T su[kStage];
    __shared__ int32_t soff[kPointBlock + 1];
    const int QC = Q * nv;  // staged values per cell
    const int ncap = kStage / QC < kPointBlock ? kStage / QC : kPointBlock;
    // consecutive runs of points on one XCD: neighbouring coarse cells share
    // the cache lines of their fine DoFs, which then stay in one L2
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    const int64_t p0 = (b * kPointBlock + tid) * PPL;  // the lane's first point
    // the points' own data first, so that these loads overlap the staging
    int f[PPL];
    T x[PPL][DIM];
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        const bool ok = p0 + u < npts;
        f[u] = ok ? fine[p0 + u] : 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) x[u][a] = ok ? xi[a * npts + p0 + u] : T(0);
    }
    // single values at Q4 in 3D: the fine values the lane adds to are loaded
    // here too, so that their latency hides behind the staging and the long
    // contraction (at lower degrees the registers cost more than that saves)
    constexpr bool kEarly = NVT == 1 && DIM == 3 && N >= 5;
    [[maybe_unused]] T old[PPL];
    if constexpr (kEarly) {
#pragma unroll
        for (int u = 0; u < PPL; ++u) old[u] = p0 + u < npts ? uf[f[u]] : T(0);
    }
    const int64_t nrun = (npts + kPointBlock - 1) / kPointBlock;
    const int64_t r0 = b * PPL, r1 = (r0 + PPL < nrun ? r0 + PPL : nrun) - 1;
    const int c0 = blk_cells[2 * r0], c1 = blk_cells[2 * r1 + 1];
    const int ns = (c1 - c0 + 1) < ncap ? (c1 - c0 + 1) : ncap;  // cells staged in LDS
    for (int i = tid; i <= ns; i += kPointBlock) soff[i] = off[c0 + i];
    for (int i = tid; i < ns * QC; i += kPointBlock) {
        const int a = nv == 1 ? i : i / nv;
        const int g = cdm[(int64_t)c0 * Q + a];
        su[i] = g >= 0 ? uc[(int64_t)g * nv + (i - a * nv)] : T(0);
    }
    __syncthreads();
    if (p0 >= npts) return;
    T px[PPL][N], py[PPL][N], pz[PPL][N];
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        lagrange_eval<N, T>(nt, x[u][0], px[u]);
        lagrange_eval<N, T>(nt, x[u][1], py[u]);
        if constexpr (DIM == 3) {
            lagrange_eval<N, T>(nt, x[u][2], pz[u]);
        } else {
#pragma unroll
            for (int a = 0; a < N; ++a) pz[u][a] = T(0);
        }
    }
    // staged cell of each point (-1: not staged), the largest local cell i
    // with soff[i] <= p (empty cells have equal offsets)
    int lc[PPL];
    bool same = true;
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        const int64_t p = p0 + u;
        lc[u] = -1;
        if (p < npts && p < soff[ns]) {
            int lo = 0, hi = ns;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (soff[mid] <= p) lo = mid; else hi = mid;
            }
            lc[u] = lo;
        }
        same = same && lc[u] == lc[0] && lc[u] >= 0;
    }
    if (same) {
        // every point of the lane in one staged cell
        const T* us = su + lc[0] * QC;
        T val[PPL];
        for (int c = 0; c < nv; ++c) {
            if (nv == 1)  // constant LDS offsets
                contract_points<DIM, N, PPL, T>(px, py, pz, [&](int a) { return us[a]; }, val);
            else
                contract_points<DIM, N, PPL, T>(px, py, pz, [&](int a) { return us[a * nv + c]; }, val);
            if constexpr (kEarly) {
#pragma unroll
                for (int u = 0; u < PPL; ++u) uf[f[u]] = old[u] + val[u];
                continue;
            }
#pragma unroll
            for (int u = 0; u < PPL; ++u) uf[(int64_t)f[u] * nv + c] += val[u];
        }
        return;
    }
    // points of different cells, or of cells beyond what LDS holds: one
    // point at a time, the latter searching the offsets and reading the
    // coarse values from global memory
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        const int64_t p = p0 + u;
        if (p >= npts) break;
        T qx[1][N], qy[1][N], qz[1][N], val[1];
#pragma unroll
        for (int a = 0; a < N; ++a) {
            qx[0][a] = px[u][a];
            qy[0][a] = py[u][a];
            qz[0][a] = pz[u][a];
        }
        T* out = uf + (int64_t)f[u] * nv;
        if (lc[u] >= 0) {
            const T* us = su + lc[u] * QC;
            for (int c = 0; c < nv; ++c) {
                contract_points<DIM, N, 1, T>(qx, qy, qz, [&](int a) { return us[a * nv + c]; }, val);
                out[c] += val[0];
            }
        } else {
            int lo = c0 + ns - 1, hi = c1 + 1;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (off[mid] <= p) lo = mid; else hi = mid;
            }
            const int32_t* dm = cdm + (int64_t)lo * Q;
            for (int c = 0; c < nv; ++c) {
                contract_points<DIM, N, 1, T>(qx, qy, qz, [&](int a) {
                    const int g = dm[a];
                    return g >= 0 ? uc[(int64_t)g * nv + c] : T(0);
                }, val);
                out[c] += val[0];
            }
        }
    }
}

#ifndef NNMG_RESTRICT_UNROLL
#define NNMG_RESTRICT_UNROLL 4
#endif

constexpr int next_pow2(int v) { return v <= 1 ? 1 : 2 * next_pow2((v + 1) / 2); }
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Butterfly reduce-scatter of QP partial sums over the 2^levels lanes of a
// lane group (lane bit j at distance S << j): at level j each lane keeps half
// of the values it still holds, the upper half if its bit j is set, and adds
// its partner's copy of that half, so the shuffles total about QP instead of
// QP * levels.  After level j < log2(QP) a lane holds QP >> (j + 1) values;
// value i then stands for output i + sum_j bit_j * (QP >> (j + 1)).  Levels
// beyond log2(QP) sum the single value left.
template <int QP, int J, int JMAX, class T>
__device__ __forceinline__ void butterfly_reduce(T (&R)[QP], int g, int S, int levels, int width) {
    if constexpr (J < JMAX) {
        if (J < levels) {
            constexpr int H = QP >> (J + 1);
            const int o = S << J;
            if constexpr (H >= 1) {
                const bool hi = (g >> J) & 1;
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    const T send = hi ? R[i] : R[i + H];
                    const T keep = hi ? R[i + H] : R[i];
                    R[i] = keep + __shfl_xor(send, o, width);
                }
            } else {
                R[0] += __shfl_xor(R[0], o, width);
            }
            butterfly_reduce<QP, J + 1, JMAX, T>(R, g, S, levels, width);
        }
    }
}

// Restriction, one team of `team` = S * G lanes per coarse cell and value
// (nv = nc nr values per coarse node: nc components times nr interleaved
// right-hand sides, value c nr + r of node i at nv i + c nr + r).  The G lane
// groups split the cell's points; the S lanes of a group read the same points
// and split the cell's q outputs by the slowest reference index (z in 3D, y in
// 2D): lane s owns the NS = ceil(N / S) slices starting at s * NS, so that
// only q / S accumulators live in registers.  The groups are reduced by the
// butterfly above; the sums of slot k for component c of right-hand side r go
// to rbuf[r plane + nc k + c], the layout of the operator's contributions.
template <int DIM, int N, class T, int S>
__global__ __launch_bounds__(256) void restrict_kernel(const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ fine,
                                                       const T* __restrict__ xi, int64_t npts,
                                                       const int32_t* __restrict__ rslot,
                                                       const T* __restrict__ rf, T* __restrict__ rbuf,
                                                       int ncells, int team_log2, NodeTable<N, T> nt, int nc,
                                                       int nr, int64_t plane) {
    const int nv = nc * nr;
    constexpr int Q = Pow<DIM, N>::value;
    constexpr int NS = (N + S - 1) / S;      // slowest-index slices per lane
    constexpr int SLICE = Q / N;             // outputs per slice
    constexpr int QL = NS * SLICE;           // outputs per lane
    constexpr int QP = next_pow2(QL);        // padded for the butterfly
    constexpr int LQ = ilog2(QP);
    constexpr int JMAX = ilog2(64 / S);      // group levels of a 64-lane team
    // consecutive cells on one XCD, as in the prolongation
    const int64_t gid = xcd_remap(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
    const int64_t KC = gid >> team_log2;     // (cell, value) pair
    const int team = 1 << team_log2;
    const int t = (int)(gid & (team - 1));
    const int s = t % S, g = t / S, G = team / S;
    const int levels = team_log2 - ilog2(S);
    // KC and the point range are uniform over a team, so whole teams leave together
    if (KC >= (int64_t)ncells * nv) return;
    const int64_t K = nv == 1 ? KC : KC / nv;
    const int comp = (int)(KC - K * nv);
    const int cc = nr == 1 ? comp : comp / nr, rr = comp - cc * nr;
    T* __restrict__ out = rbuf + rr * plane + cc;  // slot k at out[nc k]
    const int p0 = off[K], p1 = off[K + 1];
    if (p0 == p1) {
        // a cell without points contributes zeros
        for (int a = t; a < Q; a += team) {
            const int k = rslot[K * Q + a];
            if (k >= 0) out[(int64_t)k * nc] = T(0);
        }
        return;
    }
    T R[QP];
#pragma unroll
    for (int a = 0; a < QP; ++a) R[a] = T(0);
    // U points per group and round: all their loads are issued before any use
    constexpr int U = NNMG_RESTRICT_UNROLL;
    for (int base = p0 + g; base < p1; base += U * G) {
        int fi[U];
        T xs[U][DIM], r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = base + u * G;
            const bool ok = p < p1;
            fi[u] = ok ? fine[p] : -1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) xs[u][a] = ok ? xi[a * npts + p] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = fi[u] >= 0 ? rf[(int64_t)fi[u] * nv + comp] : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T ps[N];
            lagrange_eval<N, T>(nt, xs[u][DIM - 1], ps);
            // r times the lane's slices of the slowest-index basis values
            T w[NS];
#pragma unroll
            for (int c = 0; c < NS; ++c) {
                T v = T(0);
#pragma unroll
                for (int m = 0; m < N; ++m)
                    if (m == s * NS + c) v = ps[m];
                w[c] = r[u] * v;
            }
            T px[N];
            lagrange_eval<N, T>(nt, xs[u][0], px);
            if constexpr (DIM == 3) {
                T py[N];
                lagrange_eval<N, T>(nt, xs[u][1], py);
#pragma unroll
                for (int c = 0; c < NS; ++c) {
#pragma unroll
                    for (int b = 0; b < N; ++b) {
                        const T wy = w[c] * py[b];
#pragma unroll
                        for (int a = 0; a < N; ++a) R[(c * N + b) * N + a] += wy * px[a];
                    }
                }
            } else {
#pragma unroll
                for (int c = 0; c < NS; ++c) {
#pragma unroll
                    for (int a = 0; a < N; ++a) R[c * N + a] += w[c] * px[a];
                }
            }
        }
    }
    butterfly_reduce<QP, 0, JMAX, T>(R, g, S, levels, team);
    // the values this lane holds and the output they stand for
    const int held = levels < LQ ? (QP >> levels) : 1;
    int first = 0;
#pragma unroll
    for (int j = 0; j < LQ; ++j)
        if (j < levels && ((g >> j) & 1)) first += QP >> (j + 1);
    // past log2(QP) levels the lanes that differ in the higher bits hold copies
    if (levels > LQ && (g >> LQ) != 0) return;
#pragma unroll
    for (int i = 0; i < QP; ++i) {
        const int o = first + i;
        const int node = s * QL + o;
        if (i < held && o < QL && node < Q) {
            const int k = rslot[K * Q + node];
            if (k >= 0) out[(int64_t)k * nc] = R[i];
        }
    }
}

// Restriction of Q3/Q4 cells in 3D: one wavefront per coarse cell and value.
// The per-point work is an outer product, r Z[c] Y[b] X[a] added into the
// cell's q sums, so splitting the sums over lanes (as the team kernel above
// does) makes every lane that shares a point evaluate its basis again.  Here
// the cell's points are taken in chunks of CH: lane l evaluates the basis at
// point l of the chunk, once, and stages X, Y and r Z in LDS; then lane
// (g, c), one of G point groups times the N values of the slowest index,
// adds the points g, g + G, ... of the chunk into its N x N plane c of the
// cell's sums, reading 2N + 1 staged values per point for N^2 products.  At
// the end the G partial planes are summed in a fixed order through the same
// LDS, a few rows at a time, and written to the slots: deterministic, like the
// team kernel.
template <int N>
struct PlaneShape {
    static constexpr int G = kWave / N;           // point groups: 16 at N = 4, 12 at N = 5
    static constexpr int CH = G * (kWave / G);    // points per chunk: 64, 60
    static constexpr int PT = CH / G;             // points per group and chunk
    static constexpr int SB = CH * 3 * N;         // staged values per chunk
    static constexpr int BR = SB / (G * N * N);   // plane rows reduced per round
    static_assert(BR >= 1, "reduction round must hold one row");
};

template <int N, class T>
__global__ __launch_bounds__(kWave) void restrict_planes_kernel(const int32_t* __restrict__ off,
                                                                const int32_t* __restrict__ fine,
                                                                const T* __restrict__ xi, int64_t npts,
                                                                const int32_t* __restrict__ rslot,
                                                                const T* __restrict__ rf, T* __restrict__ rbuf,
                                                                NodeTable<N, T> nt, int nc, int nr, int64_t plane) {
    using Sh = PlaneShape<N>;
    constexpr int G = Sh::G, CH = Sh::CH, PT = Sh::PT, SB = Sh::SB, BR = Sh::BR;
    constexpr int Q = N * N * N;
    constexpr int NO = N * BR * N;  // outputs per reduction round
    __shared__ T buf[SB];
    const int nv = nc * nr;
    const int64_t KC = xcd_remap(blockIdx.x, gridDim.x);  // (cell, value) pair, consecutive ones on one XCD
    const int64_t K = nv == 1 ? KC : KC / nv;
    const int comp = (int)(KC - K * nv);
    const int cc = nr == 1 ? comp : comp / nr, rr = comp - cc * nr;
    T* __restrict__ out = rbuf + rr * plane + cc;  // slot k at out[nc k]
    const int lane = threadIdx.x;
    const int p0 = off[K], p1 = off[K + 1];
    if (p0 == p1) {
        // a cell without points contributes zeros
        for (int a = lane; a < Q; a += kWave) {
            const int k = rslot[K * Q + a];
            if (k >= 0) out[(int64_t)k * nc] = T(0);
        }
        return;
    }
    const int g = lane / N, c = lane - (lane / N) * N;
    const bool acc = g < G;  // lanes beyond G N only stage points
    T R[N][N];
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int a = 0; a < N; ++a) R[b][a] = T(0);
    // point data two chunks ahead and the residual value (which needs the
    // fine DoF) one chunk ahead, so that no load is waited for where it is used
    auto load_point = [&](int p, int& fi, T (&xs)[3]) {
        fi = -1;
#pragma unroll
        for (int a = 0; a < 3; ++a) xs[a] = T(0);
        if (lane < CH && p < p1) {
            fi = fine[p];
#pragma unroll
            for (int a = 0; a < 3; ++a) xs[a] = xi[a * npts + p];
        }
    };
    int fi0, fi1;
    T xs0[3], xs1[3];
    load_point(p0 + lane, fi0, xs0);
    load_point(p0 + CH + lane, fi1, xs1);
    T r0 = fi0 >= 0 ? rf[(int64_t)fi0 * nv + comp] : T(0);
    for (int base = p0; base < p1; base += CH) {
        // stage: basis of point `lane` of the chunk (zeros past the cell's points)
        T px[N], py[N], pz[N];
        lagrange_eval<N, T>(nt, xs0[0], px);
        lagrange_eval<N, T>(nt, xs0[1], py);
        lagrange_eval<N, T>(nt, xs0[2], pz);
        block_sync<kWave>();  // the previous chunk's reads are done
        if (lane < CH) {
            T* sp = buf + lane * 3 * N;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                sp[a] = px[a];
                sp[N + a] = py[a];
                sp[2 * N + a] = r0 * pz[a];
            }
        }
        block_sync<kWave>();
        // advance the pipeline: residual of the next chunk, points of the one after
        r0 = fi1 >= 0 ? rf[(int64_t)fi1 * nv + comp] : T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) xs0[a] = xs1[a];
        load_point(base + 2 * CH + lane, fi1, xs1);
        // accumulate plane c over the group's points of the chunk
        if (acc) {
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                const T* sp = buf + (g + G * k) * 3 * N;
                T xv[N];
#pragma unroll
                for (int a = 0; a < N; ++a) xv[a] = sp[a];
                const T z = sp[2 * N + c];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    const T w = z * sp[N + b];
#pragma unroll
                    for (int a = 0; a < N; ++a) R[b][a] += w * xv[a];
                }
            }
        }
    }
    // sum the G partial planes: rows b0 .. b0 + BR - 1 per round, partial of
    // group g for output o = (c BR + bb) N + a at buf[g NO + o]
#pragma unroll
    for (int b0 = 0; b0 < N; b0 += BR) {
        block_sync<kWave>();
        if (acc) {
#pragma unroll
            for (int bb = 0; bb < BR; ++bb)
                if (b0 + bb < N) {
#pragma unroll
                    for (int a = 0; a < N; ++a) buf[g * NO + (c * BR + bb) * N + a] = R[b0 + bb][a];
                }
        }
        block_sync<kWave>();
        for (int o = lane; o < NO; o += kWave) {
            const int oc = o / (BR * N), bb = (o / N) % BR, a = o % N;
            if (b0 + bb >= N) continue;
            T sum = buf[o];
#pragma unroll
            for (int q = 1; q < G; ++q) sum += buf[q * NO + o];
            const int k = rslot[K * Q + (oc * N + b0 + bb) * N + a];
            if (k >= 0) out[(int64_t)k * nc] = sum;
        }
    }
}

// lanes sharing each point in the restriction: keep the per-lane outputs
// (q / S accumulators) within the register budget of a few waves per SIMD
template <int N, class T>
constexpr int restrict_split() {
    if constexpr (sizeof(T) == 8)
        return N <= 3 ? 1 : (N == 4 ? 2 : 4);
    else
        return N <= 3 ? 1 : 2;
}

template <int N, class T>
static NodeTable<N, T> node_table(const Basis1D& b) {
    NodeTable<N, T> t;
    for (int i = 0; i < N; ++i) {
        t.node[i] = (T)b.node[i];
        t.bary[i] = (T)b.bary[i];
    }
    return t;
}

static int log2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <int DIM, int N, class T>
static void transfer_dispatch(const Transfer& tr, bool prolong, const T* xi, const void* in, void* out, int nv,
                              void* rbuf, hipStream_t s) {
    const Level& C = *tr.coarse;
    if (tr.n_points == 0 || C.n_cells == 0) return;
    const NodeTable<N, T> nt = node_table<N, T>(C.basis);
    if (prolong) {
        constexpr int PPL = prolong_ppl<DIM, N>();
        const dim3 grid((unsigned)((tr.n_points + kPointBlock * PPL - 1) / (kPointBlock * PPL)));
#define NNMG_PROLONG(NVT)                                                                                   \
    hipLaunchKernelGGL((prolongate_points_kernel<DIM, N, T, NVT, PPL>), grid, dim3(kPointBlock), 0, s, tr.d_off.ptr, \
                       tr.d_fine.ptr, xi, tr.n_points, tr.d_blk_cells.ptr, C.d_dofmap.ptr, (const T*)in, (T*)out, \
                       nt, nv)
        if (nv == 1)
            NNMG_PROLONG(1);
        else if (nv == 3)
            NNMG_PROLONG(3);
        else
            NNMG_PROLONG(0);
#undef NNMG_PROLONG
        NNMG_HIP(hipGetLastError());
        return;
    }
    if constexpr (DIM == 3 && N >= 4) {
        hipLaunchKernelGGL((restrict_planes_kernel<N, T>), dim3((unsigned)(C.n_cells * (int64_t)nv)), dim3(kWave), 0,
                           s, tr.d_off.ptr, tr.d_fine.ptr, xi, tr.n_points, tr.d_rslot.ptr, (const T*)in, (T*)rbuf,
                           nt, C.ncomp, nv / C.ncomp, (int64_t)(tr.n_rslots * C.ncomp));
        NNMG_HIP(hipGetLastError());
        return;
    }
    // 2D, and 3D up to Q2: the team kernel
    constexpr int S = DIM == 3 ? restrict_split<N, T>() : 1;
    const int team = std::max(tr.team, S);
    const int threads = 256;
    const int64_t total = C.n_cells * (int64_t)nv * team;
    const dim3 grid((unsigned)((total + threads - 1) / threads));
    hipLaunchKernelGGL((restrict_kernel<DIM, N, T, S>), grid, dim3(threads), 0, s, tr.d_off.ptr, tr.d_fine.ptr, xi,
                       tr.n_points, tr.d_rslot.ptr, (const T*)in, (T*)rbuf, (int)C.n_cells,
                       log2i(team), nt, C.ncomp, nv / C.ncomp, (int64_t)(tr.n_rslots * C.ncomp));
    NNMG_HIP(hipGetLastError());
}

template <class T>
static void transfer_prec(const Transfer& tr, bool prolong, const T* xi, const void* in, void* out, int nr,
                          void* rbuf, hipStream_t s) {
    const int d = tr.coarse->dim, n = tr.coarse->n;
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides");
    const int nv = tr.coarse->ncomp * nr;
#define NNMG_CASE(D, NN) \
    if (d == D && n == NN) return transfer_dispatch<D, NN, T>(tr, prolong, xi, in, out, nv, rbuf, s);
    NNMG_CASE(2, 2) NNMG_CASE(2, 3) NNMG_CASE(2, 4) NNMG_CASE(2, 5)
    NNMG_CASE(3, 2) NNMG_CASE(3, 3) NNMG_CASE(3, 4) NNMG_CASE(3, 5)
#undef NNMG_CASE
    fail(NNMG_ERR_UNSUPPORTED, "transfer degree/dimension");
}

void launch_prolongate(const Transfer& t, int prec, const void* coarse, void* fine, hipStream_t s, int nr) {
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides");
    if (t.nested_p) return launch_pmg_prolongate(t, prec, coarse, fine, nr, s);
    if (prec == NNMG_FP64)
        transfer_prec<double>(t, true, t.d_xi64.ptr, coarse, fine, nr, nullptr, s);
    else
        transfer_prec<float>(t, true, t.d_xi32.ptr, coarse, fine, nr, nullptr, s);
}

// the per-cell sums of P^T fine into the coarse-DoF slots; returns the buffer
// used.  rbuf: restriction_scratch_bytes(t, nr) bytes of the caller's, or
// nullptr for the transfer's own buffer (which must then hold nr right-hand sides)
static void* restrict_sums(const Transfer& t, int prec, const void* fine, void* coarse, hipStream_t s, int nr,
                           void* rbuf) {
    if (!rbuf) {
        if (nr > t.rbuf_rhs) fail(NNMG_ERR_INVALID_ARG, "restriction buffer holds fewer right-hand sides");
        rbuf = t.d_rbuf.ptr;
    }
    if (nr < 1 || nr > kMaxRhs) fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides");
    if (t.nested_p)
        launch_pmg_restrict_sums(t, prec, fine, rbuf, nr, s);
    else if (prec == NNMG_FP64)
        transfer_prec<double>(t, false, t.d_xi64.ptr, fine, coarse, nr, rbuf, s);
    else
        transfer_prec<float>(t, false, t.d_xi32.ptr, fine, coarse, nr, rbuf, s);
    return rbuf;
}

void launch_restrict(const Transfer& t, int prec, const void* fine, void* coarse, bool accumulate, hipStream_t s,
                     int nr, void* rbuf) {
    rbuf = restrict_sums(t, prec, fine, coarse, s, nr, rbuf);
    launch_gather_runs((size_t)t.coarse->n_dofs, t.coarse->ncomp, t.d_roff.ptr, prec, rbuf,
                       t.n_rslots * (size_t)t.coarse->ncomp, coarse, accumulate, s, nr);
}

void launch_restrict_first_zero(const Transfer& t, int prec, const void* fine, void* coarse, const void* dinv,
                                void* x, double c0, hipStream_t s, int nr, void* rbuf) {
    rbuf = restrict_sums(t, prec, fine, coarse, s, nr, rbuf);
    launch_gather_runs_first_zero((size_t)t.coarse->n_dofs, t.coarse->ncomp, t.d_roff.ptr, prec, rbuf,
                                  t.n_rslots * (size_t)t.coarse->ncomp, coarse, dinv, x, c0, s, nr);
}

size_t restriction_scratch_bytes(const Transfer& t, int nr) {
    return std::max<size_t>(t.n_rslots * (size_t)t.coarse->ncomp * (size_t)nr, 1) * sizeof(double);
}

}  // namespace nnmg
