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
// The points are stored grouped by owner coarse cell.  A team of `team` lanes
// (a power of two dividing 64) handles one coarse cell: for prolongation the
// team loads the cell's coarse values once and evaluates its points, each
// fine DoF being written by exactly one lane; for restriction every lane
// accumulates the cell's local vector over its points, the team reduces by
// cross-lane shuffles and the sums are scatter-added with float atomics.
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

template <int DIM, int N, class T>
__global__ __launch_bounds__(256) void prolongate_kernel(const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ fine,
                                                         const T* __restrict__ xi, int64_t npts,
                                                         const int32_t* __restrict__ cdm,
                                                         const T* __restrict__ uc, T* __restrict__ uf,
                                                         int ncells, int team_log2, NodeTable<N, T> nt) {
    constexpr int Q = Pow<DIM, N>::value;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t K = gid >> team_log2;
    const int team = 1 << team_log2;
    const int t = (int)(gid & (team - 1));
    if (K >= ncells) return;
    const int p0 = off[K], p1 = off[K + 1];
    if (p0 == p1) return;
    T u[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int g = cdm[K * Q + a];
        u[a] = g >= 0 ? uc[g] : T(0);
    }
    for (int p = p0 + t; p < p1; p += team) {
        T px[N], py[N];
        lagrange_eval<N, T>(nt, xi[p], px);
        lagrange_eval<N, T>(nt, xi[npts + p], py);
        T val = T(0);
        if constexpr (DIM == 3) {
            T pz[N];
            lagrange_eval<N, T>(nt, xi[2 * npts + p], pz);
#pragma unroll
            for (int c = 0; c < N; ++c) {
                T s1 = T(0);
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    T s0 = T(0);
#pragma unroll
                    for (int a = 0; a < N; ++a) s0 += px[a] * u[(c * N + b) * N + a];
                    s1 += py[b] * s0;
                }
                val += pz[c] * s1;
            }
        } else {
#pragma unroll
            for (int b = 0; b < N; ++b) {
                T s0 = T(0);
#pragma unroll
                for (int a = 0; a < N; ++a) s0 += px[a] * u[b * N + a];
                val += py[b] * s0;
            }
        }
        const int f = fine[p];
        uf[f] += val;
    }
}

template <int DIM, int N, class T>
__global__ __launch_bounds__(256) void restrict_kernel(const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ fine,
                                                       const T* __restrict__ xi, int64_t npts,
                                                       const int32_t* __restrict__ cdm,
                                                       const T* __restrict__ rf, T* __restrict__ rc,
                                                       int ncells, int team_log2, NodeTable<N, T> nt) {
    constexpr int Q = Pow<DIM, N>::value;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t K = gid >> team_log2;
    const int team = 1 << team_log2;
    const int t = (int)(gid & (team - 1));
    // K and the point range are uniform over a team, so whole teams leave together
    if (K >= ncells) return;
    const int p0 = off[K], p1 = off[K + 1];
    if (p0 == p1) return;
    T R[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) R[a] = T(0);
    for (int p = p0 + t; p < p1; p += team) {
        const T r = rf[fine[p]];
        T px[N], py[N];
        lagrange_eval<N, T>(nt, xi[p], px);
        lagrange_eval<N, T>(nt, xi[npts + p], py);
        if constexpr (DIM == 3) {
            T pz[N];
            lagrange_eval<N, T>(nt, xi[2 * npts + p], pz);
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const T rz = r * pz[c];
#pragma unroll
                for (int b = 0; b < N; ++b) {
                    const T rzy = rz * py[b];
#pragma unroll
                    for (int a = 0; a < N; ++a) R[(c * N + b) * N + a] += rzy * px[a];
                }
            }
        } else {
#pragma unroll
            for (int b = 0; b < N; ++b) {
                const T ry = r * py[b];
#pragma unroll
                for (int a = 0; a < N; ++a) R[b * N + a] += ry * px[a];
            }
        }
    }
    for (int o = team >> 1; o > 0; o >>= 1) {
#pragma unroll
        for (int a = 0; a < Q; ++a) R[a] += __shfl_xor(R[a], o, team);
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        if ((a & (team - 1)) == t) {
            const int g = cdm[K * Q + a];
            if (g >= 0) atomic_add(rc + g, R[a]);
        }
    }
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
static void transfer_dispatch(const Transfer& tr, bool prolong, const T* xi, const void* in, void* out,
                              hipStream_t s) {
    const Level& C = *tr.coarse;
    if (tr.n_points == 0 || C.n_cells == 0) return;
    const int threads = 256;
    const int64_t total = C.n_cells * (int64_t)tr.team;
    const dim3 grid((unsigned)((total + threads - 1) / threads));
    const NodeTable<N, T> nt = node_table<N, T>(C.basis);
    if (prolong)
        hipLaunchKernelGGL((prolongate_kernel<DIM, N, T>), grid, dim3(threads), 0, s, tr.d_off.ptr, tr.d_fine.ptr,
                           xi, tr.n_points, C.d_dofmap.ptr, (const T*)in, (T*)out, (int)C.n_cells,
                           log2i(tr.team), nt);
    else
        hipLaunchKernelGGL((restrict_kernel<DIM, N, T>), grid, dim3(threads), 0, s, tr.d_off.ptr, tr.d_fine.ptr,
                           xi, tr.n_points, C.d_dofmap.ptr, (const T*)in, (T*)out, (int)C.n_cells,
                           log2i(tr.team), nt);
    NNMG_HIP(hipGetLastError());
}

template <class T>
static void transfer_prec(const Transfer& tr, bool prolong, const T* xi, const void* in, void* out,
                          hipStream_t s) {
    const int d = tr.coarse->dim, n = tr.coarse->n;
#define NNMG_CASE(D, NN) \
    if (d == D && n == NN) return transfer_dispatch<D, NN, T>(tr, prolong, xi, in, out, s);
    NNMG_CASE(2, 2) NNMG_CASE(2, 3) NNMG_CASE(2, 4) NNMG_CASE(2, 5)
    NNMG_CASE(3, 2) NNMG_CASE(3, 3) NNMG_CASE(3, 4) NNMG_CASE(3, 5)
#undef NNMG_CASE
    fail(NNMG_ERR_UNSUPPORTED, "transfer degree/dimension");
}

void launch_prolongate(const Transfer& t, int prec, const void* coarse, void* fine, hipStream_t s) {
    if (prec == NNMG_FP64)
        transfer_prec<double>(t, true, t.d_xi64.ptr, coarse, fine, s);
    else
        transfer_prec<float>(t, true, t.d_xi32.ptr, coarse, fine, s);
}

void launch_restrict(const Transfer& t, int prec, const void* fine, void* coarse, hipStream_t s) {
    if (prec == NNMG_FP64)
        transfer_prec<double>(t, false, t.d_xi64.ptr, fine, coarse, s);
    else
        transfer_prec<float>(t, false, t.d_xi32.ptr, fine, coarse, s);
}

}  // namespace nnmg
