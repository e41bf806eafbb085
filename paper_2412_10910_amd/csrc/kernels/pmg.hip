// Transfer between two Q_k spaces on the same mesh (paper §2, Coarse grid
// solvers: the polynomial multigrid below the coarsest mesh, where the degree
// drops level by level on one triangulation).  The spaces are nested: the
// coarse function of degree k_c is, on every cell, a polynomial of degree
// k_f > k_c too, and P interpolates it at the fine support points.  On a cell
// that is the tensor product of one 1D matrix E[i][a] = phi_a^(k_c)(x_i^(k_f))
// (fine Gauss-Lobatto node i, coarse basis function a), applied by sum
// factorization: d sweeps of NF x NC instead of NF^d NC^d products.
//
// prolongate: one block per cell stages the cell's coarse values in LDS,
//             sweeps x, y (and z) and adds the result into the fine DoFs the
//             cell owns (each unconstrained fine DoF is owned by the first
//             cell that holds it, so every fine DoF is written once).
// restrict:   the transpose: the owned fine values in, transposed sweeps,
//             the cell's coarse sums out to coarse-DoF slots that a gather
//             adds in a fixed order (the slot layout of the non-nested
//             restriction).
// nv values per node (components times right-hand sides, value
// c nr + r) are transferred one after the other.
#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

template <int DIM, int N>
struct PPow {
    static constexpr int value = DIM == 2 ? N * N : N * N * N;
};

template <class T>
struct PMat {
    T e[kMaxN * kMaxN];  // E[i][a] at i * NC + a
};

constexpr int kPmgThreads = 64;

template <int DIM, int NF, int NC, class T>
__global__ __launch_bounds__(kPmgThreads) void pmg_prolongate_kernel(const int32_t* __restrict__ cdm,
                                                                     const int32_t* __restrict__ pfdm,
                                                                     const T* __restrict__ uc, T* __restrict__ uf,
                                                                     PMat<T> E, int nv) {
    constexpr int QF = PPow<DIM, NF>::value, QC = PPow<DIM, NC>::value;
    __shared__ T le[NF * NC];
    __shared__ T u[QC];
    __shared__ T t1[NC * NC * NF];
    __shared__ T t2[NC * NF * NF];
    const int64_t cell = blockIdx.x;
    const int tid = threadIdx.x;
    for (int e = tid; e < NF * NC; e += kPmgThreads) le[e] = E.e[e];
    for (int v = 0; v < nv; ++v) {
        for (int a = tid; a < QC; a += kPmgThreads) {
            const int g = cdm[cell * QC + a];
            u[a] = g >= 0 ? uc[(int64_t)g * nv + v] : T(0);
        }
        __syncthreads();
        if constexpr (DIM == 3) {
            // x: t1[c][b][i] = sum_a E[i][a] u[c][b][a]
            for (int e = tid; e < NC * NC * NF; e += kPmgThreads) {
                const int i = e % NF, cb = e / NF;
                T s = T(0);
#pragma unroll
                for (int a = 0; a < NC; ++a) s += le[i * NC + a] * u[cb * NC + a];
                t1[e] = s;
            }
            __syncthreads();
            // y: t2[c][j][i] = sum_b E[j][b] t1[c][b][i]
            for (int e = tid; e < NC * NF * NF; e += kPmgThreads) {
                const int i = e % NF, j = (e / NF) % NF, c = e / (NF * NF);
                T s = T(0);
#pragma unroll
                for (int b = 0; b < NC; ++b) s += le[j * NC + b] * t1[(c * NC + b) * NF + i];
                t2[e] = s;
            }
            __syncthreads();
            // z: out[k][j][i] = sum_c E[k][c] t2[c][j][i], added into the owned fine DoFs
            for (int e = tid; e < QF; e += kPmgThreads) {
                const int ji = e % (NF * NF), k = e / (NF * NF);
                T s = T(0);
#pragma unroll
                for (int c = 0; c < NC; ++c) s += le[k * NC + c] * t2[c * NF * NF + ji];
                const int node = pfdm[cell * QF + e];
                if (node >= 0) uf[(int64_t)node * nv + v] += s;
            }
        } else {
            for (int e = tid; e < NC * NF; e += kPmgThreads) {
                const int i = e % NF, b = e / NF;
                T s = T(0);
#pragma unroll
                for (int a = 0; a < NC; ++a) s += le[i * NC + a] * u[b * NC + a];
                t1[e] = s;
            }
            __syncthreads();
            for (int e = tid; e < QF; e += kPmgThreads) {
                const int i = e % NF, j = e / NF;
                T s = T(0);
#pragma unroll
                for (int b = 0; b < NC; ++b) s += le[j * NC + b] * t1[b * NF + i];
                const int node = pfdm[cell * QF + e];
                if (node >= 0) uf[(int64_t)node * nv + v] += s;
            }
        }
        __syncthreads();  // u and the tiles are rewritten by the next value
    }
}

template <int DIM, int NF, int NC, class T>
__global__ __launch_bounds__(kPmgThreads) void pmg_restrict_kernel(const int32_t* __restrict__ pfdm,
                                                                   const int32_t* __restrict__ rslot,
                                                                   const T* __restrict__ uf, T* __restrict__ rbuf,
                                                                   PMat<T> E, int ncomp, int nr, int64_t plane) {
    constexpr int QF = PPow<DIM, NF>::value, QC = PPow<DIM, NC>::value;
    __shared__ T le[NF * NC];
    __shared__ T r[QF];
    __shared__ T s1[NF * NF * NC];
    __shared__ T s2[NF * NC * NC];
    const int64_t cell = blockIdx.x;
    const int tid = threadIdx.x;
    const int nv = ncomp * nr;
    for (int e = tid; e < NF * NC; e += kPmgThreads) le[e] = E.e[e];
    for (int v = 0; v < nv; ++v) {
        const int cc = v / nr, rr = v - cc * nr;
        T* __restrict__ out = rbuf + rr * plane + cc;  // slot k at out[ncomp k]
        for (int e = tid; e < QF; e += kPmgThreads) {
            const int node = pfdm[cell * QF + e];
            r[e] = node >= 0 ? uf[(int64_t)node * nv + v] : T(0);
        }
        __syncthreads();
        if constexpr (DIM == 3) {
            // x: s1[k][j][a] = sum_i E[i][a] r[k][j][i]
            for (int e = tid; e < NF * NF * NC; e += kPmgThreads) {
                const int a = e % NC, kj = e / NC;
                T s = T(0);
#pragma unroll
                for (int i = 0; i < NF; ++i) s += le[i * NC + a] * r[kj * NF + i];
                s1[e] = s;
            }
            __syncthreads();
            // y: s2[k][b][a] = sum_j E[j][b] s1[k][j][a]
            for (int e = tid; e < NF * NC * NC; e += kPmgThreads) {
                const int a = e % NC, b = (e / NC) % NC, k = e / (NC * NC);
                T s = T(0);
#pragma unroll
                for (int j = 0; j < NF; ++j) s += le[j * NC + b] * s1[(k * NF + j) * NC + a];
                s2[e] = s;
            }
            __syncthreads();
            // z: the cell's sum for coarse node (c, b, a) to its slot
            for (int e = tid; e < QC; e += kPmgThreads) {
                const int ba = e % (NC * NC), c = e / (NC * NC);
                T s = T(0);
#pragma unroll
                for (int k = 0; k < NF; ++k) s += le[k * NC + c] * s2[k * NC * NC + ba];
                const int slot = rslot[cell * QC + e];
                if (slot >= 0) out[(int64_t)slot * ncomp] = s;
            }
        } else {
            for (int e = tid; e < NF * NC; e += kPmgThreads) {
                const int a = e % NC, j = e / NC;
                T s = T(0);
#pragma unroll
                for (int i = 0; i < NF; ++i) s += le[i * NC + a] * r[j * NF + i];
                s1[e] = s;
            }
            __syncthreads();
            for (int e = tid; e < QC; e += kPmgThreads) {
                const int a = e % NC, b = e / NC;
                T s = T(0);
#pragma unroll
                for (int j = 0; j < NF; ++j) s += le[j * NC + b] * s1[j * NC + a];
                const int slot = rslot[cell * QC + e];
                if (slot >= 0) out[(int64_t)slot * ncomp] = s;
            }
        }
        __syncthreads();
    }
}

template <int DIM, int NF, int NC, class T>
static void pmg_launch(const Transfer& t, bool prolong, const void* in, void* out, int nr, void* rbuf,
                       hipStream_t s) {
    const Level& C = *t.coarse;
    if (C.n_cells == 0) return;
    PMat<T> E{};
    for (int i = 0; i < NF; ++i)
        for (int a = 0; a < NC; ++a) E.e[i * NC + a] = (T)t.pmat[i * kMaxN + a];
    const dim3 grid((unsigned)C.n_cells), block(kPmgThreads);
    if (prolong)
        hipLaunchKernelGGL((pmg_prolongate_kernel<DIM, NF, NC, T>), grid, block, 0, s, C.d_dofmap.ptr, t.d_pfdm.ptr,
                           (const T*)in, (T*)out, E, C.ncomp * nr);
    else
        hipLaunchKernelGGL((pmg_restrict_kernel<DIM, NF, NC, T>), grid, block, 0, s, t.d_pfdm.ptr, t.d_rslot.ptr,
                           (const T*)in, (T*)rbuf, E, C.ncomp, nr, (int64_t)(t.n_rslots * C.ncomp));
    NNMG_HIP(hipGetLastError());
}

template <class T>
static void pmg_prec(const Transfer& t, bool prolong, const void* in, void* out, int nr, void* rbuf, hipStream_t s) {
    const int d = t.coarse->dim, nf = t.fine->n, nc = t.coarse->n;
#define NNMG_PCASE(D, F, K) \
    if (d == D && nf == F && nc == K) return pmg_launch<D, F, K, T>(t, prolong, in, out, nr, rbuf, s);
    NNMG_PCASE(2, 3, 2) NNMG_PCASE(2, 4, 2) NNMG_PCASE(2, 4, 3) NNMG_PCASE(2, 5, 2) NNMG_PCASE(2, 5, 3)
    NNMG_PCASE(2, 5, 4) NNMG_PCASE(3, 3, 2) NNMG_PCASE(3, 4, 2) NNMG_PCASE(3, 4, 3) NNMG_PCASE(3, 5, 2)
    NNMG_PCASE(3, 5, 3) NNMG_PCASE(3, 5, 4)
#undef NNMG_PCASE
    fail(NNMG_ERR_UNSUPPORTED, "polynomial transfer degrees");
}

void launch_pmg_prolongate(const Transfer& t, int prec, const void* coarse, void* fine, int nr, hipStream_t s) {
    if (prec == NNMG_FP64)
        pmg_prec<double>(t, true, coarse, fine, nr, nullptr, s);
    else
        pmg_prec<float>(t, true, coarse, fine, nr, nullptr, s);
}

void launch_pmg_restrict_sums(const Transfer& t, int prec, const void* fine, void* rbuf, int nr, hipStream_t s) {
    if (prec == NNMG_FP64)
        pmg_prec<double>(t, false, fine, nullptr, nr, rbuf, s);
    else
        pmg_prec<float>(t, false, fine, nullptr, nr, rbuf, s);
}

}  // namespace nnmg
