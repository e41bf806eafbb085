// Setup kernels of a level: geometry at the Gauss points, the operator
// diagonal and the load vector.
//
// Geometry is the Q1 (bi/trilinear) map of each cell's vertices,
// x(xi) = sum_b X_b N_b(xi) with N_b = prod_a (xi_a if bit a of b else 1 - xi_a).
// At every Gauss point the merged metric G = w det(J) J^{-1} J^{-T}
// (J_ia = dx_i / dxi_a) is stored in the operator kernel's blocked layout, in
// float64 and rounded once to float32.
#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

struct GaussTable {
    double g[kMaxN];
    double w[kMaxN];
    double S[kMaxN][kMaxN];
    double DS[kMaxN][kMaxN];
};

static GaussTable gauss_table(const Basis1D& b) {
    GaussTable t{};
    for (int i = 0; i < b.n; ++i) {
        t.g[i] = b.gauss[i];
        t.w[i] = b.weight[i];
        for (int j = 0; j < b.n; ++j) {
            t.S[i][j] = b.S[i][j];
            t.DS[i][j] = b.DS[i][j];
        }
    }
    return t;
}

// Jacobian of the Q1 map of one cell at reference point xi
template <int DIM>
__device__ inline void q1_jacobian(const double* __restrict__ cv, const double* xi, double J[DIM][DIM]) {
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int a = 0; a < DIM; ++a) J[i][a] = 0.0;
#pragma unroll
    for (int b = 0; b < (1 << DIM); ++b) {
        double dN[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double v = ((b >> a) & 1) ? 1.0 : -1.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                if (c != a) v *= ((b >> c) & 1) ? xi[c] : 1.0 - xi[c];
            dN[a] = v;
        }
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int a = 0; a < DIM; ++a) J[i][a] += cv[b * DIM + i] * dN[a];
    }
}

template <int DIM>
__device__ inline double det_inv(const double J[DIM][DIM], double Ji[DIM][DIM]) {
    if constexpr (DIM == 2) {
        const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double r = 1.0 / det;
        Ji[0][0] = J[1][1] * r;
        Ji[0][1] = -J[0][1] * r;
        Ji[1][0] = -J[1][0] * r;
        Ji[1][1] = J[0][0] * r;
        return det;
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double r = 1.0 / det;
        Ji[0][0] = c00 * r;
        Ji[1][0] = c01 * r;
        Ji[2][0] = c02 * r;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
        return det;
    }
}

// index of (cell, Gauss point) in the block layout of the operator kernel for
// component m: [blk][m][qx][wg], lane = cell_in_block * n^(d-1) + line with
// line = qy + n qz (3D) or qy (2D)
template <int DIM>
__device__ inline int64_t blk_index(int64_t c, int qx, int qy, int qz, int n, int cpb, int wg, int m) {
    const int M = DIM * (DIM + 1) / 2;
    const int Lc = DIM == 3 ? n * n : n;
    const int64_t b = c / cpb;
    const int cell = (int)(c - b * cpb);
    const int line = DIM == 3 ? qy + n * qz : qy;
    return ((b * M + m) * n + qx) * wg + cell * Lc + line;
}

// one thread per (block position, Gauss point); padding positions are skipped
template <int DIM>
__global__ void geometry_kernel(const double* __restrict__ cverts, const int32_t* __restrict__ order,
                                int64_t npos, int n, int cpb, int wg, GaussTable gt, double* __restrict__ m64,
                                float* __restrict__ m32, int* __restrict__ bad) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int qn = 1;
    for (int a = 0; a < DIM; ++a) qn *= n;
    if (gid >= npos * qn) return;
    const int64_t pos = gid / qn;
    const int q = (int)(gid - pos * qn);
    const int64_t c = order[pos];
    if (c < 0) return;
    const int qx = q % n, qy = (q / n) % n, qz = DIM == 3 ? q / (n * n) : 0;
    double xi[DIM];
    xi[0] = gt.g[qx];
    xi[1] = gt.g[qy];
    if constexpr (DIM == 3) xi[2] = gt.g[qz];
    double w = gt.w[qx] * gt.w[qy];
    if constexpr (DIM == 3) w *= gt.w[qz];
    double J[DIM][DIM], Ji[DIM][DIM];
    q1_jacobian<DIM>(cverts + c * (1 << DIM) * DIM, xi, J);
    const double det = det_inv<DIM>(J, Ji);
    if (!(det > 0.0)) atomicOr(bad, 1);
    const double s = w * det;
    // G_ab = s sum_i Ji[a][i] Ji[b][i]
    auto G = [&](int a, int b2) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < DIM; ++i) v += Ji[a][i] * Ji[b2][i];
        return s * v;
    };
    if constexpr (DIM == 3) {
        const double vals[6] = {G(0, 0), G(1, 1), G(2, 2), G(0, 1), G(0, 2), G(1, 2)};
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const int64_t k = blk_index<3>(pos, qx, qy, qz, n, cpb, wg, m);
            m64[k] = vals[m];
            m32[k] = (float)vals[m];
        }
    } else {
        const double vals[3] = {G(0, 0), G(1, 1), G(0, 1)};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int64_t k = blk_index<2>(pos, qx, qy, 0, n, cpb, wg, m);
            m64[k] = vals[m];
            m32[k] = (float)vals[m];
        }
    }
}

void launch_geometry(Level& L, int* d_bad, hipStream_t s) {
    const int64_t npos = L.nblocks * L.cpb;
    const int64_t total = npos * L.q;
    if (total == 0) return;
    if (!L.d_metric64.ptr || !L.d_metric32.ptr) fail(NNMG_ERR_INVALID_ARG, "metric arrays are not allocated");
    const int threads = 256;
    const dim3 grid((unsigned)((total + threads - 1) / threads));
    const GaussTable gt = gauss_table(L.basis);
    if (L.dim == 3)
        hipLaunchKernelGGL(geometry_kernel<3>, grid, dim3(threads), 0, s, L.d_cellverts.ptr, L.d_order.ptr, npos,
                           L.n, L.cpb, L.wg, gt, L.d_metric64.ptr, L.d_metric32.ptr, d_bad);
    else
        hipLaunchKernelGGL(geometry_kernel<2>, grid, dim3(threads), 0, s, L.d_cellverts.ptr, L.d_order.ptr, npos,
                           L.n, L.cpb, L.wg, gt, L.d_metric64.ptr, L.d_metric32.ptr, d_bad);
    NNMG_HIP(hipGetLastError());
}

// diag_i += sum_q grad_ref(phi_a)(q)^T G_q grad_ref(phi_a)(q), one thread per (cell, local node)
template <int DIM>
__global__ void diagonal_kernel(const int32_t* __restrict__ dofmap, const int32_t* __restrict__ order,
                                const double* __restrict__ m64, int64_t npos, int n, int cpb, int wg, GaussTable gt,
                                double* __restrict__ diag) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int qn = 1;
    for (int a = 0; a < DIM; ++a) qn *= n;
    if (gid >= npos * qn) return;
    const int64_t pos = gid / qn;
    const int a = (int)(gid - pos * qn);
    const int64_t c = order[pos];
    if (c < 0) return;
    const int dof = dofmap[c * qn + a];
    if (dof < 0) return;
    const int ax = a % n, ay = (a / n) % n, az = DIM == 3 ? a / (n * n) : 0;
    double sum = 0.0;
    for (int q = 0; q < qn; ++q) {
        const int qx = q % n, qy = (q / n) % n, qz = DIM == 3 ? q / (n * n) : 0;
        if constexpr (DIM == 3) {
            const double g0 = gt.DS[qx][ax] * gt.S[qy][ay] * gt.S[qz][az];
            const double g1 = gt.S[qx][ax] * gt.DS[qy][ay] * gt.S[qz][az];
            const double g2 = gt.S[qx][ax] * gt.S[qy][ay] * gt.DS[qz][az];
            const double G00 = m64[blk_index<3>(pos, qx, qy, qz, n, cpb, wg, 0)];
            const double G11 = m64[blk_index<3>(pos, qx, qy, qz, n, cpb, wg, 1)];
            const double G22 = m64[blk_index<3>(pos, qx, qy, qz, n, cpb, wg, 2)];
            const double G01 = m64[blk_index<3>(pos, qx, qy, qz, n, cpb, wg, 3)];
            const double G02 = m64[blk_index<3>(pos, qx, qy, qz, n, cpb, wg, 4)];
            const double G12 = m64[blk_index<3>(pos, qx, qy, qz, n, cpb, wg, 5)];
            sum += G00 * g0 * g0 + G11 * g1 * g1 + G22 * g2 * g2 +
                   2.0 * (G01 * g0 * g1 + G02 * g0 * g2 + G12 * g1 * g2);
        } else {
            const double g0 = gt.DS[qx][ax] * gt.S[qy][ay];
            const double g1 = gt.S[qx][ax] * gt.DS[qy][ay];
            const double G00 = m64[blk_index<2>(pos, qx, qy, 0, n, cpb, wg, 0)];
            const double G11 = m64[blk_index<2>(pos, qx, qy, 0, n, cpb, wg, 1)];
            const double G01 = m64[blk_index<2>(pos, qx, qy, 0, n, cpb, wg, 2)];
            sum += G00 * g0 * g0 + G11 * g1 * g1 + 2.0 * G01 * g0 * g1;
        }
    }
    atomicAdd(diag + dof, sum);
}

// Diagonal of the elasticity operator (paper §4, eq. linear_elasticity), one
// thread per (cell, local node a):
//   diag_(a,c) += sum_q w det J [ (lam + mu) (d_c phi_a)^2 + mu |grad phi_a|^2 ]
// with the physical gradient grad phi_a = J^{-T} grad_ref phi_a.
__global__ void elasticity_diagonal_kernel(const int32_t* __restrict__ dofmap, const double* __restrict__ cverts,
                                           int64_t ncells, int n, GaussTable gt, double lam, double mu,
                                           double* __restrict__ diag) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int qn = n * n * n;
    if (gid >= ncells * qn) return;
    const int64_t c = gid / qn;
    const int a = (int)(gid - c * qn);
    const int dof = dofmap[c * qn + a];
    if (dof < 0) return;
    const int ax = a % n, ay = (a / n) % n, az = a / (n * n);
    double sum[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < qn; ++q) {
        const int qx = q % n, qy = (q / n) % n, qz = q / (n * n);
        const double xi[3] = {gt.g[qx], gt.g[qy], gt.g[qz]};
        const double w = gt.w[qx] * gt.w[qy] * gt.w[qz];
        const double gr[3] = {gt.DS[qx][ax] * gt.S[qy][ay] * gt.S[qz][az], gt.S[qx][ax] * gt.DS[qy][ay] * gt.S[qz][az],
                              gt.S[qx][ax] * gt.S[qy][ay] * gt.DS[qz][az]};
        double J[3][3], Ji[3][3];
        q1_jacobian<3>(cverts + c * 8 * 3, xi, J);
        const double det = det_inv<3>(J, Ji);
        double g[3];  // g_i = sum_k Ji[k][i] gr_k
        for (int i = 0; i < 3; ++i) g[i] = Ji[0][i] * gr[0] + Ji[1][i] * gr[1] + Ji[2][i] * gr[2];
        const double s = w * det, g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        for (int i = 0; i < 3; ++i) sum[i] += s * ((lam + mu) * g[i] * g[i] + mu * g2);
    }
    for (int i = 0; i < 3; ++i) atomicAdd(diag + (int64_t)dof * 3 + i, sum[i]);
}

void launch_diagonal(const Level& L, double* diag, hipStream_t s) {
    if (L.op == NNMG_OP_ELASTICITY) {
        const int64_t total = L.n_cells * L.q;
        if (total == 0) return;
        const int threads = 256;
        hipLaunchKernelGGL(elasticity_diagonal_kernel, dim3((unsigned)((total + threads - 1) / threads)),
                           dim3(threads), 0, s, L.d_dofmap.ptr, L.d_cellverts.ptr, L.n_cells, L.n,
                           gauss_table(L.basis), L.lam, L.mu, diag);
        NNMG_HIP(hipGetLastError());
        return;
    }
    const int64_t npos = L.nblocks * L.cpb;
    const int64_t total = npos * L.q;
    if (total == 0) return;
    if (!L.d_metric64.ptr) fail(NNMG_ERR_INVALID_ARG, "diagonal needs the stored metric (level setup only)");
    const int threads = 256;
    const dim3 grid((unsigned)((total + threads - 1) / threads));
    const GaussTable gt = gauss_table(L.basis);
    if (L.dim == 3)
        hipLaunchKernelGGL(diagonal_kernel<3>, grid, dim3(threads), 0, s, L.d_dofmap.ptr, L.d_order.ptr,
                           L.d_metric64.ptr, npos, L.n, L.cpb, L.wg, gt, diag);
    else
        hipLaunchKernelGGL(diagonal_kernel<2>, grid, dim3(threads), 0, s, L.d_dofmap.ptr, L.d_order.ptr,
                           L.d_metric64.ptr, npos, L.n, L.cpb, L.wg, gt, diag);
    NNMG_HIP(hipGetLastError());
}

__global__ void invert_diagonal_kernel(const double* __restrict__ diag, int64_t n, double* __restrict__ d64,
                                       float* __restrict__ d32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = diag[i];
    const double r = v != 0.0 ? 1.0 / v : 0.0;  // constrained rows never received a contribution
    d64[i] = r;
    d32[i] = (float)r;
}

void launch_invert_diagonal(const Level& L, const double* diag, hipStream_t s) {
    if (L.n_dofs == 0) return;
    const int threads = 256;
    const dim3 grid((unsigned)((L.n_dofs + threads - 1) / threads));
    hipLaunchKernelGGL(invert_diagonal_kernel, grid, dim3(threads), 0, s, diag, L.n_dofs, L.d_dinv64.ptr,
                       L.d_dinv32.ptr);
    NNMG_HIP(hipGetLastError());
}

// b_(i,c) += sum_q f_(q,c) |det J_q| w_q phi_a(x_q), one thread per (cell, local
// node); nc components per node (vector DoF nc i + c, f given as [cell][q][nc])
template <int DIM>
__global__ void rhs_kernel(const int32_t* __restrict__ dofmap, const double* __restrict__ cverts,
                           const double* __restrict__ fq, int64_t ncells, int n, int nc, GaussTable gt,
                           double* __restrict__ b) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int qn = 1;
    for (int a = 0; a < DIM; ++a) qn *= n;
    if (gid >= ncells * qn) return;
    const int64_t c = gid / qn;
    const int a = (int)(gid - c * qn);
    const int dof = dofmap[c * qn + a];
    if (dof < 0) return;
    const int ax = a % n, ay = (a / n) % n, az = DIM == 3 ? a / (n * n) : 0;
    double sum[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < qn; ++q) {
        const int qx = q % n, qy = (q / n) % n, qz = DIM == 3 ? q / (n * n) : 0;
        double xi[DIM];
        xi[0] = gt.g[qx];
        xi[1] = gt.g[qy];
        double w = gt.w[qx] * gt.w[qy];
        double phi = gt.S[qx][ax] * gt.S[qy][ay];
        if constexpr (DIM == 3) {
            xi[2] = gt.g[qz];
            w *= gt.w[qz];
            phi *= gt.S[qz][az];
        }
        double J[DIM][DIM], Ji[DIM][DIM];
        q1_jacobian<DIM>(cverts + c * (1 << DIM) * DIM, xi, J);
        const double det = det_inv<DIM>(J, Ji);
        const double s = fabs(det) * w * phi;
        for (int k = 0; k < nc; ++k) sum[k] += fq[(c * qn + q) * nc + k] * s;
    }
    for (int k = 0; k < nc; ++k) atomicAdd(b + (int64_t)dof * nc + k, sum[k]);
}

void launch_assemble_rhs(const Level& L, const double* fq, double* b, hipStream_t s) {
    const int64_t total = L.n_cells * L.q;
    if (total == 0) return;
    const int threads = 256;
    const dim3 grid((unsigned)((total + threads - 1) / threads));
    const GaussTable gt = gauss_table(L.basis);
    if (L.dim == 3)
        hipLaunchKernelGGL(rhs_kernel<3>, grid, dim3(threads), 0, s, L.d_dofmap.ptr, L.d_cellverts.ptr, fq,
                           L.n_cells, L.n, L.ncomp, gt, b);
    else
        hipLaunchKernelGGL(rhs_kernel<2>, grid, dim3(threads), 0, s, L.d_dofmap.ptr, L.d_cellverts.ptr, fq,
                           L.n_cells, L.n, L.ncomp, gt, b);
    NNMG_HIP(hipGetLastError());
}

}  // namespace nnmg
