// Matrix-free operator apply by sum factorisation (paper §3.2: tensor-product
// evaluation; the operator A_l of §2, eq. linear_system, for the Poisson
// bilinear form with the (k+1)^d Gauss rule of §4).
//
// Work decomposition (gfx950, 64-lane wavefronts).  A team of N = k+1 lanes
// handles one cell; lane t of the team owns slab t along the last coordinate
// (z in 3D, y in 2D) and keeps that slab's N^(d-1) values in registers.  The
// in-slab 1D contractions (x, and y in 3D) run in registers; the contraction
// along the slab direction goes through one LDS round trip forward and one
// backward.  64 / N cells share a wavefront and a 64-lane block of the cell
// data layout, so every gather index and every geometry word is a coalesced
// 64-wide load:
//
//   dofmap_blk[(blk * P + ij) * 64 + lane]        P = N^(d-1)
//   metric_blk[((blk * M + m) * P + ij) * 64 + lane]  M = d(d+1)/2
//
// with lane = team * N + t.  The stored geometry at Gauss point q is the
// merged metric G_q = w_q det(J_q) J_q^{-1} J_q^{-T} (components 00,11,22,01,02,12
// in 3D; 00,11,01 in 2D), so that the integrand is grad_ref(v)^T G grad_ref(u).
//
// Forward: u -> values at Gauss points (S in each direction), reference
// gradient by collocation (D on the Gauss points; the slab direction uses
// DS = D S directly).  Backward: the transposes, w = D^T f_x + D^T f_y in
// registers, then S^T / DS^T along the slab direction through LDS, then S^T in
// registers.  Results are scatter-added with hardware float atomics.
#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

template <int N, class T>
__global__ __launch_bounds__(64) void vmult3_kernel(const int32_t* __restrict__ dmap,
                                                    const T* __restrict__ metric,
                                                    const T* __restrict__ src, T* __restrict__ dst,
                                                    Tables<N, T> tb) {
    constexpr int P = N * N;
    constexpr int CPW = kWave / N;
    __shared__ T lds[CPW][2][N][P];
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const int team = lane / N;
    const int t = lane - team * N;
    const bool act = team < CPW;
    const int tm = act ? team : 0;

    const int32_t* dm = dmap + b * (P * kWave) + lane;
    int32_t idx[P];
    T u[P], v[P];
#pragma unroll
    for (int ij = 0; ij < P; ++ij) idx[ij] = dm[ij * kWave];
#pragma unroll
    for (int ij = 0; ij < P; ++ij) u[ij] = idx[ij] >= 0 ? src[idx[ij]] : T(0);

    // x then y: nodal values -> Gauss points within the slab
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = T(0);
#pragma unroll
            for (int a = 0; a < N; ++a) s += tb.S[i][a] * u[j * N + a];
            v[j * N + i] = s;
        }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = T(0);
#pragma unroll
            for (int c = 0; c < N; ++c) s += tb.S[j][c] * v[c * N + i];
            u[j * N + i] = s;
        }
    // z: values and z-derivative at the Gauss points of slab t
    if (act) {
#pragma unroll
        for (int ij = 0; ij < P; ++ij) lds[tm][0][t][ij] = u[ij];
    }
    __syncthreads();
    T gz[P];
#pragma unroll
    for (int ij = 0; ij < P; ++ij) {
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int c = 0; c < N; ++c) {
            const T w = lds[tm][0][c][ij];
            s0 += tb.S[t][c] * w;
            s1 += tb.DS[t][c] * w;
        }
        u[ij] = s0;
        gz[ij] = s1;
    }
    // x and y derivatives by collocation at the Gauss points
    T gx[P], gy[P];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T sx = T(0), sy = T(0);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                sx += tb.D[i][a] * u[j * N + a];
                sy += tb.D[j][a] * u[a * N + i];
            }
            gx[j * N + i] = sx;
            gy[j * N + i] = sy;
        }
    // apply the merged metric
    const T* mt = metric + b * (6 * P * kWave) + lane;
#pragma unroll
    for (int ij = 0; ij < P; ++ij) {
        const T g00 = mt[(0 * P + ij) * kWave];
        const T g11 = mt[(1 * P + ij) * kWave];
        const T g22 = mt[(2 * P + ij) * kWave];
        const T g01 = mt[(3 * P + ij) * kWave];
        const T g02 = mt[(4 * P + ij) * kWave];
        const T g12 = mt[(5 * P + ij) * kWave];
        const T x = gx[ij], y = gy[ij], z = gz[ij];
        gx[ij] = g00 * x + g01 * y + g02 * z;
        gy[ij] = g01 * x + g11 * y + g12 * z;
        gz[ij] = g02 * x + g12 * y + g22 * z;
    }
    // backward in the slab: w = Dx^T fx + Dy^T fy
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = T(0);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                s += tb.D[a][i] * gx[j * N + a];
                s += tb.D[a][j] * gy[a * N + i];
            }
            u[j * N + i] = s;
        }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int ij = 0; ij < P; ++ij) {
            lds[tm][0][t][ij] = u[ij];
            lds[tm][1][t][ij] = gz[ij];
        }
    }
    __syncthreads();
    // z transpose: lane t now holds nodal slab t
#pragma unroll
    for (int ij = 0; ij < P; ++ij) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < N; ++q) s += tb.S[q][t] * lds[tm][0][q][ij] + tb.DS[q][t] * lds[tm][1][q][ij];
        v[ij] = s;
    }
    // y then x transposes back to the nodes
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = T(0);
#pragma unroll
            for (int q = 0; q < N; ++q) s += tb.S[q][j] * v[q * N + i];
            u[j * N + i] = s;
        }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = T(0);
#pragma unroll
            for (int q = 0; q < N; ++q) s += tb.S[q][i] * u[j * N + q];
            v[j * N + i] = s;
        }
#pragma unroll
    for (int ij = 0; ij < P; ++ij)
        if (idx[ij] >= 0) atomic_add(dst + idx[ij], v[ij]);
}

template <int N, class T>
__global__ __launch_bounds__(64) void vmult2_kernel(const int32_t* __restrict__ dmap,
                                                    const T* __restrict__ metric,
                                                    const T* __restrict__ src, T* __restrict__ dst,
                                                    Tables<N, T> tb) {
    constexpr int P = N;
    constexpr int CPW = kWave / N;
    __shared__ T lds[CPW][2][N][P];
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x;
    const int team = lane / N;
    const int t = lane - team * N;
    const bool act = team < CPW;
    const int tm = act ? team : 0;

    const int32_t* dm = dmap + b * (P * kWave) + lane;
    int32_t idx[P];
    T u[P], v[P];
#pragma unroll
    for (int i = 0; i < P; ++i) idx[i] = dm[i * kWave];
#pragma unroll
    for (int i = 0; i < P; ++i) u[i] = idx[i] >= 0 ? src[idx[i]] : T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < N; ++a) s += tb.S[i][a] * u[a];
        v[i] = s;
    }
    if (act) {
#pragma unroll
        for (int i = 0; i < P; ++i) lds[tm][0][t][i] = v[i];
    }
    __syncthreads();
    T gy[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int c = 0; c < N; ++c) {
            const T w = lds[tm][0][c][i];
            s0 += tb.S[t][c] * w;
            s1 += tb.DS[t][c] * w;
        }
        u[i] = s0;
        gy[i] = s1;
    }
    T gx[P];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < N; ++a) s += tb.D[i][a] * u[a];
        gx[i] = s;
    }
    const T* mt = metric + b * (3 * P * kWave) + lane;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const T g00 = mt[(0 * P + i) * kWave];
        const T g11 = mt[(1 * P + i) * kWave];
        const T g01 = mt[(2 * P + i) * kWave];
        const T x = gx[i], y = gy[i];
        gx[i] = g00 * x + g01 * y;
        gy[i] = g01 * x + g11 * y;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < N; ++a) s += tb.D[a][i] * gx[a];
        u[i] = s;
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            lds[tm][0][t][i] = u[i];
            lds[tm][1][t][i] = gy[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < P; ++i) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < N; ++q) s += tb.S[q][t] * lds[tm][0][q][i] + tb.DS[q][t] * lds[tm][1][q][i];
        v[i] = s;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < N; ++q) s += tb.S[q][i] * v[q];
        u[i] = s;
    }
#pragma unroll
    for (int i = 0; i < P; ++i)
        if (idx[i] >= 0) atomic_add(dst + idx[i], u[i]);
}

template <int N, class T>
Tables<N, T> make_tables(const Basis1D& b) {
    Tables<N, T> t;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            t.S[i][j] = (T)b.S[i][j];
            t.DS[i][j] = (T)b.DS[i][j];
            t.D[i][j] = (T)b.D[i][j];
        }
    return t;
}

template <int N, class T>
static void vmult_dispatch(const Level& L, const T* metric, const void* src, void* dst, hipStream_t s) {
    if (L.nblocks == 0) return;
    const dim3 grid((unsigned)L.nblocks), block(kWave);
    if (L.dim == 3)
        hipLaunchKernelGGL((vmult3_kernel<N, T>), grid, block, 0, s, L.d_dofmap_blk.ptr, metric,
                           (const T*)src, (T*)dst, make_tables<N, T>(L.basis));
    else
        hipLaunchKernelGGL((vmult2_kernel<N, T>), grid, block, 0, s, L.d_dofmap_blk.ptr, metric,
                           (const T*)src, (T*)dst, make_tables<N, T>(L.basis));
    NNMG_HIP(hipGetLastError());
}

template <class T>
static void vmult_prec(const Level& L, const T* metric, const void* src, void* dst, hipStream_t s) {
    switch (L.n) {
        case 2: vmult_dispatch<2, T>(L, metric, src, dst, s); break;
        case 3: vmult_dispatch<3, T>(L, metric, src, dst, s); break;
        case 4: vmult_dispatch<4, T>(L, metric, src, dst, s); break;
        case 5: vmult_dispatch<5, T>(L, metric, src, dst, s); break;
        default: fail(NNMG_ERR_UNSUPPORTED, "degree");
    }
}

void launch_vmult_cells(const Level& L, int prec, const void* src, void* dst, hipStream_t s) {
    if (prec == NNMG_FP64)
        vmult_prec<double>(L, L.d_metric64.ptr, src, dst, s);
    else
        vmult_prec<float>(L, L.d_metric32.ptr, src, dst, s);
}

}  // namespace nnmg
