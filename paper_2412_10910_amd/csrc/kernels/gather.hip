// Consumers of the operator's contribution buffer.  The operator kernel
// writes the contribution of every (cell, local node) to its own slot of a
// buffer sorted by node, so node i owns the contiguous run of slots
// [off[i], off[i+1]); with NC components per node (linear elasticity) slot k
// holds component c at NC k + c.  Vector DoF v = NC i + c sums its node's
// run at stride NC, in a fixed order; the sum feeds the consumer directly:
// plain gather, the Chebyshev step, the residual, or the CG product with its
// dot product.  Constrained nodes have no contributions.
#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

template <int NC, class T>
__device__ __forceinline__ T gather_sum(const int32_t* __restrict__ off, const T* __restrict__ contrib, size_t v) {
    const size_t node = NC == 1 ? v : v / NC;
    const int c = NC == 1 ? 0 : (int)(v - node * NC);
    const int k0 = off[node], k1 = off[node + 1];
    T s = T(0);
    for (int k = k0; k < k1; ++k) s += contrib[(size_t)k * NC + c];
    return s;
}

template <int NC>
__device__ __forceinline__ bool has_contributions(const int32_t* __restrict__ off, size_t v) {
    const size_t node = NC == 1 ? v : v / NC;
    return off[node] != off[node + 1];
}

static dim3 grid_n(size_t n, int threads = 256, size_t cap = 1 << 20) {
    size_t g = (n + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return dim3((unsigned)g);
}

// dispatch on the component count (1: Laplace, 3: elasticity)
#define NNMG_NC_DISPATCH(nc, BODY)                                    \
    do {                                                              \
        if ((nc) == 1) {                                              \
            constexpr int NC = 1;                                     \
            BODY;                                                     \
        } else if ((nc) == 3) {                                       \
            constexpr int NC = 3;                                     \
            BODY;                                                     \
        } else {                                                      \
            fail(NNMG_ERR_UNSUPPORTED, "components per node");        \
        }                                                             \
    } while (0)

template <int NC, class T>
__global__ void gather_kernel(size_t n, const int32_t* __restrict__ off,
                              const T* __restrict__ elem, T* __restrict__ dst, int accumulate) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (!has_contributions<NC>(off, i)) continue;  // constrained: untouched
        const T s = gather_sum<NC>(off, elem, i);
        dst[i] = accumulate ? dst[i] + s : s;
    }
}

void launch_gather_runs(size_t n, int ncomp, const int32_t* off, int prec, const void* elem, void* dst,
                        bool accumulate, hipStream_t s) {
    if (n == 0) return;
    NNMG_NC_DISPATCH(ncomp, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((gather_kernel<NC, double>), grid_n(n), dim3(256), 0, s, n, off, (const double*)elem,
                               (double*)dst, (int)accumulate);
        else
            hipLaunchKernelGGL((gather_kernel<NC, float>), grid_n(n), dim3(256), 0, s, n, off, (const float*)elem,
                               (float*)dst, (int)accumulate);
    });
    NNMG_HIP(hipGetLastError());
}

void launch_gather(const Level& L, int prec, const void* elem, void* dst, bool accumulate, hipStream_t s) {
    launch_gather_runs((size_t)L.n_dofs, L.ncomp, L.d_inv_off.ptr, prec, elem, dst, accumulate, s);
}

// r = f - A x;  d = c1 d + c2 dinv r;  x += d      (Chebyshev step, Saad Alg. 12.1)
template <int NC, class T>
__global__ void cheb_step_gather_kernel(size_t n, const int32_t* __restrict__ off,
                                        const T* __restrict__ elem, const T* __restrict__ f,
                                        const T* __restrict__ dinv, T* __restrict__ x, T* __restrict__ d, T c1,
                                        T c2, int first) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const T r = f[i] - gather_sum<NC>(off, elem, i);
        const T dn = first ? c2 * (dinv[i] * r) : c1 * d[i] + c2 * (dinv[i] * r);
        d[i] = dn;
        x[i] += dn;
    }
}

void launch_cheb_step_gather(const Level& L, int prec, const void* elem, const void* f, const void* dinv, void* x,
                             void* d, double c1, double c2, bool first, hipStream_t s) {
    const size_t n = (size_t)L.n_dofs;
    if (n == 0) return;
    NNMG_NC_DISPATCH(L.ncomp, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((cheb_step_gather_kernel<NC, double>), grid_n(n), dim3(256), 0, s, n,
                               L.d_inv_off.ptr, (const double*)elem, (const double*)f, (const double*)dinv,
                               (double*)x, (double*)d, c1, c2, (int)first);
        else
            hipLaunchKernelGGL((cheb_step_gather_kernel<NC, float>), grid_n(n), dim3(256), 0, s, n,
                               L.d_inv_off.ptr, (const float*)elem, (const float*)f, (const float*)dinv,
                               (float*)x, (float*)d, (float)c1, (float)c2, (int)first);
    });
    NNMG_HIP(hipGetLastError());
}

// r = f - A x
template <int NC, class T>
__global__ void residual_gather_kernel(size_t n, const int32_t* __restrict__ off,
                                       const T* __restrict__ elem, const T* __restrict__ f, T* __restrict__ r) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        r[i] = f[i] - gather_sum<NC>(off, elem, i);
}

void launch_residual_gather(const Level& L, int prec, const void* elem, const void* f, void* r, hipStream_t s) {
    const size_t n = (size_t)L.n_dofs;
    if (n == 0) return;
    NNMG_NC_DISPATCH(L.ncomp, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((residual_gather_kernel<NC, double>), grid_n(n), dim3(256), 0, s, n,
                               L.d_inv_off.ptr, (const double*)elem, (const double*)f, (double*)r);
        else
            hipLaunchKernelGGL((residual_gather_kernel<NC, float>), grid_n(n), dim3(256), 0, s, n,
                               L.d_inv_off.ptr, (const float*)elem, (const float*)f, (float*)r);
    });
    NNMG_HIP(hipGetLastError());
}

// q = A p (gathered) and the block partial sums of p . q; the final sum is
// taken by the two-stage reduction of vector.hip
constexpr int kRed = 256;

template <int NC>
__global__ __launch_bounds__(kRed) void gather_dot_kernel(size_t n, const int32_t* __restrict__ off,
                                                          const double* __restrict__ elem,
                                                          const double* __restrict__ p, double* __restrict__ q,
                                                          double* __restrict__ partial) {
    __shared__ double sh[kRed / kWave];
    double acc = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double v = gather_sum<NC>(off, elem, i);
        q[i] = v;
        acc += p[i] * v;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_down(acc, o, kWave);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kRed / kWave; ++w) s += sh[w];
        partial[blockIdx.x] = s;
    }
}

void launch_gather_dot(const Level& L, const double* elem, const double* p, double* q, double* partial,
                       double* out, hipStream_t s) {
    const size_t n = (size_t)L.n_dofs;
    const size_t g = dot_partials(n);
    NNMG_NC_DISPATCH(L.ncomp, {
        hipLaunchKernelGGL((gather_dot_kernel<NC>), dim3((unsigned)g), dim3(kRed), 0, s, n, L.d_inv_off.ptr, elem, p,
                           q, partial);
    });
    launch_sum_partials(partial, g, out, s);
    NNMG_HIP(hipGetLastError());
}

}  // namespace nnmg
