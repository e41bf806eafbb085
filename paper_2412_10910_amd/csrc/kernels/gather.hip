// Consumers of the operator's contribution buffer.  The operator kernel
// writes the contribution of every (cell, local node) to its own slot of a
// buffer sorted by node, so node i owns the contiguous run of slots
// [off[i], off[i+1]).  With NC components per node (linear elasticity) and NR
// right-hand sides, the vectors hold NV = NC NR values per node, value
// c NR + r being component c of right-hand side r, while the buffer is one
// plane of `plane` entries per right-hand side with component c of slot k at
// k NC + c (so the operator's stores for one right-hand side are those of a
// single-vector call).  Each value sums its node's run in a fixed order; the
// sum feeds the consumer directly: plain gather, the Chebyshev step, the
// residual, or the CG product with its dot product.  Constrained nodes have
// no contributions.
#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

// contribution slots of a node loaded at once (a hexahedral mesh node lies in
// at most 8 cells where every vertex has valence 8, as in structured meshes)
constexpr int kGatherBatch = 8;

// Value v of a vector with NC components and NR right-hand sides per node
template <int NC, int NR, class T>
__device__ __forceinline__ T gather_sum(const int32_t* __restrict__ off, const T* __restrict__ contrib, size_t plane,
                                       size_t v) {
    constexpr int NV = NC * NR;
    const size_t node = NV == 1 ? v : v / NV;
    const int sub = NV == 1 ? 0 : (int)(v - node * NV);
    const int c = NR == 1 ? sub : sub / NR;
    const int r = sub - c * NR;
    const T* base = contrib + (NR == 1 ? 0 : (size_t)r * plane) + c;
    const int k0 = off[node], k1 = off[node + 1];
    // The first kGatherBatch slots of the run are loaded together and then
    // added in slot order: one memory latency for the run instead of one per
    // slot.  Places past the run hold -0, which leaves every sum unchanged
    // (x + -0 = x, signed zeros included), so the result is the one of adding
    // the run's slots one at a time.  Longer runs (nodes shared by more cells,
    // on unstructured meshes) finish one slot at a time.
    // (the padding is hidden from the compiler: knowing x + -0 = x, it would
    // move the first addition next to its load and wait for that load alone)
    T pad = T(-0.0);
    asm volatile("" : "+v"(pad));
    T val[kGatherBatch];
#pragma unroll
    for (int j = 0; j < kGatherBatch; ++j) val[j] = k0 + j < k1 ? base[(size_t)(k0 + j) * NC] : pad;
    T s = T(0);
#pragma unroll
    for (int j = 0; j < kGatherBatch; ++j) s += val[j];
    for (int k = k0 + kGatherBatch; k < k1; ++k) s += base[(size_t)k * NC];
    return s;
}

template <int NV>
__device__ __forceinline__ bool has_contributions(const int32_t* __restrict__ off, size_t v) {
    const size_t node = NV == 1 ? v : v / NV;
    return off[node] != off[node + 1];
}

static dim3 grid_n(size_t n, int threads = 256, size_t cap = 1 << 20) {
    size_t g = (n + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return dim3((unsigned)g);
}

#define NNMG_NR_CASES(NCV, ...)                                        \
    switch (nr) {                                                      \
        case 1: { constexpr int NC = NCV, NR = 1; __VA_ARGS__; } break;       \
        case 2: { constexpr int NC = NCV, NR = 2; __VA_ARGS__; } break;       \
        case 3: { constexpr int NC = NCV, NR = 3; __VA_ARGS__; } break;       \
        case 4: { constexpr int NC = NCV, NR = 4; __VA_ARGS__; } break;       \
        case 5: { constexpr int NC = NCV, NR = 5; __VA_ARGS__; } break;       \
        case 6: { constexpr int NC = NCV, NR = 6; __VA_ARGS__; } break;       \
        case 7: { constexpr int NC = NCV, NR = 7; __VA_ARGS__; } break;       \
        case 8: { constexpr int NC = NCV, NR = 8; __VA_ARGS__; } break;       \
        default: fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides"); \
    }

// dispatch on the component count (1: Laplace, 3: elasticity) and the number
// of right-hand sides (1..kMaxRhs)
#define NNMG_NV_DISPATCH(nc, nr, ...)                               \
    do {                                                            \
        if ((nc) == 1) {                                            \
            NNMG_NR_CASES(1, __VA_ARGS__)                              \
        } else if ((nc) == 3) {                                     \
            NNMG_NR_CASES(3, __VA_ARGS__)                              \
        } else {                                                    \
            fail(NNMG_ERR_UNSUPPORTED, "components per node");      \
        }                                                           \
    } while (0)

template <int NC, int NR, class T>
__global__ void gather_kernel(size_t n, const int32_t* __restrict__ off, const T* __restrict__ elem, size_t plane,
                              T* __restrict__ dst, int accumulate) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (!has_contributions<NC * NR>(off, i)) continue;  // constrained: untouched
        const T old = accumulate ? dst[i] : T(0);  // loaded beside the slots, not after them
        const T s = gather_sum<NC, NR>(off, elem, plane, i);
        dst[i] = accumulate ? old + s : s;
    }
}

// The restriction's sums into the right-hand side f of a level whose
// smoothing starts from zero right after, fused with that first step: f =
// the gathered sums (values without contributions, the constrained ones, keep
// theirs) and x = D^-1 f c0, computed as the separate step computes it (the
// step's direction d equals x, which the next step reads in its place).
template <int NC, int NR, class T>
__global__ void gather_first_zero_kernel(size_t n, const int32_t* __restrict__ off, const T* __restrict__ elem,
                                         size_t plane, T* __restrict__ f, const T* __restrict__ dinv,
                                         T* __restrict__ x, T c0) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const T di = dinv[NR == 1 ? i : i / NR];
        T fi;
        if (has_contributions<NC * NR>(off, i)) {
            fi = gather_sum<NC, NR>(off, elem, plane, i);
            f[i] = fi;
        } else {
            fi = f[i];
        }
        x[i] = di * fi * c0;
    }
}

void launch_gather_runs_first_zero(size_t n, int ncomp, const int32_t* off, int prec, const void* elem,
                                   size_t plane, void* f, const void* dinv, void* x, double c0, hipStream_t s,
                                   int nr) {
    if (n == 0) return;
    const size_t nv = n * (size_t)nr;
    NNMG_NV_DISPATCH(ncomp, nr, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((gather_first_zero_kernel<NC, NR, double>), grid_n(nv), dim3(256), 0, s, nv, off,
                               (const double*)elem, plane, (double*)f, (const double*)dinv, (double*)x, c0);
        else
            hipLaunchKernelGGL((gather_first_zero_kernel<NC, NR, float>), grid_n(nv), dim3(256), 0, s, nv, off,
                               (const float*)elem, plane, (float*)f, (const float*)dinv, (float*)x,
                               (float)c0);
    });
    NNMG_HIP(hipGetLastError());
}

void launch_gather_runs(size_t n, int ncomp, const int32_t* off, int prec, const void* elem, size_t plane, void* dst,
                        bool accumulate, hipStream_t s, int nr) {
    if (n == 0) return;
    const size_t nv = n * (size_t)nr;
    NNMG_NV_DISPATCH(ncomp, nr, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((gather_kernel<NC, NR, double>), grid_n(nv), dim3(256), 0, s, nv, off,
                               (const double*)elem, plane, (double*)dst, (int)accumulate);
        else
            hipLaunchKernelGGL((gather_kernel<NC, NR, float>), grid_n(nv), dim3(256), 0, s, nv, off,
                               (const float*)elem, plane, (float*)dst, (int)accumulate);
    });
    NNMG_HIP(hipGetLastError());
}

size_t contrib_plane(const Level& L) { return L.contrib_len * (size_t)L.ncomp; }

void launch_gather(const Level& L, int prec, const void* elem, void* dst, bool accumulate, hipStream_t s, int nr) {
    launch_gather_runs((size_t)L.n_dofs, L.ncomp, L.inv_off(prec), prec, elem, contrib_plane(L), dst, accumulate, s,
                       nr);
}

// r = f - A x;  d = c1 d + c2 dinv r;  x += d      (Chebyshev step, Saad Alg. 12.1)
// dinv is per vector DoF, shared by the NR right-hand sides.  mode: the
// previous d is 0 (kChebFirst) or x (kChebDIsX) instead of being read, and
// the new d is not stored after the last step (kChebLast)
template <int NC, int NR, class T>
__global__ void cheb_step_gather_kernel(size_t n, const int32_t* __restrict__ off,
                                        const T* __restrict__ elem, size_t plane, const T* __restrict__ f,
                                        const T* __restrict__ dinv, T* __restrict__ x, T* __restrict__ d, T c1,
                                        T c2, int mode) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        // the DoF's own operands are loaded first, so that they arrive with
        // the slots instead of one after another behind them
        const T fi = f[i];
        const T di = dinv[NR == 1 ? i : i / NR];
        const T xi = x[i];
        const T dp = (mode & kChebFirst) ? T(0) : ((mode & kChebDIsX) ? xi : d[i]);
        const T r = fi - gather_sum<NC, NR>(off, elem, plane, i);
        const T dn = (mode & kChebFirst) ? c2 * (di * r) : c1 * dp + c2 * (di * r);
        if (!(mode & kChebLast)) d[i] = dn;
        x[i] = xi + dn;
    }
}

void launch_cheb_step_gather(const Level& L, int prec, const void* elem, const void* f, const void* dinv, void* x,
                             void* d, double c1, double c2, int mode, hipStream_t s, int nr) {
    const size_t n = (size_t)L.n_dofs * (size_t)nr;
    if (n == 0) return;
    NNMG_NV_DISPATCH(L.ncomp, nr, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((cheb_step_gather_kernel<NC, NR, double>), grid_n(n), dim3(256), 0, s, n,
                               L.inv_off(prec), (const double*)elem, contrib_plane(L), (const double*)f,
                               (const double*)dinv, (double*)x, (double*)d, c1, c2, mode);
        else
            hipLaunchKernelGGL((cheb_step_gather_kernel<NC, NR, float>), grid_n(n), dim3(256), 0, s, n,
                               L.inv_off(prec), (const float*)elem, contrib_plane(L), (const float*)f,
                               (const float*)dinv, (float*)x, (float*)d, (float)c1, (float)c2, mode);
    });
    NNMG_HIP(hipGetLastError());
}

// r = f - A x
template <int NC, int NR, class T>
__global__ void residual_gather_kernel(size_t n, const int32_t* __restrict__ off, const T* __restrict__ elem,
                                       size_t plane, const T* __restrict__ f, T* __restrict__ r) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const T fi = f[i];
        r[i] = fi - gather_sum<NC, NR>(off, elem, plane, i);
    }
}

void launch_residual_gather(const Level& L, int prec, const void* elem, const void* f, void* r, hipStream_t s,
                            int nr) {
    const size_t n = (size_t)L.n_dofs * (size_t)nr;
    if (n == 0) return;
    NNMG_NV_DISPATCH(L.ncomp, nr, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((residual_gather_kernel<NC, NR, double>), grid_n(n), dim3(256), 0, s, n,
                               L.inv_off(prec), (const double*)elem, contrib_plane(L), (const double*)f, (double*)r);
        else
            hipLaunchKernelGGL((residual_gather_kernel<NC, NR, float>), grid_n(n), dim3(256), 0, s, n,
                               L.inv_off(prec), (const float*)elem, contrib_plane(L), (const float*)f, (float*)r);
    });
    NNMG_HIP(hipGetLastError());
}

// q = A p (gathered) and the block partial sums of p . q per right-hand side.
// The lanes stride over the vector DoFs (the partition a single right-hand
// side uses) and handle the NR values of each, so that every right-hand side
// is summed in the same order as on its own; partial[block][NR], reduced by
// the second stage of vector.hip.
constexpr int kRed = 256;

template <int NC, int NR>
__global__ __launch_bounds__(kRed) void gather_dot_kernel(size_t n, const int32_t* __restrict__ off,
                                                          const double* __restrict__ elem, size_t plane,
                                                          const double* __restrict__ p, double* __restrict__ q,
                                                          double* __restrict__ partial) {
    __shared__ double sh[NR][kRed / kWave];
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const size_t v = i * NR + r;
            const double pv = p[v];
            const double g = gather_sum<NC, NR>(off, elem, plane, v);
            q[v] = g;
            acc[r] += pv * g;
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double a = acc[r];
        for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
        if (threadIdx.x % kWave == 0) sh[r][threadIdx.x / kWave] = a;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
        const int r = threadIdx.x;
        double s = 0.0;
        for (int w = 0; w < kRed / kWave; ++w) s += sh[r][w];
        partial[blockIdx.x * NR + r] = s;
    }
}

void launch_gather_dot(const Level& L, const double* elem, const double* p, double* q, double* partial,
                       double* out, hipStream_t s, int nr, double* scal, int scalar_op) {
    const size_t n = (size_t)L.n_dofs;
    const size_t g = dot_partials(n);
    NNMG_NV_DISPATCH(L.ncomp, nr, {
        hipLaunchKernelGGL((gather_dot_kernel<NC, NR>), dim3((unsigned)g), dim3(kRed), 0, s, n, L.inv_off(NNMG_FP64),
                           elem, contrib_plane(L), p, q, partial);
    });
    launch_sum_partials(partial, g, out, s, nr, kScal, scal, scalar_op);
    NNMG_HIP(hipGetLastError());
}

}  // namespace nnmg
