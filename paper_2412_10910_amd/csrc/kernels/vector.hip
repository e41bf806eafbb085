// Vector kernels of the smoother, the V-cycle and CG, and the dense
// float64 coarse solve.
//
// The Chebyshev-Jacobi smoother (paper §4: point Jacobi inside a degree-3
// Chebyshev iteration) is the three-term recurrence of the Chebyshev
// semi-iteration on D^{-1} A (Saad, Iterative Methods for Sparse Linear
// Systems, Alg. 12.1); every step fuses residual, direction and solution
// updates into one pass and clears the operator output buffer for the next
// product.
#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

static dim3 grid_for(size_t n, int threads = 256, size_t cap = 1 << 20) {
    size_t g = (n + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return dim3((unsigned)g);
}

#define NNMG_NR_DISPATCH(nr, ...)                                    \
    switch (nr) {                                                    \
        case 1: { constexpr int NR = 1; __VA_ARGS__; } break;               \
        case 2: { constexpr int NR = 2; __VA_ARGS__; } break;               \
        case 3: { constexpr int NR = 3; __VA_ARGS__; } break;               \
        case 4: { constexpr int NR = 4; __VA_ARGS__; } break;               \
        case 5: { constexpr int NR = 5; __VA_ARGS__; } break;               \
        case 6: { constexpr int NR = 6; __VA_ARGS__; } break;               \
        case 7: { constexpr int NR = 7; __VA_ARGS__; } break;               \
        case 8: { constexpr int NR = 8; __VA_ARGS__; } break;               \
        default: fail(NNMG_ERR_INVALID_ARG, "number of right-hand sides"); \
    }

template <class T>
__global__ void fill_kernel(T* __restrict__ x, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = T(0);
}

void launch_fill(void* x, size_t n, int prec, hipStream_t s) {
    if (n == 0) return;
    if (prec == NNMG_FP64)
        hipLaunchKernelGGL(fill_kernel<double>, grid_for(n), dim3(256), 0, s, (double*)x, n);
    else
        hipLaunchKernelGGL(fill_kernel<float>, grid_for(n), dim3(256), 0, s, (float*)x, n);
    NNMG_HIP(hipGetLastError());
}

template <class A, class B>
__global__ void cast_kernel(const A* __restrict__ a, B* __restrict__ b, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = (B)a[i];
}

void launch_cast_64_to_32(const double* a, float* b, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((cast_kernel<double, float>), grid_for(n), dim3(256), 0, s, a, b, n);
    NNMG_HIP(hipGetLastError());
}

void launch_cast_32_to_64(const float* a, double* b, size_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((cast_kernel<float, double>), grid_for(n), dim3(256), 0, s, a, b, n);
    NNMG_HIP(hipGetLastError());
}

// dst = src on the listed vector DoFs, for nr interleaved right-hand sides
template <class T>
__global__ void copy_idx_kernel(const int32_t* __restrict__ idx, size_t n, int nr, const T* __restrict__ src,
                                T* __restrict__ dst) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n * (size_t)nr) {
        const size_t v = (size_t)idx[i / nr] * nr + i % nr;
        dst[v] = src[v];
    }
}

void launch_copy_constrained(const int32_t* idx, size_t n, const void* src, void* dst, int prec, hipStream_t s,
                             int nr) {
    if (n == 0) return;
    const dim3 g((unsigned)((n * (size_t)nr + 255) / 256));
    if (prec == NNMG_FP64)
        hipLaunchKernelGGL(copy_idx_kernel<double>, g, dim3(256), 0, s, idx, n, nr, (const double*)src,
                           (double*)dst);
    else
        hipLaunchKernelGGL(copy_idx_kernel<float>, g, dim3(256), 0, s, idx, n, nr, (const float*)src, (float*)dst);
    NNMG_HIP(hipGetLastError());
}

template <class T>
__global__ void set_idx_kernel(const int32_t* __restrict__ idx, size_t n, T v, T* __restrict__ dst) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = v;
}

void launch_set_constrained(const int32_t* idx, size_t n, double v, void* dst, int prec, hipStream_t s) {
    if (n == 0) return;
    const dim3 g((unsigned)((n + 255) / 256));
    if (prec == NNMG_FP64)
        hipLaunchKernelGGL(set_idx_kernel<double>, g, dim3(256), 0, s, idx, n, v, (double*)dst);
    else
        hipLaunchKernelGGL(set_idx_kernel<float>, g, dim3(256), 0, s, idx, n, (float)v, (float*)dst);
    NNMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Chebyshev smoother steps
// ---------------------------------------------------------------------------
// n values; dinv is per vector DoF, shared by the NR interleaved right-hand sides
template <int NR, class T>
__global__ void cheb_first_zero_kernel(size_t n, const T* __restrict__ f, const T* __restrict__ dinv,
                                       T* __restrict__ x, T c0) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = dinv[NR == 1 ? i : i / NR] * f[i] * c0;
}

// the same first step on a float32 cycle whose right-hand side arrives in
// float64: f32 = (float) f64 is stored for the later steps and used at once
template <int NR>
__global__ void cast_cheb_first_zero_kernel(size_t n, const double* __restrict__ f64, float* __restrict__ f32,
                                            const float* __restrict__ dinv, float* __restrict__ x, float c0) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float f = (float)f64[i];
        f32[i] = f;
        x[i] = dinv[NR == 1 ? i : i / NR] * f * c0;
    }
}

void launch_cast_cheb_first_zero(size_t n, const double* f64, float* f32, const float* dinv, float* x, double c0,
                                 hipStream_t s, int nr) {
    if (n == 0) return;
    const size_t nv = n * (size_t)nr;
    NNMG_NR_DISPATCH(nr, {
        hipLaunchKernelGGL((cast_cheb_first_zero_kernel<NR>), grid_for(nv), dim3(256), 0, s, nv, f64, f32, dinv, x,
                           (float)c0);
    });
    NNMG_HIP(hipGetLastError());
}

void launch_cheb_first_zero(int prec, size_t n, const void* f, const void* dinv, void* x, double c0,
                            hipStream_t s, int nr) {
    if (n == 0) return;
    const size_t nv = n * (size_t)nr;
    NNMG_NR_DISPATCH(nr, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((cheb_first_zero_kernel<NR, double>), grid_for(nv), dim3(256), 0, s, nv,
                               (const double*)f, (const double*)dinv, (double*)x, c0);
        else
            hipLaunchKernelGGL((cheb_first_zero_kernel<NR, float>), grid_for(nv), dim3(256), 0, s, nv,
                               (const float*)f, (const float*)dinv, (float*)x, (float)c0);
    });
    NNMG_HIP(hipGetLastError());
}

// mode: kChebFirst, kChebDIsX, kChebLast (the same step as the gathering one)
template <int NR, class T>
__global__ void cheb_step_kernel(size_t n, const T* __restrict__ f, T* __restrict__ ax, const T* __restrict__ dinv,
                                 T* __restrict__ x, T* __restrict__ d, T c1, T c2, int mode) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const T r = f[i] - ax[i];
        ax[i] = T(0);
        const T xi = x[i];
        const T dp = (mode & kChebFirst) ? T(0) : ((mode & kChebDIsX) ? xi : d[i]);
        const T dr = c2 * (dinv[NR == 1 ? i : i / NR] * r);
        const T dn = (mode & kChebFirst) ? dr : c1 * dp + dr;
        if (!(mode & kChebLast)) d[i] = dn;
        x[i] = xi + dn;
    }
}

void launch_cheb_step(int prec, size_t n, const void* f, void* ax, const void* dinv, void* x, void* d, double c1,
                      double c2, int mode, hipStream_t s, int nr) {
    if (n == 0) return;
    const size_t nv = n * (size_t)nr;
    NNMG_NR_DISPATCH(nr, {
        if (prec == NNMG_FP64)
            hipLaunchKernelGGL((cheb_step_kernel<NR, double>), grid_for(nv), dim3(256), 0, s, nv, (const double*)f,
                               (double*)ax, (const double*)dinv, (double*)x, (double*)d, c1, c2, mode);
        else
            hipLaunchKernelGGL((cheb_step_kernel<NR, float>), grid_for(nv), dim3(256), 0, s, nv, (const float*)f,
                               (float*)ax, (const float*)dinv, (float*)x, (float*)d, (float)c1, (float)c2, mode);
    });
    NNMG_HIP(hipGetLastError());
}

template <class T>
__global__ void residual_kernel(size_t n, const T* __restrict__ f, T* __restrict__ ax, T* __restrict__ r) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        r[i] = f[i] - ax[i];
        ax[i] = T(0);
    }
}

void launch_residual(int prec, size_t n, const void* f, void* ax, void* r, hipStream_t s) {
    if (n == 0) return;
    if (prec == NNMG_FP64)
        hipLaunchKernelGGL(residual_kernel<double>, grid_for(n), dim3(256), 0, s, n, (const double*)f, (double*)ax,
                           (double*)r);
    else
        hipLaunchKernelGGL(residual_kernel<float>, grid_for(n), dim3(256), 0, s, n, (const float*)f, (float*)ax,
                           (float*)r);
    NNMG_HIP(hipGetLastError());
}


__global__ void lincomb_kernel(size_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

void launch_lincomb(size_t n, double a, const double* x, double b, double* y, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(lincomb_kernel, grid_for(n), dim3(256), 0, s, n, a, x, b, y);
    NNMG_HIP(hipGetLastError());
}

// SplitMix64 (Steele, Lea, Flood 2014): z = seed + (i+1) * golden gamma, then
// the mixing function; mapped to [-1, 1) from the top 53 bits.
__global__ void splitmix_kernel(double* __restrict__ v, const int32_t* __restrict__ dm_unused, size_t n,
                                uint64_t seed) {
    (void)dm_unused;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        v[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

void launch_splitmix_vector(double* v, const uint8_t* unused, size_t n, uint64_t seed, hipStream_t s) {
    (void)unused;
    if (n == 0) return;
    hipLaunchKernelGGL(splitmix_kernel, grid_for(n), dim3(256), 0, s, v, nullptr, n, seed);
    NNMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// float64 reductions, two stages with a fixed partition: deterministic.
// With NR interleaved right-hand sides the lanes stride over the rows (vector
// DoFs) exactly as for one right-hand side and keep NR sums, so that each
// right-hand side is reduced in the order it would be on its own; the first
// stage writes partial[block][NR], the second reduces each column.
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;
constexpr size_t kRedMaxBlocks = 1024;

size_t dot_partials(size_t n) {
    size_t g = (n + kRedThreads * 4 - 1) / (kRedThreads * 4);
    if (g > kRedMaxBlocks) g = kRedMaxBlocks;
    if (g == 0) g = 1;
    return g;
}

// block sums of v[0..NR), written by thread r < NR to out[r * ostride]
template <int NR>
__device__ inline void block_sums(const double (&v)[NR], double* out, size_t ostride) {
    __shared__ double sh[NR][kRedThreads / kWave];
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double a = v[r];
        for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
        if (l == 0) sh[r][w] = a;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
        double s = 0.0;
        for (int i = 0; i < kRedThreads / kWave; ++i) s += sh[threadIdx.x][i];
        out[threadIdx.x * ostride] = s;
    }
}

template <int NR>
__global__ __launch_bounds__(kRedThreads) void dot_stage1(const double* __restrict__ a, const double* __restrict__ b,
                                                          size_t n, double* __restrict__ partial) {
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] += a[i * NR + r] * b[i * NR + r];
    }
    block_sums<NR>(s, partial + blockIdx.x * NR, 1);
}

// op 0: alpha = rz / pq;  op 1: beta = rz_new / rz, rz = rz_new, with `fresh`
// the sum just formed (pq, or rz_new).  A right-hand side that is no longer
// active gets alpha = beta = 0 and keeps its iterate.  So does one whose pq is
// not positive or whose alpha is not finite (a CG breakdown): its last good
// iterate stays in x while the host reports the breakdown.
__device__ inline void cg_scalar_op(double* c, int op, double fresh) {
    const bool on = c[7] != 0.0;
    if (op == 0) {
        const double a = c[0] / fresh;
        c[2] = (on && fresh > 0.0 && isfinite(a)) ? a : 0.0;
    } else {
        c[5] = on ? fresh / c[0] : 0.0;
        c[0] = fresh;
    }
}

// out[r * ostride] = sum over the m blocks of partial[block][r]; one block per
// column, the same order as block_sums.  op >= 0: the thread that holds the
// sum also forms the CG scalar waiting for it (cg_scalar_op on the scalars of
// right-hand side r), which saves a launch per use.
__global__ __launch_bounds__(kRedThreads) void sum_stage2(const double* __restrict__ partial, size_t m, int nr,
                                                          double* out, size_t ostride, double* scal, int op) {
    __shared__ double sh[kRedThreads / kWave];
    const int r = blockIdx.x;
    double a = 0.0;
    for (size_t i = threadIdx.x; i < m; i += blockDim.x) a += partial[i * nr + r];
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kRedThreads / kWave; ++i) t += sh[i];
        out[r * ostride] = t;
        if (op >= 0) cg_scalar_op(scal + r * kScal, op, t);
    }
}

void launch_sum_partials(const double* partial, size_t m, double* out, hipStream_t s, int nr, size_t ostride,
                         double* scal, int op) {
    if (op >= 0 && (scal == nullptr || ostride != (size_t)kScal)) fail(NNMG_ERR_INVALID_ARG, "CG scalar layout");
    hipLaunchKernelGGL(sum_stage2, dim3((unsigned)nr), dim3(kRedThreads), 0, s, partial, m, nr, out, ostride, scal,
                       op);
    NNMG_HIP(hipGetLastError());
}

// z = (double) z32 and the block partial sums of r . z, in dot_stage1's order
template <int NR>
__global__ __launch_bounds__(kRedThreads) void cast_dot_stage1(const double* __restrict__ r,
                                                               const float* __restrict__ z32,
                                                               double* __restrict__ z, size_t n,
                                                               double* __restrict__ partial) {
    double s[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) s[k] = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double zv = (double)z32[i * NR + k];
            if (z) z[i * NR + k] = zv;
            s[k] += r[i * NR + k] * zv;
        }
    }
    block_sums<NR>(s, partial + blockIdx.x * NR, 1);
}

void launch_cast_dot(const double* r, const float* z32, double* z, size_t n, double* partial, double* out,
                     hipStream_t s, int nr, size_t ostride, double* scal, int op) {
    const size_t g = dot_partials(n);
    NNMG_NR_DISPATCH(nr, {
        hipLaunchKernelGGL((cast_dot_stage1<NR>), dim3((unsigned)g), dim3(kRedThreads), 0, s, r, z32, z, n,
                           partial);
    });
    launch_sum_partials(partial, g, out, s, nr, ostride, scal, op);
}

void launch_dot(const double* a, const double* b, size_t n, double* partial, double* out, hipStream_t s, int nr,
                size_t ostride, double* scal, int op) {
    const size_t g = dot_partials(n);
    NNMG_NR_DISPATCH(nr, {
        hipLaunchKernelGGL((dot_stage1<NR>), dim3((unsigned)g), dim3(kRedThreads), 0, s, a, b, n, partial);
    });
    launch_sum_partials(partial, g, out, s, nr, ostride, scal, op);
}

// CG scalars of right-hand side r at scal + r * kScal:
// [0] rz, [1] pq, [2] alpha, [3] rr, [4] rz_new, [5] beta, [6] b.b, [7] active (1 or 0)
// r -= alpha q and the partial sums of r.r; the iterate's update x += alpha p
// waits for the next direction update (or cg_finish), which reads p anyway
template <int NR>
__global__ __launch_bounds__(kRedThreads) void cg_update_stage1(size_t n, double* __restrict__ r,
                                                                const double* __restrict__ q,
                                                                const double* __restrict__ scal,
                                                                double* __restrict__ partial) {
    double alpha[NR], s[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        alpha[k] = scal[k * kScal + 2];
        s[k] = 0.0;
    }
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            // alpha = 0 (frozen or broken down): r is left as it is, even
            // where q is not finite
            const size_t v = i * NR + k;
            double rn = r[v];
            if (alpha[k] != 0.0) {
                rn -= alpha[k] * q[v];
                r[v] = rn;
            }
            s[k] += rn * rn;
        }
    }
    block_sums<NR>(s, partial + blockIdx.x * NR, 1);
}

void launch_cg_update(size_t n, double* r, const double* q, const double* scal, double* partial, double* rr_out,
                      hipStream_t s, int nr) {
    const size_t g = dot_partials(n);
    NNMG_NR_DISPATCH(nr, {
        hipLaunchKernelGGL((cg_update_stage1<NR>), dim3((unsigned)g), dim3(kRedThreads), 0, s, n, r, q, scal,
                           partial);
    });
    launch_sum_partials(partial, g, rr_out, s, nr, kScal);
}

// x += alpha p (the previous iteration's update, alpha = 0 leaving x as it
// is), then p = z + beta p; a float32 z (the float32 V-cycle's result) is
// widened exactly here.  z = nullptr: only the update of x (the end of a solve).
template <int NR, class Z>
__global__ void cg_direction_kernel(size_t n, const Z* __restrict__ z, double* __restrict__ p,
                                    double* __restrict__ x, const double* __restrict__ scal) {
    double alpha[NR], beta[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        alpha[k] = scal[k * kScal + 2];
        beta[k] = scal[k * kScal + 5];
    }
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const size_t v = i * NR + k;
            const double pv = p[v];
            if (alpha[k] != 0.0) x[v] += alpha[k] * pv;
            if (z) p[v] = (double)z[v] + beta[k] * pv;
        }
    }
}

void launch_cg_direction(size_t n, const double* z, double* p, double* x, const double* scal, hipStream_t s,
                         int nr) {
    if (n == 0) return;
    NNMG_NR_DISPATCH(nr, {
        hipLaunchKernelGGL((cg_direction_kernel<NR, double>), grid_for(n), dim3(256), 0, s, n, z, p, x, scal);
    });
    NNMG_HIP(hipGetLastError());
}

void launch_cg_direction32(size_t n, const float* z32, double* p, double* x, const double* scal, hipStream_t s,
                           int nr) {
    if (n == 0) return;
    NNMG_NR_DISPATCH(nr, {
        hipLaunchKernelGGL((cg_direction_kernel<NR, float>), grid_for(n), dim3(256), 0, s, n, z32, p, x, scal);
    });
    NNMG_HIP(hipGetLastError());
}

__global__ void jacobi_kernel(size_t n, const double* __restrict__ dinv, const double* __restrict__ r,
                              double* __restrict__ z) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        z[i] = dinv[i] * r[i];
}

void launch_jacobi(size_t n, const double* dinv, const double* r, double* z, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(jacobi_kernel, grid_for(n), dim3(256), 0, s, n, dinv, r, z);
    NNMG_HIP(hipGetLastError());
}

// y += sign * scal[idx] * x
__global__ void axpy_kernel(size_t n, double sign, const double* __restrict__ scal, int idx,
                            const double* __restrict__ x, double* __restrict__ y) {
    const double a = sign * scal[idx];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

void launch_axpy(size_t n, double a_sign, const double* scal_a, int idx, const double* x, double* y,
                 hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(axpy_kernel, grid_for(n), dim3(256), 0, s, n, a_sign, scal_a, idx, x, y);
    NNMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// dense coarse solve: explicit inverse of the unconstrained block
// ---------------------------------------------------------------------------
// Coarse solve step on the unconstrained block, one 256-lane block per row,
// for NR interleaved right-hand sides at once (the row is read once):
//   y_i,r = base_i,r + sign * sum_j M_ij v_j,r,
// with v_j,r = V[vidx[j] NR + r] (or V[j NR + r]) and base_i,r = B[bidx[i] NR + r]
// (or B[i NR + r], or 0), stored to O[oidx[i] NR + r] (or O[i NR + r]) in O's
// precision.  Rows are read coalesced; each row sum is reduced in a fixed
// order, the same for every NR.
template <int NR, class TV, class TB, class TO>
__global__ __launch_bounds__(256) void coarse_gemv_kernel(const double* __restrict__ M, size_t m,
                                                          const TV* __restrict__ V, const int32_t* __restrict__ vidx,
                                                          const TB* __restrict__ B, const int32_t* __restrict__ bidx,
                                                          double sign, TO* __restrict__ O,
                                                          const int32_t* __restrict__ oidx) {
    __shared__ double part[NR][256 / kWave];
    const size_t row = blockIdx.x;
    const double* a = M + row * m;
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] = 0.0;
    for (size_t j = threadIdx.x; j < m; j += 256) {
        const double mj = a[j];
        const size_t vj = (vidx ? (size_t)vidx[j] : j) * NR;
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] += mj * (double)V[vj + r];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double v = s[r];
        for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
        if (threadIdx.x % kWave == 0) part[r][threadIdx.x / kWave] = v;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
        const int r = threadIdx.x;
        double t = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) t += part[r][w];
        const double b = B ? (double)B[(bidx ? (size_t)bidx[row] : row) * NR + r] : 0.0;
        O[(oidx ? (size_t)oidx[row] : row) * NR + r] = (TO)(b + sign * t);
    }
}

template <class TV, class TB, class TO>
static void coarse_gemv_t(const double* M, size_t m, const void* V, const int32_t* vidx, const void* B,
                          const int32_t* bidx, double sign, void* O, const int32_t* oidx, int nr, hipStream_t s) {
    NNMG_NR_DISPATCH(nr, {
        hipLaunchKernelGGL((coarse_gemv_kernel<NR, TV, TB, TO>), dim3((unsigned)m), dim3(256), 0, s, M, m,
                           (const TV*)V, vidx, (const TB*)B, bidx, sign, (TO*)O, oidx);
    });
}

void launch_coarse_gemv(const double* M, size_t m, const void* V, int vprec, const int32_t* vidx, const void* B,
                        int bprec, const int32_t* bidx, double sign, void* O, int oprec, const int32_t* oidx,
                        hipStream_t s, int nr) {
    if (m == 0) return;
    const bool v64 = vprec == NNMG_FP64, b64 = bprec == NNMG_FP64, o64 = oprec == NNMG_FP64;
    if (v64 && b64 && o64) coarse_gemv_t<double, double, double>(M, m, V, vidx, B, bidx, sign, O, oidx, nr, s);
    else if (!v64 && b64 && o64) coarse_gemv_t<float, double, double>(M, m, V, vidx, B, bidx, sign, O, oidx, nr, s);
    else if (v64 && !b64 && o64) coarse_gemv_t<double, float, double>(M, m, V, vidx, B, bidx, sign, O, oidx, nr, s);
    else if (v64 && b64 && !o64) coarse_gemv_t<double, double, float>(M, m, V, vidx, B, bidx, sign, O, oidx, nr, s);
    else if (!v64 && !o64 && B == nullptr)
        coarse_gemv_t<float, double, float>(M, m, V, vidx, nullptr, nullptr, sign, O, oidx, nr, s);
    else fail(NNMG_ERR_INVALID_ARG, "coarse_gemv precision combination");
    NNMG_HIP(hipGetLastError());
}

// in-place Gauss-Jordan inversion of a symmetric positive definite matrix
// (no pivoting needed: every pivot is a Schur-complement diagonal entry)
__global__ void gj_save_kernel(const double* __restrict__ M, size_t m, size_t k, double* __restrict__ row,
                               double* __restrict__ col) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < m) {
        row[i] = M[k * m + i];
        col[i] = M[i * m + k];
    }
}

__global__ void gj_update_kernel(double* __restrict__ M, size_t m, size_t k, const double* __restrict__ row,
                                 const double* __restrict__ col) {
    const size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t i = blockIdx.y;
    if (j >= m) return;
    const double piv = row[k];
    double v;
    if (i == k && j == k)
        v = 1.0 / piv;
    else if (i == k)
        v = row[j] / piv;
    else if (j == k)
        v = -col[i] / piv;
    else
        v = M[i * m + j] - col[i] * row[j] / piv;
    M[i * m + j] = v;
}

void launch_gauss_jordan(double* M, size_t m, double* rowbuf, double* colbuf, hipStream_t s) {
    if (m == 0) return;
    const dim3 g1((unsigned)((m + 255) / 256));
    const dim3 g2((unsigned)((m + 255) / 256), (unsigned)m);
    for (size_t k = 0; k < m; ++k) {
        hipLaunchKernelGGL(gj_save_kernel, g1, dim3(256), 0, s, M, m, k, rowbuf, colbuf);
        hipLaunchKernelGGL(gj_update_kernel, g2, dim3(256), 0, s, M, m, k, rowbuf, colbuf);
    }
    NNMG_HIP(hipGetLastError());
}

__global__ void column_kernel(const int32_t* __restrict__ idx, size_t m, const double* __restrict__ ax,
                              double* __restrict__ M, size_t col) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < m) M[i * m + col] = ax[idx[i]];
}

void launch_column_from_unit(const int32_t* free_idx, size_t m, const double* ax, double* M, size_t col,
                             hipStream_t s) {
    if (m == 0) return;
    hipLaunchKernelGGL(column_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, free_idx, m, ax, M, col);
    NNMG_HIP(hipGetLastError());
}

__global__ void set_unit_kernel(double* x, int64_t idx, double val) {
    if (threadIdx.x == 0) x[idx] = val;
}

void launch_set_unit(double* x, size_t n, int64_t idx, double val, hipStream_t s) {
    (void)n;
    hipLaunchKernelGGL(set_unit_kernel, dim3(1), dim3(64), 0, s, x, idx, val);
    NNMG_HIP(hipGetLastError());
}

}  // namespace nnmg
