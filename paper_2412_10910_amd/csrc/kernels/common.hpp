// Device-side helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nnmg {

constexpr int kWave = 64;  // CDNA wavefront width
constexpr int kXcd = 8;    // MI355X: 8 accelerator complex dies, one L2 each

// Workgroups are dispatched round-robin over the XCDs.  Remap the hardware
// block index so that each XCD works on one contiguous range of logical
// blocks: neighbouring cells share DoFs, and keeping them on one XCD keeps the
// shared vector entries in that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t q = nb / kXcd, r = nb % kXcd;
    const int64_t xcd = b % kXcd, local = b / kXcd;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// LDS hand-off between the lanes of a block.  A block of one wavefront needs
// no hardware barrier: LDS operations of a wavefront complete in issue order,
// so it is enough to keep the compiler from moving LDS accesses across this
// point.  Unlike a workgroup barrier this does not wait for outstanding
// global loads, which stay in flight across the LDS stages.
template <int WG>
__device__ __forceinline__ void block_sync() {
    if constexpr (WG == kWave) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <class T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
    // hardware float atomics in L2 (the library is built with -munsafe-fp-atomics)
    atomicAdd(p, v);
}

// constant 1D tables of the Q_k element in the kernel's precision, passed by value
template <int N, class T>
struct Tables {
    T S[N][N];   // S[q][a]  = phi_a(g_q)
    T DS[N][N];  // DS[q][a] = phi_a'(g_q)
    T D[N][N];   // D[q][p]  = psi_p'(g_q)
};

template <int N, class T>
struct NodeTable {
    T node[N];  // Gauss-Lobatto nodes on [0,1]
    T bary[N];  // 1 / prod_{m != a} (x_a - x_m)
};

// phi_a(x) for the Lagrange polynomials on the Gauss-Lobatto nodes, by
// prefix/suffix products of (x - x_m): phi_a = bary_a prod_{m != a} (x - x_m)
template <int N, class T>
__device__ __forceinline__ void lagrange_eval(const NodeTable<N, T>& nt, T x, T* phi) {
    T diff[N];
#pragma unroll
    for (int m = 0; m < N; ++m) diff[m] = x - nt.node[m];
    T pre[N];
    pre[0] = T(1);
#pragma unroll
    for (int m = 1; m < N; ++m) pre[m] = pre[m - 1] * diff[m - 1];
    T suf = T(1);
#pragma unroll
    for (int a = N - 1; a >= 0; --a) {
        phi[a] = nt.bary[a] * pre[a] * suf;
        suf *= diff[a];
    }
}

}  // namespace nnmg
