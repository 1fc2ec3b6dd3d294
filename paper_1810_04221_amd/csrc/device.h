// Device-side helpers shared by the gfx950 kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcm {

constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels

// Workgroups are handed to the eight XCDs of the chip in turn (workgroup b runs on
// XCD b % 8).  This remaps the hardware index so that every XCD gets one
// contiguous range of logical blocks: neighbouring rows, whose gathered vector
// entries overlap, then share the same L2.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = b % X, i = b / X;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Sum over an aligned group of G lanes (G a power of two <= 64) of one wave.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// Orders LDS accesses of the lanes of one wave: everything written before is
// visible to every lane of the wave after.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide sums of K doubles; the result is valid in thread 0.  The order of
// additions depends only on the block size.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = group_sum<64>(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k * 16 + wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = lds[k * 16];
            for (int w = 1; w < nw; ++w) s += lds[k * 16 + w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// s[k] += partials[k * nb + bk] over bk = threadIdx.x, + blockDim.x, ... in
// that order (whatever U); U block indices' loads are issued before any is
// added, so the partials (just written by another kernel) cost few memory
// round trips.
template <int K, int U = 8>
__device__ __forceinline__ void add_partials(double (&s)[K], const double *__restrict__ partials, int nb) {
    for (int b0 = threadIdx.x; b0 < nb; b0 += U * blockDim.x) {
        double t[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int bk = b0 + u * blockDim.x;
#pragma unroll
            for (int k = 0; k < K; ++k) t[u][k] = bk < nb ? partials[(size_t)k * nb + bk] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (b0 + u * blockDim.x < nb) s[k] += t[u][k];
    }
}

// Block partial sums: thread 0 of every block stores the block's K sums at
// partials[k * gridDim.x + blockIdx.x].  No inter-block synchronisation: a
// following single-block kernel adds the partials in block order, so the
// result depends only on the grid and block sizes, never on timing.
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double *partials) {
    __shared__ double lds[K * 16];
    block_sum<K>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) partials[(size_t)k * gridDim.x + blockIdx.x] = v[k];
}

// The flexible-CG stop test on rr = ||r||^2 of the update just run: stores it
// in scal[4], counts the iteration in scal[11], and ends the loop (scal[10] =
// 1) when rr <= scal[12] (= tol^2 ||b||^2), the count reaches scal[13]
// (itmax) or rr is not finite (then also scal[6] = 1, breakdown).  Clears
// scal[7], the update's mark of partials not yet taken.  True when it ended.
__device__ __forceinline__ bool stop_norm(double rr, double *scal) {
    scal[4] = rr;
    const double it = scal[11] + 1.0;
    scal[11] = it;
    bool end = false;
    if (!isfinite(rr)) { scal[6] = 1.0; end = true; }
    else if (rr <= scal[12] || it >= scal[13]) end = true;
    if (end) scal[10] = 1.0;
    scal[7] = 0.0;
    return end;
}

// The stop test taken by workgroup 0 of the first kernel of a cycle (all its
// threads call it, before any returns): when the update left partials not yet
// taken (scal[7] != 0), adds its nb partials in the order of the one-block
// finalize with kBlock threads and applies stop_norm.  True when the loop has
// ended (scal[10] set now or before): the workgroup then skips its work.  The
// kernel's other workgroups run on; the kernels after it see scal[10].
__device__ __forceinline__ bool stop_test(const double *__restrict__ part, double *scal, int nb) {
    __shared__ double lds[16];
    __shared__ int end;
    if (scal[10] != 0.0) return true;
    if (scal[7] == 0.0) return false;
    double s[1] = {0.0};
    add_partials<1>(s, part, nb);
    block_sum<1>(s, lds);
    if (threadIdx.x == 0) end = stop_norm(s[0], scal) ? 1 : 0;
    __syncthreads();
    return end != 0;
}

}  // namespace bcm
