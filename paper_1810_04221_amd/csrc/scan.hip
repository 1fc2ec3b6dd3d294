// Exclusive prefix sum of int32 for gfx950: tiles of 2048 items (256 threads x
// 8), a single-workgroup scan of the tile totals, then a fix-up pass.  Used to
// number aggregates by their smallest member (Algorithm 2) and to turn coarse
// row counts into row pointers.
#include "device.h"
#include "internal.h"

namespace bcm {

namespace {

constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;

// inclusive scan of one value per lane over the 64 lanes of a wave
__device__ __forceinline__ int wave_incl(int x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    return x;
}

// exclusive scan over the block of one value per thread; *total gets the sum
__device__ __forceinline__ int block_excl(int x, int *total) {
    __shared__ int wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int inc = wave_incl(x);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

__global__ void __launch_bounds__(kBlock)
k_scan_tiles(const int *__restrict__ in, int *__restrict__ out, int n, int *__restrict__ tsum) {
    const size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kItems;
    int v[kItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + k;
        v[k] = i < (size_t)n ? in[i] : 0;
        s += v[k];
    }
    int tot;
    int run = block_excl(s, &tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + k;
        if (i < (size_t)n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_totals(int *__restrict__ tsum, int nt, int *__restrict__ total) {
    int carry = 0;
    for (int b0 = 0; b0 < nt; b0 += kBlock) {
        const int i = b0 + threadIdx.x;
        const int x = i < nt ? tsum[i] : 0;
        int tot;
        const int ex = block_excl(x, &tot);
        if (i < nt) tsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kBlock) k_scan_add(int *__restrict__ out, int n, const int *__restrict__ tsum) {
    const int add = tsum[blockIdx.x];
    const size_t base = (size_t)blockIdx.x * kTile;
    for (int k = threadIdx.x; k < kTile; k += kBlock) {
        const size_t i = base + k;
        if (i < (size_t)n) out[i] += add;
    }
}

// Whole scan in one workgroup of 1024 threads for n <= kScanSmall: thread t
// owns items [t K, t K + K), K = ceil(n / 1024).
constexpr int kScanSmall = 16384;

__global__ void __launch_bounds__(1024) k_scan_single(const int *__restrict__ in, int *__restrict__ out, int n,
                                                        int *__restrict__ total) {
    __shared__ int wsum[16];
    const int K = (n + 1023) / 1024;
    const int b = threadIdx.x * K;
    int v[kScanSmall / 1024];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanSmall / 1024; ++k) {
        v[k] = (k < K && b + k < n) ? in[b + k] : 0;
        s += v[k];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int inc = wave_incl(s);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    int run = base + inc - s;
#pragma unroll
    for (int k = 0; k < kScanSmall / 1024; ++k) {
        if (k < K && b + k < n) out[b + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) *total = tot;
}

}  // namespace

size_t scan_tmp_bytes(int n) { return sizeof(int) * (size_t)((n + kTile - 1) / kTile + 1); }

void scan_exclusive(hipStream_t s, const int *in, int *out, int n, int *total_dev, void *tmp) {
    const int nt = (n + kTile - 1) / kTile;
    int *tsum = static_cast<int *>(tmp);
    if (nt == 0) {
        launch_fill_i32(s, 1, total_dev, 0);
        return;
    }
    if (n <= kScanSmall) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, in, out, n, total_dev);
        return;
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kBlock), 0, s, in, out, n, tsum);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, s, tsum, nt, total_dev);
    hipLaunchKernelGGL(k_scan_add, dim3(nt), dim3(kBlock), 0, s, out, n, tsum);
}

}  // namespace bcm
