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

// Whole scan in one workgroup of 1024 threads for n <= kScanSmall.  Wave w owns
// C = kScanSmall / 1024 consecutive chunks of 64 items; every load and store of
// a wave is one contiguous 256-byte access (a single workgroup cannot afford
// strided ones).  Each chunk is scanned across the wave's lanes, chunk totals
// carry across the wave's chunks, then across the 16 waves.  In place is fine:
// an item is read and written by the same lane.
constexpr int kScanSmall = 16384;

__global__ void __launch_bounds__(1024) k_scan_single(const int *in, int *out, int n, int *__restrict__ total) {
    constexpr int C = kScanSmall / 1024;
    __shared__ int wsum[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int e = (wid * C + c) * 64 + lane;
        v[c] = e < n ? in[e] : 0;
    }
    int run = 0;  // the same in every lane of the wave
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int inc = wave_incl(v[c]);
        const int x = v[c];
        v[c] = run + inc - x;  // exclusive prefix within the wave's range
        run += __shfl(inc, 63, 64);
    }
    if (lane == 0) wsum[wid] = run;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int e = (wid * C + c) * 64 + lane;
        if (e < n) out[e] = base + v[c];
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
