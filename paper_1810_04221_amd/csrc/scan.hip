// Exclusive prefix sum of int32 for gfx950: up to 16384 items in one
// workgroup; longer inputs in tiles of 2048 items (256 threads x 8), a pass of
// tile sums, then one pass in which every tile adds the sums before it and
// scans itself.  Used to number aggregates by their smallest member
// (Algorithm 2) and to turn coarse row counts into row pointers.
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

// largest value over a workgroup of kBlock threads (valid in every thread)
__device__ __forceinline__ int block_max(int x) {
    __shared__ int wmax[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = x;
    __syncthreads();
    int m = wmax[0];
    for (int w = 1; w < kBlock / 64; ++w) m = max(m, wmax[w]);
    __syncthreads();
    return m;
}

// Tile sums (and largest items) of the input, tiles of kTile items.
__global__ void __launch_bounds__(kBlock)
k_scan_reduce(const int *in, int n, int *__restrict__ tsum, int *__restrict__ tmax) {
    const size_t base = (size_t)blockIdx.x * kTile + (size_t)threadIdx.x * kItems;
    int s = 0, mx = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + k;
        const int v = i < (size_t)n ? in[i] : 0;
        s += v;
        mx = max(mx, v);
    }
    int tot;
    (void)block_excl(s, &tot);
    if (tmax) mx = block_max(mx);
    if (threadIdx.x == 0) {
        tsum[blockIdx.x] = tot;
        if (tmax) tmax[blockIdx.x] = mx;
    }
}

// Tile b: its offset is the sum of the tile sums before it (added by this
// block itself, in a fixed order), then the tile is scanned and written.  The
// last tile also writes the total and the largest item.  In place is fine: an
// item is read and written by the same thread, and no other block reads it.
__global__ void __launch_bounds__(kBlock)
k_scan_apply(const int *in, int *out, int n, const int *__restrict__ tsum, int nt, int *__restrict__ total,
             const int *__restrict__ tmax, int *__restrict__ max_out) {
    const int b = blockIdx.x;
    const bool last = b == nt - 1;
    int pre = 0, mx = 0;
    for (int i = threadIdx.x; i < (last ? nt : b); i += kBlock) {
        if (i < b) pre += tsum[i];
        if (last && tmax) mx = max(mx, tmax[i]);
    }
    int ptot;
    (void)block_excl(pre, &ptot);
    const size_t base = (size_t)b * kTile + (size_t)threadIdx.x * kItems;
    int v[kItems];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + k;
        v[k] = i < (size_t)n ? in[i] : 0;
        sum += v[k];
    }
    int tot;
    int run = ptot + block_excl(sum, &tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + k;
        if (i < (size_t)n) out[i] = run;
        run += v[k];
    }
    if (last) {
        if (tmax) mx = block_max(mx);
        if (threadIdx.x == 0) {
            *total = ptot + tot;
            if (max_out) *max_out = mx;
        }
    }
}

// Whole scan in one workgroup of 1024 threads for n <= kScanSmall: the items
// are loaded with contiguous wave accesses into LDS, then thread t scans its
// kPer consecutive items (t * kPer ...) in registers, the thread totals are
// scanned across the wave's lanes and then across the 16 waves, and the
// results go back through LDS to contiguous stores.  LDS rows are padded by
// one word per kPer items, so the lanes of a wave reading their own runs hit
// distinct banks.  In place is fine: every item is loaded before any is stored.
constexpr int kScanSmall = 16384, kPer = kScanSmall / 1024;

__device__ __forceinline__ int pad_idx(int i) { return i + i / kPer; }

__global__ void __launch_bounds__(1024) k_scan_single(const int *in, int *out, int n, int *__restrict__ total,
                                                     int *__restrict__ max_out) {
    __shared__ int sh[kScanSmall + kScanSmall / kPer];
    __shared__ int wsum[16], wmax[16];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    int mx = 0;
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
        const int e = c * 1024 + t;
        const int x = e < n ? in[e] : 0;
        mx = max(mx, x);
        sh[pad_idx(e)] = x;
    }
    if (max_out) {
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) wmax[wid] = mx;
    }
    __syncthreads();
    int v[kPer];
    int run = 0;
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
        v[c] = run;  // exclusive within the thread's run
        run += sh[pad_idx(t * kPer + c)];
    }
    const int inc = wave_incl(run);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int base = inc - run, tot = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
#pragma unroll
    for (int c = 0; c < kPer; ++c) sh[pad_idx(t * kPer + c)] = base + v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
        const int e = c * 1024 + t;
        if (e < n) out[e] = sh[pad_idx(e)];
    }
    if (t == 0) {
        *total = tot;
        if (max_out) {
            for (int w = 1; w < 16; ++w) mx = max(mx, wmax[w]);
            *max_out = max(mx, wmax[0]);
        }
    }
}

}  // namespace

size_t scan_tmp_bytes(int n) { return 2 * sizeof(int) * (size_t)((n + kTile - 1) / kTile + 1); }

void scan_exclusive(hipStream_t s, const int *in, int *out, int n, int *total_dev, void *tmp, int *max_dev) {
    const int nt = (n + kTile - 1) / kTile;
    int *tsum = static_cast<int *>(tmp);
    int *tmax = max_dev ? tsum + nt + 1 : nullptr;
    if (nt == 0) {
        launch_fill_i32(s, 1, total_dev, 0);
        if (max_dev) launch_fill_i32(s, 1, max_dev, 0);
        return;
    }
    if (n <= kScanSmall) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, in, out, n, total_dev, max_dev);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nt), dim3(kBlock), 0, s, in, n, tsum, tmax);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kBlock), 0, s, in, out, n, tsum, nt, total_dev, tmax, max_dev);
}

}  // namespace bcm
