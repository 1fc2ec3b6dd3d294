// Slot-split sliced-ELL kernels for gfx950: the down leg's residual and the
// post-smoothing of the V-cycle (Algorithm 1) on levels whose rows are long
// but too few to fill the chip at one thread per row.  Included once, after
// sell_kernels.h (whose slice layout and helpers they share), inside the
// solve library's anonymous namespace.
#pragma once
#include "sell_kernels.h"

// ----------------------------------------------------------------------------
// Levels of long rows (slices averaging more than kWideSlots slots) with too
// few rows to fill the chip at one thread per row: each row's slots split over
// P waves of one workgroup.  The workgroup owns one 64-row
// slice; wave q sums slots q, q + P, q + 2P, ... of its lane's row (batches of
// kB loads issued together, as sell_slots), and the P partial sums are added
// in wave order through LDS.  P times as many waves in flight per row as one
// thread per row; each row's sum is taken in this fixed order.
// ----------------------------------------------------------------------------
constexpr int kParts = kBlock / kSlice;

template <int kB, bool Uni, typename V, typename S, typename I, typename F, bool NT = false>
__device__ __forceinline__ V sell_part(const S *a, const int *u, const I *c, int n, int i, int w, int q, F f) {
    V s = V(0);
    for (int k0 = q; k0 < w; k0 += kB * kParts) {
        S av[kB];
        V fv[kB];
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            const int k = min(k0 + t * kParts, w - 1);
            if (NT) av[t] = __builtin_nontemporal_load(&a[k * kSlice]);
            else av[t] = a[k * kSlice];
            if (Uni) {
                const int cc = i + u[k];
                fv[t] = f((unsigned)cc < (unsigned)n ? cc : i);
            } else {
                fv[t] = f(sell_col(c[k * kSlice], i));
            }
        }
#pragma unroll
        for (int t = 0; t < kB; ++t)
            if (k0 + t * kParts < w) s += (V)av[t] * fv[t];
    }
    return s;
}

// Wave q's part of row sl * 64 + lane (0 for rows past n).
template <typename V, typename S, typename I, int kB, typename F, bool NT = false>
__device__ __forceinline__ V sell_row_part(int n, const int *__restrict__ sp, const int *__restrict__ uni,
                                           const int *__restrict__ su, const I *__restrict__ sc,
                                           const S *__restrict__ sv, int sl, F f) {
    const int q = threadIdx.x / kSlice, lane = threadIdx.x % kSlice, i = sl * kSlice + lane;
    if (i >= n) return V(0);
    const int uf = uni[sl], beg = sp[sl], w = (sp[sl + 1] - beg) / kSlice;
    const S *a = sv + beg + lane;
    const int *u = su + beg / kSlice;
    const I *c = sc + beg + lane;
    if (uf) return sell_part<kB, true, V, S, I, F, NT>(a, u, c, n, i, w, q, f);
    return sell_part<kB, false, V, S, I, F, NT>(a, u, c, n, i, w, q, f);
}

// The P partial sums of each row of the slice, added in wave order (valid in wave 0).
template <typename V>
__device__ __forceinline__ V parts_sum(V s, V (&red)[kParts][kSlice]) {
    const int q = threadIdx.x / kSlice, lane = threadIdx.x % kSlice;
    red[q][lane] = s;
    __syncthreads();
    V t = red[0][lane];
#pragma unroll
    for (int r = 1; r < kParts; ++r) t += red[r][lane];
    __syncthreads();
    return t;
}

// NT: the values streamed non-temporally (Sell::stream; the slot-split
// smoother keeps them cached: streaming measured slower there).
template <typename V, typename VB, typename I, typename S, int kB, bool NT>
__global__ void __launch_bounds__(kBlock)
k_down_res_sell_p(int n, const int *__restrict__ sp, const int *__restrict__ uni, const int *__restrict__ su,
                  const I *__restrict__ sc, const S *__restrict__ sv, const V *__restrict__ dinv,
                  const V *__restrict__ p, const VB *__restrict__ b, V *__restrict__ pr, const V *__restrict__ y,
                  const double *__restrict__ done, StopTest st) {
    __shared__ V red[kParts][kSlice];
    if (st.part && blockIdx.x == 0) {
        if (stop_test(st.part, st.scal, st.nb)) return;
    } else if (done && *done != 0.0) return;
    const int sl = xcd_block(blockIdx.x, gridDim.x);
    const int i = sl * kSlice + (int)threadIdx.x % kSlice;
    V s;
    auto gy = [&](int j) { return y[j]; };
    auto gd = [&](int j) { return dinv[j] * (V)b[j]; };
    if (y) s = sell_row_part<V, S, I, kB, decltype(gy), NT>(n, sp, uni, su, sc, sv, sl, gy);
    else s = sell_row_part<V, S, I, kB, decltype(gd), NT>(n, sp, uni, su, sc, sv, sl, gd);
    const V t = parts_sum(s, red);
    if (threadIdx.x < kSlice && i < n) pr[i] = p[i] * ((V)b[i] - t);
}

template <typename V, typename VB, typename VX, typename I, typename S, int kB>
__global__ void __launch_bounds__(kBlock)
k_smooth_sell_p(int n, const int *__restrict__ sp, const int *__restrict__ uni, const int *__restrict__ su,
                const I *__restrict__ sc, const S *__restrict__ sv, const V *__restrict__ dinv,
                const VB *__restrict__ b, const V *__restrict__ xp, VX *__restrict__ x, const double *__restrict__ done) {
    __shared__ V red[kParts][kSlice];
    if (done && *done != 0.0) return;
    const int sl = xcd_block(blockIdx.x, gridDim.x);
    const int i = sl * kSlice + (int)threadIdx.x % kSlice;
    const V s = sell_row_part<V, S, I, kB>(n, sp, uni, su, sc, sv, sl, [&](int j) { return xp[j]; });
    const V t = parts_sum(s, red);
    if (threadIdx.x < kSlice && i < n) x[i] = (VX)(xp[i] + dinv[i] * ((V)b[i] - t));
}

// The flexible-CG product v = A w with the dot products (w.r, w.v, w.q) of
// Algorithm 3, one slice per workgroup: a grid of one workgroup per slice, each
// writing its own partials (summed in workgroup order by the finalize step).
template <typename I, typename S, int kB, bool NT>
__global__ void __launch_bounds__(kBlock)
k_spmv_dots_sell_p(int n, const int *__restrict__ sp, const int *__restrict__ uni, const int *__restrict__ su,
                   const I *__restrict__ sc, const S *__restrict__ sv, const double *__restrict__ w,
                   const double *__restrict__ r, const double *__restrict__ q, double *__restrict__ v,
                   double *__restrict__ partials, const double *__restrict__ done) {
    __shared__ double red[kParts][kSlice];
    if (done && *done != 0.0) return;
    const int sl = xcd_block(blockIdx.x, gridDim.x);
    const int i = sl * kSlice + (int)threadIdx.x % kSlice;
    auto g = [&](int j) { return w[j]; };
    const double s = sell_row_part<double, S, I, kB, decltype(g), NT>(n, sp, uni, su, sc, sv, sl, g);
    const double t = parts_sum(s, red);
    double acc[3] = {0.0, 0.0, 0.0};
    if (threadIdx.x < kSlice && i < n) {
        const double wi = w[i];
        v[i] = t;
        acc[0] = wi * r[i];
        acc[1] = wi * t;
        acc[2] = wi * q[i];
    }
    block_partials<3>(acc, partials);
}
