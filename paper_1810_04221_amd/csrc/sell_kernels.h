// Row-parallel kernels of the finest level and the other sliced-ELL levels:
// the residual and the flexible-CG product with its dot products, the down
// leg's residual, the up leg's smoothing, and the flexible-CG update.  Kept in
// a file of their own so that the HBM counter traffic recorded for them is
// tied to this source alone.  Included once, inside the solve library's
// anonymous namespace.
#pragma once
#include "device.h"
#include "internal.h"

// Column of a sliced-ELL slot: int32 columns, or int16 offsets col - row.
__device__ __forceinline__ int sell_col(int c, int) { return c; }
__device__ __forceinline__ int sell_col(short d, int i) { return i + (int)d; }

// Slots k0 .. w-1 of row i in batches of kB whose loads are all issued before
// any is used: a slot past the width re-reads the last one and is not added
// (w is the same for the whole wave), so no batch ends in a chain of one-slot
// steps.  Accumulates into s left to right.  Uni: column offsets from the
// slice's shared list u, else from the per-entry columns c.  NT: the values
// are loaded non-temporally (streamed past the L2, which then keeps more of
// the gathered vector).
template <int kB, bool Uni, typename V, typename S, typename I, typename F, bool NT = false>
__device__ __forceinline__ V sell_slots(const S *a, const int *u, const I *c, int n, int i, int w, V s, F f) {
    for (int k0 = 0; k0 < w; k0 += kB) {
        S av[kB];
        V fv[kB];
#pragma unroll
        for (int t = 0; t < kB; ++t) {
            const int k = min(k0 + t, w - 1);
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
            if (k0 + t < w) s += (V)av[t] * fv[t];
    }
    return s;
}

// Row i of a sliced ELL matrix: sum_k a_k * f(col_k), left to right over the
// row's slots (CSR order, with zero terms in between or after).  Lane i % 64 of
// a wave owns row i, so every slot load of the wave is one contiguous access
// (64 x 2, 4 or 8 B); the caller's waves are aligned to slices.  Values are
// stored as S and multiplied as V (S = float under V = double only when every
// value of the level is exactly a float: the conversion is exact).
// A uniform slice (uni[s] = 1: every row's offsets are a subsequence of one
// list) reads its column offsets from that list (su, from sp[s] / 64), one per
// slot for the whole wave, instead of one per entry; a slot a row does not
// have holds the value 0 (its column clamped into the matrix when it would
// leave it).
template <typename V, typename S, typename I, int kB, typename F, bool NT = false>
__device__ __forceinline__ V sell_row(int n, const int *__restrict__ sp, const int *__restrict__ uni,
                                      const int *__restrict__ su, const I *__restrict__ sc,
                                      const S *__restrict__ sv, int i, F f) {
    // uni is never null (all zero without uniform slices).  kB = 16 on levels
    // of long rows (a few dozen entries): half as many dependent memory round
    // trips per row, for twice the registers.
    const int sl = __builtin_amdgcn_readfirstlane(i / kSlice), lane = i % kSlice;
    const int uf = uni[sl], beg = sp[sl], w = (sp[sl + 1] - beg) / kSlice;
    const S *a = sv + beg + lane;
    const int *u = su + beg / kSlice;
    const I *c = sc + beg + lane;
    if (uf) return sell_slots<kB, true, V, S, I, F, NT>(a, u, c, n, i, w, V(0), f);
    return sell_slots<kB, false, V, S, I, F, NT>(a, u, c, n, i, w, V(0), f);
}


// FP32 cycle, finest level: the same residual with the values of A D (each
// slot's value times its column's inverse l1 diagonal, formed at setup), so
// each term gathers one vector:  pr_i = p_i (b_i - sum_j (a_ij dinv_j) b_j).
template <typename VB, typename I, int kB, bool NT>
__global__ void __launch_bounds__(kBlock)
k_down_res_sell_ad(int n, const int *__restrict__ sp, const int *__restrict__ uni, const int *__restrict__ su,
                   const I *__restrict__ sc, const float *__restrict__ svd, const float *__restrict__ p,
                   const VB *__restrict__ b, float *__restrict__ pr, const double *__restrict__ done,
                   StopTest st) {
    if (st.part && blockIdx.x == 0) {
        if (stop_test(st.part, st.scal, st.nb)) return;
    } else if (done && *done != 0.0) return;
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const float pi = p[i], bi = (float)b[i];  // loaded first, to overlap the product's loads
    auto g = [&](int j) { return (float)b[j]; };
    const float s = sell_row<float, float, I, kB, decltype(g), NT>(n, sp, uni, su, sc, svd, i, g);
    pr[i] = pi * (bi - s);
}

// Large levels: the down leg as a row-parallel residual on the sliced ELL copy,
//   pr_i = p_i (b_i - sum_j a_ij dinv_j b_j),
// followed by the restriction b_c[E] = sum of pr over E's members in ascending
// order (the order a serial P^T r takes).
template <typename V, typename VB, typename I, typename S, int kB, bool NT>
__global__ void __launch_bounds__(kBlock)
k_down_res_sell(int n, const int *__restrict__ sp, const int *__restrict__ uni,
                const int *__restrict__ su, const I *__restrict__ sc,
                const S *__restrict__ sv,
                const V *__restrict__ dinv, const V *__restrict__ p, const VB *__restrict__ b, V *__restrict__ pr,
                const V *__restrict__ y, const double *__restrict__ done, StopTest st) {
    // y given (levels with long rows): dinv o b formed beforehand, one gather per term
    if (st.part && blockIdx.x == 0) {
        if (stop_test(st.part, st.scal, st.nb)) return;
    } else if (done && *done != 0.0) return;
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const V pi = p[i], bi = (V)b[i];  // loaded first, to overlap the product's loads
    V s;
    auto gy = [&](int j) { return y[j]; };
    auto gd = [&](int j) { return dinv[j] * (V)b[j]; };
    if (y) s = sell_row<V, S, I, kB, decltype(gy), NT>(n, sp, uni, su, sc, sv, i, gy);
    else s = sell_row<V, S, I, kB, decltype(gd), NT>(n, sp, uni, su, sc, sv, i, gd);
    pr[i] = pi * (bi - s);
}


// k_smooth on the sliced ELL copy, one thread per row.  NT: the values are
// streamed non-temporally (Sell::stream).
template <typename V, typename VB, typename VX, typename I, typename S, int kB, bool NT>
__global__ void __launch_bounds__(kBlock)
k_smooth_sell(int n, const int *__restrict__ sp, const int *__restrict__ uni,
                const int *__restrict__ su, const I *__restrict__ sc,
              const S *__restrict__ sv,
              const V *__restrict__ dinv, const VB *__restrict__ b, const V *__restrict__ xp, VX *__restrict__ x,
              const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const V xi = xp[i], di = dinv[i], bi = (V)b[i];  // loaded first, to overlap the product's loads
    auto g = [&](int j) { return xp[j]; };
    const V s = sell_row<V, S, I, kB, decltype(g), NT>(n, sp, uni, su, sc, sv, i, g);
    x[i] = (VX)(xi + di * (bi - s));
}


// Sliced-ELL variants: one thread per row, grid-stride; each row sum is taken
// left to right exactly as a serial CSR product.
template <typename I, typename S, int kB>
__global__ void __launch_bounds__(kBlock)
k_resid_sell(int n, const int *__restrict__ sp, const int *__restrict__ uni,
                const int *__restrict__ su, const I *__restrict__ sc,
             const S *__restrict__ sv,
             const double *__restrict__ b, const double *__restrict__ u, double *__restrict__ r,
             double *__restrict__ partials) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    double acc[2] = {0.0, 0.0};
    for (int i = blk * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double bi = b[i];
        const double s = sell_row<double, S, I, kB>(n, sp, uni, su, sc, sv, i, [&](int j) { return u[j]; });
        const double ri = bi - s;
        r[i] = ri;
        acc[0] += ri * ri;
        acc[1] += bi * bi;
    }
    block_partials<2>(acc, partials);
}

// The rows a workgroup of a grid-stride kernel walks, XCD by XCD: when the
// grid is a multiple of the eight XCDs, the workgroups of one XCD (consecutive
// logical blocks under xcd_block) take one contiguous eighth of the rows and
// stride through it together, kBlock rows per workgroup and step.  The far
// neighbours of a row (the z-neighbours of a 3-D grid, about n^(2/3) rows
// away) are then rows the same XCD has just loaded or is about to, in its own
// L2, instead of rows of another XCD's window of the same step.
struct XcdRows {
    int first, end, stride;
};
__device__ __forceinline__ XcdRows xcd_rows(int n, int blk, int nb) {
    constexpr int X = 8;
    if (nb % X != 0) return XcdRows{blk * kBlock, n, nb * kBlock};
    const int per = nb / X, x = blk / per, j = blk - x * per;
    const long long chunk = ((long long)n + X - 1) / X;
    const long long len = (chunk + kBlock - 1) / kBlock * kBlock;
    const long long lo = x * len, hi = lo + len < n ? lo + len : n;
    return XcdRows{(int)(lo + (long long)j * kBlock), (int)hi, per * kBlock};
}

// NT: the matrix values streamed non-temporally (Sell::stream: the gathered
// w then stays in each XCD's L2).
template <typename I, typename S, int kB, bool NT>
__global__ void __launch_bounds__(kBlock)
k_spmv_dots_sell(int n, const int *__restrict__ sp, const int *__restrict__ uni,
                const int *__restrict__ su, const I *__restrict__ sc,
                 const S *__restrict__ sv,
                 const double *__restrict__ w, const double *__restrict__ r, const double *__restrict__ q,
                 double *__restrict__ v, double *__restrict__ partials, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const XcdRows xr = xcd_rows(n, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = xr.first + threadIdx.x; i < xr.end; i += xr.stride) {
        // the row's own entries are loaded first, to overlap the product's loads
        const double wi = w[i], ri = r[i], qi = q[i];
        auto g = [&](int j) { return w[j]; };
        const double s = sell_row<double, S, I, kB, decltype(g), NT>(n, sp, uni, su, sc, sv, i, g);
        v[i] = s;
        acc[0] += wi * ri;
        acc[1] += wi * s;
        acc[2] += wi * qi;
    }
    block_partials<3>(acc, partials);
}


// The two fused AXPY pairs of Algorithm 3 and partials of ||r||^2:
//   d = w - g d ; u += an d ; q = v - g q ; r -= an q   (first step: d = w, q = v)
// with g = gamma_i / rho_{i-1} and an = alpha_i / rho_i from the finalize step.
// With y given, also y = dinv o r in the cycle's arithmetic type YV: the
// finest level's pre-smoothed iterate (the first Jacobi step of Algorithm 1
// from a zero guess) for the next preconditioner application, whose down-leg
// residual then gathers one array instead of dinv and r.
// Vectors of at least four entries per thread of the grid go in pairs of
// entries with 16-byte accesses (the vectors are 256-byte aligned; with n odd,
// thread 0 of the grid also takes entry n - 1); shorter ones one entry at a
// time, which keeps more waves in flight.
template <bool First>
__device__ __forceinline__ void update_pair(double wi, double vi, double &di, double &qi, double &ui, double &ri,
                                            double g, double an, double &acc) {
    if (First) { di = wi; qi = vi; }
    else { di = wi - g * di; qi = vi - g * qi; }
    ui = ui + an * di;
    ri = ri - an * qi;
    acc += ri * ri;
}

template <bool First, typename YV>
__device__ __forceinline__ void update_range1(int n, const double *__restrict__ w, const double *__restrict__ v,
                                              double *__restrict__ d, double *__restrict__ u,
                                              double *__restrict__ q, double *__restrict__ r,
                                              const YV *__restrict__ dinv, YV *__restrict__ y, double g, double an,
                                              double &acc) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    for (int i = blk * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        double di = First ? 0.0 : d[i], qi = First ? 0.0 : q[i], ui = u[i], ri = r[i];
        update_pair<First>(w[i], v[i], di, qi, ui, ri, g, an, acc);
        d[i] = di;
        q[i] = qi;
        u[i] = ui;
        r[i] = ri;
        if (y) y[i] = dinv[i] * (YV)ri;
    }
}

template <typename YV> struct Pair2;
template <> struct Pair2<float> { using T = float2; };
template <> struct Pair2<double> { using T = double2; };

template <bool First, typename YV>
__device__ __forceinline__ void update_range(int n, const double *__restrict__ w, const double *__restrict__ v,
                                             double *__restrict__ d, double *__restrict__ u, double *__restrict__ q,
                                             double *__restrict__ r, const YV *__restrict__ dinv,
                                             YV *__restrict__ y, double g, double an, double &acc) {
    using Y2 = typename Pair2<YV>::T;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int n2 = n / 2;
    const double2 *w2 = reinterpret_cast<const double2 *>(w), *v2 = reinterpret_cast<const double2 *>(v);
    double2 *d2 = reinterpret_cast<double2 *>(d), *u2 = reinterpret_cast<double2 *>(u);
    double2 *q2 = reinterpret_cast<double2 *>(q), *r2 = reinterpret_cast<double2 *>(r);
    const Y2 *dinv2 = reinterpret_cast<const Y2 *>(dinv);
    Y2 *y2 = reinterpret_cast<Y2 *>(y);
    for (int i = blk * kBlock + threadIdx.x; i < n2; i += gridDim.x * kBlock) {
        const double2 wi = w2[i], vi = v2[i];
        double2 di, qi;
        if (!First) { di = d2[i]; qi = q2[i]; }
        double2 ui = u2[i], ri = r2[i];
        update_pair<First>(wi.x, vi.x, di.x, qi.x, ui.x, ri.x, g, an, acc);
        update_pair<First>(wi.y, vi.y, di.y, qi.y, ui.y, ri.y, g, an, acc);
        d2[i] = di;
        q2[i] = qi;
        u2[i] = ui;
        r2[i] = ri;
        if (y) {
            const Y2 dv = dinv2[i];
            Y2 yv;
            yv.x = dv.x * (YV)ri.x;
            yv.y = dv.y * (YV)ri.y;
            y2[i] = yv;
        }
    }
    if ((n & 1) && blk == 0 && threadIdx.x == 0) {
        const int i = n - 1;
        double di = First ? 0.0 : d[i], qi = First ? 0.0 : q[i], ui = u[i], ri = r[i];
        update_pair<First>(w[i], v[i], di, qi, ui, ri, g, an, acc);
        d[i] = di;
        q[i] = qi;
        u[i] = ui;
        r[i] = ri;
        if (y) y[i] = dinv[i] * (YV)ri;
    }
}

// The step scalars of Algorithm 3 from the sums s = (alpha, beta, gamma) of
// the product's dot products: rho_i = beta - gamma^2 / rho_{i-1} (first step:
// beta), g = gamma / rho_{i-1}, an = alpha / rho_i; false on breakdown (rho_i
// not positive, or a scalar not finite).  rho_{i-1} sits in the slot of a
// two-entry ring (scal[14], scal[15]) picked by the iteration count scal[11],
// rho_i goes to the other one, so that every workgroup of the update can form
// the scalars itself while one of them stores the new rho.  With write set the
// caller also stores alpha, beta, gamma, g, an and the breakdown flags.
__device__ __forceinline__ bool fcg_scalars(const double (&s)[3], int first, double *scal, bool write, double &g,
                                            double &an) {
    const double alpha = s[0], beta = s[1], gamma = s[2];
    const int slot = (int)scal[11] & 1;
    double rho;
    if (first) { rho = beta; g = 0.0; }
    else { const double rho_prev = scal[14 + slot]; rho = beta - gamma * gamma / rho_prev; g = gamma / rho_prev; }
    an = alpha / rho;
    const bool ok = (rho > 0.0) && isfinite(rho) && isfinite(an) && isfinite(g);
    if (write) {
        scal[0] = alpha;
        scal[1] = beta;
        scal[2] = gamma;
        scal[6] = ok ? 0.0 : 1.0;
        if (ok) { scal[15 - slot] = rho; scal[8] = g; scal[9] = an; }
        else scal[10] = 1.0;
    }
    return ok;
}

// YV: float or double, the type of dinv and y (y may be null).
// dots null: the step scalars come from scal (a k_finalize launch formed them).
// dots set: every workgroup first adds the product's ndots block partials in
// the order the one-block finalize takes with kBlock threads (bit-identical
// sums) and forms the scalars itself; workgroup 0 stores them.
template <typename YV>
__global__ void __launch_bounds__(kBlock)
k_update(int n, int first, const double *__restrict__ w, const double *__restrict__ v, double *__restrict__ d,
         double *__restrict__ u, double *__restrict__ q, double *__restrict__ r, const YV *__restrict__ dinv,
         YV *__restrict__ y, double *__restrict__ scal, double *__restrict__ partials,
         const double *__restrict__ dots, int ndots) {
    if (scal[10] != 0.0) return;
    bool ok;
    double g, an;
    if (dots) {
        __shared__ double lds[3 * 16];
        __shared__ double bc[3];
        double s[3] = {0.0, 0.0, 0.0};
        add_partials<3, 4>(s, dots, ndots);  // four loads a value: few registers
        block_sum<3>(s, lds);
        if (threadIdx.x == 0) {
            const bool k = fcg_scalars(s, first, scal, blockIdx.x == 0, g, an);
            bc[0] = k ? 1.0 : 0.0;
            bc[1] = g;
            bc[2] = an;
        }
        __syncthreads();
        ok = bc[0] != 0.0;
        g = bc[1];
        an = bc[2];
    } else {
        ok = scal[6] == 0.0;
        g = scal[8];
        an = scal[9];
    }
    double acc[1] = {0.0};
    if (ok) {
        const bool pairs = (long long)n >= 4LL * gridDim.x * kBlock;
        if (pairs && first) update_range<true>(n, w, v, d, u, q, r, dinv, y, g, an, acc[0]);
        else if (pairs) update_range<false>(n, w, v, d, u, q, r, dinv, y, g, an, acc[0]);
        else if (first) update_range1<true>(n, w, v, d, u, q, r, dinv, y, g, an, acc[0]);
        else update_range1<false>(n, w, v, d, u, q, r, dinv, y, g, an, acc[0]);
    }
    block_partials<1>(acc, partials);
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[7] = 1.0;  // partials for the stop test
}
