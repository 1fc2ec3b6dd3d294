// Solve-phase kernels for gfx950: the V-cycle of Algorithm 1 with l1-Jacobi
// smoothing (Section 3.2), the flexible CG kernels of Algorithm 3 with the three
// dot products fused into the SpMV and the vector updates fused into one pass,
// and the sampled outer product of the gradient.
//
// All of them stream CSR rows: a group of G lanes (G = power of two near the
// level's mean row length) owns one row, so a wave reads 64 consecutive
// entries of col/val at once.  Cycle kernels are templated on the value type
// (float64, or float32 for the FP32 cycle) and on the types of the level-0
// input/output vectors, which stay float64.
#include <type_traits>

#include "device.h"
#include "internal.h"

namespace bcm {

namespace {

template <typename Fn>
void with_G(int G, Fn &&fn) {
    switch (G) {
        case 4: fn(std::integral_constant<int, 4>{}); break;
        case 8: fn(std::integral_constant<int, 8>{}); break;
        case 16: fn(std::integral_constant<int, 16>{}); break;
        case 32: fn(std::integral_constant<int, 32>{}); break;
        default: fn(std::integral_constant<int, 64>{}); break;
    }
}

inline int blocks_for(long long threads) { return (int)((threads + kBlock - 1) / kBlock); }

// Calls fn(index pointer, value pointer) with the sliced-ELL arrays a kernel of
// arithmetic type V reads: int16 offsets or int32 columns, and float64 values,
// or float32 values (float32 arithmetic, or values that are exact floats).
template <typename V, typename Fn>
void with_sell(const Sell &E, Fn &&fn) {
    // fn(columns, values, batch): batch is std::integral_constant<int, 8 or 16>
    auto go = [&](auto *ix, auto *vals) {
        if (E.wide) fn(ix, vals, std::integral_constant<int, 16>());
        else fn(ix, vals, std::integral_constant<int, 8>());
    };
    if constexpr (std::is_same<V, float>::value) {
        if (E.sd) go(E.sd, E.sv32);
        else go(E.sc, E.sv32);
    } else {
        if (E.sd) {
            if (E.sv) go(E.sd, E.sv);
            else go(E.sd, E.sv32);
        } else {
            if (E.sv) go(E.sc, E.sv);
            else go(E.sc, E.sv32);
        }
    }
}

// Wide levels (batches of 16) with at most kSplitRows rows take the
// slot-split kernels: at one thread per row they would hold fewer than about
// 32 waves per CU.  Larger wide levels fill the chip already, and there the
// split's LDS reduction costs more than it gains.
constexpr int kSplitRows = 1 << 19;
inline bool split_slots(const Level &L, int kb) { return kb == 16 && L.A.n <= kSplitRows; }

// ----------------------------------------------------------------------------
// Long rows (longer than the level's lmin = kLongFactor * G): their dot
// products are summed by a pre-pass over chunks of kSegChunk entries, one
// workgroup per chunk (k_long_dot, with the same gathered operand f as the row
// kernel that follows it), and the row kernel adds the chunk sums of such a
// row in chunk order across its group instead of walking the row.
// ----------------------------------------------------------------------------
template <typename V>
struct LongView {
    int lmin = 0x7fffffff;  // no row is longer: the level has no long rows
    const int *idx = nullptr, *cb = nullptr;
    const V *part = nullptr;
};

template <typename V>
LongView<V> long_view(const LongRows &lr) {
    LongView<V> v;
    if (lr.n > 0) {
        v.lmin = lr.lmin;
        v.idx = lr.idx;
        v.cb = lr.cb;
        v.part = static_cast<const V *>(lr.part);
    }
    return v;
}

// the dot product of long row `row` from its chunk sums (every lane of the group gets it)
template <int G, typename V>
__device__ __forceinline__ V long_sum(const LongView<V> &lv, int row) {
    if (!lv.part) return V(0);  // single-launch leg: the row's finishing block writes its result
    const int lane = threadIdx.x % G, t = lv.idx[row];
    V s = V(0);
    for (int c = lv.cb[t] + lane; c < lv.cb[t + 1]; c += G) s += lv.part[c];
    return group_sum<G>(s);
}

// largest t in [0, cnt) with base[t] <= x (base strictly ascending, base[0] = 0)
__device__ __forceinline__ int chunk_owner(const int *__restrict__ base, int cnt, int x) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Chunk c of the long rows: part[c] = sum of a_q f(ci[q]) over its entries,
// eight per thread (all loads issued first), then the workgroup in a fixed order.
template <typename V, typename F>
__global__ void __launch_bounds__(kBlock)
k_long_dot(LongRows lr, const int *__restrict__ rp, const int *__restrict__ ci, const V *__restrict__ a, F f,
           V *__restrict__ part, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    constexpr int U = kSegChunk / kBlock;
    const int c = blockIdx.x;
    const int t = chunk_owner(lr.cb, lr.n, c);
    const int row = lr.rows[t];
    const int q0 = rp[row] + (c - lr.cb[t]) * kSegChunk, q1 = min(q0 + kSegChunk, rp[row + 1]);
    int j[U];
    V av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int q = q0 + (int)threadIdx.x + u * kBlock;
        const bool in = q < q1;
        j[u] = in ? ci[q] : row;
        av[u] = in ? a[q] : V(0);
    }
    V s = V(0);
#pragma unroll
    for (int u = 0; u < U; ++u) s += av[u] * f(j[u]);
    double d[1] = {(double)s};
    __shared__ double lds[16];
    block_sum<1>(d, lds);
    if (threadIdx.x == 0) part[c] = (V)d[0];
}

// Gathered operands of the row kernels (one rounding per operation, as the
// row kernels' own expressions).
template <typename V, typename VB>
struct FScaled {  // the pre-smoothed iterate from zero: dinv_j b_j
    const V *dinv;
    const VB *b;
    __device__ V operator()(int j) const { return dinv[j] * (V)b[j]; }
};
template <typename V, typename VB>
struct FProlonged {  // pre-smoothed iterate plus the coarse correction: dinv_j b_j + p_j xc[agg_j]
    const V *dinv, *p;
    const int *agg;
    const VB *b;
    const V *xc;
    __device__ V operator()(int j) const { return dinv[j] * (V)b[j] + p[j] * xc[agg[j]]; }
};
template <typename V, typename T>
struct FGather {  // a vector entry
    const T *x;
    __device__ V operator()(int j) const { return (V)x[j]; }
};

// R rows per group of G lanes.  All loads of the first pass over the R rows
// are issued before any result is used (out-of-row lanes read entry beg[k] and
// discard it), which keeps R times more memory requests in flight per lane than
// one row at a time.  Rows longer than G finish in a second loop; rows longer
// than lv.lmin take their chunk sums instead.
// s[k] = sum_q a[q] * f(ci[q]) over row rows[k] (rows[k] < 0: empty).
// *lgm (when given) gets bit k set when row rows[k] is long.
template <int G, int R, typename V, typename F>
__device__ __forceinline__ void rows_dot(const int *__restrict__ rp, const int *__restrict__ ci,
                                         const V *__restrict__ a, const int (&rows)[R], V (&s)[R], F f,
                                         const LongView<V> &lv = LongView<V>(), int *lgm = nullptr) {
    const int lane = threadIdx.x % G;
    int beg[R], end[R];
    bool lg[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        // both bounds loaded unconditionally: no branch between the R rows' loads
        const int i = rows[k] < 0 ? 0 : rows[k];
        const int b0 = rp[i], b1 = rp[i + 1];
        lg[k] = rows[k] >= 0 && b1 - b0 > lv.lmin;
        beg[k] = b0;
        end[k] = (rows[k] < 0 || lg[k]) ? b0 : b1;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int q = beg[k] + lane;
        const bool in = q < end[k];
        const int qs = in ? q : (end[k] > beg[k] ? beg[k] : 0);
        const int j = ci[qs];
        const V t = a[qs] * f(j);
        s[k] = in ? t : V(0);
    }
#pragma unroll
    for (int k = 0; k < R; ++k)
        for (int q = beg[k] + lane + G; q < end[k]; q += G) s[k] += a[q] * f(ci[q]);
#pragma unroll
    for (int k = 0; k < R; ++k) s[k] = group_sum<G>(s[k]);
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (lg[k]) s[k] = long_sum<G>(lv, rows[k]);
    if (lgm) {
        int m = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) m |= lg[k] ? (1 << k) : 0;
        *lgm = m;
    }
}

// ----------------------------------------------------------------------------
// Row-wise cycle legs (up leg, coarsest sweeps) of levels with long rows in
// one launch.  The blocks after the row kernel's nrb row blocks take the long
// rows' chunks: each sums its chunk exactly as k_long_dot, stores the partial
// and counts its arrival on the row; the block that brings a row's last chunk
// adds the row's partials (all loaded at once, in a fixed order) and writes
// the row's output (fin).  The row blocks leave the long rows alone.  The partial stores and the
// arrival count are ordered by device-scope fences (release before the count,
// acquire after it in the finishing block): a few dozen blocks per launch do
// this.  The counter is back at zero for the next launch.
// ----------------------------------------------------------------------------
struct LongFused {
    int nrb = 0;  // row blocks; 0: no chunk blocks (long rows summed by a pre-pass)
    LongRows lr;
};

template <typename V, typename F, typename Fin>
__device__ __forceinline__ void long_chunk(int c, const LongRows &lr, const int *__restrict__ rp,
                                           const int *__restrict__ ci, const V *__restrict__ a, F f, Fin fin) {
    constexpr int U = kSegChunk / kBlock;
    __shared__ double lds[16];
    __shared__ int last;
    __shared__ V srow;
    const int t = chunk_owner(lr.cb, lr.n, c);
    const int row = lr.rows[t];
    const int q0 = rp[row] + (c - lr.cb[t]) * kSegChunk, q1 = min(q0 + kSegChunk, rp[row + 1]);
    int j[U];
    V av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int q = q0 + (int)threadIdx.x + u * kBlock;
        const bool in = q < q1;
        j[u] = in ? ci[q] : row;
        av[u] = in ? a[q] : V(0);
    }
    V sum = V(0);
#pragma unroll
    for (int u = 0; u < U; ++u) sum += av[u] * f(j[u]);
    double d[1] = {(double)sum};
    block_sum<1>(d, lds);
    V *part = static_cast<V *>(lr.part);
    if (threadIdx.x == 0) {
        part[c] = (V)d[0];
        __threadfence();  // the partial before the arrival
        last = atomicAdd(&lr.cnt[t], 1) == lr.cb[t + 1] - lr.cb[t] - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // every chunk's partial after its arrival
    // the row's partials, all loads at once, added in a fixed order
    double r[1] = {0.0};
    for (int k = lr.cb[t] + (int)threadIdx.x; k < lr.cb[t + 1]; k += kBlock) r[0] += (double)part[k];
    block_sum<1>(r, lds);
    if (threadIdx.x == 0) {
        srow = (V)r[0];
        lr.cnt[t] = 0;
    }
    __syncthreads();
    fin(row, srow);
}


#include "sell_kernels.h"
#include "sell_split.h"

// ----------------------------------------------------------------------------
// Down leg of the cycle at level k (Algorithm 1, zero initial guess):
//   x = x + M^{-1}(b - A x) with x = 0   ->  x_j = dinv_j * b_j
//   b_c[E] = sum_{i in E} p_i (b_i - sum_j a_ij x_j)      (restriction)
// x is never stored: it is recomputed from b and dinv where it is gathered.
// One group of G lanes per aggregate; the member rows are processed together
// (k_down_seq, S = 1, 2 or 4 members) or one after the other (k_down_loop).
// ----------------------------------------------------------------------------
// S members (template) of one aggregate, all rows in flight at once; summed
// in ascending member order.
template <int G, int S, typename V, typename VB>
__global__ void __launch_bounds__(kBlock)
k_down_seq(int nc, const int *__restrict__ mem, const int *__restrict__ rp, const int *__restrict__ ci,
           const V *__restrict__ a, const V *__restrict__ dinv, const V *__restrict__ p,
           const VB *__restrict__ b, V *__restrict__ bc, const double *__restrict__ done, LongView<V> lv) {
    // small levels: the solve-ended flag is only tested before the store, so
    // its load overlaps the row loads instead of preceding them
    const int lane = threadIdx.x % G;
    int E = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    const bool live = E < nc;
    if (!live) E = nc - 1;
    int rows[S];
#pragma unroll
    for (int t = 0; t < S; ++t) rows[t] = mem[(size_t)E * S + t];
    V s[S];
    rows_dot<G, S, V>(rp, ci, a, rows, s, FScaled<V, VB>{dinv, b}, lv);
    V acc = V(0);
#pragma unroll
    for (int t = 0; t < S; ++t) {
        const int i = rows[t] < 0 ? 0 : rows[t];
        const V c = p[i] * ((V)b[i] - s[t]);
        acc += rows[t] < 0 ? V(0) : c;
    }
    if (lane == 0 && live && !(done && *done != 0.0)) bc[E] = acc;
}

// Any number of members (wide composed aggregates): one member row at a time.
template <int G, typename V, typename VB>
__global__ void __launch_bounds__(kBlock)
k_down_loop(int nc, int mstride, const int *__restrict__ mem, const int *__restrict__ rp,
            const int *__restrict__ ci, const V *__restrict__ a, const V *__restrict__ dinv,
            const V *__restrict__ p, const VB *__restrict__ b, V *__restrict__ bc,
            const double *__restrict__ done, LongView<V> lv) {
    if (done && *done != 0.0) return;
    const int lane = threadIdx.x % G;
    const int E = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (E >= nc) return;
    const FScaled<V, VB> f{dinv, b};
    V acc = V(0);
    for (int t = 0; t < mstride; ++t) {
        const int i = mem[(size_t)E * mstride + t];
        if (i < 0) break;
        V s = V(0);
        const int bq = rp[i], e = rp[i + 1];
        if (e - bq > lv.lmin) {
            s = long_sum<G>(lv, i);
        } else {
            for (int q = bq + lane; q < e; q += G) s += a[q] * f(ci[q]);
            s = group_sum<G>(s);
        }
        acc += p[i] * ((V)b[i] - s);
    }
    if (lane == 0) bc[E] = acc;
}


// y = dinv o b, the pre-smoothed iterate of the down leg, for the levels whose
// residual kernel gathers it instead of dinv and b (long rows)
template <typename V, typename VB>
__global__ void __launch_bounds__(kBlock)
k_scale(int n, const V *__restrict__ dinv, const VB *__restrict__ b, V *__restrict__ y,
        const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < n) y[i] = dinv[i] * (V)b[i];
}

template <typename V, int S>
__global__ void __launch_bounds__(kBlock)
k_restrict(int nc, const int *__restrict__ mem, const V *__restrict__ pr, V *__restrict__ bc,
           const V *__restrict__ cd, V *__restrict__ cy, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int E = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (E >= nc) return;
    int m[S];
#pragma unroll
    for (int t = 0; t < S; ++t) m[t] = mem[(size_t)E * S + t];
    V acc = V(0);
#pragma unroll
    for (int t = 0; t < S; ++t) acc += m[t] >= 0 ? pr[m[t]] : V(0);
    bc[E] = acc;
    if (cy) cy[E] = cd[E] * acc;  // the coarser level's dinv o b, as k_scale forms it
}

// ----------------------------------------------------------------------------
// Up leg at level k: prolongation and post-smoothing (Algorithm 1; M^{-T} =
// M^{-1} for the diagonal l1 smoother):
//   x_j = dinv_j b_j + p_j xc[agg_j]          (pre-smoothed x plus P x_c)
//   x_i <- x_i + dinv_i (b_i - sum_j a_ij x_j)
// ----------------------------------------------------------------------------
template <int G, int R, typename V, typename VB, typename VX, bool LF>
__global__ void __launch_bounds__(kBlock)
k_up(int n, const int *__restrict__ rp, const int *__restrict__ ci, const V *__restrict__ a,
     const V *__restrict__ dinv, const V *__restrict__ p, const int *__restrict__ agg,
     const VB *__restrict__ b, const V *__restrict__ xc, VX *__restrict__ x, const double *__restrict__ done,
     LongView<V> lv, LongFused lf) {
    if (LF && (int)blockIdx.x >= lf.nrb) {  // a chunk of a long row (see long_chunk)
        if (done && *done != 0.0) return;
        long_chunk<V>((int)blockIdx.x - lf.nrb, lf.lr, rp, ci, a, FProlonged<V, VB>{dinv, p, agg, b, xc},
                      [&](int i, V sl) {
                          if (threadIdx.x != 0) return;
                          const V bi = (V)b[i];
                          const V di = dinv[i];
                          const V xi = di * bi + p[i] * xc[agg[i]];
                          x[i] = (VX)(xi + di * (bi - sl));
                      });
        return;
    }
    // the solve-ended flag is tested before the stores only (as in k_down_seq)
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int base = xcd_block(blockIdx.x, LF ? lf.nrb : gridDim.x) * NG * R + threadIdx.x / G;
    int rows[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rows[k] = base + k * NG < n ? base + k * NG : -1;
    V s[R];
    int lgm = 0;
    rows_dot<G, R, V>(rp, ci, a, rows, s, FProlonged<V, VB>{dinv, p, agg, b, xc}, lv, &lgm);
    if (lane == 0 && !(done && *done != 0.0)) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = rows[k];
            if (i < 0 || (LF && ((lgm >> k) & 1))) continue;
            const V bi = (V)b[i];
            const V di = dinv[i];
            const V xi = di * bi + p[i] * xc[agg[i]];
            x[i] = (VX)(xi + di * (bi - s[k]));
        }
    }
}

// Large levels: the up leg as two streaming kernels.  k_prolong writes the
// pre-smoothed, corrected iterate xp = dinv o b + P xc (all reads coalesced);
// k_smooth then gathers only xp:  x_i = xp_i + dinv_i (b_i - sum_j a_ij xp_j).
// Same arithmetic as k_up, one gathered array per nonzero instead of five.
template <typename V, typename VB>
__global__ void __launch_bounds__(kBlock)
k_prolong(int n, const V *__restrict__ dinv, const V *__restrict__ p, const int *__restrict__ agg,
          const VB *__restrict__ b, const V *__restrict__ xc, V *__restrict__ xp, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    xp[i] = dinv[i] * (V)b[i] + p[i] * xc[agg[i]];
}

template <int G, int R, typename V, typename VB, typename VX>
__global__ void __launch_bounds__(kBlock)
k_smooth(int n, const int *__restrict__ rp, const int *__restrict__ ci, const V *__restrict__ a,
         const V *__restrict__ dinv, const VB *__restrict__ b, const V *__restrict__ xp, VX *__restrict__ x,
         const double *__restrict__ done, LongView<V> lv) {
    if (done && *done != 0.0) return;
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int base = xcd_block(blockIdx.x, gridDim.x) * NG * R + threadIdx.x / G;
    int rows[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rows[k] = base + k * NG < n ? base + k * NG : -1;
    V s[R];
    rows_dot<G, R, V>(rp, ci, a, rows, s, FGather<V, V>{xp}, lv);
    // lane k of the group finishes row k
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rows[k];
        if (lane == k % G && i >= 0) x[i] = (VX)(xp[i] + dinv[i] * ((V)b[i] - s[k]));
    }
}


// W-cycle helpers (levels >= 1, cycle precision): the coarse residual in place,
// b_i <- b_i - sum_j a_ij x_j, and x <- x + y.
template <int G, typename V>
__global__ void __launch_bounds__(kBlock)
k_resid_inplace(int n, const int *__restrict__ rp, const int *__restrict__ ci, const V *__restrict__ a,
                const V *__restrict__ x, V *__restrict__ b, const double *__restrict__ done, LongView<V> lv) {
    if (done && *done != 0.0) return;
    const int lane = threadIdx.x % G;
    const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (i >= n) return;
    V s = V(0);
    const int bq = rp[i], e = rp[i + 1];
    if (e - bq > lv.lmin) {
        s = long_sum<G>(lv, i);
    } else {
        for (int q = bq + lane; q < e; q += G) s += a[q] * x[ci[q]];
        s = group_sum<G>(s);
    }
    if (lane == 0) b[i] = b[i] - s;
}

template <typename V>
__global__ void __launch_bounds__(kBlock)
k_add(int n, const V *__restrict__ y, V *__restrict__ x, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = x[i] + y[i];
}

// ----------------------------------------------------------------------------
// K-cycle coarse solve on a level C (cycle precision V): two flexible-CG
// iterations from zero on A_C x = b, preconditioned by C's cycle, written with
// the two preconditioned directions c1 = B(b) and c2 = B(b~):
//   step 1: v1 = A c1, rho1 = c1'v1, alpha1 = c1'b, b~ = b - (alpha1/rho1) v1
//   step 2: gamma = c2'v1, beta = c2'A c2, alpha2 = c2'b~,
//           rho2 = beta - gamma^2 / rho1
//   x = (alpha1/rho1) c1 + (alpha2/rho2) (c2 - (gamma/rho1) c1)
// (the iterates of the flexible CG loop: d1 = c1, d2 = c2 - (gamma/rho1) d1).
// An iteration whose rho is not positive and finite ends the coarse CG with
// the directions kept so far.  Dot products accumulate in float64 through
// block partials summed in block order (k_kfinal).
// ks[]: [0] rho1 [1] alpha1/rho1 [2] gamma/rho1 [3] alpha2/rho2 [4] directions kept
// ----------------------------------------------------------------------------
// step 1 (c = c1, vout = v1): acc = {c'Ac, c'b};  step 2 (c = c2, vin = v1):
// acc = {c'v1, c'Ac, c'b}.  Rows in a grid-stride loop, G lanes per row.
template <int G, typename V, int STEP>
__global__ void __launch_bounds__(kBlock)
k_kdots(int n, const int *__restrict__ rp, const int *__restrict__ ci, const V *__restrict__ a,
        const V *__restrict__ c, const V *__restrict__ b, const V *__restrict__ vin, V *__restrict__ vout,
        double *__restrict__ partials, const double *__restrict__ done, LongView<V> lv) {
    if (done && *done != 0.0) return;
    constexpr int K = STEP == 1 ? 2 : 3;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int lane = threadIdx.x % G;
    const int rows_per_grid = gridDim.x * (kBlock / G);
    for (int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G; i < n; i += rows_per_grid) {
        V s = V(0);
        const int bq = rp[i], e = rp[i + 1];
        if (e - bq > lv.lmin) {
            s = long_sum<G>(lv, i);
        } else {
            for (int q = bq + lane; q < e; q += G) s += a[q] * c[ci[q]];
            s = group_sum<G>(s);
        }
        if (lane == 0) {
            const double ci_ = (double)c[i];
            if (STEP == 1) {
                vout[i] = s;
                acc[0] += ci_ * (double)s;
                acc[1] += ci_ * (double)b[i];
            } else {
                acc[0] += ci_ * (double)vin[i];
                acc[1] += ci_ * (double)s;
                acc[2] += ci_ * (double)b[i];
            }
        }
    }
    block_partials<K>(acc, partials);
}

template <int STEP>
__global__ void __launch_bounds__(kBlock) k_kfinal(int nb, const double *__restrict__ partials,
                                                   double *__restrict__ ks, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    constexpr int K = STEP == 1 ? 2 : 3;
    __shared__ double lds[K * 16];
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    add_partials<K>(s, partials, nb);
    block_sum<K>(s, lds);
    if (threadIdx.x != 0) return;
    if (STEP == 1) {
        const double rho = s[0];
        const bool ok = rho > 0.0 && isfinite(rho);
        ks[0] = rho;
        ks[1] = ok ? s[1 % K] / rho : 0.0;
        ks[2] = 0.0;
        ks[3] = 0.0;
        ks[4] = ok ? 1.0 : 0.0;
    } else {
        if (ks[4] != 1.0) return;
        const double gamma = s[0], beta = s[1 % K], alpha = s[2 % K], rho1 = ks[0];
        const double rho = beta - gamma * gamma / rho1;
        if (!(rho > 0.0) || !isfinite(rho)) return;
        ks[2] = gamma / rho1;
        ks[3] = alpha / rho;
        ks[4] = 2.0;
    }
}

// b <- b - (alpha1/rho1) v1
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_kresid(int n, const V *__restrict__ v1, const double *__restrict__ ks, V *__restrict__ b,
         const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const V a1 = (V)ks[1];
    b[i] = b[i] - a1 * v1[i];
}

// x <- (alpha1/rho1) c1 + (alpha2/rho2) (c2 - (gamma/rho1) c1), with c1 in x
template <typename V>
__global__ void __launch_bounds__(kBlock)
k_kcombine(int n, const V *__restrict__ c2, const double *__restrict__ ks, V *__restrict__ x,
           const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double kept = ks[4];
    const V a1 = (V)ks[1], g = (V)ks[2], a2 = (V)ks[3];
    const V c1 = x[i];
    V r = V(0);
    if (kept == 2.0) r = a1 * c1 + a2 * (c2[i] - g * c1);
    else if (kept == 1.0) r = a1 * c1;
    x[i] = r;
}

// ----------------------------------------------------------------------------
// Coarsest level: `sweeps` l1-Jacobi sweeps from zero in float64, inside one
// workgroup with x in LDS (n <= 8192).  When the level's matrix also fits, it
// is staged in LDS once so the sweeps never touch global memory.  Each row is
// owned by lpr lanes (the largest power of two <= 16 with n * lpr <= 1024),
// so a sweep costs a few LDS round trips.  Each sweep computes all new values
// from the old x before any is written back (Jacobi).
// ----------------------------------------------------------------------------
constexpr int kCoarseLdsBytes = 65536;

}  // namespace

// The coarsest level is solved inside one workgroup when its matrix, inverse
// diagonal and iterate fit that workgroup's LDS; otherwise one launch per sweep.
bool coarse_in_lds(int n, int nnz, bool long_rows) {
    return !long_rows && n <= kCoarseLds &&
           (size_t)n * 16 + (size_t)nnz * 12 + (size_t)(n + 1) * 4 <= (size_t)kCoarseLdsBytes;
}

namespace {

// unit_rhs: the right-hand side is the unit vector e_j with j = blockIdx.x and
// the result goes to column j of x (n x n, column-major): this builds the dense
// matrix of the whole sweep operator, one workgroup per column.
template <typename VB, typename VX>
__global__ void __launch_bounds__(1024)
k_coarse(int n, int nnz, const int *__restrict__ rp_g, const int *__restrict__ ci_g,
         const double *__restrict__ a_g, const double *__restrict__ dinv_g, const VB *__restrict__ b,
         VX *__restrict__ x, int sweeps, int unit_rhs, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    __shared__ __align__(16) char lds[kCoarseLdsBytes];
    constexpr int R = kCoarseLds / 1024;
    double *xs = reinterpret_cast<double *>(lds);
    const size_t stage = (size_t)n * 16 + (size_t)nnz * 12 + (size_t)(n + 1) * 4;
    const bool staged = stage <= (size_t)kCoarseLdsBytes;
    const int *rp = rp_g, *ci = ci_g;
    const double *a = a_g, *dinv = dinv_g;
    if (staged) {
        double *ds = xs + n, *as = ds + n;
        int *rps = reinterpret_cast<int *>(as + nnz), *cis = rps + n + 1;
        for (int i = threadIdx.x; i < n; i += blockDim.x) ds[i] = dinv_g[i];
        for (int i = threadIdx.x; i <= n; i += blockDim.x) rps[i] = rp_g[i];
        for (int q = threadIdx.x; q < nnz; q += blockDim.x) { as[q] = a_g[q]; cis[q] = ci_g[q]; }
        rp = rps; ci = cis; a = as; dinv = ds;
    }
    int lpr = 1;
    while (lpr < 16 && n * (lpr * 2) <= (int)blockDim.x) lpr *= 2;
    const int lane = threadIdx.x % lpr, grp = threadIdx.x / lpr, ngrp = blockDim.x / lpr;
    double bl[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = grp + k * ngrp;
        bl[k] = i < n ? (unit_rhs ? (i == (int)blockIdx.x ? 1.0 : 0.0) : (double)b[i]) : 0.0;
    }
    if (unit_rhs) x += (size_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = 0.0;
    __syncthreads();
    for (int t = 0; t < sweeps; ++t) {
        double xn[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = grp + k * ngrp;
            xn[k] = 0.0;
            if (i < n) {
                double s = 0.0;
                const int e = rp[i + 1];
                for (int q = rp[i] + lane; q < e; q += lpr) s = s + a[q] * xs[ci[q]];
                for (int o = lpr / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, lpr);
                xn[k] = xs[i] + dinv[i] * (bl[k] - s);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = grp + k * ngrp;
            if (i < n && lane == 0) xs[i] = xn[k];
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (VX)xs[i];
}

// Dense operator applied to b: x = S b, S row-major n x n float64 (the
// coarsest level's sweep operator, or the folded small levels).  One workgroup
// per row i, four waves splitting the row so that enough loads are in flight.
template <typename VB, typename VX>
__global__ void __launch_bounds__(kBlock)
k_coarse_dense(int n, const double *__restrict__ S, const VB *__restrict__ b, VX *__restrict__ x,
               const double *__restrict__ done) {
    // the solve-ended flag is tested before the store only (as in k_down_seq)
    const int i = blockIdx.x;
    const double *row = S + (size_t)i * n;
    double s[1] = {0.0};
#pragma unroll 4
    for (int j = threadIdx.x; j < n; j += kBlock) s[0] += row[j] * (double)b[j];
    __shared__ double lds[16];
    block_sum<1>(s, lds);
    if (threadIdx.x == 0 && !(done && *done != 0.0)) x[i] = (VX)s[0];
}

// ----------------------------------------------------------------------------
// Folded coarse levels.  With one l1-Jacobi sweep from zero before and one
// after the coarse correction, the cycle of level k is the linear map
//   T_k = D + (I - D A)(D + P T_{k+1} P^T (I - A D))
// (D = diag(dinv), P the level's prolongator, T_{k+1} the coarser level's map;
// the coarsest level's map is its sweep operator S).  On the smallest levels
// it is formed once, densely, and the cycle from such a level is one dense
// product: the same operator as the level-by-level cycle, rounded differently.
// One thread per entry (i, j), j fastest.
// ----------------------------------------------------------------------------
// H = D + G (I - A D) with G = P Tc P^T, G_ij = p_i p_j Tc[agg_i][agg_j]:
//   H_ij = [i = j] dinv_i + G_ij - dinv_j sum_{k in row j} G_ik a_jk
// (a_kj = a_jk: A is symmetric).
__global__ void __launch_bounds__(kBlock)
k_fold_h(int n, int nc, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
         const double *__restrict__ dinv, const double *__restrict__ p, const int *__restrict__ agg,
         const double *__restrict__ Tc, double *__restrict__ H) {
    const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    const double *trow = Tc + (size_t)agg[i] * nc;
    const double pi = p[i];
    double s = 0.0;
    for (int q = rp[j]; q < rp[j + 1]; ++q) {
        const int k = ci[q];
        s += ((pi * p[k]) * trow[agg[k]]) * a[q];
    }
    const double gij = (pi * p[j]) * trow[agg[j]];
    H[idx] = (i == j ? dinv[i] : 0.0) + gij - dinv[j] * s;
}

// W-cycle: the coarse problem of a level is solved by two cycles of the level
// below, the second on the residual of the first: W = T + T (I - A T) = 2T - T A T.
// M = A T (sparse rows of A against the dense columns of T):
__global__ void __launch_bounds__(kBlock)
k_fold_at(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
          const double *__restrict__ T, double *__restrict__ M) {
    const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    double s = 0.0;
    for (int q = rp[i]; q < rp[i + 1]; ++q) s += a[q] * T[(size_t)ci[q] * n + j];
    M[idx] = s;
}

// W_ij = 2 T_ij - sum_k T_ik M_kj (one thread per entry; the row of T is
// shared by the wave, the column of M read coalesced)
__global__ void __launch_bounds__(kBlock)
k_fold_w(int n, const double *__restrict__ T, const double *__restrict__ M, double *__restrict__ W) {
    const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    const double *ti = T + (size_t)i * n;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += ti[k] * M[(size_t)k * n + j];
    W[idx] = 2.0 * T[idx] - s;
}

// T = D + (I - D A) H:  T_ij = [i = j] dinv_i + H_ij - dinv_i sum_{k in row i} a_ik H_kj
// One wave per row i and 64 consecutive columns j: row i's entries are the
// same for the whole wave (scalar loads), each H load is one contiguous
// access, and four entries' loads are issued per step.  The sum runs over
// row i in order, as with one thread per entry.
constexpr int kFoldCols = 64;
inline long long fold_t_threads(int n) { return (long long)n * ((n + kFoldCols - 1) / kFoldCols) * kFoldCols; }
__global__ void __launch_bounds__(kBlock)
k_fold_t(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
         const double *__restrict__ dinv, const double *__restrict__ H, double *__restrict__ T) {
    const int nch = (n + kFoldCols - 1) / kFoldCols;
    const long long wv = ((long long)blockIdx.x * kBlock + threadIdx.x) / kFoldCols;
    if (wv >= (long long)n * nch) return;
    const int i = __builtin_amdgcn_readfirstlane((int)(wv / nch));
    const int jc = __builtin_amdgcn_readfirstlane((int)(wv % nch));
    const int j = jc * kFoldCols + (int)(threadIdx.x % kFoldCols);
    const int jj = j < n ? j : n - 1;  // lanes past the last column read a valid one and store nothing
    const int e = rp[i + 1];
    int q = rp[i];
    double s = 0.0;
    for (; q + 4 <= e; q += 4) {
        const double h0 = H[(size_t)ci[q] * n + jj], h1 = H[(size_t)ci[q + 1] * n + jj];
        const double h2 = H[(size_t)ci[q + 2] * n + jj], h3 = H[(size_t)ci[q + 3] * n + jj];
        s += a[q] * h0;
        s += a[q + 1] * h1;
        s += a[q + 2] * h2;
        s += a[q + 3] * h3;
    }
    for (; q < e; ++q) s += a[q] * H[(size_t)ci[q] * n + jj];
    if (j < n) {
        const size_t idx = (size_t)i * n + j;
        T[idx] = (i == j ? dinv[i] : 0.0) + H[idx] - dinv[i] * s;
    }
}

// ----------------------------------------------------------------------------
// Tail of the cycle: every level k >= kt (all with at most kTailRows rows) and
// the coarsest solve, inside one workgroup of 1024 threads, with phases
// separated by barriers instead of kernel launches.  Down legs (one thread per
// aggregate, members in ascending order), then the coarsest solve (dense
// operator, or l1-Jacobi sweeps with x in LDS), then the up legs.  Same
// arithmetic as the per-level kernels.
// ----------------------------------------------------------------------------
template <typename V>
__global__ void __launch_bounds__(1024)
k_tail(int kt, int nl, const TailLevel *__restrict__ tl, const double *__restrict__ S,
       const double *__restrict__ cdinv, const double *__restrict__ ca, int sweeps, const int *__restrict__ ops,
       int nops, V *__restrict__ x_out, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    __shared__ double xs[kTailRows];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int o = 0; o < nops; ++o) {
        const int op = ops[o] & 0xff, k = (ops[o] >> 8) & 0xff, sel = (ops[o] >> 16) & 0xff;
        const TailLevel L = tl[k];
        const V *a = (const V *)L.a, *dinv = (const V *)L.dinv, *p = (const V *)L.p;
        V *b = (V *)L.b;
        // output of UP / COARSE: x, or the level's save buffer, or the caller's
        // vector for the top level's x
        V *xo = sel ? (V *)L.xs : (k == kt ? x_out : (V *)L.x);
        if (op == kTailDown) {
            // b_c[E] = sum_{i in E} p_i (b_i - sum_j a_ij dinv_j b_j)
            V *bc = (V *)tl[k + 1].b;
            int lpr = 1;
            while (lpr < 16 && L.nc * (lpr * 2) <= nt) lpr *= 2;
            const int lane = tid % lpr, ngrp = nt / lpr;
            for (int E = tid / lpr; E < L.nc; E += ngrp) {
                V acc = V(0);
                for (int t = 0; t < L.mstride; ++t) {
                    const int i = L.mem[(size_t)E * L.mstride + t];
                    if (i < 0) break;
                    V s = V(0);
                    for (int q = L.rp[i] + lane; q < L.rp[i + 1]; q += lpr) {
                        const int j = L.ci[q];
                        s += a[q] * (dinv[j] * b[j]);
                    }
                    for (int m = lpr / 2; m > 0; m >>= 1) s += __shfl_xor(s, m, lpr);
                    acc += p[i] * (b[i] - s);
                }
                if (lane == 0) bc[E] = acc;
            }
        } else if (op == kTailUp) {
            // x = D b + P x_c, then x += D (b - A x), with x formed on the fly
            const V *xc = (const V *)tl[k + 1].x;
            int lpr = 1;
            while (lpr < 16 && L.n * (lpr * 2) <= nt) lpr *= 2;
            const int lane = tid % lpr, ngrp = nt / lpr;
            for (int i = tid / lpr; i < L.n; i += ngrp) {
                V s = V(0);
                for (int q = L.rp[i] + lane; q < L.rp[i + 1]; q += lpr) {
                    const int j = L.ci[q];
                    s += a[q] * (dinv[j] * b[j] + p[j] * xc[L.agg[j]]);
                }
                for (int m = lpr / 2; m > 0; m >>= 1) s += __shfl_xor(s, m, lpr);
                if (lane == 0) {
                    const V bi = b[i], di = dinv[i];
                    const V xi = di * bi + p[i] * xc[L.agg[i]];
                    xo[i] = xi + di * (bi - s);
                }
            }
        } else if (op == kTailResid) {
            // W-cycle: b <- b - A x on this level
            const V *x = (const V *)L.x;
            int lpr = 1;
            while (lpr < 16 && L.n * (lpr * 2) <= nt) lpr *= 2;
            const int lane = tid % lpr, ngrp = nt / lpr;
            for (int i = tid / lpr; i < L.n; i += ngrp) {
                V s = V(0);
                for (int q = L.rp[i] + lane; q < L.rp[i + 1]; q += lpr) s += a[q] * x[L.ci[q]];
                for (int m = lpr / 2; m > 0; m >>= 1) s += __shfl_xor(s, m, lpr);
                if (lane == 0) b[i] = b[i] - s;
            }
        } else if (op == kTailAdd) {
            V *x = (V *)L.x;
            const V *y = (const V *)L.xs;
            for (int i = tid; i < L.n; i += nt) x[i] = x[i] + y[i];
        } else {  // kTailCoarse: 20 l1-Jacobi sweeps from zero in float64 (dense operator when built)
            const int n = L.n;
            if (S) {
                int lpr = 1;
                while (lpr < 64 && n * (lpr * 2) <= nt) lpr *= 2;
                const int lane = tid % lpr, ngrp = nt / lpr;
                for (int i = tid / lpr; i < n; i += ngrp) {
                    double s = 0.0;
                    for (int j = lane; j < n; j += lpr) s += S[(size_t)i * n + j] * (double)b[j];
                    for (int m = lpr / 2; m > 0; m >>= 1) s += __shfl_xor(s, m, lpr);
                    if (lane == 0) xo[i] = (V)s;
                }
            } else {
                for (int i = tid; i < n; i += nt) xs[i] = 0.0;
                __syncthreads();
                constexpr int R = (kTailRows + 1023) / 1024;
                for (int t = 0; t < sweeps; ++t) {
                    double xn[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int i = tid + r * nt;
                        xn[r] = 0.0;
                        if (i < n) {
                            double s = 0.0;
                            for (int q = L.rp[i]; q < L.rp[i + 1]; ++q) s = s + ca[q] * xs[L.ci[q]];
                            xn[r] = xs[i] + cdinv[i] * ((double)b[i] - s);
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int i = tid + r * nt;
                        if (i < n) xs[i] = xn[r];
                    }
                    __syncthreads();
                }
                for (int i = tid; i < n; i += nt) xo[i] = (V)xs[i];
            }
        }
        __syncthreads();
    }
}

// One l1-Jacobi sweep of a coarsest level too large for one workgroup's LDS:
// xn = xo + D (b - A xo) (first: xo = 0, so xn = D b).  G lanes per row and R
// rows per group, as in the cycle kernels.  The last sweep of a solve writes
// the caller's x (type VX) instead of xn.  The solve-ended flag is tested
// before the stores only (as in k_down_seq).
template <int G, int R, typename VB, typename VX, bool LF>
__global__ void __launch_bounds__(kBlock)
k_jacobi_sweep(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
               const double *__restrict__ dinv, const VB *__restrict__ b, const double *__restrict__ xo,
               double *__restrict__ xn, VX *__restrict__ xout, int first, const double *__restrict__ done,
               LongView<double> lv, LongFused lf) {
    if (LF && (int)blockIdx.x >= lf.nrb) {  // a chunk of a long row (see long_chunk); never the first sweep
        if (done && *done != 0.0) return;
        long_chunk<double>((int)blockIdx.x - lf.nrb, lf.lr, rp, ci, a, FGather<double, double>{xo},
                           [&](int i, double sl) {
                               if (threadIdx.x != 0) return;
                               const double v = xo[i] + dinv[i] * ((double)b[i] - sl);
                               if (xout) xout[i] = (VX)v;
                               else xn[i] = v;
                           });
        return;
    }
    const int lane = threadIdx.x % G;
    const int g = (xcd_block(blockIdx.x, LF ? lf.nrb : gridDim.x) * kBlock + threadIdx.x) / G;
    int rows[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rows[k] = g * R + k < n ? g * R + k : -1;
    double s[R];
    int lgm = 0;
    if (first) {
#pragma unroll
        for (int k = 0; k < R; ++k) s[k] = 0.0;
    } else {
        rows_dot<G, R, double>(rp, ci, a, rows, s, FGather<double, double>{xo}, lv, &lgm);
    }
    const bool live = !(done && *done != 0.0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = rows[k];
        if (lane == k % G && i >= 0 && live && !(LF && ((lgm >> k) & 1))) {
            const double v = (first ? 0.0 : xo[i]) + dinv[i] * ((double)b[i] - s[k]);
            if (xout) xout[i] = (VX)v;
            else xn[i] = v;
        }
    }
}

// block_sum with its final additions spread over the threads:
// thread k (k < K, K <= blockDim.x) returns sum k, added in block_sum's order.
template <int K>
__device__ __forceinline__ double block_sum_spread(double (&v)[K], double *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = group_sum<64>(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k * 16 + wid] = v[k];
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x < K) {
        s = lds[threadIdx.x * 16];
        for (int w = 1; w < nw; ++w) s += lds[threadIdx.x * 16 + w];
    }
    __syncthreads();
    return s;
}

// The coarse solve on a star level (StarView): E_m over the hub row's
// entries, m < sweeps - 1, one partial per workgroup and m.
template <typename VB>
__global__ void __launch_bounds__(kBlock)
k_star_sums(StarView sv, int sweeps, const double *__restrict__ dinv, const VB *__restrict__ b,
            const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    constexpr int K = kStarMaxSweeps - 1;
    __shared__ double lds[K * 16];
    double acc[K];
#pragma unroll
    for (int m = 0; m < K; ++m) acc[m] = 0.0;
    for (int q = blockIdx.x * kBlock + threadIdx.x; q < sv.nh; q += gridDim.x * kBlock) {
        const int j = sv.hj[q];
        const double cj = sv.c[j];
        double t = sv.ha[q] * (dinv[j] * (double)b[j]);
#pragma unroll
        for (int m = 0; m < K; ++m)
            if (m < sweeps - 1) {
                acc[m] += t;
                t *= cj;
            }
    }
    // the workgroup's sums, each finished by its own thread
    const double e = block_sum_spread<K>(acc, lds);
    if (threadIdx.x < K) sv.part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = e;
}

// One workgroup: E_m from the partials (in workgroup order), then the hub's
// values x_h^(t), t = 0 .. sweeps, by the recurrence; writes x at the hub.
// The hub's recurrence for S sweeps known at compile time, every value in a
// register; the same operations in the same order as the loop in k_star_hub.
constexpr int kCoarseSweeps = 20;  // the coarse solve's default sweep count
template <int S>
__device__ __forceinline__ void star_recurrence(const double *se, const double *sf, double bh, const StarView &sv) {
    double e[S], f[S], xh[S + 1];
#pragma unroll
    for (int m = 0; m < S - 1; ++m) { e[m] = se[m]; f[m] = sf[m]; }
    xh[0] = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        double sum = 0.0;
#pragma unroll
        for (int t = 0; t < k; ++t) sum += e[k - 1 - t] - f[k - 1 - t] * xh[t];
        xh[k + 1] = xh[k] + sv.dh * (bh - (sv.ahh * xh[k] + sum));
    }
#pragma unroll
    for (int t = 0; t <= S; ++t) sv.xh[t] = xh[t];
}

template <typename VB, typename VX>
__global__ void __launch_bounds__(kBlock)
k_star_hub(StarView sv, int sweeps, const VB *__restrict__ b, VX *__restrict__ x, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    constexpr int K = kStarMaxSweeps - 1;
    __shared__ double lds[K * 16];
    __shared__ double se[K], sf[K], xh[kStarMaxSweeps + 1];  // the recurrence reads these at run-time indices
    if (threadIdx.x < K) sf[threadIdx.x] = threadIdx.x < sweeps - 1 ? sv.F[threadIdx.x] : 0.0;
    double e[K];
#pragma unroll
    for (int m = 0; m < K; ++m) e[m] = 0.0;
    add_partials<K, 1>(e, sv.part, kStarBlocks);
    const double em = block_sum_spread<K>(e, lds);
    if (threadIdx.x < K) se[threadIdx.x] = em;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double bh = (double)b[sv.hub];
    if (sweeps == kCoarseSweeps) {
        star_recurrence<kCoarseSweeps>(se, sf, bh, sv);  // in registers: no LDS round trip per term
    } else {
        xh[0] = 0.0;
        for (int k = 0; k < sweeps; ++k) {
            double sum = 0.0;  // the hub row's product after k sweeps, off the diagonal
            for (int t = 0; t < k; ++t) sum += se[k - 1 - t] - sf[k - 1 - t] * xh[t];
            xh[k + 1] = xh[k] + sv.dh * (bh - (sv.ahh * xh[k] + sum));
        }
        for (int t = 0; t <= sweeps; ++t) sv.xh[t] = xh[t];
    }
    x[sv.hub] = (VX)sv.xh[sweeps];
}

// Every row but the hub: its sweeps with the hub's values x_h^(t), each in
// the order and rounding of k_jacobi_sweep (the row's two products in column
// order).
template <typename VB, typename VX>
__global__ void __launch_bounds__(kBlock)
k_star_rows(StarView sv, int n, int sweeps, const int *__restrict__ rp, const int *__restrict__ ci,
            const double *__restrict__ a, const double *__restrict__ dinv, const VB *__restrict__ b,
            VX *__restrict__ x, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n || j == sv.hub) return;
    const int s0 = rp[j], e0 = rp[j + 1];
    double ajj = 0.0, ajh = 0.0;
    bool hub_first = false;
    for (int q = s0; q < e0; ++q) {
        if (ci[q] == j) ajj = a[q];
        else { ajh = a[q]; hub_first = q == s0; }
    }
    const double dj = dinv[j], bj = (double)b[j];
    double xj = 0.0;
    for (int t = 0; t < sweeps; ++t) {
        const double xt = sv.xh[t];
        const double rs = hub_first ? ajh * xt + ajj * xj : ajj * xj + ajh * xt;
        xj = xj + dj * (bj - rs);
    }
    x[j] = (VX)xj;
}

// ----------------------------------------------------------------------------
// Flexible CG kernels (Algorithm 3).  Fixed grid of nb blocks with a
// grid-stride loop over row groups; every block stores its partial sums and a
// one-block finalize kernel adds them in block order (deterministic).
// scal: [0] alpha [1] beta [2] gamma [4] ||r||^2 [5] ||b||^2 [6] breakdown
//       flag [7] update partials not yet taken by the stop test
//       [8] gamma_i / rho_{i-1} [9] alpha_i / rho_i [10] loop ended
//       [11] iterations [12] tol^2 ||b||^2 [13] itmax [14], [15] rho ring
// ----------------------------------------------------------------------------

constexpr int kRows = 4;  // rows per lane group in the streaming row kernels

// r = b - A u; partials of ||r||^2 and ||b||^2
template <int G>
__global__ void __launch_bounds__(kBlock)
k_resid(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
        const double *__restrict__ b, const double *__restrict__ u, double *__restrict__ r,
        double *__restrict__ partials, LongView<double> lv) {
    constexpr int NG = kBlock / G, R = kRows;
    const int lane = threadIdx.x % G;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    double acc[2] = {0.0, 0.0};
    for (int base = blk * NG * R + threadIdx.x / G; base < n; base += gridDim.x * NG * R) {
        int rows[R];
#pragma unroll
        for (int k = 0; k < R; ++k) rows[k] = base + k * NG < n ? base + k * NG : -1;
        double s[R];
        rows_dot<G, R, double>(rp, ci, a, rows, s, FGather<double, double>{u}, lv);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (rows[k] < 0) continue;
                const double bi = b[rows[k]];
                const double ri = bi - s[k];
                r[rows[k]] = ri;
                acc[0] += ri * ri;
                acc[1] += bi * bi;
            }
        }
    }
    block_partials<2>(acc, partials);
}

// v = A w with partials of alpha = w.r, beta = w.v, gamma = w.q in the same pass
template <int G>
__global__ void __launch_bounds__(kBlock)
k_spmv_dots(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
            const double *__restrict__ w, const double *__restrict__ r, const double *__restrict__ q,
            double *__restrict__ v, double *__restrict__ partials, const double *__restrict__ done,
            LongView<double> lv) {
    if (done && *done != 0.0) return;
    constexpr int NG = kBlock / G, R = kRows;
    const int lane = threadIdx.x % G;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int base = blk * NG * R + threadIdx.x / G; base < n; base += gridDim.x * NG * R) {
        int rows[R];
#pragma unroll
        for (int k = 0; k < R; ++k) rows[k] = base + k * NG < n ? base + k * NG : -1;
        double s[R];
        rows_dot<G, R, double>(rp, ci, a, rows, s, FGather<double, double>{w}, lv);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = rows[k];
                if (i < 0) continue;
                const double wi = w[i];
                v[i] = s[k];
                acc[0] += wi * r[i];
                acc[1] += wi * s[k];
                acc[2] += wi * q[i];
            }
        }
    }
    block_partials<3>(acc, partials);
}


// Finalize: sums the block partials in block order, then
//   mode 0 (residual):  scal[4] = ||r||^2, scal[5] = ||b||^2
//   mode 1 (dots):      alpha, beta, gamma and the scalars of Algorithm 3
//                       (fcg_scalars): scal[8] = gamma / rho_{i-1},
//                       scal[9] = alpha / rho_i, scal[6] = 1 on breakdown
//                       (the update forms them itself when it gets the
//                       product's partials: no mode-1 launch then)
//   mode 2 (norm):      the stop test (stop_norm): scal[4] = ||r||^2,
//                       scal[11] += 1 (iterations done); a no-op when the
//                       first kernel of the next cycle has taken it already
// In the iteration loop (modes 1, 2) scal[10] != 0 means the solve has ended:
// every kernel of a later iteration returns at once.  Mode 2 sets it when
// ||r||^2 <= scal[12] (= tol^2 ||b||^2) or scal[11] >= scal[13] (itmax); mode 1
// sets it, with scal[6], on breakdown.
// One workgroup: kBlock threads for up to 8 x kBlock partials (their loads in
// flight in one round trip), kFinalize threads beyond that (the product that
// takes one workgroup per slice writes one partial per slice).
constexpr int kFinalize = 1024;
inline int finalize_threads(int nb) { return nb > 8 * kBlock ? kFinalize : kBlock; }
template <int K>
__global__ void __launch_bounds__(kFinalize) k_finalize(int nb, const double *__restrict__ partials,
                                                     double *__restrict__ scal, int mode, int first) {
    if (mode != 0 && scal[10] != 0.0) return;
    if (mode == 2 && scal[7] == 0.0) return;  // the next cycle's stop test took them
    __shared__ double lds[K * 16];
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    add_partials<K>(s, partials, nb);
    block_sum<K>(s, lds);
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        scal[4] = s[0];
        scal[5] = s[1 % K];
        scal[7] = 0.0;
    } else if (mode == 2) {
        (void)stop_norm(s[0], scal);
    } else {
        const double d3[3] = {s[0], s[1 % K], s[2 % K]};
        double g, an;
        (void)fcg_scalars(d3, first, scal, true, g, an);
    }
}


// dL/da_ij = -lambda_i x_j on the stored pattern.  R rows per group of G
// lanes, the loads of their first G entries all issued before any store (as in
// rows_dot), so a wave keeps R times more requests in flight.
template <int G, int R>
__global__ void __launch_bounds__(kBlock)
k_sampled_outer(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ lam,
                const double *__restrict__ x, double *__restrict__ out, int lmin) {
    // rows longer than lmin are written by k_long_outer
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int base = xcd_block(blockIdx.x, gridDim.x) * NG * R + threadIdx.x / G;
    int beg[R], end[R];
    double li[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = base + k * NG;
        const int ic = i < n ? i : 0;
        beg[k] = rp[ic];
        const int e = rp[ic + 1];
        end[k] = (i < n && e - beg[k] <= lmin) ? e : beg[k];
        li[k] = lam[ic];
    }
    int j[R];
#pragma unroll
    for (int k = 0; k < R; ++k) j[k] = beg[k] + lane < end[k] ? ci[beg[k] + lane] : 0;
    double xv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) xv[k] = x[j[k]];
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (beg[k] + lane < end[k]) out[beg[k] + lane] = -(li[k] * xv[k]);
#pragma unroll
    for (int k = 0; k < R; ++k)
        for (int q = beg[k] + lane + G; q < end[k]; q += G) out[q] = -(li[k] * x[ci[q]]);
}

// The long rows of the sampled outer product, chunk by chunk.
__global__ void __launch_bounds__(kBlock)
k_long_outer(LongRows lr, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ lam,
             const double *__restrict__ x, double *__restrict__ out) {
    const int c = blockIdx.x;
    const int t = chunk_owner(lr.cb, lr.n, c);
    const int row = lr.rows[t];
    const int q0 = rp[row] + (c - lr.cb[t]) * kSegChunk, q1 = min(q0 + kSegChunk, rp[row + 1]);
    const double li = lam[row];
    for (int q = q0 + threadIdx.x; q < q1; q += kBlock) out[q] = -(li * x[ci[q]]);
}

// The chunk sums of level L's long rows for a row kernel with operand f.
template <typename V, typename F>
void long_pre(hipStream_t s, const Level &L, const V *a, F f, const double *done) {
    if (L.lr.n > 0)
        hipLaunchKernelGGL((k_long_dot<V, F>), dim3(L.lr.nchunks), dim3(kBlock), 0, s, L.lr, L.A.rp, L.A.ci, a, f,
                           static_cast<V *>(L.lr.part), done);
}

// The long rows of a level in the row kernel's own launch (LongFused), when
// the level has their arrival counters.
LongFused long_fused(const Level &L, int nrb) {
    LongFused lf;
    if (L.lr.n > 0 && L.lr.cnt) {
        lf.nrb = nrb;
        lf.lr = L.lr;
    }
    return lf;
}

template <int G, typename V, typename VB>
void down_dispatch(hipStream_t s, const Level &L, const V *a, const V *dinv, const V *p, const VB *b, V *bc,
                   const double *done) {
    const int S = L.mstride;
    const dim3 grid(blocks_for((long long)L.nc * G));
    const LongView<V> lv = long_view<V>(L.lr);
    // (the down leg keeps the pre-pass: its finishing block would have to
    // build a whole aggregate, which measured slower than the separate launch)
    long_pre(s, L, a, FScaled<V, VB>{dinv, b}, done);
    auto seq = [&](auto sc) {
        constexpr int SS = decltype(sc)::value;
        launch_k((k_down_seq<G, SS, V, VB>), grid, dim3(kBlock), s, L.nc, L.mem, L.A.rp, L.A.ci, a, dinv, p, b, bc,
                 done, lv);
    };
    if (S == 1) seq(std::integral_constant<int, 1>{});
    else if (S == 2) seq(std::integral_constant<int, 2>{});
    else if (S == 4) seq(std::integral_constant<int, 4>{});
    else
        launch_k((k_down_loop<G, V, VB>), grid, dim3(kBlock), s, L.nc, L.mstride, L.mem, L.A.rp,
                           L.A.ci, a, dinv, p, b, bc, done, lv);
}

// part: 0 = the whole leg, 1 = its first kernel, 2 = its second kernel (a
// leg of one kernel has it as part 1 of the down leg and part 2 of the up leg)
// yr: dinv o b already formed by the caller (the flexible-CG update, or the
// finer level's restriction), or null.  cd, cy: the coarser level's dinv and
// dinv o b, formed by the restriction here when cy is given.
template <typename V, typename VB>
void down_t(hipStream_t s, const Level &L, const V *a, const V *dinv, const V *p, const VB *b, V *bc,
            const double *done, int part, const V *yr, const V *cd, V *cy, StopTest st) {
    if (down_on_sell(L)) {
        V *pr = (V *)L.xp;  // free during the down leg: the up leg of this level runs later
        const V *y = yr ? yr : (const V *)L.yb;
        if (part != 2) {
            if (!yr && L.yb)
                hipLaunchKernelGGL((k_scale<V, VB>), dim3(blocks_for(L.A.n)), dim3(kBlock), 0, s, L.A.n, dinv, b,
                                   (V *)L.yb, done);
            with_sell<V>(L.E, [&](auto *ix, auto *vals, auto kb) {
                using I = std::remove_const_t<std::remove_pointer_t<decltype(ix)>>;
                using S = std::remove_const_t<std::remove_pointer_t<decltype(vals)>>;
                // NT: the values streamed non-temporally (Sell::stream)
                auto go = [&](auto nt) {
                    constexpr bool NT = decltype(nt)::value;
                    constexpr int B = decltype(kb)::value;
                    if (split_slots(L, B))
                        launch_k((k_down_res_sell_p<V, VB, I, S, 8, NT>), dim3(L.E.nslices), dim3(kBlock), s, L.A.n,
                                 L.E.sp, L.E.uni, L.E.su, ix, vals, dinv, p, b, pr, (const V *)y, done, st);
                    else if (std::is_same<V, float>::value && L.E.svd && !y)  // values of A D: one gather per term
                        launch_k((k_down_res_sell_ad<VB, I, B, NT>), dim3(blocks_for(L.A.n)), dim3(kBlock), s, L.A.n,
                                 L.E.sp, L.E.uni, L.E.su, ix, (const float *)L.E.svd, (const float *)p, b, (float *)pr,
                                 done, st);
                    else
                        launch_k((k_down_res_sell<V, VB, I, S, B, NT>), dim3(blocks_for(L.A.n)), dim3(kBlock), s,
                                 L.A.n, L.E.sp, L.E.uni, L.E.su, ix, vals, dinv, p, b, pr, (const V *)y, done, st);
                };
                if (L.E.stream) go(std::true_type{});
                else go(std::false_type{});
            });
        }
        if (part == 1) return;
        if (L.mstride == 4)
            hipLaunchKernelGGL((k_restrict<V, 4>), dim3(blocks_for(L.nc)), dim3(kBlock), 0, s, L.nc, L.mem, pr, bc,
                               cd, cy, done);
        else
            hipLaunchKernelGGL((k_restrict<V, 2>), dim3(blocks_for(L.nc)), dim3(kBlock), 0, s, L.nc, L.mem, pr, bc,
                               cd, cy, done);
        return;
    }
    if (part == 2) return;
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        down_dispatch<g, V, VB>(s, L, a, dinv, p, b, bc, done);
    });
}

template <typename V, typename VB, typename VX>
void up_t(hipStream_t s, const Level &L, const V *a, const V *dinv, const V *p, const VB *b, const V *xc,
          VX *x, const double *done, int part) {
    if (L.xp) {
        V *xp = (V *)L.xp;
        if (part != 2)
            hipLaunchKernelGGL((k_prolong<V, VB>), dim3(blocks_for(L.A.n)), dim3(kBlock), 0, s, L.A.n, dinv, p, L.agg,
                               b, xc, xp, done);
        if (part == 1) return;
        if (L.E.sp) {
            with_sell<V>(L.E, [&](auto *ix, auto *vals, auto kb) {
                using I = std::remove_const_t<std::remove_pointer_t<decltype(ix)>>;
                using S = std::remove_const_t<std::remove_pointer_t<decltype(vals)>>;
                if (split_slots(L, decltype(kb)::value))
                    launch_k((k_smooth_sell_p<V, VB, VX, I, S, 8>), dim3(L.E.nslices), dim3(kBlock), s, L.A.n, L.E.sp,
                             L.E.uni, L.E.su, ix, vals, dinv, b, xp, x, done);
                else if (L.E.stream)  // values streamed non-temporally
                    launch_k((k_smooth_sell<V, VB, VX, I, S, decltype(kb)::value, true>), dim3(blocks_for(L.A.n)),
                             dim3(kBlock), s, L.A.n, L.E.sp, L.E.uni, L.E.su, ix, vals, dinv, b, xp, x, done);
                else
                    launch_k((k_smooth_sell<V, VB, VX, I, S, decltype(kb)::value, false>), dim3(blocks_for(L.A.n)),
                             dim3(kBlock), s, L.A.n, L.E.sp, L.E.uni, L.E.su, ix, vals, dinv, b, xp, x, done);
            });
            return;
        }
        long_pre(s, L, a, FGather<V, V>{xp}, done);
        with_G(L.G, [&](auto gc) {
            constexpr int g = decltype(gc)::value;
            constexpr int R = 2;
            launch_k((k_smooth<g, R, V, VB, VX>), dim3(blocks_for(((long long)L.A.n * g + R - 1) / R)),
                               dim3(kBlock), s, L.A.n, L.A.rp, L.A.ci, a, dinv, b, xp, x, done, long_view<V>(L.lr));
        });
        return;
    }
    if (part == 1) return;
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        constexpr int R = 2;
        dim3 grid(blocks_for(((long long)L.A.n * g + R - 1) / R));
        LongView<V> lv = long_view<V>(L.lr);
        const LongFused lf = long_fused(L, (int)grid.x);
        if (lf.nrb > 0) {
            grid.x += L.lr.nchunks;
            lv.part = nullptr;
        } else {
            long_pre(s, L, a, FProlonged<V, VB>{dinv, p, L.agg, b, xc}, done);
        }
        if (lf.nrb > 0)
            launch_k((k_up<g, R, V, VB, VX, true>), grid, dim3(kBlock), s, L.A.n, L.A.rp, L.A.ci, a, dinv, p, L.agg, b,
                     xc, x, done, lv, lf);
        else
            launch_k((k_up<g, R, V, VB, VX, false>), grid, dim3(kBlock), s, L.A.n, L.A.rp, L.A.ci, a, dinv, p, L.agg,
                     b, xc, x, done, lv, lf);
    });
}

template <typename VB, typename VX>
void coarse_t(hipStream_t s, const Level &L, int sweeps, const VB *b, VX *x, double *ta, double *tb,
              const double *done) {
    const int n = L.A.n;
    if (L.S) {
        hipLaunchKernelGGL((k_coarse_dense<VB, VX>), dim3(n), dim3(kBlock), 0, s, n, L.S, b, x, done);
        return;
    }
    if (coarse_in_lds(n, L.A.nnz, L.lr.n > 0)) {
        hipLaunchKernelGGL((k_coarse<VB, VX>), dim3(1), dim3(1024), 0, s, n, L.A.nnz, L.A.rp, L.A.ci, L.A.v, L.dinv,
                           b, x, sweeps, 0, done);
        return;
    }
    if (L.star.hub >= 0 && sweeps >= 1 && sweeps <= kStarMaxSweeps) {
        // a star: the sweeps as the hub's recurrence (three launches instead of one per sweep)
        hipLaunchKernelGGL((k_star_sums<VB>), dim3(kStarBlocks), dim3(kBlock), 0, s, L.star, sweeps, L.dinv, b, done);
        hipLaunchKernelGGL((k_star_hub<VB, VX>), dim3(1), dim3(kBlock), 0, s, L.star, sweeps, b, x, done);
        hipLaunchKernelGGL((k_star_rows<VB, VX>), dim3(blocks_for(n)), dim3(kBlock), 0, s, L.star, n, sweeps, L.A.rp,
                           L.A.ci, L.A.v, L.dinv, b, x, done);
        return;
    }
    double *xo = ta, *xn = tb;
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        constexpr int R = 2;
        for (int t = 0; t < sweeps; ++t) {
            dim3 grid(blocks_for(((long long)n + R - 1) / R * g));
            LongView<double> lv = long_view<double>(L.lr);
            // (the first sweep, from zero, has no products)
            const LongFused lf = t > 0 ? long_fused(L, (int)grid.x) : LongFused();
            if (lf.nrb > 0) {
                grid.x += L.lr.nchunks;
                lv.part = nullptr;
            } else if (t > 0) {
                long_pre(s, L, (const double *)L.A.v, FGather<double, double>{xo}, done);
            }
            if (lf.nrb > 0)
                hipLaunchKernelGGL((k_jacobi_sweep<g, R, VB, VX, true>), grid, dim3(kBlock), 0, s, n, L.A.rp, L.A.ci,
                                   L.A.v, L.dinv, b, xo, xn, t == sweeps - 1 ? x : (VX *)nullptr, 0, done, lv, lf);
            else
                hipLaunchKernelGGL((k_jacobi_sweep<g, R, VB, VX, false>), grid, dim3(kBlock), 0, s, n, L.A.rp, L.A.ci,
                                   L.A.v, L.dinv, b, xo, xn, t == sweeps - 1 ? x : (VX *)nullptr, t == 0 ? 1 : 0, done,
                                   lv, lf);
            double *tmp = xo; xo = xn; xn = tmp;
        }
    });
}

}  // namespace

int reduce_blocks(int n) {
    long long b = ((long long)n + kBlock - 1) / kBlock;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

void launch_down(hipStream_t s, const Level &L, int fp32, const void *b, void *bc, int b_is_f64,
                 const double *done, int part, const void *yr, const Level *next, StopTest st) {
    void *cy = next ? next->yb : nullptr;
    if (!fp32) {
        down_t<double, double>(s, L, L.A.v, L.dinv, L.p, (const double *)b, (double *)bc, done, part,
                               (const double *)yr, cy ? next->dinv : nullptr, (double *)cy, st);
    } else if (b_is_f64) {
        down_t<float, double>(s, L, L.A.v32, L.dinv32, L.p32, (const double *)b, (float *)bc, done, part,
                              (const float *)yr, cy ? next->dinv32 : nullptr, (float *)cy, st);
    } else {
        down_t<float, float>(s, L, L.A.v32, L.dinv32, L.p32, (const float *)b, (float *)bc, done, part,
                             (const float *)yr, cy ? next->dinv32 : nullptr, (float *)cy, st);
    }
}

void launch_up(hipStream_t s, const Level &L, int fp32, const void *b, const void *xc, void *x, int b_is_f64,
               int x_is_f64, const double *done, int part) {
    if (!fp32) {
        up_t<double, double, double>(s, L, L.A.v, L.dinv, L.p, (const double *)b, (const double *)xc, (double *)x,
                                     done, part);
    } else if (b_is_f64 && x_is_f64) {
        up_t<float, double, double>(s, L, L.A.v32, L.dinv32, L.p32, (const double *)b, (const float *)xc,
                                    (double *)x, done, part);
    } else {
        up_t<float, float, float>(s, L, L.A.v32, L.dinv32, L.p32, (const float *)b, (const float *)xc, (float *)x,
                                  done, part);
    }
}

void launch_coarse(hipStream_t s, const Level &L, int sweeps, const void *b, void *x, int b_f64, int x_f64,
                   void *tmp_a, void *tmp_b, const double *done) {
    double *ta = (double *)tmp_a, *tb = (double *)tmp_b;
    if (b_f64 && x_f64) coarse_t<double, double>(s, L, sweeps, (const double *)b, (double *)x, ta, tb, done);
    else coarse_t<float, float>(s, L, sweeps, (const float *)b, (float *)x, ta, tb, done);
}

void launch_tail(hipStream_t s, int fp32, int kt, int nl, const TailLevel *tl, const Level &C, int sweeps,
                 const int *ops, int nops, void *x_out, const double *done) {
    if (fp32)
        hipLaunchKernelGGL((k_tail<float>), dim3(1), dim3(1024), 0, s, kt, nl, tl, C.S, C.dinv, C.A.v, sweeps, ops,
                           nops, (float *)x_out, done);
    else
        hipLaunchKernelGGL((k_tail<double>), dim3(1), dim3(1024), 0, s, kt, nl, tl, C.S, C.dinv, C.A.v, sweeps, ops,
                           nops, (double *)x_out, done);
}

void launch_resid_inplace(hipStream_t s, const Level &L, int fp32, const void *x, void *b, const double *done) {
    if (fp32) long_pre(s, L, (const float *)L.A.v32, FGather<float, float>{(const float *)x}, done);
    else long_pre(s, L, (const double *)L.A.v, FGather<double, double>{(const double *)x}, done);
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (fp32)
            hipLaunchKernelGGL((k_resid_inplace<g, float>), dim3(blocks_for((long long)L.A.n * g)), dim3(kBlock), 0, s,
                               L.A.n, L.A.rp, L.A.ci, L.A.v32, (const float *)x, (float *)b, done,
                               long_view<float>(L.lr));
        else
            hipLaunchKernelGGL((k_resid_inplace<g, double>), dim3(blocks_for((long long)L.A.n * g)), dim3(kBlock), 0,
                               s, L.A.n, L.A.rp, L.A.ci, L.A.v, (const double *)x, (double *)b, done,
                               long_view<double>(L.lr));
    });
}

void launch_add(hipStream_t s, int n, int fp32, const void *y, void *x, const double *done) {
    if (fp32)
        hipLaunchKernelGGL((k_add<float>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, (const float *)y, (float *)x,
                           done);
    else
        hipLaunchKernelGGL((k_add<double>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, (const double *)y,
                           (double *)x, done);
}

int kcycle_blocks(const Level &L) {
    long long b = ((long long)L.A.n * L.G + kBlock - 1) / kBlock;
    if (b > kKPartBlocks) b = kKPartBlocks;
    if (b < 1) b = 1;
    return (int)b;
}

void launch_kcycle_step1(hipStream_t s, const Level &C, int fp32, const void *c1, const void *b, void *v1,
                         double *partials, double *ks, const double *done) {
    const int nb = kcycle_blocks(C);
    if (fp32) long_pre(s, C, (const float *)C.A.v32, FGather<float, float>{(const float *)c1}, done);
    else long_pre(s, C, (const double *)C.A.v, FGather<double, double>{(const double *)c1}, done);
    with_G(C.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (fp32)
            hipLaunchKernelGGL((k_kdots<g, float, 1>), dim3(nb), dim3(kBlock), 0, s, C.A.n, C.A.rp, C.A.ci, C.A.v32,
                               (const float *)c1, (const float *)b, (const float *)nullptr, (float *)v1, partials,
                               done, long_view<float>(C.lr));
        else
            hipLaunchKernelGGL((k_kdots<g, double, 1>), dim3(nb), dim3(kBlock), 0, s, C.A.n, C.A.rp, C.A.ci, C.A.v,
                               (const double *)c1, (const double *)b, (const double *)nullptr, (double *)v1,
                               partials, done, long_view<double>(C.lr));
    });
    hipLaunchKernelGGL(k_kfinal<1>, dim3(1), dim3(kBlock), 0, s, nb, partials, ks, done);
    if (fp32)
        hipLaunchKernelGGL((k_kresid<float>), dim3(blocks_for(C.A.n)), dim3(kBlock), 0, s, C.A.n, (const float *)v1,
                           ks, (float *)b, done);
    else
        hipLaunchKernelGGL((k_kresid<double>), dim3(blocks_for(C.A.n)), dim3(kBlock), 0, s, C.A.n,
                           (const double *)v1, ks, (double *)b, done);
}

void launch_kcycle_step2(hipStream_t s, const Level &C, int fp32, const void *c2, const void *b, const void *v1,
                         void *x, double *partials, double *ks, const double *done) {
    const int nb = kcycle_blocks(C);
    if (fp32) long_pre(s, C, (const float *)C.A.v32, FGather<float, float>{(const float *)c2}, done);
    else long_pre(s, C, (const double *)C.A.v, FGather<double, double>{(const double *)c2}, done);
    with_G(C.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (fp32)
            hipLaunchKernelGGL((k_kdots<g, float, 2>), dim3(nb), dim3(kBlock), 0, s, C.A.n, C.A.rp, C.A.ci, C.A.v32,
                               (const float *)c2, (const float *)b, (const float *)v1, (float *)nullptr, partials,
                               done, long_view<float>(C.lr));
        else
            hipLaunchKernelGGL((k_kdots<g, double, 2>), dim3(nb), dim3(kBlock), 0, s, C.A.n, C.A.rp, C.A.ci, C.A.v,
                               (const double *)c2, (const double *)b, (const double *)v1, (double *)nullptr,
                               partials, done, long_view<double>(C.lr));
    });
    hipLaunchKernelGGL(k_kfinal<2>, dim3(1), dim3(kBlock), 0, s, nb, partials, ks, done);
    if (fp32)
        hipLaunchKernelGGL((k_kcombine<float>), dim3(blocks_for(C.A.n)), dim3(kBlock), 0, s, C.A.n,
                           (const float *)c2, ks, (float *)x, done);
    else
        hipLaunchKernelGGL((k_kcombine<double>), dim3(blocks_for(C.A.n)), dim3(kBlock), 0, s, C.A.n,
                           (const double *)c2, ks, (double *)x, done);
}

void launch_fold_level(hipStream_t s, const Level &L, const double *Tc, int nc, double *H, double *T) {
    const int n = L.A.n;
    const int nb = blocks_for((long long)n * n);
    hipLaunchKernelGGL(k_fold_h, dim3(nb), dim3(kBlock), 0, s, n, nc, L.A.rp, L.A.ci, L.A.v, L.dinv, L.p, L.agg, Tc, H);
    hipLaunchKernelGGL(k_fold_t, dim3(blocks_for(fold_t_threads(n))), dim3(kBlock), 0, s, n, L.A.rp, L.A.ci, L.A.v,
                       L.dinv, H, T);
}

void launch_fold_w(hipStream_t s, const Level &L, const double *T, double *M, double *W) {
    const int n = L.A.n;
    const int nb = blocks_for((long long)n * n);
    hipLaunchKernelGGL(k_fold_at, dim3(nb), dim3(kBlock), 0, s, n, L.A.rp, L.A.ci, L.A.v, T, M);
    hipLaunchKernelGGL(k_fold_w, dim3(nb), dim3(kBlock), 0, s, n, T, M, W);
}

void launch_fold_left(hipStream_t s, const Level &L, const double *H, double *T) {
    const int n = L.A.n;
    hipLaunchKernelGGL(k_fold_t, dim3(blocks_for(fold_t_threads(n))), dim3(kBlock), 0, s, n, L.A.rp, L.A.ci, L.A.v,
                       L.dinv, H, T);
}

void launch_dense(hipStream_t s, int n, const double *T, const void *b, void *x, int b_f64, int x_f64,
                  const double *done) {
    if (b_f64 && x_f64)
        hipLaunchKernelGGL((k_coarse_dense<double, double>), dim3(n), dim3(kBlock), 0, s, n, T, (const double *)b,
                           (double *)x, done);
    else
        hipLaunchKernelGGL((k_coarse_dense<float, float>), dim3(n), dim3(kBlock), 0, s, n, T, (const float *)b,
                           (float *)x, done);
}

void launch_coarse_build(hipStream_t s, const Level &L, int sweeps, double *S) {
    hipLaunchKernelGGL((k_coarse<double, double>), dim3(L.A.n), dim3(1024), 0, s, L.A.n, L.A.nnz, L.A.rp, L.A.ci,
                       L.A.v, L.dinv, (const double *)nullptr, S, sweeps, 1, (const double *)nullptr);
}

void launch_resid(hipStream_t s, const Level &L, int nb, const double *b, const double *u, double *r,
                  double *partials, double *scal) {
    if (L.E.sp) {
        with_sell<double>(L.E, [&](auto *ix, auto *vals, auto kb) {
            using I = std::remove_const_t<std::remove_pointer_t<decltype(ix)>>;
            using S = std::remove_const_t<std::remove_pointer_t<decltype(vals)>>;
            hipLaunchKernelGGL((k_resid_sell<I, S, decltype(kb)::value>), dim3(nb), dim3(kBlock), 0, s, L.A.n, L.E.sp, L.E.uni, L.E.su, ix, vals, b, u, r,
                               partials);
        });
        return;
    }
    long_pre(s, L, (const double *)L.A.v, FGather<double, double>{u}, nullptr);
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL(k_resid<g>, dim3(nb), dim3(kBlock), 0, s, L.A.n, L.A.rp, L.A.ci, L.A.v, b, u, r,
                           partials, long_view<double>(L.lr));
    });
}

// The grid-stride product runs on at most 1024 workgroups (eight or more rows
// per thread on the largest grids: 160^3 product 84 -> 81 us, and half the
// partials for its finalize step); the vector update keeps the 2048 of nb
// (with 1024 it measured 55 -> 60 us there).
constexpr int kSpmvBlocks = 1024;
bool slot_split_level(const Level &L) { return L.E.sp && split_slots(L, L.E.wide ? 16 : 8); }

int spmv_dots_grid(const Level &L, int nb) {
    return L.E.sp && split_slots(L, L.E.wide ? 16 : 8) ? L.E.nslices : std::min(nb, kSpmvBlocks);
}

void launch_spmv_dots(hipStream_t s, const Level &L, int nb, int first, const double *w, const double *r,
                      const double *q, double *v, double *partials, double *scal) {
    if (L.E.sp) {
        with_sell<double>(L.E, [&](auto *ix, auto *vals, auto kb) {
            using I = std::remove_const_t<std::remove_pointer_t<decltype(ix)>>;
            using S = std::remove_const_t<std::remove_pointer_t<decltype(vals)>>;
            // nb = L.E.nslices (spmv_dots_grid); batches of four slots per wave, which
            // measured faster than eight here (the residual and smoother keep eight)
            auto go = [&](auto nt) {  // NT: the values streamed non-temporally (Sell::stream)
                constexpr bool NT = decltype(nt)::value;
                if (split_slots(L, decltype(kb)::value))
                    launch_k((k_spmv_dots_sell_p<I, S, 4, NT>), dim3(nb), dim3(kBlock), s, L.A.n, L.E.sp, L.E.uni,
                             L.E.su, ix, vals, w, r, q, v, partials, scal + 10);
                else
                    launch_k((k_spmv_dots_sell<I, S, decltype(kb)::value, NT>), dim3(nb), dim3(kBlock), s, L.A.n,
                             L.E.sp, L.E.uni, L.E.su, ix, vals, w, r, q, v, partials, scal + 10);
            };
            if (L.E.stream) go(std::true_type{});
            else go(std::false_type{});
        });
        return;
    }
    long_pre(s, L, (const double *)L.A.v, FGather<double, double>{w}, scal + 10);
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        launch_k((k_spmv_dots<g>), dim3(nb), dim3(kBlock), s, L.A.n, L.A.rp, L.A.ci, L.A.v, w, r, q, v,
                           partials, scal + 10, long_view<double>(L.lr));
    });
}

// Up to kSpmvBlocks product partials every update workgroup adds them itself
// (24 KB of L2-resident loads each) instead of a one-block finalize launch; the
// one-workgroup-per-slice product's thousands of partials keep that launch.
bool update_takes_dots(int nbs) { return nbs <= kSpmvBlocks; }

void launch_update(hipStream_t s, int n, int nb, int first, const double *w, const double *v, double *d,
                   double *u, double *q, double *r, double *partials, double *scal, const void *dinv, void *y,
                   int y_f32, const double *dots, int ndots) {
    if (y && y_f32)
        launch_k((k_update<float>), dim3(nb), dim3(kBlock), s, n, first, w, v, d, u, q, r, (const float *)dinv,
                 (float *)y, scal, partials, dots, ndots);
    else
        launch_k((k_update<double>), dim3(nb), dim3(kBlock), s, n, first, w, v, d, u, q, r, (const double *)dinv,
                 (double *)y, scal, partials, dots, ndots);
}

void launch_finalize(hipStream_t s, int mode, int nb, int first, const double *partials, double *scal) {
    const dim3 t(finalize_threads(nb));
    if (mode == 0) hipLaunchKernelGGL(k_finalize<2>, dim3(1), t, 0, s, nb, partials, scal, 0, 0);
    else if (mode == 1) hipLaunchKernelGGL(k_finalize<3>, dim3(1), t, 0, s, nb, partials, scal, 1, first);
    else hipLaunchKernelGGL(k_finalize<1>, dim3(1), t, 0, s, nb, partials, scal, 2, 0);
}

void launch_sampled_outer(hipStream_t s, const Level &L, const double *lam, const double *x, double *G) {
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        constexpr int R = 4;
        hipLaunchKernelGGL((k_sampled_outer<g, R>), dim3(blocks_for(((long long)L.A.n + R - 1) / R * g)),
                           dim3(kBlock), 0, s, L.A.n, L.A.rp, L.A.ci, lam, x, G,
                           L.lr.n > 0 ? L.lr.lmin : 0x7fffffff);
    });
    if (L.lr.n > 0)
        hipLaunchKernelGGL(k_long_outer, dim3(L.lr.nchunks), dim3(kBlock), 0, s, L.lr, L.A.rp, L.A.ci, lam, x, G);
}

}  // namespace bcm
