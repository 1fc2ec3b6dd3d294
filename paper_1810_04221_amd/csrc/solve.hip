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

// ----------------------------------------------------------------------------
// Down leg of the cycle at level k (Algorithm 1, zero initial guess):
//   x = x + M^{-1}(b - A x) with x = 0   ->  x_j = dinv_j * b_j
//   b_c[E] = sum_{i in E} p_i (b_i - sum_j a_ij x_j)      (restriction)
// One group per coarse aggregate E walks its members in ascending order; x is
// never stored, it is recomputed from b and dinv where it is gathered.
// ----------------------------------------------------------------------------
template <int G, typename V, typename VB>
__global__ void __launch_bounds__(kBlock)
k_down(int nc, int mstride, const int *__restrict__ mem, const int *__restrict__ rp,
       const int *__restrict__ ci, const V *__restrict__ a, const V *__restrict__ dinv,
       const V *__restrict__ p, const VB *__restrict__ b, V *__restrict__ bc) {
    const int lane = threadIdx.x % G;
    const int E = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (E >= nc) return;
    V acc = V(0);
    for (int t = 0; t < mstride; ++t) {
        const int i = mem[(size_t)E * mstride + t];
        if (i < 0) break;
        V s = V(0);
        const int e = rp[i + 1];
        for (int q = rp[i] + lane; q < e; q += G) {
            const int j = ci[q];
            s += a[q] * (dinv[j] * (V)b[j]);
        }
        s = group_sum<G>(s);
        const V r = (V)b[i] - s;
        acc += p[i] * r;
    }
    if (lane == 0) bc[E] = acc;
}

// ----------------------------------------------------------------------------
// Up leg at level k: prolongation and post-smoothing (Algorithm 1; M^{-T} =
// M^{-1} for the diagonal l1 smoother):
//   x_j = dinv_j b_j + p_j xc[agg_j]          (pre-smoothed x plus P x_c)
//   x_i <- x_i + dinv_i (b_i - sum_j a_ij x_j)
// ----------------------------------------------------------------------------
template <int G, typename V, typename VB, typename VX>
__global__ void __launch_bounds__(kBlock)
k_up(int n, const int *__restrict__ rp, const int *__restrict__ ci, const V *__restrict__ a,
     const V *__restrict__ dinv, const V *__restrict__ p, const int *__restrict__ agg,
     const VB *__restrict__ b, const V *__restrict__ xc, VX *__restrict__ x) {
    const int lane = threadIdx.x % G;
    const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (i >= n) return;
    V s = V(0);
    const int e = rp[i + 1];
    for (int q = rp[i] + lane; q < e; q += G) {
        const int j = ci[q];
        const V xj = dinv[j] * (V)b[j] + p[j] * xc[agg[j]];
        s += a[q] * xj;
    }
    s = group_sum<G>(s);
    if (lane == 0) {
        const V bi = (V)b[i];
        const V di = dinv[i];
        const V xi = di * bi + p[i] * xc[agg[i]];
        x[i] = (VX)(xi + di * (bi - s));
    }
}

// ----------------------------------------------------------------------------
// Coarsest level: `sweeps` l1-Jacobi sweeps from zero in float64, inside one
// workgroup with x held in LDS (n <= 8192).  Each sweep computes all new values
// from the old x before any is written back, i.e. plain Jacobi.
// ----------------------------------------------------------------------------
template <typename VB, typename VX>
__global__ void __launch_bounds__(1024)
k_coarse(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
         const double *__restrict__ dinv, const VB *__restrict__ b, VX *__restrict__ x, int sweeps) {
    __shared__ double xs[kCoarseLds];
    constexpr int R = kCoarseLds / 1024;
    for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = 0.0;
    __syncthreads();
    for (int t = 0; t < sweeps; ++t) {
        double xn[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = threadIdx.x + k * blockDim.x;
            xn[k] = 0.0;
            if (i < n) {
                double s = 0.0;
                const int e = rp[i + 1];
                for (int q = rp[i]; q < e; ++q) s = s + a[q] * xs[ci[q]];
                const double r = (double)b[i] - s;
                xn[k] = xs[i] + dinv[i] * r;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = threadIdx.x + k * blockDim.x;
            if (i < n) xs[i] = xn[k];
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (VX)xs[i];
}

// One global l1-Jacobi sweep (coarsest levels larger than the LDS bound).
template <typename VB>
__global__ void __launch_bounds__(kBlock)
k_jacobi_sweep(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
               const double *__restrict__ dinv, const VB *__restrict__ b, const double *__restrict__ xo,
               double *__restrict__ xn, int first) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    if (!first) {
        const int e = rp[i + 1];
        for (int q = rp[i]; q < e; ++q) s = s + a[q] * xo[ci[q]];
    }
    const double r = (double)b[i] - s;
    xn[i] = (first ? 0.0 : xo[i]) + dinv[i] * r;
}

template <typename VX>
__global__ void k_store(int n, const double *__restrict__ src, VX *__restrict__ dst) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = (VX)src[i];
}

// ----------------------------------------------------------------------------
// Flexible CG kernels (Algorithm 3).  Fixed grid of nb blocks with a
// grid-stride loop over row groups; reductions are deterministic for a fixed
// grid (block partials summed in block order by the last block).
// scal: [0] alpha [1] beta [2] gamma [3] rho_{i-1} [4] ||r||^2 [5] ||b||^2
//       [6] breakdown flag
// ----------------------------------------------------------------------------

// r = b - A u, ||r||^2 -> scal[4], ||b||^2 -> scal[5]
template <int G>
__global__ void __launch_bounds__(kBlock)
k_resid(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
        const double *__restrict__ b, const double *__restrict__ u, double *__restrict__ r,
        double *partials, unsigned *counter, double *scal) {
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    double acc[2] = {0.0, 0.0};
    for (int i = blk * NG + threadIdx.x / G; i < n; i += gridDim.x * NG) {
        double s = 0.0;
        const int e = rp[i + 1];
        for (int q = rp[i] + lane; q < e; q += G) s += a[q] * u[ci[q]];
        s = group_sum<G>(s);
        if (lane == 0) {
            const double bi = b[i];
            const double ri = bi - s;
            r[i] = ri;
            acc[0] += ri * ri;
            acc[1] += bi * bi;
        }
    }
    grid_sum<2>(acc, partials, counter, scal + 4);
}

// v = A w with alpha = w.r, beta = w.v, gamma = w.q in the same pass -> scal[0..2]
template <int G>
__global__ void __launch_bounds__(kBlock)
k_spmv_dots(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ a,
            const double *__restrict__ w, const double *__restrict__ r, const double *__restrict__ q,
            double *__restrict__ v, double *partials, unsigned *counter, double *scal) {
    constexpr int NG = kBlock / G;
    const int lane = threadIdx.x % G;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = blk * NG + threadIdx.x / G; i < n; i += gridDim.x * NG) {
        double s = 0.0;
        const int e = rp[i + 1];
        for (int k = rp[i] + lane; k < e; k += G) s += a[k] * w[ci[k]];
        s = group_sum<G>(s);
        if (lane == 0) {
            const double wi = w[i];
            v[i] = s;
            acc[0] += wi * r[i];
            acc[1] += wi * s;
            acc[2] += wi * q[i];
        }
    }
    grid_sum<3>(acc, partials, counter, scal);
}

// The two fused AXPY pairs of Algorithm 3 and ||r||^2:
//   rho_i = beta - gamma^2 / rho_{i-1}
//   d = w - (gamma/rho_{i-1}) d ; u += (alpha/rho_i) d
//   q = v - (gamma/rho_{i-1}) q ; r -= (alpha/rho_i) q
// first step: rho_0 = beta, d = w, q = v.  On rho <= 0 or not finite nothing is
// updated and scal[6] = 1.
__global__ void __launch_bounds__(kBlock)
k_update(int n, int first, const double *__restrict__ w, const double *__restrict__ v, double *__restrict__ d,
         double *__restrict__ u, double *__restrict__ q, double *__restrict__ r, double *partials,
         unsigned *counter, double *scal) {
    const double alpha = scal[0], beta = scal[1], gamma = scal[2], rho_prev = scal[3];
    double rho, g;
    if (first) { rho = beta; g = 0.0; }
    else { rho = beta - gamma * gamma / rho_prev; g = gamma / rho_prev; }
    const double an = alpha / rho;
    const bool ok = (rho > 0.0) && isfinite(rho) && isfinite(an) && isfinite(g);
    double acc[1] = {0.0};
    if (ok) {
        const int blk = xcd_block(blockIdx.x, gridDim.x);
        for (int i = blk * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
            const double wi = w[i], vi = v[i];
            double di, qi;
            if (first) { di = wi; qi = vi; }
            else { di = wi - g * d[i]; qi = vi - g * q[i]; }
            d[i] = di;
            q[i] = qi;
            u[i] = u[i] + an * di;
            const double ri = r[i] - an * qi;
            r[i] = ri;
            acc[0] += ri * ri;
        }
    }
    if (grid_sum<1>(acc, partials, counter, scal + 4) && threadIdx.x == 0) {
        scal[3] = rho;
        scal[6] = ok ? 0.0 : 1.0;
    }
}

// dL/da_ij = -lambda_i x_j on the stored pattern
template <int G>
__global__ void __launch_bounds__(kBlock)
k_sampled_outer(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ lam,
                const double *__restrict__ x, double *__restrict__ out) {
    const int lane = threadIdx.x % G;
    const int i = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (i >= n) return;
    const double li = lam[i];
    const int e = rp[i + 1];
    for (int q = rp[i] + lane; q < e; q += G) out[q] = -(li * x[ci[q]]);
}

template <typename V, typename VB>
void down_t(hipStream_t s, const Level &L, const V *a, const V *dinv, const V *p, const VB *b, V *bc) {
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL((k_down<g, V, VB>), dim3(blocks_for((long long)L.nc * g)), dim3(kBlock), 0, s, L.nc,
                           L.mstride, L.mem, L.A.rp, L.A.ci, a, dinv, p, b, bc);
    });
}

template <typename V, typename VB, typename VX>
void up_t(hipStream_t s, const Level &L, const V *a, const V *dinv, const V *p, const VB *b, const V *xc,
          VX *x) {
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL((k_up<g, V, VB, VX>), dim3(blocks_for((long long)L.A.n * g)), dim3(kBlock), 0, s,
                           L.A.n, L.A.rp, L.A.ci, a, dinv, p, L.agg, b, xc, x);
    });
}

template <typename VB, typename VX>
void coarse_t(hipStream_t s, const Level &L, int sweeps, const VB *b, VX *x, double *ta, double *tb) {
    const int n = L.A.n;
    if (n <= kCoarseLds) {
        hipLaunchKernelGGL((k_coarse<VB, VX>), dim3(1), dim3(1024), 0, s, n, L.A.rp, L.A.ci, L.A.v, L.dinv, b, x,
                           sweeps);
        return;
    }
    double *xo = ta, *xn = tb;
    for (int t = 0; t < sweeps; ++t) {
        hipLaunchKernelGGL((k_jacobi_sweep<VB>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, L.A.rp, L.A.ci,
                           L.A.v, L.dinv, b, xo, xn, t == 0 ? 1 : 0);
        double *tmp = xo; xo = xn; xn = tmp;
    }
    hipLaunchKernelGGL((k_store<VX>), dim3(blocks_for(n)), dim3(kBlock), 0, s, n, xo, x);
}

}  // namespace

int reduce_blocks(int n) {
    long long b = ((long long)n + kBlock - 1) / kBlock;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

void launch_down(hipStream_t s, const Level &L, int fp32, const void *b, void *bc, int b_is_f64) {
    if (!fp32) {
        down_t<double, double>(s, L, L.A.v, L.dinv, L.p, (const double *)b, (double *)bc);
    } else if (b_is_f64) {
        down_t<float, double>(s, L, L.A.v32, L.dinv32, L.p32, (const double *)b, (float *)bc);
    } else {
        down_t<float, float>(s, L, L.A.v32, L.dinv32, L.p32, (const float *)b, (float *)bc);
    }
}

void launch_up(hipStream_t s, const Level &L, int fp32, const void *b, const void *xc, void *x, int b_is_f64,
               int x_is_f64) {
    if (!fp32) {
        up_t<double, double, double>(s, L, L.A.v, L.dinv, L.p, (const double *)b, (const double *)xc, (double *)x);
    } else if (b_is_f64 && x_is_f64) {
        up_t<float, double, double>(s, L, L.A.v32, L.dinv32, L.p32, (const double *)b, (const float *)xc,
                                    (double *)x);
    } else {
        up_t<float, float, float>(s, L, L.A.v32, L.dinv32, L.p32, (const float *)b, (const float *)xc, (float *)x);
    }
}

void launch_coarse(hipStream_t s, const Level &L, int sweeps, const void *b, void *x, int b_f64, int x_f64,
                   void *tmp_a, void *tmp_b) {
    double *ta = (double *)tmp_a, *tb = (double *)tmp_b;
    if (b_f64 && x_f64) coarse_t<double, double>(s, L, sweeps, (const double *)b, (double *)x, ta, tb);
    else coarse_t<float, float>(s, L, sweeps, (const float *)b, (float *)x, ta, tb);
}

void launch_resid(hipStream_t s, const Level &L, int nb, const double *b, const double *u, double *r,
                  double *partials, unsigned *counter, double *scal) {
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL(k_resid<g>, dim3(nb), dim3(kBlock), 0, s, L.A.n, L.A.rp, L.A.ci, L.A.v, b, u, r,
                           partials, counter, scal);
    });
}

void launch_spmv_dots(hipStream_t s, const Level &L, int nb, const double *w, const double *r, const double *q,
                      double *v, double *partials, unsigned *counter, double *scal) {
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL(k_spmv_dots<g>, dim3(nb), dim3(kBlock), 0, s, L.A.n, L.A.rp, L.A.ci, L.A.v, w, r, q, v,
                           partials, counter, scal);
    });
}

void launch_update(hipStream_t s, int n, int nb, int first, const double *w, const double *v, double *d,
                   double *u, double *q, double *r, double *partials, unsigned *counter, double *scal) {
    hipLaunchKernelGGL(k_update, dim3(nb), dim3(kBlock), 0, s, n, first, w, v, d, u, q, r, partials, counter,
                       scal);
}

void launch_sampled_outer(hipStream_t s, const Level &L, const double *lam, const double *x, double *G) {
    with_G(L.G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL(k_sampled_outer<g>, dim3(blocks_for((long long)L.A.n * g)), dim3(kBlock), 0, s, L.A.n,
                           L.A.rp, L.A.ci, lam, x, G);
    });
}

}  // namespace bcm
