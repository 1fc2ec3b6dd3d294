/*
 * bcm.h -- C ABI of the MI355X (gfx950) library for AMG preconditioning based on
 * compatible weighted matching inside flexible CG (Bernaschi, D'Ambra,
 * Pasquini, "AMG based on compatible weighted matching for GPUs", arXiv
 * 1810.04221).
 *
 * Problem (Section 1, the system A x = b): A is sparse, symmetric positive
 * definite, in CSR form (Section 3: CSR storage for all sparse matrices).
 *
 * Conventions for every entry point:
 *  - Array arguments are device pointers of the GPU that is current when the
 *    call is made, unless stated otherwise.  They stay owned by the caller and
 *    are not retained after the call returns.
 *  - Work is enqueued on bcm_params.stream (a hipStream_t; NULL = the default
 *    stream).  Calls that return sizes or convergence information synchronise
 *    that stream before returning.
 *  - Return codes: BCM_OK (0), BCM_MAXIT (1) or BCM_STAGNATED (2), both not
 *    fatal, or a negative error.
 *    bcm_last_error() gives a message for the last failing call of the
 *    calling thread.  A handle must not be used by two threads at once.
 *  - CSR requirements: int32 row_ptr[n + 1] with row_ptr[0] = 0 and
 *    row_ptr[n] = nnz, int32 col[nnz] strictly ascending inside each row and
 *    in [0, n), float64 val[nnz]; every row stores its diagonal entry, which
 *    must be positive; all values finite.  The matching needs the weight of an
 *    edge to be the same double from both ends, so A must be bitwise
 *    symmetric: same pattern, and val(i, j) and val(j, i) the same double.
 *    Violations are reported as BCM_EINVAL (symmetry only when
 *    bcm_params.check is nonzero).
 */
#ifndef BCM_H
#define BCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BCM_OK = 0,
    BCM_MAXIT = 1,        /* itmax reached before tol; x holds the last iterate */
    BCM_STAGNATED = 2,    /* the recurrence residual met tol but the true residual
                             b - A x stayed above it through every restart (rounding
                             floor): x holds the last iterate, bcm_info its true
                             relative residual */
    BCM_EINVAL = -1,      /* invalid argument or matrix (see bcm_last_error) */
    BCM_EBREAKDOWN = -2,  /* flexible CG breakdown: rho <= 0 or not finite */
    BCM_ENOMEM = -3,      /* device allocation failed */
    BCM_EHIP = -4         /* HIP runtime error */
};

enum { BCM_FP64 = 0, BCM_FP32_CYCLE = 1 };
enum { BCM_VCYCLE = 1, BCM_WCYCLE = 2, BCM_KCYCLE = 3 };

typedef struct bcm_handle bcm_handle;

typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col;
    const double *val;
} bcm_csr;

/*
 * Parameters (Section 5, experimental settings, gives the defaults):
 *   max_levels     40    maximum number of levels
 *   max_coarse     0     stop coarsening once n_k <= max_coarse;
 *                        0 means round(40 * n^(1/3)).  With max_levels and a
 *                        level that leaves the size unchanged, this is the
 *                        stopping rule of Section 5.
 *   min_ratio      0     <= 1: Section 5's rule alone.  > 1: also stop at the
 *                        first level formed with n_{k-1} / n_k < min_ratio
 *                        (coarsening that has stalled; a rule of this library,
 *                        not of the paper: 2 = a level that did not halve the
 *                        size under double pairwise aggregation)
 *   sweeps         2     pairwise matching sweeps composed per level
 *                        (2 = double pairwise aggregation, ratio <= 4); 1..4
 *   coarse_sweeps  20    l1-Jacobi sweeps from zero at the coarsest level
 *   pre, post      1, 1  l1-Jacobi sweeps before/after the coarse correction
 *                        (only 1, 1 is implemented)
 *   cycle          BCM_VCYCLE (Algorithm 1), BCM_WCYCLE (Section 2.1: the
 *                        coarse problem of every level solved by two cycles,
 *                        the second on the coarse residual) or BCM_KCYCLE
 *                        (Sections 2.1 and 3.2, Krylov-based cycle: the coarse
 *                        problem of a level solved by two flexible-CG
 *                        iterations from zero, preconditioned by the coarse
 *                        level's cycle; the preconditioner is then nonlinear)
 *   kcycle_levels  0     BCM_KCYCLE: levels k < kcycle_levels (0 = finest)
 *                        use the Krylov coarse solve, the others one cycle;
 *                        0 = every level
 *   precision      BCM_FP64: hierarchy and cycle in float64.
 *                  BCM_FP32_CYCLE: hierarchy stored and cycle run in float32
 *                  with float32 accumulation; the coarsest solve, the outer
 *                  CG (residual, dot products, updates) and the setup's
 *                  matching weights stay float64.
 *   itmax          5000  maximum number of preconditioned iterations
 *   check          1     also verify bitwise symmetry of A in bcm_setup
 *   adjoint_tol    0     tolerance of bcm_solve_adjoint; 0 = last solve's tol
 *   alloc/dealloc        optional device allocator (e.g. a framework's caching
 *                        allocator); NULL = hipMalloc / hipFree.
 *                        dealloc receives the pointer and size returned/asked.
 *   stream               hipStream_t for all work of the handle.
 *   profile              bit mask of kernel classes (BCM_PROF_*) whose
 *                        launches are bracketed by HIP events during
 *                        bcm_solve; read back with bcm_profile().
 *   graph          0     1 = replay one flexible-CG iteration (cycle, SpMV,
 *                        updates) from a HIP graph captured on the handle's
 *                        first solve; 0 = launch every kernel (measured faster
 *                        on MI355X for this iteration).  A profile mask of exactly one
 *                        of the classes down0, up0, spmv_dots, update, coarse is
 *                        timed inside the graph; other masks launch eagerly.
 *   group          0     lanes per matrix row in the CSR row kernels (the
 *                        miniwarp of Sections 3.1 and 3.2): 0 = the smallest
 *                        power of two >= the level's average nonzeros per row,
 *                        clamped to 4..64; 4, 8, 16, 32 or 64 = that width on
 *                        every level; -1 = the rule during setup, then the
 *                        fastest width per cycle level, timed at the end of
 *                        setup (the solve's rounding then depends on timing)
 *   sell           1     sliced-ELL copies (64-row slices) of the finest level
 *                        and of levels >= 65536 rows for the row-parallel solve
 *                        kernels; 0 = CSR row kernels everywhere
 *   fold           1     V-cycle: the cycle from the first level k >= 1 with at
 *                        most 2048 rows down to the coarsest (a fixed linear
 *                        map, pre = post = 1) is formed once in float64 at
 *                        setup and applied as one dense product; the same
 *                        operator as the level-by-level cycle up to rounding,
 *                        also under BCM_FP32_CYCLE.  0 = level by level.
 */
typedef struct {
    int32_t max_levels;
    int32_t max_coarse;
    int32_t sweeps;
    int32_t coarse_sweeps;
    int32_t pre;
    int32_t post;
    int32_t cycle;
    int32_t kcycle_levels;
    int32_t precision;
    int32_t itmax;
    int32_t check;
    int32_t profile;
    int32_t graph;
    int32_t group;
    int32_t sell;
    int32_t fold;
    double adjoint_tol;
    double min_ratio;
    void *(*alloc)(size_t bytes, void *ctx);
    void (*dealloc)(void *ptr, size_t bytes, void *ctx);
    void *alloc_ctx;
    void *stream;
} bcm_params;

/* Fills *p with the defaults listed above. */
void bcm_default_params(bcm_params *p);

/*
 * Setup phase (Section 2.1 hierarchy, Section 2.2 and Algorithm 2 coarsening,
 * Section 3.1 GPU setup): builds the hierarchy A^1 = A, ..., A^nl with
 * A^{k+1} = (P^k)^T A^k P^k.  Each level composes `sweeps` pairwise
 * aggregations: edge weights c_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 +
 * a_jj w_j^2) from the current smooth vector, half-approximate maximum weight
 * matching (Suitor; equal to the greedy matching under weight descending,
 * then larger, then smaller endpoint descending), Algorithm 2 with aggregates
 * numbered by their smallest index, the prolongator from the orthonormal
 * projection of w on each aggregate, coarse w = restriction of w, and the
 * Galerkin product.
 *   A   matrix (device arrays), copied into the handle.
 *   w   float64[n] device smooth vector; every entry finite and nonzero.
 *   p   parameters (NULL = defaults).
 *   out receives the new handle (NULL on failure).
 */
int bcm_setup(const bcm_csr *A, const double *w, const bcm_params *p, bcm_handle **out);

/*
 * Solve phase: flexible preconditioned CG (Section 3.2, Algorithm 3 read with
 * r_{i+1} = r_i - (alpha_i/rho_i) q_i and gamma_i/rho_{i-1} in the d and q
 * updates) preconditioned by one cycle of Algorithm 1 per iteration.
 *   b   float64[n] device right-hand side.
 *   x   float64[n] device; in: initial guess, out: solution.
 *   tol stop when ||r||_2 / ||b||_2 <= tol (Section 5: relative residual);
 *       the true residual b - A x is recomputed at exit; while it misses
 *       tol the solve restarts from x (at most three restarts).
 * Returns BCM_OK, BCM_MAXIT, BCM_STAGNATED, BCM_EBREAKDOWN or an error.
 */
int bcm_solve(bcm_handle *h, const double *b, double *x, double tol);

/*
 * Preconditioner application: z = B(r), one cycle of Algorithm 1 from a zero
 * initial guess (the operator flexible CG applies every iteration).
 *   r  float64[n] device input;  z  float64[n] device output.
 */
int bcm_precond(bcm_handle *h, const double *r, double *z);

/*
 * Adjoint solve for the gradient of a loss L(x), x = A^{-1} b: solves
 * A lambda = g with the same hierarchy (A is symmetric), from lambda = 0, to
 * bcm_params.adjoint_tol (0 = tol of the last bcm_solve).  dL/db = lambda.
 *   g       float64[n] device, dL/dx.
 *   lambda  float64[n] device output.
 */
int bcm_solve_adjoint(bcm_handle *h, const double *g, double *lambda);

/*
 * Sampled outer product on A's pattern: grad_val[q] = -lambda_i * x_j for the
 * q-th stored entry (i, j), i.e. dL/da_ij with every stored entry treated as
 * an independent parameter.
 *   lambda, x  float64[n] device;  grad_val float64[nnz] device output.
 */
int bcm_sampled_outer(bcm_handle *h, const double *lambda, const double *x, double *grad_val);

/* Hierarchy and last-solve statistics.  Vcmplx = sum_k nnz(A^k) / nnz(A^1)
 * and cratio = mean of n_{k-1} / n_k (Section 5.2 quality measures); cratio
 * averages over the nl - 1 ratios, cratio_nl divides the same sum by nl. */
typedef struct {
    int32_t nl;
    int32_t precision;
    int32_t iters;
    int32_t status;
    int32_t n[64];
    int64_t nnz[64];
    double vcmplx;
    double cratio;
    double cratio_nl;
    double relres;
    double t_setup_ms;
    double t_solve_ms;
    double cycle_bytes;  /* algorithmic bytes of one preconditioner application */
    double iter_bytes;   /* algorithmic bytes of one outer iteration, cycle included */
    double setup_bytes;  /* algorithmic bytes of the setup: sum over its pairwise sweeps on
                            (m rows, z entries) of 72 z + 80 m, a lower bound */
    int32_t sweeps_run;  /* pairwise sweeps the setup ran */
    int32_t long_rows;   /* rows of all levels on the long-row path of the solve kernels */
} bcm_info_t;

int bcm_info(const bcm_handle *h, bcm_info_t *out);

/*
 * Copies level k of the hierarchy into caller buffers (device or host
 * pointers; NULL skips an array): row_ptr[n_k + 1], col[nnz_k], val[nnz_k],
 * w[n_k] smooth vector, dinv[n_k] = 1 / sum_j |a_ij| (l1-Jacobi, Section
 * 3.2), and for k < nl - 1 the composed prolongator P^k: agg[n_k] (column of
 * row i) and p[n_k] (its value).  Synchronises the stream.
 */
int bcm_level_copy(const bcm_handle *h, int32_t k, int32_t *row_ptr, int32_t *col, double *val,
                   double *w, double *dinv, int32_t *agg, double *p);

/*
 * One matching sweep on A with smooth vector w (Section 2.2, Section 3.1):
 * writes mate[i] = j if {i, j} is matched, -1 otherwise (device int32[n]),
 * and, when c is not NULL, the edge weights c[nnz] (0 on the diagonal).
 * Uses p's allocator and stream (NULL = defaults).
 */
int bcm_match(const bcm_csr *A, const double *w, const bcm_params *p, int32_t *mate, double *c);

/* Size of the device scratch array of bcm_match_noalloc: 64 MiB per GPU. */
#define BCM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * bcm_match without any allocation, for callers that cannot allocate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as bcm_match (p's allocator
 * is ignored).  Its scratch lives in one static device array of
 * BCM_NOALLOC_SCRATCH_BYTES on each GPU the library runs on, held until the
 * process ends; its address is looked up once per device, on the first call
 * made with that device current.  Host read-backs go to plain host memory
 * (no pinned staging buffer).
 *  - Limit: the scratch of a call is, in 256-byte-rounded pieces, about
 *    20 n + 12 nnz bytes (+ 8 nnz when c is NULL), plus the long-row lists
 *    and 16 bytes per entry of rows longer than 16 x the lanes per row.  A
 *    call that needs more returns BCM_EINVAL with a message and leaves mate
 *    unspecified.
 *  - Every call on one GPU shares that GPU's array and finds the previous
 *    call's contents there (everything a call reads it first writes).  Calls
 *    that overlap on one GPU (two streams, two threads) race: the caller
 *    serialises them.  bcm_params.stream must belong to the current device.
 */
int bcm_match_noalloc(const bcm_csr *A, const double *w, const bcm_params *p, int32_t *mate, double *c);

/* Kernel classes that bcm_params.profile can time. */
enum {
    BCM_PROF_CYCLE_DOWN0 = 1,  /* finest-level pre-smooth + residual + restriction */
    BCM_PROF_CYCLE_UP0 = 2,    /* finest-level prolongation + post-smooth */
    BCM_PROF_SPMV_DOTS = 4,    /* v = A w fused with the three dot products */
    BCM_PROF_UPDATE = 8,       /* the four fused vector updates + ||r||^2 */
    BCM_PROF_CYCLE_COARSE = 16, /* the coarsest-level solve */
    BCM_PROF_CYCLE_MID = 32,    /* every cycle kernel of levels 1 .. nl - 2 (several per cycle) */
    /* setup classes, one bracket per pairwise sweep, timed during bcm_setup */
    BCM_PROF_SETUP_MATCH = 64,     /* edge weights and Suitor candidate lists (long rows included) */
    BCM_PROF_SETUP_SUITOR = 128,   /* the Suitor matching kernel itself */
    BCM_PROF_SETUP_GALERKIN = 256  /* Galerkin product: count, row pointers, fill */
};

/*
 * Event timings for one kernel class: number of launches (brackets), their
 * summed duration in ms, and the summed algorithmic bytes (the bytes the
 * operation must move at least once).  Solve classes: the last bcm_solve;
 * setup classes: bcm_setup.
 */
int bcm_profile(const bcm_handle *h, int32_t kclass, int64_t *launches, double *ms, double *bytes);

/* Releases every device buffer of the handle (NULL is allowed). */
void bcm_free(bcm_handle *h);

/* Message of the last error of the calling thread ("" if none). */
const char *bcm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BCM_H */
