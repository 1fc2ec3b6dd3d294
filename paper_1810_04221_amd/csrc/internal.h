// Host-side internals of the library: hierarchy data layout in HBM, the device
// arena and the kernel launchers shared between translation units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "bcm.h"

namespace bcm {

// Timing of a single kernel by its own dispatch.  While armed (start set), the
// next launch through launch_k takes start/stop as that kernel's own start and
// end timestamps (hipExtLaunchKernelGGL) and disarms them; otherwise launch_k
// is an ordinary launch.  Per host thread.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local KernelEvents g_kernel_events;

template <typename F, typename... Args>
inline void launch_k(F kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
    if (g_kernel_events.start) {
        const KernelEvents e = g_kernel_events;
        g_kernel_events = KernelEvents{};
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e.start, e.stop, 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}

constexpr int kMaxLevels = 64;
constexpr int kCoarseLds = 8192;   // largest coarsest level solved inside one workgroup
constexpr int kCoarseDense = 2048; // largest coarsest level applied as a precomputed dense operator
constexpr int kCoarseBuildSweeps = 1024;  // up to this size S is built by sweeps on unit vectors
constexpr int kFoldRows = 2048;    // V-cycle: levels from the first this small on form one dense operator
constexpr int kSplitUp = 65536;    // levels at least this large run the up leg as prolong + smooth
constexpr int kGatherRow = 16;     // sliced-ELL levels averaging this many entries per row gather dinv o b
                                   // formed beforehand in the down leg (one vector instead of two)
// Levels of long rows (kGatherRow or more entries per row on average) holding
// at least kSplitEntries entries run split legs too, below kSplitUp rows: on
// the sliced-ELL copy they take the slot-split kernels.  A level that runs
// split legs gets the buffer L.xp, whose presence then selects them.
constexpr long long kSplitEntries = 1LL << 20;
inline bool split_legs(long long n, long long nnz) {
    return n >= kSplitUp || (nnz >= (long long)kGatherRow * n && nnz >= kSplitEntries);
}

// Long rows.  The per-row kernels give each row a group of G lanes, G chosen
// from the level's mean row length (Sections 3.1, 3.2: miniwarp per row).  A
// row longer than kLongFactor * G entries (a hub: a vertex coupled to most of
// its level, as coarsening produces on strongly heterogeneous problems) would
// serialise its group, so such rows leave the per-row kernels and are spread
// over whole workgroups instead: chunks of kSegChunk entries.
constexpr int kLongFactor = 16;
constexpr int kSegChunk = 2048;  // entries per chunk (one workgroup); keys per LDS sort chunk
inline int long_min(int G) { return kLongFactor * G; }

// A list of long segments (rows, or Galerkin coarse rows) found on the device:
// the finding kernel appends (row, length) in any order; k_seg_fix then turns
// the lengths into key offsets and first chunks.  cap bounds the count (a
// segment is longer than lmin, so at most nnz / lmin + 1 of them exist).
struct SegList {
    int *ctl = nullptr;  // [0] segments [1] total length [2] chunks [3] longest [4] overflow
    int *row = nullptr;  // [cap]
    int *len = nullptr;  // [cap]
    int *off = nullptr;  // [cap + 1] exclusive prefix of len
    int *cb = nullptr;   // [cap + 1] exclusive prefix of ceil(len / kSegChunk)
    int cap = 0;
};

// Long rows of one level for the solve kernels: rows longer than lmin, with
// idx[i] = position of row i in rows (or -1) and cb their first chunks.  The
// row kernels take such a row's dot product from the chunk partial sums that
// a pre-pass (k_long_dot) leaves in part, summed in chunk order.
struct LongRows {
    int lmin = 0;     // 0: the level has no long rows
    int n = 0;        // long rows
    int nchunks = 0;  // chunks over them
    const int *rows = nullptr, *cb = nullptr, *idx = nullptr;
    void *part = nullptr;  // nchunks partial sums (cycle precision; float64 for the flexible-CG kernels)
    // Row-wise cycle legs in one launch (chunk blocks after the row blocks):
    // per long row, an arrival counter of its chunks (zero between launches).
    int *cnt = nullptr;
};

// Error flags raised by the validation kernel.
enum : int {
    kErrRowPtr = 1, kErrCol = 2, kErrUnsorted = 4, kErrNonFinite = 8, kErrNoDiag = 16,
    kErrDiagNonPos = 32, kErrW = 64, kErrAsym = 128
};

struct Status {
    int code = BCM_OK;
    std::string msg;
};
void set_error(const std::string &m);

// Bump allocator over a few large device chunks obtained from the caller's
// allocator (or hipMalloc).  Nothing is freed before release().
struct Arena {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*dealloc)(void *, size_t, void *) = nullptr;
    void *ctx = nullptr;
    std::vector<std::pair<void *, size_t>> chunks;
    char *cur = nullptr;
    size_t left = 0;
    size_t chunk_min = size_t(64) << 20;
    bool failed = false;

    void *raw_alloc(size_t bytes);
    void raw_free(void *p, size_t bytes);
    void *get(size_t bytes);
    template <typename T>
    T *get_n(size_t n) { return static_cast<T *>(get(n * sizeof(T))); }
    void reserve(size_t bytes);
    void rewind();   // forget all sub-allocations, keep the chunks
    void release();  // free every chunk
};

struct Csr {
    int n = 0, nnz = 0;
    int *rp = nullptr, *ci = nullptr;
    double *v = nullptr;
    float *v32 = nullptr;
    // set while the exact entry count is still on the device only (setup): nnz
    // then holds an upper bound, the capacity of ci and v; nnz_dev[1] holds the
    // longest row's length
    const int *nnz_dev = nullptr;
    // bound on the longest row (exact once read back; 0 = unknown: n)
    int dmax = 0;
};

// Sliced ELL copy of a CSR matrix for the row-parallel solve kernels: rows in
// slices of 64 (one wave), slice s holds width w_s = its longest row; entry k
// of row 64 s + l sits at sp[s] + 64 k + l.  Rows keep their CSR column order
// and are padded with (col = row, value = 0), so a row sum taken left to right
// equals the CSR one.  Columns are stored as int16 offsets col - row when every
// offset of the level fits (sd), else as int32 columns (sc).  Values: float64
// (sv) and, for float32 cycles, float32 (sv32); when every value of the level
// is exactly a float32 only sv32 is kept and the float64 kernels widen it
// (exactly) on load.
constexpr int kSlice = 64;
// Sliced-ELL levels whose slices average more than this many slots read their
// rows in batches of 16 slots instead of 8.
constexpr int kWideSlots = 12;
struct Sell {
    int nslices = 0;
    int *sp = nullptr, *sc = nullptr;
    short *sd = nullptr;
    // int16 copies only: uni[s] = 1 when the rows of slice s share one list of
    // column offsets, held in su from index sp[s] / 64 (one per slot column)
    int *uni = nullptr;
    int *su = nullptr;
    double *sv = nullptr;
    float *sv32 = nullptr;
    // finest level, FP32 cycle: sv32 scaled by the inverse l1 diagonal of each
    // slot's column (the values of A D), read by the down leg's residual
    float *svd = nullptr;
    double mixed = 1.0;  // fraction of the slots in slices that are not uniform
    int wide = 0;        // slices average more than kWideSlots slots: batches of 16
    // the solve's product, its down-leg residuals and its one-thread-per-row
    // smoother load the values non-temporally: set on every level when the
    // values a solve iteration reads exceed kStreamSolve
    int stream = 0;
};

// Bytes of matrix values per solve iteration (both cycle legs of every
// sliced-ELL level and the finest level's product) above which the values
// are streamed: below it they stay in the 256 MB Infinity Cache between
// iterations, and non-temporal loads that skip it measured slower (100^3:
// about 0.1 GB, solve +4.6%); above it the cache cannot hold them and the L2
// keeps the gathered vectors instead (160^3 residual 43.0 -> 40.4 us, product
// 78.6 -> 74.8 us; 128^3 and 160^3 ratio-rule solves -4.6% and -1.4%,
// elasticity -4.9%).  The slot-split smoother measured slower streamed and
// keeps cached loads.
constexpr long long kStreamSolve = 192LL << 20;

// A coarsest level shaped as a star: one hub row coupled to every other row,
// each of which holds only its diagonal and the hub entry.  The coarse solve's
// sweeps from zero (the coarsest step of Algorithm 1: l1-Jacobi sweeps, 20 in
// the Section 5 settings) are then a recurrence in the hub's value alone
// (k_star_*), the same operator evaluated in another order:
// with c_j = 1 - d_j a_jj, row j after k sweeps is
//   sum_{t<k} c_j^(k-1-t) d_j (b_j - a_jh x_h^(t)),
// so the hub row's product after k sweeps is
//   sum_{t<k} (E_(k-1-t) - F_(k-1-t) x_h^(t)),
//   E_m = sum_j a_hj c_j^m d_j b_j,  F_m = sum_j a_hj c_j^m d_j a_jh
// (j over the hub row's columns off the diagonal).  F depends on the matrix
// alone and is formed at setup; E takes one pass over the hub row.
constexpr int kStarBlocks = 64;      // workgroups of the pass that forms E
constexpr int kStarMaxSweeps = 32;   // sweeps beyond this keep the sweep kernels
struct StarView {
    int hub = -1;                  // -1: not a star
    int nh = 0;                    // hub-row entries off the diagonal
    const int *hj = nullptr;       // their columns
    const double *ha = nullptr;    // their values a_hj
    const double *c = nullptr;     // c_j = 1 - d_j a_jj per row
    const double *F = nullptr;     // F_m, m < sweeps - 1
    double *part = nullptr;        // E partials: (kStarMaxSweeps - 1) x kStarBlocks
    double *xh = nullptr;          // x_h after t sweeps, t = 0 .. sweeps
    double ahh = 0.0, dh = 0.0;    // the hub's diagonal and inverse l1 diagonal
};

// One level of the hierarchy.  Row i of A^k, its l1 inverse diagonal, the
// composed prolongator P^k (one nonzero per row: column agg[i], value p[i]),
// and the members of every coarse aggregate (P^k transposed) in ascending
// order, mstride slots per aggregate padded with -1.
struct Level {
    Csr A;
    LongRows lr;  // rows longer than long_min(G) of the rule (set at the end of setup)
    Sell E;  // sliced ELL copy (finest level, and levels that run the split up leg)
    double *w = nullptr;
    double *dinv = nullptr;
    float *dinv32 = nullptr;
    int G = 8;  // lanes per row for this level's row kernels
    int nc = 0;
    int *agg = nullptr;
    double *p = nullptr;
    float *p32 = nullptr;
    int mstride = 0;
    int *mem = nullptr;
    void *b = nullptr, *x = nullptr;  // cycle vectors for k >= 1 (cycle precision)
    void *xp = nullptr;               // prolonged iterate of the split up leg (cycle precision)
    void *yb = nullptr;               // dinv o b of the down leg on sliced-ELL levels with long rows
    void *xs = nullptr;               // W/K-cycle: result of the second coarse cycle (cycle precision)
    void *kv = nullptr;               // K-cycle: A c1, the product of the first coarse direction
    double *S = nullptr;  // coarsest level only: dense sweep operator (n <= kCoarseDense)
    StarView star;        // coarsest level only: the star recurrence (hub >= 0)
};

// Device-side view of one level for the single-workgroup tail kernel
// (value arrays in cycle precision).
struct TailLevel {
    int n, nc, mstride, pad;
    const int *rp, *ci, *agg, *mem;
    const void *a, *dinv, *p;
    void *b, *x, *xs;
};
constexpr int kTailRows = 512;  // levels up to this size run inside the tail kernel
// Operations of the tail kernel's program, one int each: op | level << 8 | sel << 16
// (sel = 1: UP / COARSE write the level's save buffer xs instead of x).
enum : int { kTailDown = 1, kTailUp = 2, kTailCoarse = 3, kTailResid = 4, kTailAdd = 5 };
constexpr int kKPartBlocks = 1024;  // K-cycle dot products: at most this many block partials

struct ProfClass {
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
};

}  // namespace bcm

// The flexible-CG loop's stop test after an update, handed to the first kernel
// of the next cycle: part holds the update's nb block partials of ||r||^2 and
// scal the loop's scalars; part null: no stop test.
struct StopTest {
    const double *part;
    double *scal;
    int nb;
};

struct bcm_handle {
    bcm_params prm{};
    hipStream_t s = nullptr;
    int nl = 0;
    bcm::Level lv[bcm::kMaxLevels];
    bcm::Arena persist, scratch;
    // flexible CG vectors (float64, n of the finest level)
    double *r = nullptr, *w = nullptr, *d = nullptr, *v = nullptr, *q = nullptr;
    double *u = nullptr;                  // iterate of the solve (the caller's x is copied in and out)
    void *y0 = nullptr;  // dinv o r of the finest level in the cycle's type, written by the update
                         // (finest levels whose sliced-ELL down leg gathers dinv o b; else null)
    hipStream_t cap = nullptr;            // internal stream used only to capture the iteration graph
    // one general flexible-CG iteration as one graph, or three when one kernel
    // class is profiled (before it, the class, after it); null: empty segment
    hipGraphExec_t iter_exec[3] = {nullptr, nullptr, nullptr};
    int n_exec = 0;
    int graph_prof_cls = -1;  // class the segments are cut at (-1: none)
    // device scalars: [0] alpha [1] beta [2] gamma [3] rho of the last step [4] ||r||^2
    // [5] ||b||^2 [6] breakdown flag [8] gamma_i / rho_{i-1} [9] alpha_i / rho_i
    // [10] solve-ended flag [11] iterations done [12] tol^2 ||b||^2 [13] itmax
    double *scal = nullptr;
    double *ctmp[2] = {nullptr, nullptr};  // coarsest-level sweep buffers when n > kCoarseLds
    bcm::TailLevel *tail = nullptr;        // device table of levels for the tail kernel
    int kt = -1;                           // first level handled by the tail kernel (-1: none)
    int kf = 0;                            // first level of the folded dense operator (0: none):
                                           // the V- or W-cycle from level kf down, as one n_kf x n_kf map
    double *fold = nullptr;                // that operator, n_kf x n_kf row-major, float64
    int *tail_ops = nullptr;               // the tail kernel's program (device)
    int n_tail_ops = 0;
    double *partials = nullptr;
    double *spart = nullptr;  // the finest product's partials (never aliases partials: the update reads them)
    double *lpart = nullptr;  // chunk sums of the long rows (the largest level's chunk count)
    double *kpart = nullptr;  // K-cycle block partials (3 * kKPartBlocks)
    double *ks = nullptr;     // K-cycle scalars, 8 per level
    double *host_scal = nullptr;  // pinned
    int red_blocks = 0;
    double last_tol = 0.0;
    int iters = 0, status = 0;
    double relres = 0.0, t_setup_ms = 0.0, t_solve_ms = 0.0;
    // profiling
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_pairs;  // (class, event index of the start)
    std::vector<double> ev_bytes;
    std::vector<int> ev_iter;
    bcm::ProfClass prof[9];
    double setup_bytes = 0.0;  // sum over the pairwise sweeps of 72 z + 80 m
    int sweeps_run = 0;
};

namespace bcm {

int pick_G(double avg_nnz_per_row);

// ---- setup kernels (setup.hip) ----
// Validation (bounds, order, finiteness, diagonal; symmetry when check_sym);
// the diagonal goes to diag.  With seg.ctl given, rows longer than lmin are
// appended to seg and their entries are checked by launch_long_validate
// (launched by the caller after this, once seg is fixed up).  dmax, when given
// (starting at 0), gets the longest row's length.
void launch_validate(hipStream_t s, int G, int n, int nnz, const int *rp, const int *ci,
                     const double *v, const double *w, int check_sym, double *diag, int *flags,
                     const SegList &seg = SegList(), int lmin = 0, int *dmax = nullptr);
// weights of the rows up to lmin entries (lmin = 0: every row)
void launch_weights(hipStream_t s, int G, int n, const int *rp, const int *ci, const double *v, const double *diag,
                    const double *w, double *c, unsigned long long *ws, int lmin = 0);
// Suitor candidate lists; matrices averaging at least kSortedCandidatesAvg
// entries per row sort each row (own-row ranks in rk[nnz], scratch).  Rows
// longer than lmin (0: none) are left to launch_long_candidates; the direct
// kernel then takes the rank of an entry seen from such a row from rk.
constexpr int kSortedCandidatesAvg = 24;
void launch_candidates(hipStream_t s, int G, int n, bool sorted, const int *rp, const int *ci, const double *c,
                       unsigned *rk, unsigned long long *cand, int lmin = 0, int part = 0);
// ---- long segments (setup.hip) ----
// rows of (n, rp) longer than lmin appended to seg; idx (optional) gets each
// row's position in seg or -1
void launch_find_long(hipStream_t s, int n, const int *rp, int lmin, const SegList &seg, int *idx);
// Galerkin coarse rows with more than lmin candidate entries (members' rows)
void launch_find_long_gal(hipStream_t s, int nc, const int *mem2, const int *rp, int lmin, const SegList &seg);
// offsets, chunk bases and totals of seg (one workgroup)
void launch_seg_fix(hipStream_t s, const SegList &seg);
// per-entry checks of the long rows in seg (as the validation kernel does)
void launch_long_validate(hipStream_t s, int n, int nnz, const int *rp, const int *ci, const double *v,
                          int check_sym, const SegList &seg, int *flags);
void launch_long_weights(hipStream_t s, const SegList &seg, const int *rp, const int *ci, const double *v,
                         const double *diag, const double *w, double *c);
// Own-row ranks and candidate lists of the long rows (a segmented sort of each
// row; keys scratch k0/k1 of 2 * total length, maxlen bounds the longest).
// direct: rk holds ranks for the long rows only (the other rows count theirs).
void launch_long_ranks(hipStream_t s, const SegList &seg, int maxlen, const int *rp, const double *c,
                       unsigned *rk, unsigned long long *k0, unsigned long long *k1);
void launch_long_candidates(hipStream_t s, const SegList &seg, int maxlen, const int *rp, const int *ci,
                            const double *c, const unsigned *rk, int lmin, bool direct, unsigned long long *cand,
                            unsigned long long *k0, unsigned long long *k1);
// Galerkin coarse rows of seg: sort their candidates (keys left in *sorted),
// then pass 0 counts distinct columns into cnt, pass 1 fills the entries
void launch_gal_long_sort(hipStream_t s, const SegList &seg, int maxlen, const int *rp, const int *ci,
                          const int *agg, const int *mem2, unsigned long long *k0, unsigned long long *k1,
                          unsigned long long **sorted);
void launch_gal_long(hipStream_t s, int pass, const SegList &seg, const unsigned long long *sorted, const int *rp,
                     const int *ci, const double *v, const int *agg, const double *p, const int *mem2, int *cnt,
                     int *cc, const int *crp, int *cci, double *cv);
// l1 row norms of the long rows of a level: chunk partial sums into part
// (float64), float32 copies of their values into v32 when given
void launch_long_abs(hipStream_t s, const LongRows &lr, const int *rp, const double *v, double *part, float *v32);
void launch_suitor(hipStream_t s, int n, const int *rp, const unsigned long long *cand, unsigned long long *ws);
void launch_mate(hipStream_t s, int n, const int *rp, const int *ci, const unsigned long long *ws, int *mate,
                 int *leader, const int *csrc = nullptr, int *cdst = nullptr);
void launch_aggfill(hipStream_t s, int n, const int *mate, const int *ofs, const double *w,
                    int *agg, double *p, double *wc, int *mem2);
// Galerkin product of one pairwise sweep (coarse rows with more than lmin
// candidates are left to launch_gal_long; lmin = 0: none)
void launch_gal_count(hipStream_t s, int G, int nc, const int *rp, const int *ci, const int *agg,
                      const int *mem2, int *cnt, int *gF, int *gU, bool sorted, int lmin = 0);
void launch_gal_fill(hipStream_t s, int G, int nc, const int *rp, const int *ci, const double *v,
                     const int *agg, const double *p, const int *mem2, const int *crp, int *cci,
                     double *cv, int *gF, int *gU, bool sorted, int lmin = 0);
void launch_compose(hipStream_t s, int n, int nc_new, const int *agg_prev, const double *p_prev,
                    const int *mem_prev, int stride_prev, const int *agg_s, const double *p_s,
                    const int *mem_s, int *agg_out, double *p_out, int *mem_out);
// l1-Jacobi inverse diagonal; the level's long rows take their norms from
// the partial sums of launch_long_abs (lr.n = 0: none)
void launch_diag_l1(hipStream_t s, int G, int n, const int *rp, const double *v, double *dinv,
                    float *dinv32, float *v32, const LongRows &lr = LongRows(), const double *part = nullptr);
void launch_cast(hipStream_t s, size_t n, const double *src, float *dst);
// slice widths (64 * longest row of each slice) -> cnt[nslices]; *maxoff is
// raised to the largest |col - row| of the matrix, *inexact to 1 if a value is
// not exactly a float32 (start both at 0)
void launch_sell_width(hipStream_t s, int n, const int *rp, const int *ci, const double *v, int *cnt, int *uni,
                       int *maxoff, int *inexact, int *mixed);
// fills the slots: int32 columns into sc, or int16 offsets into sd (one is null)
void launch_sell_fill(hipStream_t s, int n, const int *rp, const int *ci, const double *v, const int *sp,
                      const int *uni, int *su, int *sc, short *sd, double *sv, float *sv32);
// svd[slot] = sv32[slot] * dinv32[column of the slot] over every slot of the
// sliced-ELL copy (rows past n: 0)
void launch_sell_scale_cols(hipStream_t s, int n, int nslices, const int *sp, const int *uni, const int *su,
                            const int *sc, const short *sd, const float *sv32, const float *dinv32, float *svd);
void launch_fill_i32(hipStream_t s, size_t n, int *dst, int val);
void launch_fill_u64(hipStream_t s, size_t n, unsigned long long *dst, unsigned long long val);
void launch_copy_f64(hipStream_t s, size_t n, const double *src, double *dst);
// dst = src on the finest level's vector length; also a graph-safe fill (no memset node)

// ---- scan (scan.hip) ----
size_t scan_tmp_bytes(int n);
// out[i] = sum_{j<i} in[j] (in and out may alias); total written to *total_dev,
// and the largest in[i] to *max_dev when given.
void scan_exclusive(hipStream_t s, const int *in, int *out, int n, int *total_dev, void *tmp,
                    int *max_dev = nullptr);

// ---- solve kernels (solve.hip) ----
// Cycle kernels return at once when done != NULL and *done != 0 (the flexible
// CG loop's "solve ended" flag); done = NULL outside that loop.
// part: 0 = the whole leg; 1 / 2 = its first / second kernel only (a leg of one
// kernel: that kernel is part 1 of the down leg and part 2 of the up leg)
// true when level L's down leg runs as the sliced-ELL residual + restriction
inline bool down_on_sell(const Level &L) { return L.E.sp && L.xp && (L.mstride == 2 || L.mstride == 4); }
// yr (part 0 or 1 of a sliced-ELL level's down leg): dinv o b already formed,
// in the cycle's type; null: formed here when the level needs it.  next (part
// 0 or 2 of such a leg): the coarser level, whose dinv o b the restriction
// then also writes into next->yb; null: it does not.
// st (part 1 of a sliced-ELL level's leg): the flexible-CG stop test that
// workgroup 0 of its residual kernel takes first (StopTest); default: none.
void launch_down(hipStream_t s, const Level &L, int fp32, const void *b, void *bc, int b_is_f64,
                 const double *done, int part = 0, const void *yr = nullptr, const Level *next = nullptr,
                 StopTest st = {});
void launch_up(hipStream_t s, const Level &L, int fp32, const void *b, const void *xc, void *x,
               int b_is_f64, int x_is_f64, const double *done, int part = 0);
void launch_coarse(hipStream_t s, const Level &L, int sweeps, const void *b, void *x, int b_f64,
                   int x_f64, void *tmp_a, void *tmp_b, const double *done);
// true when the coarsest level (without a dense operator) runs in one workgroup
// with everything in LDS; otherwise launch_coarse needs two n-vectors tmp_a/b
bool coarse_in_lds(int n, int nnz, bool long_rows);
// Each of these is a streaming kernel writing block partials; launch_finalize
// (mode 0 after resid, 1 after spmv_dots, 2 after update) then sums them in
// block order into scal[].
// W-cycle: b <- b - A x in place on a level >= 1, and x <- x + y
void launch_resid_inplace(hipStream_t s, const Level &L, int fp32, const void *x, void *b, const double *done);
void launch_add(hipStream_t s, int n, int fp32, const void *y, void *x, const double *done);
// K-cycle coarse solve on level C: step 1 after the first coarse cycle (c1 in
// x): v1 = A c1, scalars, b <- b - (alpha1/rho1) v1; step 2 after the second
// (c2): scalars, x <- (alpha1/rho1) c1 + (alpha2/rho2)(c2 - (gamma/rho1) c1).
void launch_kcycle_step1(hipStream_t s, const Level &C, int fp32, const void *c1, const void *b, void *v1,
                         double *partials, double *ks, const double *done);
void launch_kcycle_step2(hipStream_t s, const Level &C, int fp32, const void *c2, const void *b, const void *v1,
                         void *x, double *partials, double *ks, const double *done);
// the cycle of levels kt .. nl-1 in one workgroup: runs the nops operations of
// ops (from b of level kt into x_out); tail table tl, coarsest level C
void launch_tail(hipStream_t s, int fp32, int kt, int nl, const TailLevel *tl, const Level &C, int sweeps,
                 const int *ops, int nops, void *x_out, const double *done);
// S = sum_{t < sweeps} (I - D A)^t D of the coarsest level, column by column
void launch_coarse_build(hipStream_t s, const Level &L, int sweeps, double *S);
// Folded V-cycle of level L (pre = post = 1) from the coarser level's map Tc
// (nc x nc): T = D + (I - D A)(D + P Tc P^T (I - A D)), n x n row-major; H is
// n x n scratch.  A must be exactly symmetric (every coarse level is).
void launch_fold_level(hipStream_t s, const Level &L, const double *Tc, int nc, double *H, double *T);
// W-cycle coarse solve of the level above L by two cycles of L: W = 2T - T A T
// (T, W n x n row-major; M n x n scratch)
void launch_fold_w(hipStream_t s, const Level &L, const double *T, double *M, double *W);
// T = D + (I - D A) H for dense n x n row-major H and T (level L's matrix)
void launch_fold_left(hipStream_t s, const Level &L, const double *H, double *T);
// x = T b with a dense n x n row-major float64 operator (float64 accumulation)
void launch_dense(hipStream_t s, int n, const double *T, const void *b, void *x, int b_f64, int x_f64,
                  const double *done);
void launch_resid(hipStream_t s, const Level &L, int nb, const double *b, const double *u, double *r,
                  double *partials, double *scal);
// workgroups of the flexible-CG product on level L (nb: the reduction grid of
// the vector kernels): one per slice on the levels whose rows it splits, else nb.
// launch_spmv_dots takes this count and writes that many partials per product.
int spmv_dots_grid(const Level &L, int nb);
// level L's sliced-ELL legs take the slot-split kernels (wide slices, at most 2^19 rows)
bool slot_split_level(const Level &L);
void launch_spmv_dots(hipStream_t s, const Level &L, int nb, int first, const double *w, const double *r,
                      const double *q, double *v, double *partials, double *scal);
// with y: also y = dinv o r (float when y_f32, else double; dinv of that type).
// with dots: the update adds the product's ndots partials and forms the step
// scalars itself (no mode-1 finalize before it); allowed when
// update_takes_dots(ndots).
void launch_update(hipStream_t s, int n, int nb, int first, const double *w, const double *v,
                   double *d, double *u, double *q, double *r, double *partials, double *scal,
                   const void *dinv = nullptr, void *y = nullptr, int y_f32 = 0, const double *dots = nullptr,
                   int ndots = 0);
bool update_takes_dots(int nbs);
void launch_finalize(hipStream_t s, int mode, int nb, int first, const double *partials, double *scal);
void launch_sampled_outer(hipStream_t s, const Level &L, const double *lam, const double *x,
                          double *G);
int reduce_blocks(int n);

}  // namespace bcm
