// C ABI of the library: hierarchy setup (Sections 2.1, 2.2, 3.1 of the paper),
// flexible-CG solve with the V-cycle preconditioner (Algorithms 1 and 3,
// Section 3.2), adjoint solve and sampled outer product for gradients.
// Host code here only sequences kernels, reads back sizes and convergence
// scalars, and manages device memory; all arithmetic runs in the kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>

#include "internal.h"

namespace bcm {

thread_local KernelEvents g_kernel_events;

namespace {
thread_local std::string g_err;
thread_local double *g_pinned = nullptr;  // 64 doubles of pinned host memory per thread

double *pinned() {
    if (!g_pinned) {
        if (hipHostMalloc((void **)&g_pinned, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
            g_pinned = nullptr;
    }
    return g_pinned;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

void set_error(const std::string &m) { g_err = m; }

// ---------------------------------------------------------------- arena
void *Arena::raw_alloc(size_t bytes) {
    void *p = nullptr;
    if (alloc) {
        p = alloc(bytes, ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    return p;
}

void Arena::raw_free(void *p, size_t bytes) {
    if (!p) return;
    if (dealloc) dealloc(p, bytes, ctx);
    else (void)hipFree(p);
}

void *Arena::get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (bytes > left) {
        const size_t sz = std::max(bytes, chunk_min);
        void *p = raw_alloc(sz);
        if (!p) { failed = true; return nullptr; }
        chunks.push_back({p, sz});
        cur = static_cast<char *>(p);
        left = sz;
    }
    void *r = cur;
    cur += bytes;
    left -= bytes;
    return r;
}

void Arena::reserve(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (left >= bytes) return;
    void *p = raw_alloc(bytes);
    if (!p) { failed = true; return; }
    chunks.push_back({p, bytes});
    cur = static_cast<char *>(p);
    left = bytes;
}

void Arena::rewind() {
    if (chunks.empty()) return;
    if (chunks.size() > 1) {
        size_t tot = 0;
        for (auto &c : chunks) tot += c.second;
        release();
        reserve(tot);
        return;
    }
    cur = static_cast<char *>(chunks[0].first);
    left = chunks[0].second;
}

void Arena::release() {
    for (auto &c : chunks) raw_free(c.first, c.second);
    chunks.clear();
    cur = nullptr;
    left = 0;
}

}  // namespace bcm

using namespace bcm;

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_error(std::string("HIP error ") + hipGetErrorString(e_) + " in " #expr);   \
            return BCM_EHIP;                                                                \
        }                                                                                   \
    } while (0)

#define NOMEM(ptr)                                                    \
    do {                                                              \
        if (!(ptr)) {                                                 \
            set_error("device allocation failed (" #ptr ")");         \
            return BCM_ENOMEM;                                        \
        }                                                             \
    } while (0)

// Device scratch of the allocation-free matching entry point: one array on
// each GPU, kept until the process ends.  Host code passes the address that
// noalloc_scratch() looked up for the current device, never this name.
static __device__ __align__(256) unsigned char scratch[BCM_NOALLOC_SCRATCH_BYTES];

namespace {

std::string flag_text(int f) {
    std::string s;
    if (f & kErrRowPtr) s += " row_ptr not monotone / not 0..nnz;";
    if (f & kErrCol) s += " column index out of [0, n);";
    if (f & kErrUnsorted) s += " columns not strictly ascending in a row;";
    if (f & kErrNonFinite) s += " non-finite value;";
    if (f & kErrNoDiag) s += " missing diagonal entry;";
    if (f & kErrDiagNonPos) s += " non-positive diagonal entry;";
    if (f & kErrW) s += " smooth vector entry zero or not finite;";
    if (f & kErrAsym) s += " matrix not bitwise symmetric;";
    return s;
}

int read_back(hipStream_t s, const void *dev, size_t bytes, void *host) {
    double *pin = pinned();
    if (!pin || bytes > 64 * sizeof(double)) {
        HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return BCM_OK;
    }
    HIPCHK(hipMemcpyAsync(pin, dev, bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(host, pin, bytes);
    return BCM_OK;
}

// The same without the pinned staging buffer (no host allocation at all).
int read_back_plain(hipStream_t s, const void *dev, size_t bytes, void *host) {
    HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return BCM_OK;
}

// The coarsest level's StarView when it is a star (one hub row, every other
// row holding only its diagonal and the hub entry); otherwise L.star stays
// unset and the coarse solve keeps its sweep kernels.  The matrix is read back
// once; E's weights F_m are formed here in FP64, in the hub row's order.
int build_star(bcm_handle *h, hipStream_t s, Level &L, int sweeps) {
    const int n = L.A.n, nnz = L.A.nnz;
    std::vector<int> rp(n + 1), ci(nnz);
    std::vector<double> a(nnz), dinv(n);
    int rc = read_back(s, L.A.rp, sizeof(int) * (n + 1), rp.data());
    if (!rc) rc = read_back(s, L.A.ci, sizeof(int) * nnz, ci.data());
    if (!rc) rc = read_back(s, L.A.v, sizeof(double) * nnz, a.data());
    if (!rc) rc = read_back(s, L.dinv, sizeof(double) * n, dinv.data());
    if (rc) return rc;
    int hub = -1;
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] - rp[i] > 2) {
            if (hub >= 0) return BCM_OK;  // two rows beyond two entries: not a star
            hub = i;
        }
    if (hub < 0) return BCM_OK;
    // every other row: its diagonal, and at most the hub besides
    std::vector<double> c(n, 0.0), f(n, 0.0);
    for (int j = 0; j < n; ++j) {
        if (j == hub) continue;
        bool diag = false;
        double ajj = 0.0, ajh = 0.0;
        for (int q = rp[j]; q < rp[j + 1]; ++q) {
            if (ci[q] == j) { diag = true; ajj = a[q]; }
            else if (ci[q] == hub) ajh = a[q];
            else return BCM_OK;
        }
        if (!diag) return BCM_OK;
        c[j] = 1.0 - dinv[j] * ajj;
        f[j] = dinv[j] * ajh;
    }
    std::vector<int> hj;
    std::vector<double> ha;
    double ahh = 0.0;
    for (int q = rp[hub]; q < rp[hub + 1]; ++q) {
        if (ci[q] == hub) ahh = a[q];
        else { hj.push_back(ci[q]); ha.push_back(a[q]); }
    }
    const int M = sweeps - 1;
    std::vector<double> F(std::max(M, 1), 0.0);
    for (size_t q = 0; q < hj.size(); ++q) {
        const int j = hj[q];
        double t = ha[q] * f[j];
        for (int m = 0; m < M; ++m) { F[m] += t; t *= c[j]; }
    }
    StarView &sv = L.star;
    const int nh = (int)hj.size();
    int *dhj = h->persist.get_n<int>(std::max(nh, 1));
    double *dha = h->persist.get_n<double>(std::max(nh, 1));
    double *dc = h->persist.get_n<double>(n);
    double *dF = h->persist.get_n<double>(F.size());
    double *dpart = h->persist.get_n<double>((size_t)(kStarMaxSweeps - 1) * kStarBlocks);
    double *dxh = h->persist.get_n<double>(kStarMaxSweeps + 1);
    NOMEM(dhj && dha && dc && dF && dpart && dxh);
    if (nh) {
        HIPCHK(hipMemcpyAsync(dhj, hj.data(), sizeof(int) * nh, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(dha, ha.data(), sizeof(double) * nh, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipMemcpyAsync(dc, c.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dF, F.data(), sizeof(double) * F.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    sv.hub = hub;
    sv.nh = nh;
    sv.hj = dhj;
    sv.ha = dha;
    sv.c = dc;
    sv.F = dF;
    sv.part = dpart;
    sv.xh = dxh;
    sv.ahh = ahh;
    sv.dh = dinv[hub];
    return BCM_OK;
}

struct SweepOut {
    int prof_gal = -1;  // setup profile bracket of this sweep's Galerkin product
    int nc = 0;
    int *agg = nullptr;
    double *p = nullptr;
    double *wc = nullptr;
    int *mem2 = nullptr;
    Csr Ac;
};

// Lanes per row of the CSR row kernels: the forced width of the parameters,
// else the rule on the average row length.
int lanes_for(int group, const Csr &A) {
    return group > 0 ? group : pick_G((double)A.nnz / std::max(1, A.n));
}

bool valid_group(int g) { return g == 0 || g == -1 || g == 4 || g == 8 || g == 16 || g == 32 || g == 64; }

// Sub-allocation from one block of device memory in 256-byte steps (a null
// base with an unbounded size measures a layout without touching memory).
struct Carver {
    char *cur = nullptr;
    size_t left = 0;
    size_t used = 0;
    bool ok = true;
    template <typename T>
    T *get(size_t n) {
        size_t b = (n * sizeof(T) + 255) & ~size_t(255);
        if (b == 0) b = 256;
        if (b > left) { ok = false; return nullptr; }
        T *r = reinterpret_cast<T *>(cur);
        if (cur) cur += b;
        left -= b;
        used += b;
        return r;
    }
};

// Event timing of the setup kernel classes (bcm_params.profile bits
// BCM_PROF_SETUP_*): one event pair per bracket, taken by the kernel's own
// dispatch for a single-kernel class, else recorded on the stream; summed
// into the handle's class totals once setup has finished.
struct SetupProf {
    hipStream_t s = nullptr;
    int mask = 0;
    struct Rec {
        int bit;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> rec;
    int begin(int bit, bool single) {
        if (!(mask & bit)) return -1;
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return -1;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return -1;
        }
        rec.push_back({bit, a, b, 0.0});
        if (single) g_kernel_events = KernelEvents{a, b};
        else (void)hipEventRecord(a, s);
        return (int)rec.size() - 1;
    }
    void end(int idx, bool single, double bytes) {
        if (idx < 0) return;
        rec[idx].bytes = bytes;
        if (!single) (void)hipEventRecord(rec[idx].b, s);
        else if (g_kernel_events.start) {  // no kernel took the events: no sample
            g_kernel_events = KernelEvents{};
            rec[idx].bit = 0;
        }
    }
    void set_bytes(int idx, double bytes) {
        if (idx >= 0) rec[idx].bytes = bytes;
    }
    // adds the samples to prof[] (index = log2 of the class bit); call after a sync
    void collect(bcm::ProfClass *prof) {
        for (auto &r : rec) {
            float ms = 0.f;
            if (r.bit && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                int i = 0;
                for (int b = r.bit; b > 1; b >>= 1) ++i;
                prof[i].launches += 1;
                prof[i].ms += ms;
                prof[i].bytes += r.bytes;
            }
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        rec.clear();
    }
    ~SetupProf() {
        for (auto &r : rec) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
    }
};

// Algorithmic bytes of the setup classes on a sweep over m rows, z entries,
// nc aggregates and zc coarse entries (every array once, gathers cached).
// weights: row pointers, columns, values, diagonal and w, c and ws written;
// candidate lists: columns and c read, the lists written (+ the own-row ranks
// written and read when the rows are sorted).
double bytes_setup_match(double m, double z, bool sorted) {
    return 2 * 4 * (m + 1) + 20 * z + 24 * m + 20 * z + (sorted ? 8 * z : 0.0);
}
// Suitor: each vertex reads its row bounds, at least one candidate and
// raises at least one proposal word.
double bytes_setup_suitor(double m) { return 8 * (m + 1) + 16 * m; }
// Galerkin, both passes: members and their row bounds, columns and their
// aggregates (twice), values and p once, counts, the scan, row pointers,
// and the coarse columns and values written.
double bytes_setup_galerkin(double m, double z, double nc, double zc) {
    return 2 * (8 * nc + 8 * m + 4 * z + 4 * m) + 8 * z + 8 * m + 4 * nc + 8 * nc + 4 * nc + 12 * zc;
}

// Device scratch of one matching sweep on an m-row matrix with nnz entries.
// c and mate may be the caller's arrays (c_ext, mate_ext); diag is absent when
// the caller hands in the diagonal of an already validated matrix.  With
// lmin > 0 it also holds the list of rows longer than lmin (at most
// nnz / (lmin + 1) of them); the sort keys of those rows (2 x their total
// length) are carved separately once that length or a bound is known.
struct MatchScratch {
    double *diag = nullptr;
    int *flags = nullptr;
    double *c = nullptr;
    unsigned long long *cand = nullptr;
    unsigned *rk = nullptr;
    unsigned long long *ws = nullptr;
    int *mate = nullptr;
    int *leader = nullptr;
    SegList seg;
    int lmin = 0;  // 0: no long-row list
    unsigned long long *k0 = nullptr, *k1 = nullptr;
};

int seg_cap(long long nnz, int lmin) { return (int)(nnz / (lmin + 1) + 1); }

void carve_seg(Carver &cv, int cap, SegList &sg) {
    sg.cap = cap;
    sg.ctl = cv.get<int>(8);
    sg.row = cv.get<int>(cap);
    sg.len = cv.get<int>(cap);
    sg.off = cv.get<int>((size_t)cap + 1);
    sg.cb = cv.get<int>((size_t)cap + 1);
}

void carve_match(Carver &cv, int m, long long nnz, bool own_diag, double *c_ext, int *mate_ext, int lmin,
                 MatchScratch &ms) {
    ms.diag = own_diag ? cv.get<double>(m) : nullptr;
    ms.flags = cv.get<int>(32);
    ms.c = c_ext ? c_ext : cv.get<double>(nnz);
    ms.cand = cv.get<unsigned long long>(nnz);
    ms.rk = cv.get<unsigned>(nnz);
    ms.ws = cv.get<unsigned long long>(m);
    ms.mate = mate_ext ? mate_ext : cv.get<int>(m);
    ms.leader = cv.get<int>(m);
    ms.lmin = lmin;
    if (lmin > 0) carve_seg(cv, seg_cap(nnz, lmin), ms.seg);
}

size_t match_scratch_bytes(int m, long long nnz, bool own_diag, bool c_ext, bool mate_ext, int lmin) {
    Carver cv;
    cv.left = ~size_t(0);
    MatchScratch ms;
    carve_match(cv, m, nnz, own_diag, c_ext ? reinterpret_cast<double *>(8) : nullptr,
                mate_ext ? reinterpret_cast<int *>(8) : nullptr, lmin, ms);
    return cv.used;
}

// Weights, ranks, Suitor matching and mate/leader flags on (A, w): Sections
// 2.2 and 3.1, in the scratch ms.
// With flags_dev given, the validation flags are left there for the caller
// to read with its next read-back (only for matrices already known to be well
// formed: the validated input and the coarse matrices built from it; a bad
// value there makes weights ineligible, never an out-of-bounds access).
// Without it the flags are read back here (pinned: through the thread's pinned
// staging buffer, else a plain copy into host memory), together with the
// long-row list's size, and the long rows' sort keys are then taken from
// keys_from or keys_arena (exact size).  With flags_dev, rows longer than
// ms.lmin may exist only when A.dmax (a bound) exceeds it; their keys must
// already be in ms.k0/k1 (2 x nnz).
// With diag_in given (the diagonal of a matrix already validated), the
// validation pass is skipped.
int match_sweep(hipStream_t s, MatchScratch &ms, const Csr &A, const double *w, int check_sym, int group,
                int *flags_dev = nullptr, int G_hint = 0, const int *copy_src = nullptr,
                const double *diag_in = nullptr, bool pinned_ok = true, Carver *keys_from = nullptr,
                Arena *keys_arena = nullptr, SetupProf *sp = nullptr, int *prof_idx = nullptr) {
    const int m = A.n, G = G_hint > 0 ? G_hint : lanes_for(group, A);
    const int dbound = A.dmax > 0 ? A.dmax : m;
    bool lng = ms.lmin > 0 && dbound > ms.lmin;
    int maxlen = dbound;
    const SegList none;
    const double *diag = diag_in ? diag_in : ms.diag;
    int *flags = flags_dev ? flags_dev : ms.flags;
    launch_fill_i32(s, 1, flags, 0);
    if (lng) launch_fill_i32(s, 8, ms.seg.ctl, 0);
    if (!diag_in) {
        launch_validate(s, G, m, A.nnz_dev ? -1 : A.nnz, A.rp, A.ci, A.v, w, check_sym, ms.diag, flags,
                        lng ? ms.seg : none, ms.lmin);
    } else if (lng) {
        launch_find_long(s, m, A.rp, ms.lmin, ms.seg, nullptr);
    }
    if (lng) {
        launch_seg_fix(s, ms.seg);
        if (!diag_in) launch_long_validate(s, m, A.nnz_dev ? -1 : A.nnz, A.rp, A.ci, A.v, check_sym, ms.seg, flags);
    }
    if (!flags_dev && !diag_in) {
        int f[8] = {0};
        int rc = pinned_ok ? read_back(s, flags, sizeof(int), f) : read_back_plain(s, flags, sizeof(int), f);
        if (rc) return rc;
        if (f[0]) {
            set_error("invalid input:" + flag_text(f[0]));
            return BCM_EINVAL;
        }
        if (lng) {
            rc = pinned_ok ? read_back(s, ms.seg.ctl, 8 * sizeof(int), f)
                           : read_back_plain(s, ms.seg.ctl, 8 * sizeof(int), f);
            if (rc) return rc;
            lng = f[0] > 0;
            maxlen = f[3];
            if (lng) {  // sort keys of the long rows, now that their total is known
                const size_t tot = (size_t)f[1];
                if (keys_from) {
                    ms.k0 = keys_from->get<unsigned long long>(tot);
                    ms.k1 = keys_from->get<unsigned long long>(tot);
                } else if (keys_arena) {
                    ms.k0 = keys_arena->get_n<unsigned long long>(tot);
                    ms.k1 = keys_arena->get_n<unsigned long long>(tot);
                }
                if (!ms.k0 || !ms.k1) {
                    set_error(keys_from ? "the long rows' sort keys do not fit the static scratch"
                                        : "device allocation failed (long-row sort keys)");
                    return keys_from ? BCM_EINVAL : BCM_ENOMEM;
                }
            }
        }
    }
    // candidate lists: direct comparisons for rows of a few dozen entries, else
    // sorted; long rows through the segmented sorts
    const bool sorted = A.nnz >= (long long)kSortedCandidatesAvg * m;
    const int lm = lng ? ms.lmin : 0;
    // (bytes of the brackets: set here when A's entry count is known, else by the caller)
    const int pm = sp ? sp->begin(BCM_PROF_SETUP_MATCH, false) : -1;
    launch_weights(s, G, m, A.rp, A.ci, A.v, diag, w, ms.c, ms.ws, lm);
    if (lng) launch_long_weights(s, ms.seg, A.rp, A.ci, A.v, diag, w, ms.c);
    if (sorted) {
        launch_candidates(s, G, m, true, A.rp, A.ci, ms.c, ms.rk, ms.cand, lm, 1);
        if (lng) launch_long_ranks(s, ms.seg, maxlen, A.rp, ms.c, ms.rk, ms.k0, ms.k1);
        launch_candidates(s, G, m, true, A.rp, A.ci, ms.c, ms.rk, ms.cand, lm, 2);
        if (lng) launch_long_candidates(s, ms.seg, maxlen, A.rp, A.ci, ms.c, ms.rk, lm, false, ms.cand, ms.k0, ms.k1);
    } else {
        if (lng) launch_long_ranks(s, ms.seg, maxlen, A.rp, ms.c, ms.rk, ms.k0, ms.k1);
        launch_candidates(s, G, m, false, A.rp, A.ci, ms.c, ms.rk, ms.cand, lm, 2);
        if (lng) launch_long_candidates(s, ms.seg, maxlen, A.rp, A.ci, ms.c, ms.rk, lm, true, ms.cand, ms.k0, ms.k1);
    }
    if (sp) sp->end(pm, false, A.nnz_dev ? 0.0 : bytes_setup_match(m, A.nnz, sorted));
    const int ps = sp ? sp->begin(BCM_PROF_SETUP_SUITOR, true) : -1;
    launch_suitor(s, m, A.rp, ms.cand, ms.ws);
    if (sp) sp->end(ps, true, bytes_setup_suitor(m));
    if (prof_idx) prof_idx[0] = pm;
    // (copy_src: two ints for the caller's next read-back, to flags_dev[17..18])
    launch_mate(s, m, A.rp, A.ci, ms.ws, ms.mate, ms.leader, copy_src, copy_src ? flags_dev + 17 : nullptr);
    HIPCHK(hipGetLastError());
    return BCM_OK;
}

// One pairwise sweep on (A, w): matching, Algorithm 2, prolongator, Galerkin.
// Outputs that outlive the sweep come from `keep`, except that the coarse
// matrix and w come from finA and the prolongator from finP when those are
// given (the level's final outputs, allocated where they stay).  out.nc == A.n
// means that no pair was formed (nothing else is produced then).
int pairwise_sweep(hipStream_t s, Arena &tmp, Arena &keep, Csr &A, const double *w, int group, int G_hint,
                   SweepOut &out, Arena *finA, Arena *finP, const double *diag_in = nullptr,
                   SetupProf *sp = nullptr, double *sweep_bytes = nullptr) {
    // A's exact entry count and longest row, when still on the device, come
    // back with this sweep's first read-back (G_hint sizes the lanes of the
    // kernels before it, A.dmax bounds its rows)
    Arena &oa = finA ? *finA : keep;
    Arena &op = finP ? *finP : keep;
    const int m = A.n;
    const int Gm = A.nnz_dev && G_hint > 0 ? G_hint : lanes_for(group, A);
    int *ctl = tmp.get_n<int>(32);  // [0] flags, [16] aggregates, [17] A's entries, [18] A's longest row
    NOMEM(ctl);
    MatchScratch ms;
    {
        const size_t bytes = match_scratch_bytes(m, A.nnz, !diag_in, false, false, long_min(Gm));
        Carver cv;
        cv.cur = static_cast<char *>(tmp.get(bytes));
        cv.left = bytes;
        NOMEM(cv.cur);
        carve_match(cv, m, A.nnz, !diag_in, nullptr, nullptr, long_min(Gm), ms);
    }
    // sort keys of the long rows (matching, then the Galerkin product): at most
    // every entry of A
    unsigned long long *k0 = nullptr, *k1 = nullptr;
    auto keys = [&]() {
        if (!k0) {
            k0 = tmp.get_n<unsigned long long>(A.nnz);
            k1 = tmp.get_n<unsigned long long>(A.nnz);
        }
        return k0 && k1;
    };
    if ((A.dmax > 0 ? A.dmax : m) > ms.lmin) {
        NOMEM(keys());
        ms.k0 = k0;
        ms.k1 = k1;
    }
    int pm = -1;
    int rc = match_sweep(s, ms, A, w, 0, group, ctl, Gm, A.nnz_dev, diag_in, true, nullptr, nullptr, sp, &pm);
    if (rc) return rc;
    int *mate = ms.mate, *leader = ms.leader;
    int *ofs = leader;  // scanned in place
    void *stmp = tmp.get(scan_tmp_bytes(m));
    NOMEM(stmp);
    scan_exclusive(s, leader, ofs, m, ctl + 16, stmp);
    int hc[19];
    rc = read_back(s, ctl, sizeof(hc), hc);
    if (rc) return rc;
    if (hc[0]) {
        set_error("invalid coarse-level matrix:" + flag_text(hc[0]));
        return BCM_EINVAL;
    }
    if (A.nnz_dev) {
        A.nnz = hc[17];
        A.dmax = hc[18];
        A.nnz_dev = nullptr;
        if (sp) sp->set_bytes(pm, bytes_setup_match(m, A.nnz, A.nnz >= (long long)kSortedCandidatesAvg * m));
    }
    if (sweep_bytes) *sweep_bytes = 72.0 * A.nnz + 80.0 * m;
    const int nc = hc[16], G = lanes_for(group, A);
    out.nc = nc;
    if (nc == m) return BCM_OK;
    out.agg = op.get_n<int>(m);
    out.p = op.get_n<double>(m);
    out.wc = oa.get_n<double>(nc);
    out.mem2 = op.get_n<int>(2 * (size_t)nc);
    NOMEM(out.agg && out.p && out.wc && out.mem2);
    launch_aggfill(s, m, mate, ofs, w, out.agg, out.p, out.wc, out.mem2);
    // Galerkin product: count, scan to row pointers, fill.  Every coarse entry
    // (E, F) comes from at least one stored a_ij (i in E, j in F), so A's entry
    // count bounds the coarse one; the exact count and the longest coarse row
    // stay on the device (row_ptr[nc], row_ptr[nc + 1]) until the next
    // read-back.  A coarse row's candidates are its members' entries: more
    // than lmin of them only when A has rows longer than lmin / 2.
    const int lmin_g = long_min(G);
    const bool gal_long = 2LL * A.dmax > lmin_g;
    int *crp = oa.get_n<int>((size_t)nc + 2);
    int *gF = tmp.get_n<int>(A.nnz);
    int *gU = tmp.get_n<int>(A.nnz);
    void *stmp2 = tmp.get(scan_tmp_bytes(nc));
    NOMEM(crp && gF && gU && stmp2);
    const bool gsorted = A.nnz >= (long long)kSortedCandidatesAvg * A.n;
    SegList sg;
    unsigned long long *gkeys = nullptr;
    int *gcc = nullptr;  // column starts per chunk of the long coarse rows' sorted keys
    const int pg = sp ? sp->begin(BCM_PROF_SETUP_GALERKIN, false) : -1;
    if (gal_long) {
        Carver cv;
        Carver probe;
        probe.left = ~size_t(0);
        carve_seg(probe, seg_cap(A.nnz, lmin_g), sg);
        cv.cur = static_cast<char *>(tmp.get(probe.used));
        cv.left = probe.used;
        gcc = tmp.get_n<int>((size_t)(A.nnz / kSegChunk) + seg_cap(A.nnz, lmin_g) + 1);
        NOMEM(cv.cur && keys() && gcc);
        carve_seg(cv, seg_cap(A.nnz, lmin_g), sg);
        launch_fill_i32(s, 8, sg.ctl, 0);
        launch_find_long_gal(s, nc, out.mem2, A.rp, lmin_g, sg);
        launch_seg_fix(s, sg);
        launch_gal_long_sort(s, sg, (int)std::min(2LL * A.dmax, (long long)A.nnz), A.rp, A.ci, out.agg, out.mem2, k0,
                             k1, &gkeys);
    }
    launch_gal_count(s, G, nc, A.rp, A.ci, out.agg, out.mem2, crp, gF, gU, gsorted, gal_long ? lmin_g : 0);
    if (gal_long)
        launch_gal_long(s, 0, sg, gkeys, A.rp, A.ci, A.v, out.agg, out.p, out.mem2, crp, gcc, nullptr, nullptr,
                        nullptr);
    scan_exclusive(s, crp, crp, nc, crp + nc, stmp2, crp + nc + 1);
    out.Ac.n = nc;
    out.Ac.nnz = A.nnz;
    out.Ac.nnz_dev = crp + nc;
    out.Ac.dmax = (int)std::min<long long>(2LL * A.dmax, nc);
    out.Ac.rp = crp;
    out.Ac.ci = oa.get_n<int>(A.nnz);
    out.Ac.v = oa.get_n<double>(A.nnz);
    NOMEM(out.Ac.ci && out.Ac.v);
    launch_gal_fill(s, G, nc, A.rp, A.ci, A.v, out.agg, out.p, out.mem2, crp, out.Ac.ci, out.Ac.v, gF, gU, gsorted,
                    gal_long ? lmin_g : 0);
    if (gal_long)
        launch_gal_long(s, 1, sg, gkeys, A.rp, A.ci, A.v, out.agg, out.p, out.mem2, nullptr, gcc, crp, out.Ac.ci,
                        out.Ac.v);
    // (the coarse entry count is still on the device: A's bounds it; the bytes
    // are corrected with the exact count in build_hierarchy's summary)
    if (sp) sp->end(pg, false, bytes_setup_galerkin(m, A.nnz, nc, A.nnz));
    out.prof_gal = pg;
    HIPCHK(hipGetLastError());
    return BCM_OK;
}

template <typename T>
T *persist_copy(bcm_handle *h, const T *src, size_t n) {
    T *d = h->persist.get_n<T>(n);
    if (d && n && hipMemcpyAsync(d, src, n * sizeof(T), hipMemcpyDeviceToDevice, h->s) != hipSuccess) d = nullptr;
    return d;
}

// group = -1: every level whose cycle legs run CSR row kernels (levels of the
// tail kernel and levels running entirely on the sliced-ELL copy excluded)
// gets the lane width whose down + up legs ran fastest, over three timed
// repetitions per width on zero vectors.
int autotune_lanes(bcm_handle *h) {
    hipStream_t s = h->s;
    const int fp32 = h->prm.precision == BCM_FP32_CYCLE;
    const size_t es = fp32 ? sizeof(float) : sizeof(double);
    hipEvent_t ev[2];
    HIPCHK(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        set_error("hipEventCreate failed");
        return BCM_EHIP;
    }
    launch_fill_i32(s, 2 * (size_t)h->lv[0].A.n, (int *)h->r, 0);
    const int last = h->kt > 0 ? h->kt : h->nl - 1;
    hipError_t err = hipSuccess;
    for (int l = 0; l < last && err == hipSuccess; ++l) {
        Level &L = h->lv[l];
        Level &C = h->lv[l + 1];
        if (down_on_sell(L) && L.xp) continue;
        if (l > 0) launch_fill_i32(s, es * L.A.n / 4, (int *)L.b, 0);
        launch_fill_i32(s, es * C.A.n / 4, (int *)C.x, 0);
        const void *b = l == 0 ? (const void *)h->r : L.b;
        void *x = l == 0 ? (void *)h->w : L.x;
        const int io = (l == 0 || !fp32) ? 1 : 0;
        float best = 0.f;
        int best_g = L.G;
        for (int g = 4; g <= 64 && err == hipSuccess; g *= 2) {
            L.G = g;
            for (int t = 0; t < 4; ++t) {
                if (t == 1) (void)hipEventRecord(ev[0], s);
                launch_down(s, L, fp32, b, C.b, io, nullptr);
                launch_up(s, L, fp32, b, C.x, x, io, io, nullptr);
            }
            (void)hipEventRecord(ev[1], s);
            err = hipEventSynchronize(ev[1]);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (err == hipSuccess && (g == 4 || ms < best)) { best = ms; best_g = g; }
        }
        L.G = best_g;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (err != hipSuccess) {
        set_error(std::string("lane-width timing failed: ") + hipGetErrorString(err));
        return BCM_EHIP;
    }
    return BCM_OK;
}

int build_hierarchy(bcm_handle *h, const bcm_csr *Ain, const double *win) {
    hipStream_t s = h->s;
    const bcm_params &P = h->prm;
    const int n = Ain->n, nnz = Ain->nnz;
    const bool fp32 = P.precision == BCM_FP32_CYCLE;
    // device memory: persistent hierarchy, level-lifetime and sweep-lifetime scratch
    const double z = nnz, nn = n;
    h->persist.reserve((size_t)(1.5 * (16.0 * z + 48.0 * nn) + 64.0 * nn + 1.3 * 24.0 * z) + (size_t(4) << 20));
    Arena keep, tmp;
    keep.alloc = tmp.alloc = P.alloc;
    keep.dealloc = tmp.dealloc = P.dealloc;
    keep.ctx = tmp.ctx = P.alloc_ctx;
    keep.reserve((size_t)(16.0 * z + 96.0 * nn) + (size_t(1) << 20));
    tmp.reserve((size_t)(32.0 * z + 56.0 * nn) + (size_t(1) << 20));
    struct Guard {
        Arena &a, &b;
        hipStream_t s;
        ~Guard() { (void)hipStreamSynchronize(s); a.release(); b.release(); }
    } guard{keep, tmp, s};
    if (h->persist.failed || keep.failed || tmp.failed) { set_error("device allocation failed"); return BCM_ENOMEM; }

    Level &L0 = h->lv[0];
    L0.A.n = n;
    L0.A.nnz = nnz;
    L0.A.rp = persist_copy(h, Ain->row_ptr, (size_t)n + 1);
    L0.A.ci = persist_copy(h, Ain->col, (size_t)nnz);
    L0.A.v = persist_copy(h, Ain->val, (size_t)nnz);
    L0.w = persist_copy(h, win, (size_t)n);
    NOMEM(L0.A.rp && L0.A.ci && L0.A.v && L0.w);
    {
        // full validation of the input, symmetry included when asked.  The
        // diagonal goes to the finest level's smoother array, which holds it
        // for the first matching sweep until the smoother overwrites it.  The
        // longest row comes back with the flags: it decides the long-row paths.
        // (flags: [0] errors, [1] longest row, [8..15] the long-row list's control)
        L0.dinv = h->persist.get_n<double>(n);
        double *diag = L0.dinv;
        int *flags = tmp.get_n<int>(16);
        const int G0 = lanes_for(P.group, L0.A), lmin0 = long_min(G0);
        SegList sg;
        Carver probe;
        probe.left = ~size_t(0);
        carve_seg(probe, seg_cap(nnz, lmin0), sg);
        Carver cv;
        cv.cur = static_cast<char *>(tmp.get(probe.used));
        cv.left = probe.used;
        NOMEM(diag && flags && cv.cur);
        carve_seg(cv, seg_cap(nnz, lmin0), sg);
        launch_fill_i32(s, 2, flags, 0);
        launch_fill_i32(s, 8, sg.ctl, 0);
        launch_validate(s, G0, n, nnz, L0.A.rp, L0.A.ci, L0.A.v, L0.w, P.check ? 1 : 0, diag, flags, sg, lmin0,
                        flags + 1);
        launch_seg_fix(s, sg);
        launch_long_validate(s, n, nnz, L0.A.rp, L0.A.ci, L0.A.v, P.check ? 1 : 0, sg, flags);
        HIPCHK(hipMemcpyAsync(flags + 8, sg.ctl, 8 * sizeof(int), hipMemcpyDeviceToDevice, s));
        int f[16];
        int rc = read_back(s, flags, sizeof(f), f);
        if (rc) return rc;
        if (f[0]) { set_error("invalid input:" + flag_text(f[0])); return BCM_EINVAL; }
        L0.A.dmax = f[1];
    }
    const int max_coarse = P.max_coarse > 0 ? P.max_coarse : (int)std::lround(40.0 * std::cbrt((double)n));
    // Section 5 stops at max_coarse, max_levels or an unchanged size; min_ratio
    // > 1 adds the stalled-coarsening rule (not the paper's)
    const double rmin = P.min_ratio > 1.0 ? P.min_ratio : 1.0;
    int k = 0;
    int g_prev = lanes_for(P.group, L0.A);
    SetupProf sp;
    sp.s = s;
    sp.mask = P.profile;
    // the Galerkin bracket whose coarse entry count is still pending
    struct {
        int idx = -1;
        double m = 0, z = 0, nc = 0;
    } pend;
    for (;;) {
        Level &L = h->lv[k];
        const int nk = L.A.n;
        if (nk <= max_coarse || k + 1 >= P.max_levels || k + 1 >= kMaxLevels) break;
        keep.rewind();
        Csr Acur = L.A;
        const double *wcur = L.w;
        int g_hint = g_prev;
        bool have = false;
        int *cagg = nullptr, *cmem = nullptr;
        double *cp = nullptr;
        int cstride = 1;
        bool final_done = false;  // the last sweep ran: its outputs already live in persist
        for (int sw = 0; sw < P.sweeps; ++sw) {
            tmp.rewind();
            SweepOut so;
            const bool last = sw == P.sweeps - 1;
            double swb = 0.0;
            int rc = pairwise_sweep(s, tmp, keep, Acur, wcur, P.group, g_hint, so, last ? &h->persist : nullptr,
                                    last && !have ? &h->persist : nullptr, k == 0 && sw == 0 ? L0.dinv : nullptr,
                                    &sp, &swb);
            if (rc) return rc;
            h->setup_bytes += swb;
            h->sweeps_run += 1;
            // this sweep's matrix came from the previous sweep's Galerkin product: its size is known now
            if (pend.idx >= 0) {
                sp.set_bytes(pend.idx, bytes_setup_galerkin(pend.m, pend.z, pend.nc, Acur.nnz));
                pend.idx = -1;
            }
            if (so.nc != Acur.n) {
                pend.idx = so.prof_gal;
                pend.m = Acur.n;
                pend.z = Acur.nnz;
                pend.nc = so.nc;
            }
            if (sw == 0 && L.A.nnz_dev) {  // the level's own entry count is known now
                L.A.nnz = Acur.nnz;
                L.A.dmax = Acur.dmax;
                L.A.nnz_dev = nullptr;
            }
            g_hint = g_prev = lanes_for(P.group, Acur);
            if (so.nc == Acur.n) break;  // no pair formed: further sweeps would not either
            if (!have) {
                cagg = so.agg; cp = so.p; cmem = so.mem2; cstride = 2;
            } else {
                Arena &ca = last ? h->persist : keep;
                int *nagg = ca.get_n<int>(nk);
                double *np_ = ca.get_n<double>(nk);
                int *nmem = ca.get_n<int>((size_t)so.nc * 2 * cstride);
                NOMEM(nagg && np_ && nmem);
                launch_compose(s, nk, so.nc, cagg, cp, cmem, cstride, so.agg, so.p, so.mem2, nagg, np_, nmem);
                cagg = nagg; cp = np_; cmem = nmem; cstride *= 2;
            }
            Acur = so.Ac;
            wcur = so.wc;
            have = true;
            final_done = last;
        }
        if (!have) break;  // stagnation: level k is the coarsest
        Level &C = h->lv[k + 1];
        C.A.n = Acur.n;
        C.A.nnz = Acur.nnz;
        C.A.dmax = Acur.dmax;
        L.nc = Acur.n;
        L.mstride = cstride;
        if (final_done) {
            C.A.rp = Acur.rp; C.A.ci = Acur.ci; C.A.v = Acur.v; C.w = const_cast<double *>(wcur);
            C.A.nnz_dev = Acur.nnz_dev;
            L.agg = cagg; L.p = cp; L.mem = cmem;
        } else {  // a later sweep formed no pair: the outputs are still in level scratch
            C.A.rp = persist_copy(h, Acur.rp, (size_t)Acur.n + 1);
            C.A.ci = persist_copy(h, Acur.ci, (size_t)Acur.nnz);
            C.A.v = persist_copy(h, Acur.v, (size_t)Acur.nnz);
            C.w = persist_copy(h, wcur, (size_t)Acur.n);
            L.agg = persist_copy(h, cagg, (size_t)nk);
            L.p = persist_copy(h, cp, (size_t)nk);
            L.mem = persist_copy(h, cmem, (size_t)Acur.n * cstride);
        }
        NOMEM(C.A.rp && C.A.ci && C.A.v && C.w && L.agg && L.p && L.mem);
        // keep/tmp are rewound next: their memory is reused by later work on the
        // same stream, which runs after everything that reads it now
        ++k;
        if (rmin > 1.0 && (double)nk < rmin * (double)C.A.n) break;  // stalled coarsening: C is the coarsest
    }
    h->nl = k + 1;
    {
        Csr &Ac = h->lv[h->nl - 1].A;  // the coarsest level ran no sweep: its entry count is still pending
        if (Ac.nnz_dev) {
            int two[2];
            int rc = read_back(s, Ac.nnz_dev, sizeof(two), two);
            if (rc) return rc;
            Ac.nnz = two[0];
            Ac.dmax = two[1];
            Ac.nnz_dev = nullptr;
        }
        if (pend.idx >= 0) sp.set_bytes(pend.idx, bytes_setup_galerkin(pend.m, pend.z, pend.nc, Ac.nnz));
    }
    {
        // rows longer than long_min(G) of every level (G of the rule): their
        // lists for the row kernels, found on the levels whose longest row
        // exceeds that bound; their counts come back in one read-back
        std::vector<int> lv_long;
        std::vector<SegList> segs;
        for (int l = 0; l < h->nl; ++l) {
            Level &L = h->lv[l];
            L.G = lanes_for(P.group, L.A);
            const int lmin = long_min(L.G);
            if (L.A.dmax <= lmin) continue;
            SegList sg;
            Carver probe;
            probe.left = ~size_t(0);
            carve_seg(probe, seg_cap(L.A.nnz, lmin), sg);
            Carver cv;
            cv.cur = static_cast<char *>(h->persist.get(probe.used));
            cv.left = probe.used;
            int *idx = h->persist.get_n<int>(L.A.n);
            NOMEM(cv.cur && idx);
            carve_seg(cv, seg_cap(L.A.nnz, lmin), sg);
            // arrival counters of the single-launch cycle legs (zero between launches)
            int *cnt = h->persist.get_n<int>((size_t)sg.cap);
            NOMEM(cnt);
            launch_fill_i32(s, (size_t)sg.cap, cnt, 0);
            launch_fill_i32(s, 8, sg.ctl, 0);
            launch_find_long(s, L.A.n, L.A.rp, lmin, sg, idx);
            launch_seg_fix(s, sg);
            L.lr.lmin = lmin;
            L.lr.idx = idx;
            L.lr.rows = sg.row;
            L.lr.cb = sg.cb;
            L.lr.cnt = cnt;
            lv_long.push_back(l);
            segs.push_back(sg);
        }
        if (!lv_long.empty()) {
            int *cnts = tmp.get_n<int>(8 * lv_long.size());
            NOMEM(cnts);
            for (size_t t = 0; t < lv_long.size(); ++t)
                HIPCHK(hipMemcpyAsync(cnts + 8 * t, segs[t].ctl, 8 * sizeof(int), hipMemcpyDeviceToDevice, s));
            std::vector<int> hc(8 * lv_long.size());
            int rc = read_back(s, cnts, hc.size() * sizeof(int), hc.data());
            if (rc) return rc;
            int maxch = 1;
            for (size_t t = 0; t < lv_long.size(); ++t) {
                Level &L = h->lv[lv_long[t]];
                L.lr.n = hc[8 * t];
                L.lr.nchunks = hc[8 * t + 2];
                maxch = std::max(maxch, L.lr.nchunks);
                if (L.lr.n == 0) L.lr = LongRows();  // the bound was not reached after all
            }
            h->lpart = h->persist.get_n<double>(maxch);
            NOMEM(h->lpart);
            for (int l : lv_long)
                if (h->lv[l].lr.n > 0) h->lv[l].lr.part = h->lpart;
        }
    }
    // smoother, FP32 copies, cycle vectors
    for (int l = 0; l < h->nl; ++l) {
        Level &L = h->lv[l];
        const int nl_ = L.A.n;
        if (!L.dinv) L.dinv = h->persist.get_n<double>(nl_);  // (the finest level's was allocated first)
        NOMEM(L.dinv);
        if (fp32) {
            L.dinv32 = h->persist.get_n<float>(nl_);
            L.A.v32 = h->persist.get_n<float>(L.A.nnz);
            NOMEM(L.dinv32 && L.A.v32);
            if (l < h->nl - 1) {
                L.p32 = h->persist.get_n<float>(nl_);
                NOMEM(L.p32);
                launch_cast(s, nl_, L.p, L.p32);
            }
        }
        launch_long_abs(s, L.lr, L.A.rp, L.A.v, h->lpart, L.A.v32);
        launch_diag_l1(s, L.G, nl_, L.A.rp, L.A.v, L.dinv, L.dinv32, L.A.v32, L.lr, h->lpart);
        if (l < h->nl - 1 && split_legs(nl_, L.A.nnz)) {
            L.xp = h->persist.get((fp32 ? sizeof(float) : sizeof(double)) * nl_);
            NOMEM(L.xp);
            if (L.A.nnz >= (long long)kGatherRow * nl_) {
                L.yb = h->persist.get((fp32 ? sizeof(float) : sizeof(double)) * nl_);
                NOMEM(L.yb);
            }
        }
        if (l > 0) {
            const size_t es = fp32 ? sizeof(float) : sizeof(double);
            L.b = h->persist.get(es * nl_);
            L.x = h->persist.get(es * nl_);
            NOMEM(L.b && L.x);
            if (P.cycle != BCM_VCYCLE) {
                L.xs = h->persist.get(es * nl_);
                NOMEM(L.xs);
            }
            if (P.cycle == BCM_KCYCLE && (P.kcycle_levels == 0 || l - 1 < P.kcycle_levels)) {
                L.kv = h->persist.get(es * nl_);
                NOMEM(L.kv);
            }
        }
    }
    {
        // sliced ELL copies: the finest level (flexible CG products) and every
        // level that runs the split up leg
        std::vector<int> lv_sell;
        for (int l = 0; l < h->nl && P.sell; ++l)
            if ((l == 0 || h->lv[l].xp) && h->lv[l].lr.n == 0) lv_sell.push_back(l);
        // per level t: tot[t] = total slots, tot[32 + t] = largest |col - row|,
        // tot[64 + t] = 1 if some value is not exactly a float32, tot[96 + t] =
        // slots of the slices without uniform column offsets
        if (lv_sell.size() > 32) lv_sell.resize(32);  // deeper levels keep the CSR kernels
        int *tot = h->persist.get_n<int>(128);
        NOMEM(tot);
        launch_fill_i32(s, 128, tot, 0);
        std::vector<int *> uni(lv_sell.size());
        for (size_t t = 0; t < lv_sell.size(); ++t) {
            Level &L = h->lv[lv_sell[t]];
            const int ns = (L.A.n + kSlice - 1) / kSlice;
            L.E.nslices = ns;
            L.E.sp = h->persist.get_n<int>((size_t)ns + 1);
            uni[t] = h->persist.get_n<int>(ns);
            void *stmp = keep.get(scan_tmp_bytes(ns));
            NOMEM(L.E.sp && uni[t] && stmp);
            launch_sell_width(s, L.A.n, L.A.rp, L.A.ci, L.A.v, L.E.sp, uni[t], tot + 32 + t, tot + 64 + t,
                              tot + 96 + t);
            scan_exclusive(s, L.E.sp, L.E.sp, ns, L.E.sp + ns, stmp);  // sp[ns] = total slots
            HIPCHK(hipMemcpyAsync(tot + t, L.E.sp + ns, sizeof(int), hipMemcpyDeviceToDevice, s));
        }
        int tots[128];
        int rc = read_back(s, tot, sizeof(tots), tots);
        if (rc) return rc;
        for (size_t t = 0; t < lv_sell.size(); ++t) {
            Level &L = h->lv[lv_sell[t]];
            const size_t ne = (size_t)tots[t];
            if (tots[32 + t] <= 32767) {
                L.E.sd = h->persist.get_n<short>(ne);
                L.E.su = h->persist.get_n<int>(ne / kSlice);
                L.E.uni = uni[t];
                NOMEM(L.E.sd && L.E.su);
                L.E.mixed = ne ? (double)tots[96 + t] / (double)ne : 1.0;
            } else {
                L.E.sc = h->persist.get_n<int>(ne);
                // int32 columns: no uniform slices (the kernels read the flags regardless)
                L.E.uni = uni[t];
                launch_fill_i32(s, (size_t)L.E.nslices, uni[t], 0);
            }
            L.E.wide = ne > (size_t)kWideSlots * kSlice * (size_t)L.E.nslices;
            const bool exact32 = tots[64 + t] == 0;
            if (!exact32) L.E.sv = h->persist.get_n<double>(ne);
            if (fp32 || exact32) L.E.sv32 = h->persist.get_n<float>(ne);
            NOMEM((L.E.sc || L.E.sd) && (L.E.sv || L.E.sv32));
            launch_sell_fill(s, L.A.n, L.A.rp, L.A.ci, L.A.v, L.E.sp, uni[t], L.E.su, L.E.sc, L.E.sd, L.E.sv,
                             L.E.sv32);
            // FP32 cycle, levels whose down leg is the sliced-ELL residual with
            // one thread per row: the values of A D for it (the long-row levels
            // gather dinv o b instead, the slot-split ones keep dinv and b).
            // Below 2^19 rows the residual runs near its latency either way
            // (250k rows: 4.6 against 4.7 us a launch, less over a solve than
            // the scaling costs the setup), so only larger levels take it.
            if (fp32 && down_on_sell(L) && !L.yb && !slot_split_level(L) && (lv_sell[t] == 0 || L.A.n >= (1 << 19))) {
                L.E.svd = h->persist.get_n<float>(ne);
                NOMEM(L.E.svd);
                launch_sell_scale_cols(s, L.A.n, L.E.nslices, L.E.sp, L.E.uni, L.E.su, L.E.sc, L.E.sd, L.E.sv32,
                                       L.dinv32, L.E.svd);
            }
        }
        // the values one solve iteration reads: both legs of every sliced-ELL
        // level in the cycle's type, and the finest level's product
        long long vb = 0;
        for (size_t t = 0; t < lv_sell.size(); ++t) {
            const Level &L = h->lv[lv_sell[t]];
            const long long ne = tots[t];
            vb += 2 * ne * (fp32 || !L.E.sv ? 4 : 8);
            if (lv_sell[t] == 0) vb += ne * (L.E.sv ? 8 : 4);
        }
        for (size_t t = 0; t < lv_sell.size(); ++t) h->lv[lv_sell[t]].E.stream = vb > kStreamSolve;
    }
    {
        // coarsest level: precompute the sweep operator when it is small
        Level &C = h->lv[h->nl - 1];
        if (C.A.n <= kCoarseDense) {
            const size_t nn2 = (size_t)C.A.n * C.A.n;
            C.S = h->persist.get_n<double>(nn2);
            NOMEM(C.S);
            if (C.A.n <= kCoarseBuildSweeps && C.lr.n == 0) {
                // one workgroup per unit vector runs the sweeps
                launch_coarse_build(s, C, P.coarse_sweeps, C.S);
            } else {
                // S_{t+1} = D + (I - DA) S_t from S_0 = 0 on the whole matrix at once
                tmp.rewind();
                double *W = tmp.get_n<double>(nn2);
                NOMEM(W);
                double *cur = (P.coarse_sweeps % 2) ? W : C.S, *nxt = (P.coarse_sweeps % 2) ? C.S : W;
                launch_fill_i32(s, 2 * nn2, (int *)cur, 0);
                for (int t = 0; t < P.coarse_sweeps; ++t) {
                    launch_fold_left(s, C, cur, nxt);
                    std::swap(cur, nxt);
                }
            }
        }
    }
    if (P.fold && h->nl >= 3 && h->lv[h->nl - 1].S) {
        // The cycle from the first level k >= 1 with at most kFoldRows rows down to
        // the coarsest, formed once as one dense operator (built upwards from the
        // coarsest level's sweep operator): V- and W-cycles, and K-cycles whose
        // Krylov coarse solves all sit above that level.
        int kf = h->nl - 1;
        while (kf > 1 && h->lv[kf - 1].A.n <= kFoldRows) --kf;
        const bool wcyc = P.cycle == BCM_WCYCLE;
        const bool linear = P.cycle != BCM_KCYCLE || (P.kcycle_levels > 0 && P.kcycle_levels <= kf);
        if (kf < h->nl - 1 && linear) {
            tmp.rewind();
            const double *Tc = h->lv[h->nl - 1].S;
            for (int k = h->nl - 2; k >= kf; --k) {
                const Level &L = h->lv[k], &C = h->lv[k + 1];
                const size_t nn2 = (size_t)L.A.n * L.A.n, nc2 = (size_t)C.A.n * C.A.n;
                if (wcyc) {  // the coarse problem solved by two cycles of level k + 1
                    double *M = tmp.get_n<double>(nc2), *W = tmp.get_n<double>(nc2);
                    NOMEM(M && W);
                    launch_fold_w(s, C, Tc, M, W);
                    Tc = W;
                }
                double *T = k == kf ? h->persist.get_n<double>(nn2) : tmp.get_n<double>(nn2);
                double *H = tmp.get_n<double>(nn2);
                NOMEM(T && H);
                launch_fold_level(s, L, Tc, C.A.n, H, T);
                Tc = T;
            }
            h->kf = kf;
            h->fold = const_cast<double *>(Tc);
        }
    }
    if (h->kf == 0) {
        // tail kernel: the smallest levels (and the coarsest solve) in one workgroup
        // (levels with long rows stay out of it: it gives a row at most 16 lanes)
        int kt = h->nl - 1;
        while (kt > 1 && h->lv[kt - 1].A.n <= kTailRows && h->lv[kt - 1].lr.n == 0) --kt;
        const Level &C = h->lv[h->nl - 1];
        // K levels need dot products between cycles: the tail takes V and W levels only
        const bool plain = P.cycle != BCM_KCYCLE || (P.kcycle_levels > 0 && P.kcycle_levels <= kt);
        if (plain && kt < h->nl - 1 && C.A.n <= kTailRows && C.lr.n == 0) {
            std::vector<TailLevel> tv(h->nl);
            for (int l = 0; l < h->nl; ++l) {
                const Level &L = h->lv[l];
                TailLevel t{};
                t.n = L.A.n; t.nc = L.nc; t.mstride = L.mstride;
                t.rp = L.A.rp; t.ci = L.A.ci; t.agg = L.agg; t.mem = L.mem;
                t.a = fp32 ? (const void *)L.A.v32 : (const void *)L.A.v;
                t.dinv = fp32 ? (const void *)L.dinv32 : (const void *)L.dinv;
                t.p = fp32 ? (const void *)L.p32 : (const void *)L.p;
                t.b = L.b; t.x = L.x; t.xs = L.xs;
                tv[l] = t;
            }
            // the tail's program: the cycle of level kt (Algorithm 1; W-cycle: the
            // coarse problem of every level solved by two cycles, the second on the
            // coarse residual and written to the save buffer, then added)
            std::vector<int> ops;
            const int nl_ = h->nl;
            const bool w = P.cycle == BCM_WCYCLE;
            auto op = [&](int o, int k, int sel) { ops.push_back(o | (k << 8) | (sel << 16)); };
            std::function<void(int, int)> cyc = [&](int k, int sel) {
                if (k == nl_ - 1) { op(kTailCoarse, k, sel); return; }
                op(kTailDown, k, 0);
                cyc(k + 1, 0);
                if (w) {
                    op(kTailResid, k + 1, 0);
                    cyc(k + 1, 1);
                    op(kTailAdd, k + 1, 0);
                }
                op(kTailUp, k, sel);
            };
            cyc(kt, 0);
            h->tail = h->persist.get_n<TailLevel>(h->nl);
            h->tail_ops = h->persist.get_n<int>(ops.size());
            NOMEM(h->tail && h->tail_ops);
            HIPCHK(hipMemcpyAsync(h->tail, tv.data(), sizeof(TailLevel) * h->nl, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(h->tail_ops, ops.data(), sizeof(int) * ops.size(), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            h->n_tail_ops = (int)ops.size();
            h->kt = kt;
        }
    }
    if (!h->lv[h->nl - 1].S &&
        !coarse_in_lds(h->lv[h->nl - 1].A.n, h->lv[h->nl - 1].A.nnz, h->lv[h->nl - 1].lr.n > 0)) {
        h->ctmp[0] = h->persist.get_n<double>(h->lv[h->nl - 1].A.n);
        h->ctmp[1] = h->persist.get_n<double>(h->lv[h->nl - 1].A.n);
        NOMEM(h->ctmp[0] && h->ctmp[1]);
        if (P.coarse_sweeps >= 1 && P.coarse_sweeps <= kStarMaxSweeps && h->lv[h->nl - 1].lr.n == 1) {
            const int rc = build_star(h, s, h->lv[h->nl - 1], P.coarse_sweeps);
            if (rc) return rc;
        }
    }
    // flexible CG state
    h->r = h->persist.get_n<double>(n);
    h->w = h->persist.get_n<double>(n);
    h->d = h->persist.get_n<double>(n);
    h->v = h->persist.get_n<double>(n);
    h->q = h->persist.get_n<double>(n);
    h->u = h->persist.get_n<double>(n);
    h->scal = h->persist.get_n<double>(16);
    h->red_blocks = reduce_blocks(n);
    h->partials = h->persist.get_n<double>(4 * (size_t)h->red_blocks);
    NOMEM(h->r && h->w && h->d && h->v && h->q && h->u && h->scal && h->partials);
    {
        const Level &F = h->lv[0];
        // levels whose down leg gathers dinv o b (long rows) get it from the
        // update instead of a launch of its own; on the others the extra
        // stream through the update costs as much as the second gather saves
        if (h->nl > 1 && F.yb && down_on_sell(F)) {
            h->y0 = h->persist.get((P.precision == BCM_FP32_CYCLE ? sizeof(float) : sizeof(double)) * (size_t)n);
            NOMEM(h->y0);
        }
    }
    {
        // the product's partials: one per slice where it takes one workgroup per slice
        const int nbs = spmv_dots_grid(h->lv[0], h->red_blocks);
        // a buffer of its own: the update reads these partials while its
        // workgroups write their own into h->partials
        h->spart = h->persist.get_n<double>(3 * (size_t)nbs);
        NOMEM(h->spart);
    }
    if (P.cycle == BCM_KCYCLE) {
        h->kpart = h->persist.get_n<double>(3 * (size_t)kKPartBlocks);
        h->ks = h->persist.get_n<double>(8 * (size_t)h->nl);
        NOMEM(h->kpart && h->ks);
    }
    launch_fill_i32(s, 32, (int *)h->scal, 0);
    launch_fill_i32(s, 2 * (size_t)n, (int *)h->q, 0);
    launch_fill_i32(s, 2 * (size_t)n, (int *)h->d, 0);
    HIPCHK(hipGetLastError());
    if (P.group == -1) {
        const int rc = autotune_lanes(h);
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int c = 6; c < 9; ++c) h->prof[c] = ProfClass{};
    sp.collect(h->prof);
    return BCM_OK;
}

// Level k solves its coarse problem with the K-cycle's two flexible-CG iterations.
bool kcycle_at(const bcm_handle *h, int k) {
    return h->prm.cycle == BCM_KCYCLE && (h->prm.kcycle_levels == 0 || k < h->prm.kcycle_levels);
}

// --------------------------------------------------------------- byte model
// Algorithmic bytes (every array touched once; gathers assumed cached).
// down leg: fused k_down_*, or residual + restriction on large levels (p r written and read once)
// Bytes of one column index of the matrix a row-parallel kernel reads: int16
// offsets on a sliced-ELL copy that has them (none in its uniform slices, which
// hold one offset per slot column), else int32.
double index_bytes(const Level &L, bool sell_path) { return sell_path && L.E.sd ? 2.0 * L.E.mixed : 4.0; }
// Bytes of one matrix value: float32 arithmetic, or a float64 kernel on a
// sliced-ELL copy whose values are all exact float32, reads 4.
double value_bytes(const Level &L, bool sell_path, bool f32) {
    return f32 || (sell_path && !L.E.sv && L.E.sv32) ? 4.0 : 8.0;
}

// levels 0 .. cycle_levels(h) - 1 run their own down and up legs in the
// V-cycle; the rest are the folded operator, the tail kernel or the coarsest solve
int cycle_levels(const bcm_handle *h) { return h->kf > 0 ? h->kf : (h->kt > 0 ? h->kt : h->nl - 1); }
// level k (>= 1) of the V-cycle gets its dinv o b from level k - 1's restriction
bool y_by_restrict(const bcm_handle *h, int k) {
    return h->prm.cycle == BCM_VCYCLE && k >= 1 && k < cycle_levels(h) && h->lv[k].yb && down_on_sell(h->lv[k]) &&
           down_on_sell(h->lv[k - 1]);
}

double bytes_down(const bcm_handle *h, int k) {
    const Level &L = h->lv[k];
    const bool f32 = h->prm.precision == BCM_FP32_CYCLE;
    const double sv = f32 ? 4 : 8, sb = (k == 0 || !f32) ? 8 : 4;
    const double n = L.A.n, z = L.A.nnz, nc = L.nc;
    const bool sell = down_on_sell(L);
    const double base = 4 * (n + 1) + (index_bytes(L, sell) + value_bytes(L, sell, f32)) * z + sb * n + 2 * sv * n +
                        4.0 * nc * L.mstride + sv * nc;
    // split leg: p r written and read; with yb, dinv o b formed first (b, dinv read, y written),
    // except where the flexible-CG update (finest level, y0) or the finer
    // level's restriction forms it; the restriction forming the coarser
    // level's reads its dinv and writes its y
    const bool scale = L.yb && !(k == 0 && h->y0) && !y_by_restrict(h, k);
    const double cy = y_by_restrict(h, k + 1) ? 2 * sv * nc : 0.0;
    const double ad = L.E.svd ? sv * n : 0.0;  // values of A D: dinv not read
    return sell ? base + 2 * sv * n + (scale ? (sb + 2 * sv) * n : 0.0) + cy - ad : base;
}
// up leg: fused k_up, or k_prolong + k_smooth on large levels (xp written and read once)
double bytes_up(const bcm_handle *h, int k) {
    const Level &L = h->lv[k];
    const bool f32 = h->prm.precision == BCM_FP32_CYCLE;
    const double sv = f32 ? 4 : 8, sb = (k == 0 || !f32) ? 8 : 4;
    const double n = L.A.n, z = L.A.nnz, nc = L.nc;
    if (L.xp)
        return (sb * n + 2 * sv * n + 4 * n + sv * nc + sv * n) +
               (4 * (n + 1) + (index_bytes(L, L.E.sp != nullptr) + value_bytes(L, L.E.sp != nullptr, f32)) * z +
                2 * sv * n + 2 * sb * n);
    return 4 * (n + 1) + (4 + sv) * z + 2 * sb * n + 2 * sv * n + 4 * n + sv * nc;
}
// the main kernel of a level's leg alone: the residual of a split down leg
// (p r written once), the smoothing of a split up leg; else the fused leg
double bytes_down_main(const bcm_handle *h, int k) {
    const Level &L = h->lv[k];
    const bool f32 = h->prm.precision == BCM_FP32_CYCLE;
    const double sv = f32 ? 4 : 8, sb = (k == 0 || !f32) ? 8 : 4, n = L.A.n, z = L.A.nnz;
    if (!down_on_sell(L)) return bytes_down(h, k);
    // b read; p read and p r written; dinv read unless the values are those of A D
    return 4 * (n + 1) + (index_bytes(L, true) + value_bytes(L, true, f32)) * z + sb * n + (L.E.svd ? 2 : 3) * sv * n;
}
double bytes_up_main(const bcm_handle *h, int k) {
    const Level &L = h->lv[k];
    const bool f32 = h->prm.precision == BCM_FP32_CYCLE;
    const double sv = f32 ? 4 : 8, sb = (k == 0 || !f32) ? 8 : 4, n = L.A.n, z = L.A.nnz;
    if (!L.xp) return bytes_up(h, k);
    return 4 * (n + 1) + (index_bytes(L, L.E.sp != nullptr) + value_bytes(L, L.E.sp != nullptr, f32)) * z +
           2 * sv * n + 2 * sb * n;
}
double bytes_coarse(const bcm_handle *h) {
    const Level &L = h->lv[h->nl - 1];
    const double n = L.A.n, z = L.A.nnz;
    const double sb = (h->nl == 1 || h->prm.precision != BCM_FP32_CYCLE) ? 8 : 4;
    return 4 * (n + 1) + 12 * z + 8 * n + 2 * sb * n;
}
// the folded operator: every entry once, b in and x out
double bytes_fold(const bcm_handle *h) {
    const double n = h->lv[h->kf].A.n;
    const double sb = h->prm.precision == BCM_FP32_CYCLE ? 4 : 8;
    return 8 * n * n + 2 * sb * n;
}
// one preconditioner application: every level's legs times the number of
// times the level is visited (doubling below each W- or K-accelerated level),
// plus the W residual/add and the K-cycle products and combinations
double bytes_cycle(const bcm_handle *h) {
    const double sv = h->prm.precision == BCM_FP32_CYCLE ? 4 : 8;
    double total = 0.0, visits = 1.0;
    const int kend = h->kf > 0 ? h->kf : h->nl - 1;  // levels below kend: the folded operator
    for (int k = 0; k < kend; ++k) {
        total += visits * (bytes_down(h, k) + bytes_up(h, k));
        const Level &C = h->lv[k + 1];
        const double n = C.A.n, spmv = 4 * (n + 1) + (4 + sv) * C.A.nnz;
        if (kcycle_at(h, k)) {
            total += visits * (2 * (spmv + 3 * sv * n) + 6 * sv * n);
            visits *= 2;
        } else if (h->prm.cycle == BCM_WCYCLE) {
            total += visits * (spmv + 6 * sv * n);
            visits *= 2;
        }
    }
    return total + visits * (h->kf > 0 ? bytes_fold(h) : bytes_coarse(h));
}
double bytes_spmv_dots(const bcm_handle *h) {
    const Level &L = h->lv[0];
    const double n = L.A.n, z = L.A.nnz;
    // algorithmic: every stored entry once (ELL padding not counted)
    return 4 * (n + 1) + (index_bytes(L, L.E.sp != nullptr) + value_bytes(L, L.E.sp != nullptr, false)) * z + 32 * n;
}
// ten float64 vector streams; with y0, dinv read and y0 written in the cycle's type
double bytes_update(const bcm_handle *h) {
    const double sv = h->prm.precision == BCM_FP32_CYCLE ? 4 : 8;
    return (80.0 + (h->y0 ? 2 * sv : 0.0)) * h->lv[0].A.n;
}

// Bytes of one bracket of a class launched once per iteration (0..4).
double class_bytes(const bcm_handle *h, int cls) {
    switch (cls) {
    case 0: return bytes_down_main(h, 0);
    case 1: return bytes_up_main(h, 0);
    case 2: return bytes_spmv_dots(h);
    case 3: return bytes_update(h);
    default: {
        if (h->kf > 0) return bytes_fold(h);
        double by = bytes_coarse(h);
        const int kt = h->kt > 0 ? h->kt : h->nl - 1;
        for (int k = kt; k < h->nl - 1; ++k) by += bytes_down(h, k) + bytes_up(h, k);
        return by;
    }
    }
}

// --------------------------------------------------------------- profiling
// Capture of one iteration cut into segments: in capture mode the bracket of
// the profiled class ends the current graph and starts a new one, so that the
// bracket's kernels form a graph of their own, replayed between two event
// records issued on the stream.
struct SegCapture {
    hipStream_t st = nullptr;
    std::vector<hipGraph_t> graphs;
    hipError_t err = hipSuccess;
    void begin() {
        if (err == hipSuccess) err = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    }
    void end() {
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (err == hipSuccess) err = e;
        graphs.push_back(g);
    }
    void cut() {
        end();
        begin();
    }
};

// Event timing of kernel classes: one event pair per bracketed launch, from the
// handle's pool.  In capture mode (cap != NULL) the bracket of class gcls only
// cuts the captured iteration into segments.
struct Prof {
    bcm_handle *h;
    int mask;
    int gcls = -1;
    SegCapture *cap = nullptr;
    // Classes 0-3 are single kernels: their events are taken by that kernel's
    // own dispatch (launch_k), so the time excludes the launch gap.  Other
    // classes, and any class bracketing a graph segment (stream = true), record
    // the events on the stream around the bracket.
    int begin(int cls, bool stream = false) {
        if (cap) {
            if (cls == gcls) cap->cut();
            return -1;
        }
        if (!(mask & (1 << cls))) return -1;
        const int idx = (int)(h->ev_pairs.size() * 2);
        while ((int)h->ev_pool.size() < idx + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            h->ev_pool.push_back(e);
        }
        if (cls <= 3 && !stream) g_kernel_events = KernelEvents{h->ev_pool[idx], h->ev_pool[idx + 1]};
        else (void)hipEventRecord(h->ev_pool[idx], h->s);
        return idx;
    }
    void end(int cls, int idx, double bytes, int iter, bool stream = false) {
        if (cap) {
            if (cls == gcls) cap->cut();
            return;
        }
        if (idx < 0) return;
        if (cls <= 3 && !stream) {
            // no kernel took the events (a bracket without a launch_k): no sample
            if (g_kernel_events.start) { g_kernel_events = KernelEvents{}; return; }
        } else {
            (void)hipEventRecord(h->ev_pool[idx + 1], h->s);
        }
        h->ev_pairs.push_back({cls, idx});
        h->ev_bytes.push_back(bytes);
        h->ev_iter.push_back(iter);
    }
};

int prof_class_index(int bit) {
    int i = 0;
    while (bit > 1) { bit >>= 1; ++i; }
    return i;
}

// Accumulates the event pairs of iterations < iters (launches of a batch after
// the solve ended returned at once and are not counted).
void prof_collect(bcm_handle *h, int iters) {
    for (int c = 0; c < 6; ++c) h->prof[c] = ProfClass{};  // the solve classes (setup ones stay)
    for (size_t t = 0; t < h->ev_pairs.size(); ++t) {
        if (h->ev_iter[t] >= iters) continue;
        const int cls = h->ev_pairs[t].first, idx = h->ev_pairs[t].second;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev_pool[idx], h->ev_pool[idx + 1]) == hipSuccess) {
            h->prof[cls].launches += 1;
            h->prof[cls].ms += ms;
            h->prof[cls].bytes += h->ev_bytes[t];
        }
    }
    h->ev_pairs.clear();
    h->ev_bytes.clear();
    h->ev_iter.clear();
}

// --------------------------------------------------------------- W- and K-cycles
// Recursive cycle of a level k >= 1 (right-hand side in lv[k].b, result in
// lv[k].x), and the solve of the coarse problem of a level k (right-hand side
// lv[k+1].b, result lv[k+1].x): one cycle (V); two cycles, the second on the
// coarse residual and written to the level's save buffer (W); or two
// flexible-CG iterations preconditioned by the coarse cycle (K, on levels
// k < kcycle_levels).
void cycle_level(bcm_handle *h, Prof &pf, int k, const double *done, int iter);

void coarse_solve(bcm_handle *h, Prof &pf, int k, const double *done, int iter) {
    hipStream_t s = h->s;
    const int fp32 = h->prm.precision == BCM_FP32_CYCLE;
    Level &C = h->lv[k + 1];
    cycle_level(h, pf, k + 1, done, iter);
    if (kcycle_at(h, k)) {
        double *ks = h->ks + 8 * k;
        launch_kcycle_step1(s, C, fp32, C.x, C.b, C.kv, h->kpart, ks, done);
        std::swap(C.x, C.xs);
        cycle_level(h, pf, k + 1, done, iter);
        std::swap(C.x, C.xs);
        launch_kcycle_step2(s, C, fp32, C.xs, C.b, C.kv, C.x, h->kpart, ks, done);
    } else if (h->prm.cycle == BCM_WCYCLE) {
        launch_resid_inplace(s, C, fp32, C.x, C.b, done);
        std::swap(C.x, C.xs);
        cycle_level(h, pf, k + 1, done, iter);
        std::swap(C.x, C.xs);
        launch_add(s, C.A.n, fp32, C.xs, C.x, done);
    }
}

void cycle_level(bcm_handle *h, Prof &pf, int k, const double *done, int iter) {
    hipStream_t s = h->s;
    const int fp32 = h->prm.precision == BCM_FP32_CYCLE;
    Level &L = h->lv[k];
    if (k == h->kf) {  // this level and every coarser one as one dense operator
        int e = pf.begin(5);
        launch_dense(s, L.A.n, h->fold, L.b, L.x, !fp32, !fp32, done);
        pf.end(5, e, bytes_fold(h), iter);
        return;
    }
    if (k == h->kt) {  // this level and every coarser one in one workgroup
        int e = pf.begin(5);
        launch_tail(s, fp32, k, h->nl, h->tail, h->lv[h->nl - 1], h->prm.coarse_sweeps, h->tail_ops, h->n_tail_ops,
                    L.x, done);
        pf.end(5, e, 0.0, iter);
        return;
    }
    if (k == h->nl - 1) {
        int e = pf.begin(5);
        launch_coarse(s, L, h->prm.coarse_sweeps, L.b, L.x, !fp32, !fp32, h->ctmp[0], h->ctmp[1], done);
        pf.end(5, e, bytes_coarse(h), iter);
        return;
    }
    Level &C = h->lv[k + 1];
    const int f64io = !fp32;
    launch_down(s, L, fp32, L.b, C.b, f64io, done);
    coarse_solve(h, pf, k, done, iter);
    launch_up(s, L, fp32, L.b, C.x, L.x, f64io, f64io, done);
}

// --------------------------------------------------------------- V-cycle
// One cycle of Algorithm 1 from a zero guess: z = B(r).  done: see launch_down.
// y0: dinv o r of the finest level already formed (the update's h->y0), or null.
// st: the stop test of the flexible-CG update before this cycle, taken by the
// finest level's first kernel (only where cycle_takes_stop(h)); default none.
void vcycle(bcm_handle *h, Prof &pf, const double *rin, double *wout, const double *done, int iter,
            const void *y0 = nullptr, StopTest st = {}) {
    hipStream_t s = h->s;
    const int fp32 = h->prm.precision == BCM_FP32_CYCLE;
    const int nl = h->nl;
    const int cs = h->prm.coarse_sweeps;
    Level &C = h->lv[nl - 1];
    if (nl == 1) {
        int e = pf.begin(4);
        launch_coarse(s, C, cs, rin, wout, 1, 1, h->ctmp[0], h->ctmp[1], done);
        pf.end(4, e, bytes_coarse(h), iter);
        return;
    }
    if (h->prm.cycle != BCM_VCYCLE) {
        // finest level here (f64 in/out), coarse levels recursively
        Level &L = h->lv[0], &N = h->lv[1];
        int e = pf.begin(0);
        launch_down(s, L, fp32, rin, N.b, 1, done, 1, y0, nullptr, st);
        pf.end(0, e, class_bytes(h, 0), iter);
        launch_down(s, L, fp32, rin, N.b, 1, done, 2);
        coarse_solve(h, pf, 0, done, iter);
        launch_up(s, L, fp32, rin, N.x, wout, 1, 1, done, 1);
        e = pf.begin(1);
        launch_up(s, L, fp32, rin, N.x, wout, 1, 1, done, 2);
        pf.end(1, e, class_bytes(h, 1), iter);
        return;
    }
    // levels below kt: the folded operator, the tail kernel, or the coarsest solve
    const int kt = cycle_levels(h);
    for (int k = 0; k < kt; ++k) {
        Level &L = h->lv[k];
        const void *bk = k == 0 ? (const void *)rin : L.b;
        const int io = (k == 0 || !fp32) ? 1 : 0;
        // the restriction forms the coarser level's dinv o b when that level gathers it
        const Level *next = y_by_restrict(h, k + 1) ? &h->lv[k + 1] : nullptr;
        if (k == 0) {  // the finest level's main kernel alone is class 0
            int e = pf.begin(0);
            launch_down(s, L, fp32, bk, h->lv[1].b, io, done, 1, y0, nullptr, st);
            pf.end(0, e, class_bytes(h, 0), iter);
            launch_down(s, L, fp32, bk, h->lv[1].b, io, done, 2, nullptr, next);
        } else {
            int e = pf.begin(5);
            launch_down(s, L, fp32, bk, h->lv[k + 1].b, io, done, 0, y_by_restrict(h, k) ? L.yb : nullptr, next);
            pf.end(5, e, bytes_down(h, k), iter);
        }
    }
    {
        int e = pf.begin(4);
        if (h->kf > 0) {
            launch_dense(s, h->lv[kt].A.n, h->fold, h->lv[kt].b, h->lv[kt].x, !fp32, !fp32, done);
        } else if (h->kt > 0) {
            launch_tail(s, fp32, kt, nl, h->tail, C, cs, h->tail_ops, h->n_tail_ops, h->lv[kt].x, done);
        } else {
            launch_coarse(s, C, cs, C.b, C.x, !fp32, !fp32, h->ctmp[0], h->ctmp[1], done);
        }
        pf.end(4, e, class_bytes(h, 4), iter);
    }
    for (int k = kt - 1; k >= 0; --k) {
        Level &L = h->lv[k];
        const int f64io = (k == 0 || !fp32) ? 1 : 0;
        const void *bk = k == 0 ? (const void *)rin : L.b;
        void *xk = k == 0 ? (void *)wout : L.x;
        if (k == 0) {  // the finest level's main kernel alone is class 1
            launch_up(s, L, fp32, bk, h->lv[1].x, xk, f64io, f64io, done, 1);
            int e = pf.begin(1);
            launch_up(s, L, fp32, bk, h->lv[1].x, xk, f64io, f64io, done, 2);
            pf.end(1, e, class_bytes(h, 1), iter);
        } else {
            int e = pf.begin(5);
            launch_up(s, L, fp32, bk, h->lv[k + 1].x, xk, f64io, f64io, done);
            pf.end(5, e, bytes_up(h, k), iter);
        }
    }
}

// Flexible CG, Algorithm 3 (read with r_{i+1} = r_i - (alpha/rho_i) q_i and
// gamma_i/rho_{i-1} in the d and q updates).  Iterations are launched in
// batches: the finalize kernel counts iterations on the device and raises the
// solve-ended flag when ||r|| <= tol ||b|| or itmax is reached, after which every
// kernel of the batch returns at once.  The host reads the scalars once per
// batch and sizes the next batch from the observed convergence rate, so the
// iteration count is exactly the one a per-iteration test gives.
// Captures one general iteration (cycle, SpMV + dots, updates; first = 0) on
// the handle's vectors into HIP graphs: one graph, or with prof_cls >= 0 (a
// class bracketed once per iteration) three: before the class, the class's
// kernels, after it.  Recaptured when prof_cls changes.
// the finest level's dinv in the cycle's type (read by the update with h->y0)
const void *y0_dinv(const bcm_handle *h) {
    return h->prm.precision == BCM_FP32_CYCLE ? (const void *)h->lv[0].dinv32 : (const void *)h->lv[0].dinv;
}

// The flexible-CG stop test after an update is taken by workgroup 0 of the
// next cycle's first kernel where that is a sliced-ELL residual kernel (it
// hides behind the other workgroups); elsewhere a one-block finalize launch
// after the update takes it.
bool cycle_takes_stop(const bcm_handle *h) { return h->nl > 1 && down_on_sell(h->lv[0]); }

StopTest stop_test_of(const bcm_handle *h) {
    return cycle_takes_stop(h) ? StopTest{h->partials, h->scal, h->red_blocks} : StopTest{};
}

void destroy_iteration_graphs(bcm_handle *h) {
    for (auto &g : h->iter_exec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    h->n_exec = 0;
}

int capture_iteration(bcm_handle *h, int prof_cls) {
    if (h->n_exec > 0 && h->graph_prof_cls == prof_cls) return BCM_OK;
    destroy_iteration_graphs(h);
    if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    const Level &L0 = h->lv[0];
    const int n = L0.A.n, nb = h->red_blocks;
    SegCapture sc;
    sc.st = h->cap;
    Prof gp{h, 0, prof_cls, &sc};
    hipStream_t keep = h->s;
    h->s = h->cap;
    sc.begin();
    vcycle(h, gp, h->r, h->w, h->scal + 10, 0, h->y0, stop_test_of(h));
    int e = gp.begin(2);
    const int nbs = spmv_dots_grid(L0, nb);
    launch_spmv_dots(h->cap, L0, nbs, 0, h->w, h->r, h->q, h->v, h->spart, h->scal);
    gp.end(2, e, 0.0, 0);
    const bool fuse = update_takes_dots(nbs);
    if (!fuse) launch_finalize(h->cap, 1, nbs, 0, h->spart, h->scal);
    e = gp.begin(3);
    launch_update(h->cap, n, nb, 0, h->w, h->v, h->d, h->u, h->q, h->r, h->partials, h->scal, y0_dinv(h), h->y0,
                  h->prm.precision == BCM_FP32_CYCLE, fuse ? h->spart : nullptr, nbs);
    gp.end(3, e, 0.0, 0);
    if (!cycle_takes_stop(h)) launch_finalize(h->cap, 2, nb, 0, h->partials, h->scal);
    sc.end();
    h->s = keep;
    hipError_t err = sc.err;
    if (err == hipSuccess && sc.graphs.size() != 1 && sc.graphs.size() != 3) err = hipErrorInvalidValue;
    for (size_t i = 0; i < sc.graphs.size(); ++i) {
        hipGraph_t g = sc.graphs[i];
        size_t nodes = 0;
        if (err == hipSuccess && g) err = hipGraphGetNodes(g, nullptr, &nodes);
        if (err == hipSuccess && g && nodes > 0) err = hipGraphInstantiate(&h->iter_exec[i], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
    }
    if (err != hipSuccess) {
        destroy_iteration_graphs(h);
        set_error(std::string("HIP graph capture failed: ") + hipGetErrorString(err));
        return BCM_EHIP;
    }
    h->n_exec = (int)sc.graphs.size();
    h->graph_prof_cls = prof_cls;
    return BCM_OK;
}

int fcg_run(bcm_handle *h, const double *b, double *x_user, double tol) {
    hipStream_t s = h->s;
    const Level &L0 = h->lv[0];
    const int n = L0.A.n, nb = h->red_blocks, nbs = spmv_dots_grid(L0, nb);
    Prof pf{h, h->prm.profile};
    // graph mode: a profile mask of one class bracketed once per iteration
    // (down0, up0, spmv_dots, update, coarse) is timed by events recorded
    // around that class's own graph; other masks launch every iteration eagerly
    int gcls = -1;
    for (int c = 0; c < 5; ++c)
        if (h->prm.profile == (1 << c)) gcls = c;
    const bool use_graph = h->prm.graph && (!h->prm.profile || gcls >= 0);
    if (use_graph) {
        const int rcg = capture_iteration(h, gcls);
        if (rcg) return rcg;
    }

    double *x = h->u;
    launch_copy_f64(s, n, x_user, x);
    h->ev_pairs.clear();
    h->ev_bytes.clear();
    h->ev_iter.clear();
    double hs[16];
    launch_resid(s, L0, nb, b, x, h->r, h->partials, h->scal);
    launch_finalize(s, 0, nb, 0, h->partials, h->scal);
    int rc = read_back(s, h->scal, 16 * sizeof(double), hs);
    if (rc) return rc;
    const double bb = hs[5];
    int it = 0, status = BCM_OK;
    double relres = 0.0;
    if (!(bb > 0.0) || !std::isfinite(bb)) {
        if (bb == 0.0) {
            launch_fill_i32(s, 2 * (size_t)n, (int *)x, 0);
            h->iters = 0; h->relres = 0.0; h->status = BCM_OK;
            HIPCHK(hipStreamSynchronize(s));
            return BCM_OK;
        }
        set_error("right-hand side or initial guess not finite");
        return BCM_EINVAL;
    }
    const double bn = std::sqrt(bb);
    relres = std::sqrt(hs[4]) / bn;
    const int itmax = h->prm.itmax;
    const double *done = h->scal + 10;
    double ctl_local[4];
    double *ctl = pinned() ? pinned() + 32 : ctl_local;
    for (int restart = 0; restart < 4; ++restart) {
        if (relres <= tol) { status = BCM_OK; break; }
        if (it >= itmax) { status = BCM_MAXIT; break; }
        // arm the device-side loop control: flag, count, threshold, itmax
        ctl[0] = 0.0; ctl[1] = (double)it; ctl[2] = tol * tol * bb; ctl[3] = (double)itmax;
        HIPCHK(hipMemcpyAsync(h->scal + 10, ctl, 4 * sizeof(double), hipMemcpyHostToDevice, s));
        int first = 1, batch = 4, launched = it;
        double rel_prev = relres;
        int it_prev = it;
        for (;;) {
            const int nb_it = std::min(batch, itmax - launched);
            for (int t = 0; t < nb_it; ++t) {
                if (use_graph && !first) {
                    // segments: [before] [profiled class] [after], or one graph
                    int e = -1;
                    for (int g = 0; g < h->n_exec; ++g) {
                        if (h->n_exec == 3 && g == 1) e = pf.begin(gcls, true);
                        if (h->iter_exec[g]) HIPCHK(hipGraphLaunch(h->iter_exec[g], s));
                        if (h->n_exec == 3 && g == 1) pf.end(gcls, e, class_bytes(h, gcls), launched, true);
                    }
                    ++launched;
                    continue;
                }
                // the first iteration's r comes from the residual kernel: no y0 yet
                vcycle(h, pf, h->r, h->w, done, launched, first ? nullptr : h->y0, stop_test_of(h));
                int e = pf.begin(2);
                launch_spmv_dots(s, L0, nbs, first, h->w, h->r, h->q, h->v, h->spart, h->scal);
                pf.end(2, e, bytes_spmv_dots(h), launched);
                const bool fuse = update_takes_dots(nbs);
                if (!fuse) launch_finalize(s, 1, nbs, first, h->spart, h->scal);
                e = pf.begin(3);
                launch_update(s, n, nb, first, h->w, h->v, h->d, x, h->q, h->r, h->partials, h->scal, y0_dinv(h),
                              h->y0, h->prm.precision == BCM_FP32_CYCLE, fuse ? h->spart : nullptr, nbs);
                pf.end(3, e, bytes_update(h), launched);
                if (!cycle_takes_stop(h)) launch_finalize(s, 2, nb, 0, h->partials, h->scal);
                first = 0;
                ++launched;
            }
            // the batch's last stop test (a no-op where it has been taken)
            launch_finalize(s, 2, nb, 0, h->partials, h->scal);
            rc = read_back(s, h->scal, 16 * sizeof(double), hs);
            if (rc) return rc;
            it = (int)hs[11];
            if (hs[6] != 0.0) {
                h->iters = it; h->status = BCM_EBREAKDOWN;
                prof_collect(h, it);
                set_error("flexible CG breakdown: rho <= 0 or not finite (matrix or preconditioner not s.p.d.)");
                return BCM_EBREAKDOWN;
            }
            relres = std::sqrt(hs[4]) / bn;
            if (hs[10] != 0.0 || it >= itmax) break;
            // next batch: iterations the observed rate needs to reach tol
            const double rate = it > it_prev && rel_prev > 0.0 ? std::pow(relres / rel_prev, 1.0 / (it - it_prev)) : 1.0;
            int need = 4;
            if (rate > 0.0 && rate < 0.999) need = (int)std::ceil(std::log(tol / relres) / std::log(rate));
            batch = std::max(1, std::min(32, need));
            rel_prev = relres;
            it_prev = it;
        }
        // true residual b - A x
        launch_resid(s, L0, nb, b, x, h->r, h->partials, h->scal);
        launch_finalize(s, 0, nb, 0, h->partials, h->scal);
        rc = read_back(s, h->scal, 16 * sizeof(double), hs);
        if (rc) return rc;
        relres = std::sqrt(hs[4]) / bn;
        if (relres <= tol) { status = BCM_OK; break; }
        if (it >= itmax) { status = BCM_MAXIT; break; }
        // the recurrence met tol, the true residual did not: restart from x
        status = BCM_STAGNATED;
    }
    if (status == BCM_STAGNATED)
        set_error("true residual stagnated above tol after 3 restarts: relative residual " + std::to_string(relres) +
                  " after " + std::to_string(it) + " iterations");
    HIPCHK(hipGetLastError());
    prof_collect(h, it);
    h->iters = it;
    h->relres = relres;
    h->status = status;
    return status;
}

// flexible CG on the handle's iterate; the caller's x is copied in and back out
int fcg(bcm_handle *h, const double *b, double *x, double tol) {
    const int rc = fcg_run(h, b, x, tol);
    if (rc == BCM_OK || rc == BCM_MAXIT || rc == BCM_STAGNATED || rc == BCM_EBREAKDOWN) {
        launch_copy_f64(h->s, h->lv[0].A.n, h->u, x);
        HIPCHK(hipStreamSynchronize(h->s));
    }
    return rc;
}

// Argument checks of bcm_match.
int match_args(const bcm_csr *A, const double *w, const bcm_params *p, const int32_t *mate, bcm_params &prm) {
    if (!A || !w || !mate || !A->row_ptr || !A->col || !A->val || A->n <= 0 || A->nnz < 0) {
        set_error("NULL or empty argument");
        return BCM_EINVAL;
    }
    if (p) prm = *p; else bcm_default_params(&prm);
    if (!valid_group(prm.group) || (prm.alloc == nullptr) != (prm.dealloc == nullptr)) {
        set_error("unsupported parameters (group 0, -1, 4, 8, 16, 32 or 64; alloc and dealloc both or neither)");
        return BCM_EINVAL;
    }
    return BCM_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Address of the static scratch array on the current device, looked up on the
// first call made with that device current.
int noalloc_scratch(void **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("bcm_match_noalloc: device index out of range");
        return BCM_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("bcm_match_noalloc: no address for the static scratch array");
            return BCM_EHIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return BCM_OK;
}

Csr csr_view(const bcm_csr *A) {
    Csr M;
    M.n = A->n;
    M.nnz = A->nnz;
    M.rp = const_cast<int *>(A->row_ptr);
    M.ci = const_cast<int *>(A->col);
    M.v = const_cast<double *>(A->val);
    return M;
}

}  // namespace

extern "C" {

void bcm_default_params(bcm_params *p) {
    std::memset(p, 0, sizeof(*p));
    p->max_levels = 40;
    p->max_coarse = 0;
    p->sweeps = 2;
    p->coarse_sweeps = 20;
    p->pre = 1;
    p->post = 1;
    p->cycle = BCM_VCYCLE;
    p->kcycle_levels = 0;
    p->precision = BCM_FP64;
    p->itmax = 5000;
    p->check = 1;
    p->profile = 0;
    p->graph = 0;
    p->group = 0;
    p->sell = 1;
    p->fold = 1;
    p->adjoint_tol = 0.0;
    p->min_ratio = 0.0;
}

const char *bcm_last_error(void) { return g_err.c_str(); }

int bcm_setup(const bcm_csr *A, const double *w, const bcm_params *p, bcm_handle **out) {
    g_err.clear();
    if (!out) { set_error("out is NULL"); return BCM_EINVAL; }
    *out = nullptr;
    if (!A || !w || !A->row_ptr || !A->col || !A->val) { set_error("NULL matrix or smooth vector"); return BCM_EINVAL; }
    if (A->n <= 0 || A->nnz < A->n) { set_error("need n > 0 and nnz >= n (diagonal stored)"); return BCM_EINVAL; }
    bcm_params prm;
    if (p) prm = *p; else bcm_default_params(&prm);
    if (prm.max_levels < 1 || prm.sweeps < 1 || prm.sweeps > 4 || prm.coarse_sweeps < 1 || prm.itmax < 1 ||
        prm.pre != 1 || prm.post != 1 || prm.cycle < BCM_VCYCLE || prm.cycle > BCM_KCYCLE || prm.kcycle_levels < 0 ||
        !valid_group(prm.group) || !(prm.min_ratio >= 0.0) || (prm.fold != 0 && prm.fold != 1) ||
        (prm.precision != BCM_FP64 && prm.precision != BCM_FP32_CYCLE) || (prm.alloc == nullptr) != (prm.dealloc == nullptr)) {
        set_error("unsupported parameters (sweeps 1..4, pre = post = 1, V-, W- or K-cycle, kcycle_levels >= 0, "
                  "group 0, -1, 4, 8, 16, 32 or 64, fold 0 or 1, FP64 or FP32 cycle)");
        return BCM_EINVAL;
    }
    const double t0 = now_ms();
    bcm_handle *h = new bcm_handle();
    h->prm = prm;
    h->s = (hipStream_t)prm.stream;
    h->persist.alloc = prm.alloc;
    h->persist.dealloc = prm.dealloc;
    h->persist.ctx = prm.alloc_ctx;
    int rc = build_hierarchy(h, A, w);
    if (rc) {
        bcm_free(h);
        return rc;
    }
    h->t_setup_ms = now_ms() - t0;
    *out = h;
    return BCM_OK;
}

int bcm_solve(bcm_handle *h, const double *b, double *x, double tol) {
    g_err.clear();
    if (!h || !b || !x) { set_error("NULL handle or vector"); return BCM_EINVAL; }
    if (!(tol > 0.0)) { set_error("tol must be positive"); return BCM_EINVAL; }
    const double t0 = now_ms();
    h->last_tol = tol;
    const int rc = fcg(h, b, x, tol);
    h->t_solve_ms = now_ms() - t0;
    return rc;
}

int bcm_precond(bcm_handle *h, const double *r, double *z) {
    g_err.clear();
    if (!h || !r || !z) { set_error("NULL handle or vector"); return BCM_EINVAL; }
    Prof pf{h, 0};
    vcycle(h, pf, r, z, nullptr, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->s));
    return BCM_OK;
}

int bcm_solve_adjoint(bcm_handle *h, const double *g, double *lambda) {
    g_err.clear();
    if (!h || !g || !lambda) { set_error("NULL handle or vector"); return BCM_EINVAL; }
    const double tol = h->prm.adjoint_tol > 0.0 ? h->prm.adjoint_tol : h->last_tol;
    if (!(tol > 0.0)) { set_error("no adjoint tolerance: set adjoint_tol or call bcm_solve first"); return BCM_EINVAL; }
    launch_fill_i32(h->s, 2 * (size_t)h->lv[0].A.n, (int *)lambda, 0);
    const double t0 = now_ms();
    const int rc = fcg(h, g, lambda, tol);
    h->t_solve_ms = now_ms() - t0;
    return rc;
}

int bcm_sampled_outer(bcm_handle *h, const double *lambda, const double *x, double *grad_val) {
    g_err.clear();
    if (!h || !lambda || !x || !grad_val) { set_error("NULL handle or vector"); return BCM_EINVAL; }
    launch_sampled_outer(h->s, h->lv[0], lambda, x, grad_val);
    HIPCHK(hipGetLastError());
    return BCM_OK;
}

int bcm_info(const bcm_handle *h, bcm_info_t *o) {
    if (!h || !o) { set_error("NULL handle or output"); return BCM_EINVAL; }
    std::memset(o, 0, sizeof(*o));
    o->nl = h->nl;
    o->precision = h->prm.precision;
    o->iters = h->iters;
    o->status = h->status;
    double sz = 0, sr = 0;
    for (int k = 0; k < h->nl; ++k) {
        o->n[k] = h->lv[k].A.n;
        o->nnz[k] = h->lv[k].A.nnz;
        sz += h->lv[k].A.nnz;
        if (k > 0) sr += (double)h->lv[k - 1].A.n / h->lv[k].A.n;
    }
    o->vcmplx = sz / h->lv[0].A.nnz;
    o->cratio = h->nl > 1 ? sr / (h->nl - 1) : 1.0;
    o->cratio_nl = sr / h->nl;
    o->relres = h->relres;
    o->t_setup_ms = h->t_setup_ms;
    o->t_solve_ms = h->t_solve_ms;
    const double cyc = bytes_cycle(h);
    o->cycle_bytes = cyc;
    o->iter_bytes = cyc + bytes_spmv_dots(h) + bytes_update(h);
    o->setup_bytes = h->setup_bytes;
    o->sweeps_run = h->sweeps_run;
    for (int k = 0; k < h->nl; ++k) o->long_rows += h->lv[k].lr.n;
    return BCM_OK;
}

int bcm_level_copy(const bcm_handle *h, int32_t k, int32_t *row_ptr, int32_t *col, double *val, double *w,
                   double *dinv, int32_t *agg, double *p) {
    if (!h || k < 0 || k >= h->nl) { set_error("bad handle or level"); return BCM_EINVAL; }
    const Level &L = h->lv[k];
    hipStream_t s = h->s;
    const size_t n = L.A.n, z = L.A.nnz;
    if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, L.A.rp, (n + 1) * 4, hipMemcpyDefault, s));
    if (col) HIPCHK(hipMemcpyAsync(col, L.A.ci, z * 4, hipMemcpyDefault, s));
    if (val) HIPCHK(hipMemcpyAsync(val, L.A.v, z * 8, hipMemcpyDefault, s));
    if (w) HIPCHK(hipMemcpyAsync(w, L.w, n * 8, hipMemcpyDefault, s));
    if (dinv) HIPCHK(hipMemcpyAsync(dinv, L.dinv, n * 8, hipMemcpyDefault, s));
    if (k < h->nl - 1) {
        if (agg) HIPCHK(hipMemcpyAsync(agg, L.agg, n * 4, hipMemcpyDefault, s));
        if (p) HIPCHK(hipMemcpyAsync(p, L.p, n * 8, hipMemcpyDefault, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return BCM_OK;
}

int bcm_match(const bcm_csr *A, const double *w, const bcm_params *p, int32_t *mate, double *c) {
    g_err.clear();
    bcm_params prm;
    int rc = match_args(A, w, p, mate, prm);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)prm.stream;
    Arena tmp;
    tmp.alloc = prm.alloc;
    tmp.dealloc = prm.dealloc;
    tmp.ctx = prm.alloc_ctx;
    const Csr M = csr_view(A);
    const int lmin = long_min(lanes_for(prm.group, M));
    const size_t bytes = match_scratch_bytes(A->n, A->nnz, true, c != nullptr, true, lmin);
    Carver cv;
    cv.cur = static_cast<char *>(tmp.get(bytes));
    cv.left = bytes;
    if (!cv.cur) {
        set_error("device allocation failed");
        return BCM_ENOMEM;
    }
    MatchScratch ms;
    carve_match(cv, A->n, A->nnz, true, c, mate, lmin, ms);
    rc = match_sweep(s, ms, M, w, prm.check ? 1 : 0, prm.group, nullptr, 0, nullptr, nullptr, true, nullptr, &tmp);
    (void)hipStreamSynchronize(s);
    tmp.release();
    return rc;
}

int bcm_match_noalloc(const bcm_csr *A, const double *w, const bcm_params *p, int32_t *mate, double *c) {
    g_err.clear();
    bcm_params prm;
    int rc = match_args(A, w, p, mate, prm);
    if (rc) return rc;
    void *base = nullptr;
    rc = noalloc_scratch(&base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)prm.stream;
    const Csr M = csr_view(A);
    const int lmin = long_min(lanes_for(prm.group, M));
    const size_t bytes = match_scratch_bytes(A->n, A->nnz, true, c != nullptr, true, lmin);
    if (bytes > BCM_NOALLOC_SCRATCH_BYTES) {
        set_error("bcm_match_noalloc: the matching needs " + std::to_string(bytes) + " bytes of scratch, more than the " +
                  std::to_string((size_t)BCM_NOALLOC_SCRATCH_BYTES) + "-byte static array");
        return BCM_EINVAL;
    }
    Carver cv;
    cv.cur = static_cast<char *>(base);
    cv.left = BCM_NOALLOC_SCRATCH_BYTES;
    MatchScratch ms;
    carve_match(cv, A->n, A->nnz, true, c, mate, lmin, ms);
    // the long rows' sort keys, if any, come from what is left of the array
    rc = match_sweep(s, ms, M, w, prm.check ? 1 : 0, prm.group, nullptr, 0, nullptr, nullptr, false, &cv, nullptr);
    if (rc == BCM_OK) HIPCHK(hipStreamSynchronize(s));
    else (void)hipStreamSynchronize(s);
    return rc;
}

int bcm_profile(const bcm_handle *h, int32_t kclass, int64_t *launches, double *ms, double *bytes) {
    if (!h || kclass <= 0 || (kclass & (kclass - 1)) || kclass > BCM_PROF_SETUP_GALERKIN) {
        set_error("bad handle or kernel class");
        return BCM_EINVAL;
    }
    const ProfClass &c = h->prof[prof_class_index(kclass)];
    if (launches) *launches = c.launches;
    if (ms) *ms = c.ms;
    if (bytes) *bytes = c.bytes;
    return BCM_OK;
}

void bcm_free(bcm_handle *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->s);
    destroy_iteration_graphs(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (auto e : h->ev_pool) (void)hipEventDestroy(e);
    h->persist.release();
    delete h;
}

}  // extern "C"
