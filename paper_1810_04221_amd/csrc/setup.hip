// Setup-phase kernels for gfx950: input validation, compatible-matching edge
// weights, Suitor matching, pairwise aggregation (Algorithm 2), the
// w-normalised prolongator and the Galerkin product P^T A P (Sections 2.1, 2.2,
// 3.1 of the paper).
//
// Every floating-point expression here is written so that the device and a
// serial IEEE binary64 evaluation round identically: the file is compiled with
// -ffp-contract=off (no FMA contraction) and each operation below is one
// correctly rounded binary64 add, multiply, divide or square root.
#include <type_traits>
#include <utility>

#include "device.h"
#include "internal.h"

#pragma clang fp contract(off)

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
// Validation and diagonal: one group of G lanes per row.  Every read is guarded
// so that malformed input raises a flag instead of an out-of-bounds access.
// ----------------------------------------------------------------------------
// Appends (row, len) to a list of long segments.
__device__ __forceinline__ void seg_append(const SegList &sg, int row, int len) {
    const int t = atomicAdd(&sg.ctl[0], 1);
    if (t < sg.cap) {
        sg.row[t] = row;
        sg.len[t] = len;
    }
}

template <int G>
__global__ void __launch_bounds__(kBlock)
k_validate(int n, int nnz, const int *__restrict__ rp, const int *__restrict__ ci,
           const double *__restrict__ v, const double *__restrict__ w, int check_sym,
           double *__restrict__ diag, int *__restrict__ flags, SegList sg, int lmin, int *__restrict__ dmax) {
    const int lane = threadIdx.x % G;
    const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
    if (row >= n) return;
    const int s = rp[row], e = rp[row + 1];
    int f = 0;
    // nnz < 0: a matrix built here whose entry count is not known on the host
    if (s < 0 || e < s || (nnz >= 0 && (e > nnz || (row == n - 1 && e != nnz))) || (row == 0 && s != 0)) {
        if (lane == 0) atomicOr(flags, kErrRowPtr);
        return;
    }
    // longest row: the atomic only when the (coherent) current value is exceeded
    if (dmax && lane == 0 && e - s > load_agent(dmax)) atomicMax(dmax, e - s);
    int has_diag = 0;
    double dval = 0.0;
    // a long row: its entries are checked by k_long_validate; here only its
    // diagonal, found by a binary search of the (ascending) columns
    const bool lng = sg.ctl && e - s > lmin;
    if (lng) {
        if (lane == 0) {
            seg_append(sg, row, e - s);
            int lo = s, hi = e;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ci[mid] < row) lo = mid + 1; else hi = mid;
            }
            if (lo < e && ci[lo] == row) { has_diag = 1; dval = v[lo]; }
        }
    }
    for (int q = s + lane; q < (lng ? s : e); q += G) {
        const int j = ci[q];
        const double a = v[q];
        if (j < 0 || j >= n) { f |= kErrCol; continue; }
        if (q > s && ci[q - 1] >= j) f |= kErrUnsorted;
        if (!isfinite(a)) f |= kErrNonFinite;
        if (j == row) { has_diag = 1; dval = a; }
        if (check_sym && j != row) {
            const int s2 = rp[j], e2 = rp[j + 1];
            int found = -1;
            if (s2 >= 0 && e2 >= s2 && (nnz < 0 || e2 <= nnz)) {
                int lo = s2, hi = e2 - 1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    const int cm = ci[mid];
                    if (cm == row) { found = mid; break; }
                    if (cm < row) lo = mid + 1; else hi = mid - 1;
                }
            }
            if (found < 0 || __double_as_longlong(v[found]) != __double_as_longlong(a)) f |= kErrAsym;
        }
    }
    // one lane at most holds the diagonal
    const int hd = group_sum<G>(has_diag);
    const double dv = group_sum<G>(has_diag ? dval : 0.0);
    if (lane == 0) {
        if (hd == 0) f |= kErrNoDiag;
        else if (!(dv > 0.0)) f |= kErrDiagNonPos;
        diag[row] = dv;
        const double wi = w[row];
        if (!(isfinite(wi) && wi != 0.0)) f |= kErrW;
    }
    if (f) atomicOr(flags, f);
}

// ----------------------------------------------------------------------------
// Edge weights of compatible weighted matching (Section 2.2):
//   c_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2)
// with m = min(i, j), M = max(i, j) fixing the operand order, so both ends of
// an edge compute the same double.  Diagonal positions get 0; ws (the
// matching's best proposal per vertex) is cleared on the way.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double edge_weight(int row, int j, double a, const double *__restrict__ diag,
                                              const double *__restrict__ w) {
    if (j == row) return 0.0;
    const int m = min(row, j), M = max(row, j);
    const double wm = w[m], wM = w[M];
    const double num = ((2.0 * a) * wm) * wM;
    const double den = (diag[m] * wm) * wm + (diag[M] * wM) * wM;
    return 1.0 - num / den;
}

template <int G>
__global__ void __launch_bounds__(kBlock)
k_weights(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
          const double *__restrict__ diag, const double *__restrict__ w, double *__restrict__ c,
          unsigned long long *__restrict__ ws, int lmin) {
    // rows longer than lmin (> 0) are left to k_long_weights
    const int lane = threadIdx.x % G;
    const int row = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (row >= n) return;
    if (ws && lane == 0) ws[row] = 0ull;
    const int b = rp[row], e = rp[row + 1];
    if (lmin > 0 && e - b > lmin) return;
    for (int q = b + lane; q < e; q += G) c[q] = edge_weight(row, ci[q], v[q], diag, w);
}

// ----------------------------------------------------------------------------
// Suitor candidate lists for short rows (same output as k_candidates below;
// see there): the row's weights and columns are held in LDS (rows of at most
// 4 G entries) and each eligible entry counts its place in the row's order
// there; the rank of c_uv seen from v is counted over row v's weights (c_vu
// is the same double as c_uv), all of whose loads are issued together.
// ----------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(kBlock)
k_candidates_direct(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ c,
                    const unsigned *__restrict__ rk, unsigned long long *__restrict__ cand, int lmin) {
    // rows longer than lmin (> 0) are left to the long-row kernels, which leave
    // their own-row ranks in rk: the rank of c_uv seen from such a row v is read
    // there (at the transposed position) instead of counted
    constexpr int LS = 4 * G;
    constexpr int NG = kBlock / G;
    // groups' slots one element apart (stride LS + 1): the groups of a wave
    // reading the same slot index hit different LDS banks
    constexpr int LSP = LS + 1;
    __shared__ double sc[NG * LSP];
    __shared__ int sv[NG * LSP];
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int row = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (row >= n) return;
    const int s0 = rp[row], e = rp[row + 1], d = e - s0;
    if (lmin > 0 && d > lmin) return;
    auto rank_at = [&](int vtx, double cq) -> unsigned {
        const int b2 = rp[vtx], e2 = rp[vtx + 1];
        if (lmin > 0 && e2 - b2 > lmin) {
            int lo = b2, hi = e2;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ci[mid] < row) lo = mid + 1; else hi = mid;
            }
            return (lo < e2 && ci[lo] == row) ? rk[lo] : 0u;
        }
        unsigned r = 0;
#pragma unroll 8
        for (int t = b2; t < e2; ++t) r += (c[t] < cq) ? 1u : 0u;
        return r;
    };
    const bool staged = d <= LS;
    double *C = sc + g * LSP;
    int *V = sv + g * LSP;
    if (staged) {
        for (int k = lane; k < d; k += G) {
            C[k] = c[s0 + k];
            V[k] = ci[s0 + k];
        }
        wave_sync();
    }
    const double *Cr = staged ? C : c + s0;
    const int *Vr = staged ? V : ci + s0;
    int nelig = 0;
    for (int k = lane; k < d; k += G) {
        const int vtx = Vr[k];
        const double cq = Cr[k];
        if (!(vtx != row && cq > 0.0 && cq < INFINITY)) continue;
        ++nelig;
        int before = 0;
        for (int t = 0; t < d; ++t) {
            const int vt = Vr[t];
            const double ct = Cr[t];
            const bool elig = vt != row && ct > 0.0 && ct < INFINITY;
            before += (elig && (ct > cq || (ct == cq && vt > vtx))) ? 1 : 0;
        }
        if (before < d - 1) cand[s0 + before] = ((unsigned long long)rank_at(vtx, cq) << 32) | (unsigned)vtx;
    }
    nelig = min(group_sum<G>(nelig), max(d - 1, 0));
    for (int q = s0 + nelig + lane; q < e; q += G) cand[q] = ~0ull;
}

// ----------------------------------------------------------------------------
// Sorting inside a group of G lanes (a wave or part of one): bitonic network
// over P (a power of two) 64-bit keys in the group's LDS slots, ascending.
// Only the group's own lanes touch its slots, so wave-level ordering suffices.
// ----------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ void group_sort(unsigned long long *keys, int P, int lane) {
    // size = 2^ls, stride = 2^lt: the pair indices by shifts and masks (a
    // division by a stride the compiler cannot see to be a power of two costs
    // dozens of instructions)
    for (int ls = 1; (1 << ls) <= P; ++ls) {
        for (int lt = ls - 1; lt >= 0; --lt) {
            const int stride = 1 << lt;
            for (int t = lane; t < (P >> 1); t += G) {
                const int lo = ((t >> lt) << (lt + 1)) | (t & (stride - 1)), hi = lo + stride;
                const bool up = (lo & (1 << ls)) == 0;
                const unsigned long long a = keys[lo], b = keys[hi];
                if ((a > b) == up) {
                    keys[lo] = b;
                    keys[hi] = a;
                }
            }
            wave_sync();
        }
    }
}

__device__ __forceinline__ int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Order-preserving image of a double in the unsigned integers (NaN above +inf).
__device__ __forceinline__ unsigned long long order_key(double x) {
    if (x != x) return ~0ull - 1;
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// first index k < cnt with keys[k] >= key (keys ascending)
__device__ __forceinline__ int lower_bound_u64(const unsigned long long *keys, int cnt, unsigned long long key) {
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ----------------------------------------------------------------------------
// Rank of every weight within its own row: rk[q] = #{ t in row(q) : c[t] < c[q] }
// (the count a row's neighbours need for their Suitor keys).  The row's weights
// are sorted in LDS and each rank is a binary search; rows longer than the LDS
// slots count directly.
// ----------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(kBlock)
k_rank(int n, const int *__restrict__ rp, const double *__restrict__ c, unsigned *__restrict__ rk, int lmin) {
    constexpr int LMAX = 16 * G;
    constexpr int NG = kBlock / G;
    __shared__ unsigned long long sk[NG * (LMAX + 1)];  // groups one element apart: distinct banks
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int row = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (row >= n) return;
    const int s0 = rp[row], d = rp[row + 1] - s0;
    if (lmin > 0 && d > lmin) return;  // a long row: k_long_rank
    if (d <= LMAX) {
        unsigned long long *keys = sk + g * (LMAX + 1);
        const int P = pow2_at_least(d);
        for (int k = lane; k < P; k += G) keys[k] = k < d ? order_key(c[s0 + k]) : ~0ull;
        wave_sync();
        group_sort<G>(keys, P, lane);
        for (int k = lane; k < d; k += G) rk[s0 + k] = (unsigned)lower_bound_u64(keys, d, order_key(c[s0 + k]));
    } else {
        for (int k = lane; k < d; k += G) {
            const double cq = c[s0 + k];
            unsigned r = 0;
            for (int t = 0; t < d; ++t) r += (c[s0 + t] < cq) ? 1u : 0u;
            rk[s0 + k] = r;
        }
    }
}

// ----------------------------------------------------------------------------
// Suitor candidate lists.  For row u, the eligible entries (off-diagonal, weight
// positive and finite) are written in preference order of u -- weight
// descending, then neighbour index descending -- as 64-bit words
//   cand = rk << 32 | v,   rk = #{ entries t of row v : c[t] < c_uv }
// where rk is the position of c_uv among the weights seen from v (the own-row
// rank of the transposed entry, c being the same double from both ends).  A
// proposal from u to v then compares at v as (rk << 32 | t + 1), t being the
// slot of v in u's list: slots grow with u (rows are stored in order), so this
// orders proposals exactly as (c_uv, u).  After the eligible entries the row
// holds the sentinel ~0, at least in its last slot (the diagonal is never
// eligible; a row without one drops its last candidate, which validation
// rejects anyway).  The preference order is a sort of
// (own-row rank desc, v desc) in LDS; rows longer than the LDS slots are
// placed by direct counting.
// ----------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(kBlock)
k_candidates(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ c,
             const unsigned *__restrict__ rk_own, unsigned long long *__restrict__ cand, int lmin) {
    constexpr int LMAX = 16 * G;
    constexpr int NG = kBlock / G;
    __shared__ unsigned long long sk[NG * (LMAX + 1)];  // groups one element apart: distinct banks
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int row = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (row >= n) return;
    const int s0 = rp[row], e = rp[row + 1], d = e - s0;
    if (lmin > 0 && d > lmin) return;  // a long row: k_long_cand
    // rank of c_uv seen from v: the own-row rank of (v, u), found by binary search
    // (a pattern that is not symmetric, accepted without the symmetry check,
    // may lack the entry: rank 0 then, and no read outside row v)
    auto rank_at = [&](int vtx) -> unsigned {
        const int e2 = rp[vtx + 1];
        int lo = rp[vtx], hi = e2;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ci[mid] < row) lo = mid + 1; else hi = mid;
        }
        return (lo < e2 && ci[lo] == row) ? rk_own[lo] : 0u;
    };
    if (d <= LMAX) {
        unsigned long long *keys = sk + g * (LMAX + 1);
        const int P = pow2_at_least(d);
        int nelig = 0;
        for (int k = lane; k < P; k += G) {
            unsigned long long key = ~0ull;
            if (k < d) {
                const int vtx = ci[s0 + k];
                const double cq = c[s0 + k];
                if (vtx != row && cq > 0.0 && cq < INFINITY) {
                    // ascending (rank, index) complement = descending preference
                    key = ((unsigned long long)(0x7fffffffu - rk_own[s0 + k]) << 32) | (0x7fffffffu - (unsigned)vtx);
                    ++nelig;
                }
            }
            keys[k] = key;
        }
        wave_sync();
        group_sort<G>(keys, P, lane);
        nelig = min(group_sum<G>(nelig), d - 1);
        for (int k = lane; k < d; k += G) {
            unsigned long long out = ~0ull;
            if (k < nelig) {
                const int vtx = (int)(0x7fffffffu - (unsigned)(keys[k] & 0xffffffffull));
                out = ((unsigned long long)rank_at(vtx) << 32) | (unsigned)vtx;
            }
            cand[s0 + k] = out;
        }
    } else {
        int nelig = 0;
        for (int q = s0 + lane; q < e; q += G) {
            const int vtx = ci[q];
            const double cq = c[q];
            if (!(vtx != row && cq > 0.0 && cq < INFINITY)) continue;
            ++nelig;
            int before = 0;
            for (int t = s0; t < e; ++t) {
                const int vt = ci[t];
                const double ct = c[t];
                const bool elig = vt != row && ct > 0.0 && ct < INFINITY;
                before += (elig && (ct > cq || (ct == cq && vt > vtx))) ? 1 : 0;
            }
            if (before < d - 1) cand[s0 + before] = ((unsigned long long)rank_at(vtx) << 32) | (unsigned)vtx;
        }
        nelig = min(group_sum<G>(nelig), d - 1);
        for (int q = s0 + nelig + lane; q < e; q += G) cand[q] = ~0ull;
    }
}

// ----------------------------------------------------------------------------
// Suitor matching (Section 3.1).  One thread per vertex holds that vertex's
// proposal.  A proposal is the candidate slot t of u's list (cand[t] names v);
// u proposes to each candidate in turn until one accepts.  ws[v] holds the key
// (rk << 32 | t + 1) of v's best proposal so far and is raised with atomicMax,
// whose old value says whether u won.  A displaced proposal is taken over by
// the displacing thread and resumes at the slot after the one it lost (its
// key holds that slot, so no per-vertex position is kept): ws[] only grows,
// so every candidate it passed stays unavailable.  One proposal step is thus
// an atomic and the load of the next candidate.  Every successful atomicMax
// strictly raises one ws[] entry (finitely many times) and a failed one moves
// to the next slot, which ends at the row's sentinel, so every thread exits.
// The final suitor pairs are mutual and equal the greedy matching under
// (c desc, larger endpoint desc, smaller desc).
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_suitor(int n, const int *__restrict__ rp, const unsigned long long *__restrict__ cand, unsigned long long *ws) {
    // Highest vertices first: workgroups are dispatched roughly in index order,
    // and the greedy order settles large indices first on equal weights.  (Cut
    // into several launches, highest chunk first, this ran slower.)
    __shared__ unsigned long long wbest[kBlock / 64];
    const int u = n - 1 - (int)(blockIdx.x * kBlock + threadIdx.x);
    if (u < 0) return;
    int t = rp[u];
    if (t == rp[u + 1]) return;  // empty row: no slot of its own
    for (;;) {
        // ws[v] is not read first: the atomic itself tells whether the proposal
        // lost, and a read would add a memory round trip per step
        const unsigned long long e = cand[t];
        if (e == ~0ull) break;  // no candidate left: this vertex stays unmatched
        const unsigned long long key = (e & 0xffffffff00000000ull) | (unsigned long long)(unsigned)(t + 1);
        const int v = (int)(e & 0xffffffffull);
        // Every active lane of the wave proposing to the same vertex (the
        // leaves of a hub): only the best of these proposals can win there (ws
        // only grows, keys are distinct), so the others lose at once -- the
        // outcome of any order in which the best one came first -- and the
        // wave issues one atomic instead of 64.
        // (one active lane, the usual case in the tail of displacement
        // chains, goes straight to the atomic)
        const int v0 = __builtin_amdgcn_readfirstlane(v);
        const unsigned long long act = __ballot(1);
        if ((act & (act - 1)) != 0ull && __ballot(v != v0) == 0ull) {
            unsigned long long *slot = &wbest[threadIdx.x >> 6];
            const int first = __ffsll(act) - 1;
            if ((int)(threadIdx.x & 63) == first) *slot = 0ull;
            wave_sync();
            atomicMax(slot, key);
            wave_sync();
            const unsigned long long best = *slot;
            wave_sync();
            if (key != best) { ++t; continue; }
        }
        const unsigned long long old = atomicMax(&ws[v], key);
        if (old > key) { ++t; continue; }  // lost v for good (ws only grows): next slot
        if (old == 0ull) break;            // v had no suitor: done
        t = (int)(old & 0xffffffffull);    // displaced proposal (slot old - 1) resumes after it
    }
}

// mate[i] = s if i and its suitor s chose each other; leader[i] marks the
// smallest member of each aggregate of Algorithm 2.
__global__ void __launch_bounds__(kBlock)
k_mate(int n, const int *__restrict__ rp, const int *__restrict__ ci, const unsigned long long *__restrict__ ws,
       int *__restrict__ mate, int *__restrict__ leader, const int *__restrict__ csrc, int *__restrict__ cdst) {
    // (csrc given: two ints copied to cdst on the way, for the host's next read-back)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < 2 && csrc) cdst[i] = csrc[i];
    if (i >= n) return;
    // the suitor of i is the neighbour whose row holds the winning slot ts:
    // the last neighbour j of i with rp[j] <= ts (columns ascending, rp monotone)
    const int ts = (int)(ws[i] & 0xffffffffull) - 1;
    int m = -1;
    if (ts >= 0 && rp[i] < rp[i + 1]) {
        int lo = rp[i], hi = rp[i + 1] - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[ci[mid]] <= ts) lo = mid; else hi = mid - 1;
        }
        const int s = ci[lo];
        const int tb = (int)(ws[s] & 0xffffffffull) - 1;
        if (ts >= rp[s] && ts < rp[s + 1] && tb >= rp[i] && tb < rp[i + 1]) m = s;
    }
    mate[i] = m;
    leader[i] = (m < 0 || i < m) ? 1 : 0;
}

// ----------------------------------------------------------------------------
// Algorithm 2 with aggregates numbered in the order of their smallest member
// (ofs = exclusive scan of leader flags), and the prolongator: orthonormal
// projection of w on each aggregate (Section 2.2).  Pair {i < j}:
// s = sqrt(w_i*w_i + w_j*w_j), p = w / s; singleton: s = |w_i|.  The coarse
// smooth vector is the restriction P^T w = s.  mem2 lists each aggregate's
// members (second = -1 for a singleton).
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_aggfill(int n, const int *__restrict__ mate, const int *__restrict__ ofs, const double *__restrict__ w,
          int *__restrict__ agg, double *__restrict__ p, double *__restrict__ wc, int *__restrict__ mem2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int m = mate[i];
    if (!(m < 0 || i < m)) return;
    const int E = ofs[i];
    agg[i] = E;
    mem2[2 * E] = i;
    const double wi = w[i];
    if (m >= 0) {
        const double wm = w[m];
        const double s = sqrt(wi * wi + wm * wm);
        agg[m] = E;
        mem2[2 * E + 1] = m;
        p[i] = wi / s;
        p[m] = wm / s;
        wc[E] = s;
    } else {
        const double s = fabs(wi);
        mem2[2 * E + 1] = -1;
        p[i] = wi / s;
        wc[E] = s;
    }
}

// ----------------------------------------------------------------------------
// Galerkin product A_c = P^T A P for one pairwise sweep (Section 2.1; the
// paper's most expensive setup step).  One group of G lanes per coarse row E.
// The candidate columns F = agg[j] of E's member rows are staged in LDS
// (16 G per group; longer rows fall back to scratch arrays indexed by the
// candidate's position in A).  Pass 0 counts distinct columns; pass 1 writes
// them in ascending order and the value of each entry, whose terms are the
// (at most four) staged candidates with the same column:
//   (A_c)_EF = sum over stored (i in E, j in F) of (p_m * a_ij) * p_M,
//   m = min(i, j), M = max(i, j), summed from the first term in ascending
//   (m, M).  Terms sharing (m, M) (i <-> j inside one aggregate) are
//   bitwise equal, so the sum is exactly symmetric and independent of timing.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void cswap(unsigned long long &ka, double &ta, unsigned long long &kb,
                                      double &tb) {
    if (kb < ka) {
        const unsigned long long k = ka; ka = kb; kb = k;
        const double t = ta; ta = tb; tb = t;
    }
}

// One coarse row E (members e0 < e1 or e1 = -1) of k_gal: F / U are the
// group's LDS slots (staged) or the scratch arrays indexed by position in A.
template <int G>
__device__ __forceinline__ void gal_row(int pass, int E, int lane, const int *__restrict__ rp,
                                        const int *__restrict__ ci, const double *__restrict__ v,
                                        const int *__restrict__ agg, const double *__restrict__ p, int e0, int e1,
                                        int s0, int L0, int s1, int L1, int *__restrict__ cnt,
                                        const int *__restrict__ crp, int *__restrict__ cci, double *__restrict__ cv,
                                        int *F, int *U, bool staged) {
    const int L = L0 + L1;
    // slot of candidate k: LDS index, or its position in A (disjoint per coarse row)
    auto slot = [&](int k) { return staged ? k : (k < L0 ? s0 + k : s1 + (k - L0)); };
    for (int k = lane; k < L; k += G) {
        const int q = k < L0 ? s0 + k : s1 + (k - L0);
        F[slot(k)] = agg[ci[q]];
    }
    if (staged) wave_sync(); else __threadfence_block();
    int nu = 0;
    for (int k = lane; k < L; k += G) {
        const int f = F[slot(k)];
        int first = 1;
        for (int k2 = 0; k2 < k; ++k2)
            if (F[slot(k2)] == f) { first = 0; break; }
        U[slot(k)] = first;
        nu += first;
    }
    if (pass == 0) {
        nu = group_sum<G>(nu);
        if (lane == 0) cnt[E] = nu;
        return;
    }
    if (staged) wave_sync(); else __threadfence_block();
    const int base = crp[E];
    const unsigned long long NONE = ~0ull;
    for (int k = lane; k < L; k += G) {
        if (!U[slot(k)]) continue;
        const int f = F[slot(k)];
        // rank among the distinct columns, and the (at most four) candidates of
        // column f: one per stored (i in E, j in F)
        int rank = 0, c0 = -1, c1 = -1, c2 = -1, c3 = -1;
        for (int k2 = 0; k2 < L; ++k2) {
            const int f2 = F[slot(k2)];
            rank += (U[slot(k2)] && f2 < f) ? 1 : 0;
            if (f2 == f) {
                if (c0 < 0) c0 = k2;
                else if (c1 < 0) c1 = k2;
                else if (c2 < 0) c2 = k2;
                else c3 = k2;
            }
        }
        unsigned long long key[4];
        double t[4];
        const int cs[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            key[r] = NONE;
            t[r] = 0.0;
            const int kk = cs[r];
            if (kk < 0) continue;
            const int q = kk < L0 ? s0 + kk : s1 + (kk - L0);
            const int i = kk < L0 ? e0 : e1, j = ci[q];
            const int m = min(i, j), M = max(i, j);
            key[r] = ((unsigned long long)(unsigned)m << 32) | (unsigned)M;
            t[r] = (p[m] * v[q]) * p[M];
        }
        cswap(key[0], t[0], key[1], t[1]);
        cswap(key[2], t[2], key[3], t[3]);
        cswap(key[0], t[0], key[2], t[2]);
        cswap(key[1], t[1], key[3], t[3]);
        cswap(key[1], t[1], key[2], t[2]);
        double sum = t[0];
#pragma unroll
        for (int r = 1; r < 4; ++r)
            if (key[r] != NONE) sum = sum + t[r];
        cci[base + rank] = f;
        cv[base + rank] = sum;
    }
}

// ----------------------------------------------------------------------------
// Composition of the previous sweeps' prolongator with this sweep's pairwise
// one: agg = agg_s[agg_prev], p = p_prev * p_s[agg_prev]; the members of each
// new aggregate are the members of its (at most two) sweep aggregates, sorted
// ascending, stride 2 * stride_prev, padded with -1.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_compose_rows(int n, const int *__restrict__ agg_prev, const double *__restrict__ p_prev,
               const int *__restrict__ agg_s, const double *__restrict__ p_s, int *__restrict__ agg_out,
               double *__restrict__ p_out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int a = agg_prev[i];
    p_out[i] = p_prev[i] * p_s[a];
    agg_out[i] = agg_s[a];
}

__global__ void __launch_bounds__(kBlock)
k_compose_members(int nc_new, const int *__restrict__ mem_prev, int stride_prev,
                  const int *__restrict__ mem_s, int *__restrict__ mem_out) {
    const int E = blockIdx.x * kBlock + threadIdx.x;
    if (E >= nc_new) return;
    int buf[16];
    int cnt = 0;
    for (int h = 0; h < 2; ++h) {
        const int F = mem_s[2 * E + h];
        if (F < 0) continue;
        for (int t = 0; t < stride_prev; ++t) {
            const int i = mem_prev[(size_t)F * stride_prev + t];
            if (i < 0) break;
            int pos = cnt++;
            while (pos > 0 && buf[pos - 1] > i) { buf[pos] = buf[pos - 1]; --pos; }
            buf[pos] = i;
        }
    }
    const int so = 2 * stride_prev;
    for (int t = 0; t < so; ++t) mem_out[(size_t)E * so + t] = t < cnt ? buf[t] : -1;
}

// l1-Jacobi (Section 3.2): dinv_i = 1 / sum_j |a_ij|.
template <int G>
__global__ void __launch_bounds__(kBlock)
k_diag_l1(int n, const int *__restrict__ rp, const double *__restrict__ v, double *__restrict__ dinv,
          float *__restrict__ dinv32, float *__restrict__ v32, LongRows lr, const double *__restrict__ part) {
    // (with v32 given, the row's values are also written rounded to float32).
    // A long row (lr) takes its norm from the chunk sums of k_long_abs, which
    // also wrote its float32 values.
    const int lane = threadIdx.x % G;
    const int row = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
    if (row >= n) return;
    double s = 0.0;
    const int b = rp[row], e = rp[row + 1];
    if (lr.n > 0 && e - b > lr.lmin) {
        const int t = lr.idx[row];
        for (int c = lr.cb[t] + lane; c < lr.cb[t + 1]; c += G) s += part[c];
    } else {
        for (int q = b + lane; q < e; q += G) {
            const double a = v[q];
            s += fabs(a);
            if (v32) v32[q] = (float)a;
        }
    }
    s = group_sum<G>(s);
    if (lane == 0) {
        const double d = 1.0 / s;
        dinv[row] = d;
        if (dinv32) dinv32[row] = (float)d;
    }
}

// Sliced ELL: width of slice s (times 64) = 64 * max row length over its rows.
// A slice of width at most 64 is uniform when every row's column offsets
// (col - row, ascending) are a subsequence of those of its first full-width
// row, the template: uni[s] = 1; the slots of the slices that are not add up in
// *mixed.  The template's offsets are staged in LDS and each row's are loaded
// eight at a time, so the comparison waits on few memory round trips.
__global__ void __launch_bounds__(kBlock)
k_sell_width(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
             int *__restrict__ cnt, int *__restrict__ uni, int *__restrict__ maxoff, int *__restrict__ inexact,
             int *__restrict__ mixed) {
    // one wave per slice (lane l on row 64 s + l), waves striding over slices;
    // the largest offset is reduced per block, then one atomic per block
    static_assert(kBlock % kSlice == 0, "a block must hold whole slices");
    constexpr int kWaves = kBlock / kSlice;
    __shared__ int red[kWaves], redx[kWaves], redm[kWaves];
    __shared__ int tmpl[kWaves][kSlice];
    const int ns = (n + kSlice - 1) / kSlice;
    const int lane = threadIdx.x % kSlice, wv = threadIdx.x / kSlice;
    int off = 0, inx = 0, mix = 0;
    for (int sl = blockIdx.x * kWaves + wv; sl < ns; sl += gridDim.x * kWaves) {
        const int i = sl * kSlice + lane;
        int w = 0, len = -1, q0 = 0;
        if (i < n) {
            q0 = rp[i];
            const int q1 = rp[i + 1];
            w = len = q1 - q0;
            // columns are sorted: the extreme offsets are the first and the last
            if (q1 > q0) off = max(off, max(abs(ci[q0] - i), abs(ci[q1 - 1] - i)));
            for (int q = q0; q < q1; ++q) inx |= (double)(float)v[q] != v[q] ? 1 : 0;
        }
        for (int o = kSlice / 2; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, kSlice));
        const int t = __ffsll((unsigned long long)__ballot(len == w)) - 1;
        const int it = sl * kSlice + t, qt = rp[it];
        int *T = tmpl[wv];
        if (lane < w) T[lane] = ci[qt + lane] - it;
        wave_sync();
        int ok = w <= kSlice ? 1 : 0;
        if (i < n && ok) {
            // merge walk: each offset of this row must appear in the template, in order
            int k = 0;
            for (int j0 = 0; j0 < len && ok; j0 += 8) {
                int o[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) o[u] = j0 + u < len ? ci[q0 + j0 + u] - i : 0;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (j0 + u >= len || !ok) continue;
                    while (k < w && T[k] != o[u]) ++k;
                    if (k == w) ok = 0;
                    ++k;
                }
            }
        }
        wave_sync();  // the template slots are rewritten by this wave's next slice
        const bool u = __ballot(!ok) == 0;
        if (lane == 0) {
            cnt[sl] = w * kSlice;
            uni[sl] = u ? 1 : 0;
            if (!u) mix += w * kSlice;
        }
    }
    for (int o = kSlice / 2; o > 0; o >>= 1) {
        off = max(off, __shfl_xor(off, o, kSlice));
        inx |= __shfl_xor(inx, o, kSlice);
    }
    if (lane == 0) { red[wv] = off; redx[wv] = inx; redm[wv] = mix; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = red[0], x = redx[0], mx = redm[0];
        for (int k = 1; k < kWaves; ++k) { m = max(m, red[k]); x |= redx[k]; mx += redm[k]; }
        atomicMax(maxoff, m);
        if (x) atomicMax(inexact, 1);
        if (mx) atomicAdd(mixed, mx);
    }
}

// One thread per row writes its entries in column-major slot order.  Slices
// that are not uniform (or without su): CSR order, then padding slots with
// (col = row, value = 0).  Uniform slices: the template's offsets go to su and
// each entry to the slot of its offset; the other slots get value 0 and the
// template's column, clamped to the row itself where it would leave the matrix
// (the column the uniform read takes too).
__global__ void __launch_bounds__(kBlock)
k_sell_fill(int n, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
            const int *__restrict__ sp, const int *__restrict__ uni, int *__restrict__ su, int *__restrict__ sc,
            short *__restrict__ sd, double *__restrict__ sv, float *__restrict__ sv32) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int sl = i / kSlice, lane = i % kSlice;
    if (sl * kSlice >= n) return;  // (whole waves past the last slice)
    const int base = sp[sl] + lane, w = (sp[sl + 1] - sp[sl]) / kSlice;
    auto put = [&](int k, int col, double val) {
        if (sd) sd[base + k * kSlice] = (short)(col - i);
        else sc[base + k * kSlice] = col;
        if (sv) sv[base + k * kSlice] = val;
        if (sv32) sv32[base + k * kSlice] = (float)val;
    };
    if (su && uni[sl]) {
        if (i >= n) return;
        const int q0 = rp[i], len = rp[i + 1] - q0;
        // the slice's template: its first row of full width (rows past n are
        // inactive); uniform slices have w <= 64
        __shared__ int tmpl[kBlock / kSlice][kSlice];
        const int t = __ffsll((unsigned long long)__ballot(len == w)) - 1;
        const int it = sl * kSlice + t, qt = rp[it];
        int *T = tmpl[(threadIdx.x % kBlock) / kSlice];
        if (lane == t) {  // the template row is always active; the slice's last rows may not be
            int *u = su + sp[sl] / kSlice;
            for (int k = 0; k < w; ++k) {
                const int o = ci[qt + k] - it;
                u[k] = o;
                T[k] = o;
            }
        }
        wave_sync();
        int k = 0;
        for (int j0 = 0; j0 < len; j0 += 8) {
            int c[8];
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                c[u] = j0 + u < len ? ci[q0 + j0 + u] : i;
                a[u] = j0 + u < len ? v[q0 + j0 + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (j0 + u >= len) continue;
                // slots before this entry's offset hold zeros (the offset is in
                // the template: the slice was checked uniform with the same one)
                for (; k < w && T[k] != c[u] - i; ++k) {
                    int col = i + T[k];
                    if ((unsigned)col >= (unsigned)n) col = i;
                    put(k, col, 0.0);
                }
                if (k < w) put(k++, c[u], a[u]);
            }
        }
        for (; k < w; ++k) {
            int col = i + T[k];
            if ((unsigned)col >= (unsigned)n) col = i;
            put(k, col, 0.0);
        }
        return;
    }
    // Other slices: CSR order, then padding slots (col = row, value 0).  The
    // slots go KC at a time through LDS: eight lanes per row load KC
    // consecutive entries of that row (a contiguous access per row, eight rows
    // per pass), then every lane writes its own row's KC slots (a contiguous
    // access per slot).  Every lane of the wave takes part in the loads.
    constexpr int KC = 8, RP = kSlice / KC;  // rows per pass
    __shared__ int tci[kBlock / kSlice][kSlice][KC + 1];
    __shared__ double tva[kBlock / kSlice][kSlice][KC + 1];
    const int wv = (threadIdx.x % kBlock) / kSlice, c = lane % KC;
    int qr[KC], lr[KC];
#pragma unroll
    for (int ps = 0; ps < KC; ++ps) {
        const int ir = sl * kSlice + ps * RP + lane / KC;
        qr[ps] = ir < n ? rp[ir] : 0;
        lr[ps] = ir < n ? rp[ir + 1] - qr[ps] : 0;
    }
    for (int k0 = 0; k0 < w; k0 += KC) {
#pragma unroll
        for (int ps = 0; ps < KC; ++ps) {
            const int r = ps * RP + lane / KC;
            const bool in = k0 + c < lr[ps];
            tci[wv][r][c] = in ? ci[qr[ps] + k0 + c] : sl * kSlice + r;
            tva[wv][r][c] = in ? v[qr[ps] + k0 + c] : 0.0;
        }
        wave_sync();
        if (i < n)
            for (int cc = 0; cc < KC && k0 + cc < w; ++cc) put(k0 + cc, tci[wv][lane][cc], tva[wv][lane][cc]);
        wave_sync();  // the tile is refilled by the next step
    }
}

// The finest level's sliced-ELL values scaled by the inverse l1 diagonal of
// their columns, svd = sv32 * dinv32[col] in float32, for the FP32 cycle's
// down-leg residual b - (A D) b.  One thread per row lane of a slice; columns
// as the row kernels read them (uniform offsets clamped to the row itself,
// int16 offsets, or int32 columns).  Padding slots hold 0 and stay 0.
__global__ void __launch_bounds__(kBlock)
k_sell_scale_cols(int n, int nslices, const int *__restrict__ sp, const int *__restrict__ uni,
                  const int *__restrict__ su, const int *__restrict__ sc, const short *__restrict__ sd,
                  const float *__restrict__ sv32, const float *__restrict__ dinv32, float *__restrict__ svd) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int sl = t / kSlice, lane = t % kSlice;
    if (sl >= nslices) return;
    const int i = sl * kSlice + lane, beg = sp[sl], w = (sp[sl + 1] - beg) / kSlice;
    const bool uf = su && uni[sl];
    for (int k = 0; k < w; ++k) {
        const int q = beg + k * kSlice + lane;
        if (i >= n) {
            svd[q] = 0.0f;
            continue;
        }
        int col;
        if (uf) {
            const int cc = i + su[beg / kSlice + k];
            col = (unsigned)cc < (unsigned)n ? cc : i;
        } else {
            col = sd ? i + (int)sd[q] : sc[q];
        }
        svd[q] = sv32[q] * dinv32[col];
    }
}

__global__ void k_cast(size_t n, const double *__restrict__ src, float *__restrict__ dst) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

__global__ void k_copy_f64(size_t n, const double *__restrict__ src, double *__restrict__ dst) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_fill_i32(size_t n, int *__restrict__ dst, int val) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = val;
}

__global__ void k_fill_u64(size_t n, unsigned long long *__restrict__ dst, unsigned long long val) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = val;
}

// ============================================================================
// Long segments: rows longer than the level's bound, and Galerkin coarse rows
// with more candidates than that.  Their entries are processed in parallel
// across workgroups, and the orderings the per-row kernels form in a group's
// LDS (own-row ranks, the Suitor preference order, the distinct columns of a
// coarse row) come from a segmented sort: every chunk of kSegChunk keys is
// sorted in one workgroup's LDS, then runs are merged pairwise, each key
// placed by one binary search in the partner run.
// ============================================================================
constexpr int kSegBlock = 1024;  // threads of the one-workgroup kernels below

// largest t in [0, cnt) with base[t] <= x (base strictly ascending, base[0] = 0)
__device__ __forceinline__ int seg_of(const int *__restrict__ base, int cnt, int x) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// first index k < cnt with keys[k] > key (keys ascending)
__device__ __forceinline__ int upper_bound_u64(const unsigned long long *keys, int cnt, unsigned long long key) {
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// exclusive scan over a workgroup of kSegBlock threads; *total gets the sum
__device__ __forceinline__ int seg_block_excl(int x, int *total) {
    __shared__ int wsum[kSegBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < kSegBlock / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + inc - x;
}

// Offsets and first chunks of the segments found, in the order found.
__global__ void __launch_bounds__(kSegBlock) k_seg_fix(SegList sg) {
    const int found = sg.ctl[0];
    const int cnt = min(found, sg.cap);
    int carry_l = 0, carry_c = 0, mx = 0;
    for (int b0 = 0; b0 < cnt; b0 += kSegBlock) {
        const int t = b0 + threadIdx.x;
        const int l = t < cnt ? sg.len[t] : 0;
        const int ch = (l + kSegChunk - 1) / kSegChunk;
        mx = max(mx, l);
        int tl, tc;
        const int el = seg_block_excl(l, &tl);
        const int ec = seg_block_excl(ch, &tc);
        if (t < cnt) {
            sg.off[t] = carry_l + el;
            sg.cb[t] = carry_c + ec;
        }
        carry_l += tl;
        carry_c += tc;
    }
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    __shared__ int wmax[kSegBlock / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kSegBlock / 64; ++w) mx = max(mx, wmax[w]);
        sg.off[cnt] = carry_l;
        sg.cb[cnt] = carry_c;
        sg.ctl[0] = cnt;
        sg.ctl[1] = carry_l;
        sg.ctl[2] = carry_c;
        sg.ctl[3] = mx;
        sg.ctl[4] = found > sg.cap ? 1 : 0;
    }
}

// Rows of (n, rp) longer than lmin; idx[i] = position in the list or -1.
__global__ void __launch_bounds__(kBlock)
k_find_long(int n, const int *__restrict__ rp, int lmin, SegList sg, int *__restrict__ idx) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int d = rp[i + 1] - rp[i];
    int t = -1;
    if (d > lmin) {
        t = atomicAdd(&sg.ctl[0], 1);
        if (t < sg.cap) {
            sg.row[t] = i;
            sg.len[t] = d;
        } else {
            t = -1;
        }
    }
    if (idx) idx[i] = t;
}

// Coarse rows E of a pairwise sweep whose member rows hold more than lmin
// entries together (the candidates of E's Galerkin row).
__global__ void __launch_bounds__(kBlock)
k_find_long_gal(int nc, const int *__restrict__ mem2, const int *__restrict__ rp, int lmin, SegList sg) {
    const int E = blockIdx.x * kBlock + threadIdx.x;
    if (E >= nc) return;
    const int e0 = mem2[2 * E], e1 = mem2[2 * E + 1];
    const int L = (rp[e0 + 1] - rp[e0]) + (e1 >= 0 ? rp[e1 + 1] - rp[e1] : 0);
    if (L > lmin) seg_append(sg, E, L);
}

// Every entry of every segment, in a grid-stride loop: body(t, k, row).
template <typename Body>
__device__ __forceinline__ void for_seg_entries(const SegList &sg, Body body) {
    const int cnt = sg.ctl[0], tot = sg.ctl[1];
    for (int g = blockIdx.x * kBlock + threadIdx.x; g < tot; g += gridDim.x * kBlock) {
        const int t = seg_of(sg.off, cnt, g);
        body(t, g - sg.off[t], sg.row[t]);
    }
}

// Per-entry checks of the long rows (the part of k_validate they skipped).
__global__ void __launch_bounds__(kBlock)
k_long_validate(int n, int nnz, const int *__restrict__ rp, const int *__restrict__ ci,
                const double *__restrict__ v, int check_sym, SegList sg, int *__restrict__ flags) {
    int f = 0;
    for_seg_entries(sg, [&](int, int k, int row) {
        const int q = rp[row] + k;
        const int j = ci[q];
        const double a = v[q];
        if (j < 0 || j >= n) { f |= kErrCol; return; }
        if (k > 0 && ci[q - 1] >= j) f |= kErrUnsorted;
        if (!isfinite(a)) f |= kErrNonFinite;
        if (check_sym && j != row) {
            const int s2 = rp[j], e2 = rp[j + 1];
            int found = -1;
            if (s2 >= 0 && e2 >= s2 && (nnz < 0 || e2 <= nnz)) {
                int lo = s2, hi = e2 - 1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    const int cm = ci[mid];
                    if (cm == row) { found = mid; break; }
                    if (cm < row) lo = mid + 1; else hi = mid - 1;
                }
            }
            if (found < 0 || __double_as_longlong(v[found]) != __double_as_longlong(a)) f |= kErrAsym;
        }
    });
    if (f) atomicOr(flags, f);
}

__global__ void __launch_bounds__(kBlock)
k_long_weights(SegList sg, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
               const double *__restrict__ diag, const double *__restrict__ w, double *__restrict__ c) {
    for_seg_entries(sg, [&](int, int k, int row) {
        const int q = rp[row] + k;
        c[q] = edge_weight(row, ci[q], v[q], diag, w);
    });
}

// Sort keys of the segmented sorts.  Own-row ranks: the weight's order key.
struct KeyRank {
    const int *rp;
    const double *c;
    __device__ unsigned long long operator()(int row, int, int k) const { return order_key(c[rp[row] + k]); }
};
// Suitor preference order of a row u: eligible entries by (own-row rank
// desc, neighbour desc) -- the order k_candidates sorts -- then the others.
struct KeyCand {
    const int *rp, *ci;
    const double *c;
    const unsigned *rk;
    __device__ unsigned long long operator()(int row, int, int k) const {
        const int q = rp[row] + k, vtx = ci[q];
        const double cq = c[q];
        if (vtx != row && cq > 0.0 && cq < INFINITY)
            return ((unsigned long long)(0x7fffffffu - rk[q]) << 32) | (0x7fffffffu - (unsigned)vtx);
        return 0xffffffff00000000ull | (unsigned)k;
    }
};
// Galerkin coarse row E: candidate k (an entry of E's member rows) keyed by
// its coarse column, then k.
struct KeyGal {
    const int *rp, *ci, *agg, *mem2;
    __device__ unsigned long long operator()(int E, int, int k) const {
        const int e0 = mem2[2 * E], s0 = rp[e0], L0 = rp[e0 + 1] - s0;
        const int q = k < L0 ? s0 + k : rp[mem2[2 * E + 1]] + (k - L0);
        return ((unsigned long long)(unsigned)agg[ci[q]] << 32) | (unsigned)k;
    }
};

// Sorts every chunk of kSegChunk keys of every segment in LDS (bitonic
// network over the whole chunk, ~0 padding), writing them to out at the
// segment's offset.  One compare-exchange per thread and stage (kSegChunk / 2
// threads).  A stage of stride <= 64 pairs keys inside one wave's 128-key
// block (the wave's 64 threads cover exactly that block), so only the stages
// of longer strides wait for the whole workgroup; the others order the LDS
// accesses of one wave.
constexpr int kSortThreads = kSegChunk / 2;
template <typename Key>
__global__ void __launch_bounds__(kSortThreads)
k_seg_sort_chunks(SegList sg, Key key, unsigned long long *__restrict__ out) {
    static_assert((kSegChunk & (kSegChunk - 1)) == 0 && kSortThreads % 64 == 0, "power-of-two chunk");
    __shared__ unsigned long long keys[kSegChunk];
    const int cnt = sg.ctl[0], nch = sg.ctl[2];
    const int u = threadIdx.x;
    constexpr int LOG = __builtin_ctz(kSegChunk);
    for (int ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const int t = seg_of(sg.cb, cnt, ch);
        const int L = sg.len[t], k0 = (ch - sg.cb[t]) * kSegChunk, m = min(kSegChunk, L - k0);
        const int row = sg.row[t];
        const unsigned long long a0 = u < m ? key(row, L, k0 + u) : ~0ull;
        const unsigned long long a1 = u + kSortThreads < m ? key(row, L, k0 + u + kSortThreads) : ~0ull;
        keys[u] = a0;
        keys[u + kSortThreads] = a1;
        __syncthreads();
        for (int ls = 1; ls <= LOG; ++ls) {         // sorted runs of 2^ls keys
            for (int lt = ls - 1; lt >= 0; --lt) {  // stride 2^lt
                const int lo = ((u >> lt) << (lt + 1)) | (u & ((1 << lt) - 1)), hi = lo + (1 << lt);
                const bool up = ((lo >> ls) & 1) == 0;
                const unsigned long long a = keys[lo], b = keys[hi];
                if ((a > b) == up) {
                    keys[lo] = b;
                    keys[hi] = a;
                }
                // the next stage pairs keys of other waves: stride >= 128 (this
                // stage's, or the next size's first one after stride 1)
                if (lt > 6 || (lt == 0 && ls >= 7 && ls < LOG)) __syncthreads();
                else wave_sync();
            }
        }
        __syncthreads();
        unsigned long long *dst = out + sg.off[t] + k0;
        if (u < m) dst[u] = keys[u];
        if (u + kSortThreads < m) dst[u + kSortThreads] = keys[u + kSortThreads];
        __syncthreads();
    }
}

// One merge pass: sorted runs of `run` keys become runs of 2 run.  A key of a
// left run goes before the equal keys of its right partner (stable), so equal
// keys keep their chunk order.
__global__ void __launch_bounds__(kBlock)
k_seg_merge(SegList sg, int run, const unsigned long long *__restrict__ in, unsigned long long *__restrict__ out) {
    const int cnt = sg.ctl[0], tot = sg.ctl[1];
    for (int g = blockIdx.x * kBlock + threadIdx.x; g < tot; g += gridDim.x * kBlock) {
        const int t = seg_of(sg.off, cnt, g);
        const int k = g - sg.off[t], L = sg.len[t];
        const unsigned long long *seg = in + sg.off[t];
        const unsigned long long key = seg[k];
        const int r = k / run, base = (r & ~1) * run;
        int pos;
        if ((r & 1) == 0) {
            const int b0 = base + run, b1 = min(base + 2 * run, L);
            pos = b0 >= L ? k : k + lower_bound_u64(seg + b0, b1 - b0, key);
        } else {
            pos = k - run + upper_bound_u64(seg + base, run, key);
        }
        out[sg.off[t] + pos] = key;
    }
}

// Own-row ranks of the long rows: rk[q] = #{t in the row : c[t] < c[q]}, the
// first position of c[q]'s key in the sorted row.
__global__ void __launch_bounds__(kBlock)
k_long_rank(SegList sg, const unsigned long long *__restrict__ sorted, const int *__restrict__ rp,
            const double *__restrict__ c, unsigned *__restrict__ rk) {
    for_seg_entries(sg, [&](int t, int k, int row) {
        const int q = rp[row] + k;
        rk[q] = (unsigned)lower_bound_u64(sorted + sg.off[t], sg.len[t], order_key(c[q]));
    });
}

// Candidate lists of the long rows (the output k_candidates gives other rows):
// each entry's key is found in the sorted row, which gives its slot.  The
// rank of c_uv seen from v: from rk at the transposed position (every row in
// the sorted family; long rows in the direct one), else counted over row v.
__global__ void __launch_bounds__(kBlock)
k_long_cand(SegList sg, const unsigned long long *__restrict__ sorted, const int *__restrict__ rp,
            const int *__restrict__ ci, const double *__restrict__ c, const unsigned *__restrict__ rk, int lmin,
            int direct, unsigned long long *__restrict__ cand) {
    const KeyCand kc{rp, ci, c, rk};
    for_seg_entries(sg, [&](int t, int k, int row) {
        const unsigned long long key = kc(row, 0, k);
        const int pos = lower_bound_u64(sorted + sg.off[t], sg.len[t], key);
        const int q = rp[row] + k, vtx = ci[q];
        unsigned long long out = ~0ull;
        if ((key >> 32) != 0xffffffffull) {
            const double cq = c[q];
            const int b2 = rp[vtx], e2 = rp[vtx + 1];
            unsigned r = 0;
            if (!direct || e2 - b2 > lmin) {
                int lo = b2, hi = e2;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (ci[mid] < row) lo = mid + 1; else hi = mid;
                }
                r = (lo < e2 && ci[lo] == row) ? rk[lo] : 0u;
            } else {
                for (int u = b2; u < e2; ++u) r += (c[u] < cq) ? 1u : 0u;
            }
            out = ((unsigned long long)r << 32) | (unsigned)vtx;
        }
        cand[rp[row] + pos] = out;
    });
}

// Galerkin coarse rows with many candidates, over their sorted candidate keys
// (column << 32 | candidate), one workgroup per chunk of kSegChunk keys: a
// column starts where the key's column differs from the previous key's.
// Pass 0 stores the chunk's column starts in cc[chunk] and adds them to the
// row's count (zeroed by the count pass of k_gal); pass 1 numbers them from
// the row's first entry plus the starts of the row's earlier chunks and writes
// each entry, its (at most four) terms summed in canonical (m, M) order as
// k_gal.  A column's run of keys may continue into the next chunk: its start
// owns it.
__global__ void __launch_bounds__(kSegBlock)
k_gal_long(int pass, SegList sg, const unsigned long long *__restrict__ sorted, const int *__restrict__ rp,
           const int *__restrict__ ci, const double *__restrict__ v, const int *__restrict__ agg,
           const double *__restrict__ p, const int *__restrict__ mem2, int *__restrict__ cnt,
           int *__restrict__ cc, const int *__restrict__ crp, int *__restrict__ cci, double *__restrict__ cv) {
    constexpr int PER = kSegChunk / kSegBlock;  // keys per thread
    const int nseg = sg.ctl[0], nch = sg.ctl[2];
    for (int ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const int t = seg_of(sg.cb, nseg, ch);
        const int E = sg.row[t], L = sg.len[t];
        const unsigned long long *keys = sorted + sg.off[t];
        const int k0 = min((ch - sg.cb[t]) * kSegChunk + (int)threadIdx.x * PER, L);
        // the thread's keys and the one before them, all loaded first
        int col[PER + 1];
        col[0] = k0 > 0 ? (int)(keys[k0 - 1] >> 32) : -1;
#pragma unroll
        for (int r = 0; r < PER; ++r) col[r + 1] = k0 + r < L ? (int)(keys[k0 + r] >> 32) : -1;
        int mine = 0;
#pragma unroll
        for (int r = 0; r < PER; ++r) mine += (k0 + r < L && (k0 + r == 0 || col[r + 1] != col[r])) ? 1 : 0;
        int total;
        int rank = seg_block_excl(mine, &total);
        if (pass == 0) {
            if (threadIdx.x == 0) {
                cc[ch] = total;
                atomicAdd(&cnt[E], total);
            }
            continue;
        }
        int before = 0;
        for (int c = sg.cb[t] + (int)threadIdx.x; c < ch; c += kSegBlock) before += cc[c];
        int btot;
        (void)seg_block_excl(before, &btot);
        const int e0 = mem2[2 * E], e1 = mem2[2 * E + 1];
        const int s0 = rp[e0], L0 = rp[e0 + 1] - s0;
        const int s1 = e1 >= 0 ? rp[e1] : 0;
        const int base = crp[E] + btot;
        const unsigned long long NONE = ~0ull;
#pragma unroll
        for (int r0 = 0; r0 < PER; ++r0) {
            const int k = k0 + r0;
            if (!(k < L && (k == 0 || col[r0 + 1] != col[r0]))) continue;
            const int f = col[r0 + 1];
            // the run's keys k .. k + 3 (a column has at most four candidates)
            unsigned long long kk[4];
            double tt[4];
            int cidx[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const unsigned long long key = k + r < L ? keys[k + r] : NONE;
                cidx[r] = (key != NONE && (int)(key >> 32) == f) ? (int)(key & 0xffffffffull) : -1;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                kk[r] = NONE;
                tt[r] = 0.0;
                if (cidx[r] < 0) continue;
                const int q = cidx[r] < L0 ? s0 + cidx[r] : s1 + (cidx[r] - L0);
                const int i = cidx[r] < L0 ? e0 : e1, j = ci[q];
                const int m = min(i, j), M = max(i, j);
                kk[r] = ((unsigned long long)(unsigned)m << 32) | (unsigned)M;
                tt[r] = (p[m] * v[q]) * p[M];
            }
            cswap(kk[0], tt[0], kk[1], tt[1]);
            cswap(kk[2], tt[2], kk[3], tt[3]);
            cswap(kk[0], tt[0], kk[2], tt[2]);
            cswap(kk[1], tt[1], kk[3], tt[3]);
            cswap(kk[1], tt[1], kk[2], tt[2]);
            double sum = tt[0];
#pragma unroll
            for (int r = 1; r < 4; ++r)
                if (kk[r] != NONE) sum = sum + tt[r];
            cci[base + rank] = f;
            cv[base + rank] = sum;
            ++rank;
        }
        __syncthreads();
    }
}

// l1 norms of the long rows of a level: chunk c sums |a_q| over its kSegChunk
// entries (eight per thread, then the workgroup in a fixed order).
__global__ void __launch_bounds__(kBlock)
k_long_abs(LongRows lr, const int *__restrict__ rp, const double *__restrict__ v, double *__restrict__ part,
           float *__restrict__ v32) {
    const int c = blockIdx.x;
    const int t = seg_of(lr.cb, lr.n, c);
    const int row = lr.rows[t];
    const int q0 = rp[row] + (c - lr.cb[t]) * kSegChunk, q1 = min(q0 + kSegChunk, rp[row + 1]);
    double s[1] = {0.0};
    for (int q = q0 + threadIdx.x; q < q1; q += kBlock) {
        const double a = v[q];
        s[0] += fabs(a);
        if (v32) v32[q] = (float)a;
    }
    __shared__ double lds[16];
    block_sum<1>(s, lds);
    if (threadIdx.x == 0) part[c] = s[0];
}

inline int stream_grid(size_t n) {
    size_t b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int pick_G(double avg) {
    int G = 4;
    while (G < 64 && G < avg) G <<= 1;
    return G;
}

void launch_validate(hipStream_t s, int G, int n, int nnz, const int *rp, const int *ci,
                     const double *v, const double *w, int check_sym, double *diag, int *flags,
                     const SegList &seg, int lmin, int *dmax) {
    with_G(G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL(k_validate<g>, dim3(blocks_for((long long)n * g)), dim3(kBlock), 0, s, n, nnz,
                           rp, ci, v, w, check_sym, diag, flags, seg, lmin, dmax);
    });
}

void launch_weights(hipStream_t s, int G, int n, const int *rp, const int *ci, const double *v, const double *diag,
                    const double *w, double *c, unsigned long long *ws, int lmin) {
    with_G(G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL(k_weights<g>, dim3(blocks_for((long long)n * g)), dim3(kBlock), 0, s, n, rp, ci,
                           v, diag, w, c, ws, lmin);
    });
}

// Rows of a few dozen entries compare directly; longer rows sort (k_rank +
// k_candidates: O(d log d) per row instead of O(d^2)).  part: 0 = all, 1 =
// the own-row ranks only (sorted), 2 = the candidate lists only.
void launch_candidates(hipStream_t s, int G, int n, bool sorted, const int *rp, const int *ci, const double *c,
                       unsigned *rk, unsigned long long *cand, int lmin, int part) {
    with_G(G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (!sorted) {
            if (part != 1)
                hipLaunchKernelGGL(k_candidates_direct<g>, dim3(blocks_for((long long)n * g)), dim3(kBlock), 0, s, n,
                                   rp, ci, c, rk, cand, lmin);
            return;
        }
        if (part != 2)
            hipLaunchKernelGGL(k_rank<g>, dim3(blocks_for((long long)n * g)), dim3(kBlock), 0, s, n, rp, c, rk, lmin);
        if (part != 1)
            hipLaunchKernelGGL(k_candidates<g>, dim3(blocks_for((long long)n * g)), dim3(kBlock), 0, s, n, rp, ci, c,
                               rk, cand, lmin);
    });
}

void launch_suitor(hipStream_t s, int n, const int *rp, const unsigned long long *cand, unsigned long long *ws) {
    launch_k(k_suitor, dim3(blocks_for(n)), dim3(kBlock), s, n, rp, cand, ws);
}

void launch_mate(hipStream_t s, int n, const int *rp, const int *ci, const unsigned long long *ws, int *mate,
                 int *leader, const int *csrc, int *cdst) {
    hipLaunchKernelGGL(k_mate, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, rp, ci, ws, mate, leader, csrc, cdst);
}

void launch_aggfill(hipStream_t s, int n, const int *mate, const int *ofs, const double *w, int *agg,
                    double *p, double *wc, int *mem2) {
    hipLaunchKernelGGL(k_aggfill, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, mate, ofs, w, agg, p, wc, mem2);
}

// Rows with at most 4 G candidates: each candidate's column F, key (m, M) and
// term (p_m a_ij) p_M are formed once, with all loads of the row in flight
// together, and kept in LDS; the distinct columns, their ranks and their (at
// most four) terms are then found by comparing LDS entries only.  Longer rows
// take gal_row's scratch path.
template <int G>
__global__ void __launch_bounds__(kBlock)
k_gal(int pass, int nc, const int *__restrict__ rp, const int *__restrict__ ci,
      const double *__restrict__ v, const int *__restrict__ agg, const double *__restrict__ p,
      const int *__restrict__ mem2, int *__restrict__ cnt, const int *__restrict__ crp,
      int *__restrict__ cci, double *__restrict__ cv, int *__restrict__ gF, int *__restrict__ gU, int lmin) {
    constexpr int SL = 4;  // candidate slots per lane
    constexpr int LS = SL * G;
    constexpr int NG = kBlock / G;
    // groups' slots one element apart (stride LS + 1): the groups of a wave
    // reading the same slot index hit different LDS banks
    constexpr int LSP = LS + 1;
    __shared__ int sf[NG * LSP];
    __shared__ int sfirst[NG * LSP];
    __shared__ unsigned long long skey[NG * LSP];
    __shared__ double st[NG * LSP];
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int E = xcd_block(blockIdx.x, gridDim.x) * NG + g;
    if (E >= nc) return;
    const int e0 = mem2[2 * E], e1 = mem2[2 * E + 1];
    const int s0 = rp[e0], L0 = rp[e0 + 1] - s0;
    const int s1 = e1 >= 0 ? rp[e1] : 0;
    const int L1 = e1 >= 0 ? rp[e1 + 1] - s1 : 0;
    const int L = L0 + L1;
    if (lmin > 0 && L > lmin) {  // a long coarse row: k_gal_long adds its count
        if (pass == 0 && lane == 0) cnt[E] = 0;
        return;
    }
    if (L > LS) {
        gal_row<G>(pass, E, lane, rp, ci, v, agg, p, e0, e1, s0, L0, s1, L1, cnt, crp, cci, cv, gF, gU, false);
        return;
    }
    int *F = sf + g * LSP, *first = sfirst + g * LSP;
    unsigned long long *K = skey + g * LSP;
    double *T = st + g * LSP;
    const double pe0 = pass ? p[e0] : 0.0, pe1 = (pass && e1 >= 0) ? p[e1] : 0.0;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
        const int k = lane + sl * G;
        if (k >= L) continue;
        const int q = k < L0 ? s0 + k : s1 + (k - L0);
        const int j = ci[q];
        F[k] = agg[j];
        if (pass) {
            const int i = k < L0 ? e0 : e1;
            const double pi = k < L0 ? pe0 : pe1, pj = p[j], a = v[q];
            const bool ilo = i <= j;
            K[k] = ((unsigned long long)(unsigned)(ilo ? i : j) << 32) | (unsigned)(ilo ? j : i);
            T[k] = ((ilo ? pi : pj) * a) * (ilo ? pj : pi);
        }
    }
    wave_sync();
    // first occurrence of each column among the candidates; first[k] holds the
    // column and that flag together, (F << 1) | flag, so the rank loop below
    // reads one word per candidate
    int nu = 0;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
        const int k = lane + sl * G;
        if (k >= L) continue;
        const int f = F[k];
        int fk = 1;
        for (int k2 = 0; k2 < k; ++k2) fk = (F[k2] == f) ? 0 : fk;
        first[k] = (f << 1) | fk;
        nu += fk;
    }
    if (pass == 0) {
        nu = group_sum<G>(nu);
        if (lane == 0) cnt[E] = nu;
        return;
    }
    wave_sync();
    const int base = crp[E];
    const unsigned long long NONE = ~0ull;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
        const int k = lane + sl * G;
        if (k >= L || !(first[k] & 1)) continue;
        const int f = F[k];
        // rank among the distinct columns; the (at most four) candidates of
        // column f in candidate order, their terms loaded after the scan
        int rank = 0, c0 = -1, c1 = -1, c2 = -1, c3 = -1;
        for (int k2 = 0; k2 < L; ++k2) {
            const int pf = first[k2], f2 = pf >> 1;
            rank += ((pf & 1) && f2 < f) ? 1 : 0;
            if (f2 == f) {
                if (c0 < 0) c0 = k2;
                else if (c1 < 0) c1 = k2;
                else if (c2 < 0) c2 = k2;
                else if (c3 < 0) c3 = k2;
            }
        }
        const int cs[4] = {c0, c1, c2, c3};
        unsigned long long key[4];
        double t[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            key[r] = cs[r] >= 0 ? K[max(cs[r], 0)] : NONE;
            t[r] = cs[r] >= 0 ? T[max(cs[r], 0)] : 0.0;
        }
        cswap(key[0], t[0], key[1], t[1]);
        cswap(key[2], t[2], key[3], t[3]);
        cswap(key[0], t[0], key[2], t[2]);
        cswap(key[1], t[1], key[3], t[3]);
        cswap(key[1], t[1], key[2], t[2]);
        double sum = t[0];
#pragma unroll
        for (int r = 1; r < 4; ++r)
            if (key[r] != NONE) sum = sum + t[r];
        cci[base + rank] = f;
        cv[base + rank] = sum;
    }
}

// Galerkin product for long rows: the same entries and sums as k_gal, with the
// candidate columns of a coarse row sorted in LDS as (F << 32 | candidate)
// instead of compared pairwise.  Equal columns are then adjacent (at most four
// candidates each), the distinct columns come out in ascending order, and a
// scan over the group's lanes gives each column its position in the row.
// Rows with more candidates than the LDS slots use k_gal's scratch path.
template <int G>
__global__ void __launch_bounds__(kBlock)
k_gal_sorted(int pass, int nc, const int *__restrict__ rp, const int *__restrict__ ci,
             const double *__restrict__ v, const int *__restrict__ agg, const double *__restrict__ p,
             const int *__restrict__ mem2, int *__restrict__ cnt, const int *__restrict__ crp,
             int *__restrict__ cci, double *__restrict__ cv, int *__restrict__ gF, int *__restrict__ gU, int lmin) {
    constexpr int LMAX = 16 * G;
    constexpr int NG = kBlock / G;
    __shared__ unsigned long long sk[NG * (LMAX + 1)];  // groups one element apart: distinct banks
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int E = xcd_block(blockIdx.x, gridDim.x) * NG + g;
    if (E >= nc) return;
    const int e0 = mem2[2 * E], e1 = mem2[2 * E + 1];
    const int s0 = rp[e0], L0 = rp[e0 + 1] - s0;
    const int s1 = e1 >= 0 ? rp[e1] : 0;
    const int L1 = e1 >= 0 ? rp[e1 + 1] - s1 : 0;
    const int L = L0 + L1;
    if (lmin > 0 && L > lmin) {  // a long coarse row: k_gal_long adds its count
        if (pass == 0 && lane == 0) cnt[E] = 0;
        return;
    }
    if (L > LMAX) {  // more candidates than LDS slots: k_gal's scratch path
        gal_row<G>(pass, E, lane, rp, ci, v, agg, p, e0, e1, s0, L0, s1, L1, cnt, crp, cci, cv, gF, gU, false);
        return;
    }
    unsigned long long *keys = sk + g * (LMAX + 1);
    const int P = pow2_at_least(L);
    for (int k = lane; k < P; k += G) {
        unsigned long long key = ~0ull;
        if (k < L) {
            const int q = k < L0 ? s0 + k : s1 + (k - L0);
            key = ((unsigned long long)(unsigned)agg[ci[q]] << 32) | (unsigned)k;
        }
        keys[k] = key;
    }
    wave_sync();
    group_sort<G>(keys, P, lane);
    auto col = [&](int k) { return (int)(keys[k] >> 32); };
    auto starts = [&](int k) { return k < L && (k == 0 || col(k) != col(k - 1)); };
    // contiguous chunk of sorted positions per lane; exclusive scan of segment starts
    const int C = (L + G - 1) / G;
    const int k0 = min(lane * C, L), k1 = min(k0 + C, L);
    int mine = 0;
    for (int k = k0; k < k1; ++k) mine += starts(k) ? 1 : 0;
    int incl = mine;
    for (int o = 1; o < G; o <<= 1) {
        const int t = __shfl_up(incl, o, G);
        if (lane >= o) incl += t;
    }
    if (pass == 0) {
        if (lane == G - 1) cnt[E] = incl;
        return;
    }
    int rank = incl - mine;
    const int base = crp[E];
    const unsigned long long NONE = ~0ull;
    for (int k = k0; k < k1; ++k) {
        if (!starts(k)) continue;
        const int f = col(k);
        unsigned long long key[4];
        double t[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            key[r] = NONE;
            t[r] = 0.0;
            const int kk = k + r;
            if (kk >= L || col(kk) != f) continue;
            const int cidx = (int)(keys[kk] & 0xffffffffull);
            const int q = cidx < L0 ? s0 + cidx : s1 + (cidx - L0);
            const int i = cidx < L0 ? e0 : e1, j = ci[q];
            const int m = min(i, j), M = max(i, j);
            key[r] = ((unsigned long long)(unsigned)m << 32) | (unsigned)M;
            t[r] = (p[m] * v[q]) * p[M];
        }
        cswap(key[0], t[0], key[1], t[1]);
        cswap(key[2], t[2], key[3], t[3]);
        cswap(key[0], t[0], key[2], t[2]);
        cswap(key[1], t[1], key[3], t[3]);
        cswap(key[1], t[1], key[2], t[2]);
        double sum = t[0];
#pragma unroll
        for (int r = 1; r < 4; ++r)
            if (key[r] != NONE) sum = sum + t[r];
        cci[base + rank] = f;
        cv[base + rank] = sum;
        ++rank;
    }
}

void launch_gal_count(hipStream_t s, int G, int nc, const int *rp, const int *ci, const int *agg,
                      const int *mem2, int *cnt, int *gF, int *gU, bool sorted, int lmin) {
    with_G(G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (sorted)
            hipLaunchKernelGGL(k_gal_sorted<g>, dim3(blocks_for((long long)nc * g)), dim3(kBlock), 0, s, 0, nc, rp, ci,
                               nullptr, agg, nullptr, mem2, cnt, nullptr, nullptr, nullptr, gF, gU, lmin);
        else
            hipLaunchKernelGGL(k_gal<g>, dim3(blocks_for((long long)nc * g)), dim3(kBlock), 0, s, 0, nc, rp, ci,
                               nullptr, agg, nullptr, mem2, cnt, nullptr, nullptr, nullptr, gF, gU, lmin);
    });
}

void launch_gal_fill(hipStream_t s, int G, int nc, const int *rp, const int *ci, const double *v,
                     const int *agg, const double *p, const int *mem2, const int *crp, int *cci,
                     double *cv, int *gF, int *gU, bool sorted, int lmin) {
    with_G(G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (sorted)
            hipLaunchKernelGGL(k_gal_sorted<g>, dim3(blocks_for((long long)nc * g)), dim3(kBlock), 0, s, 1, nc, rp, ci,
                               v, agg, p, mem2, nullptr, crp, cci, cv, gF, gU, lmin);
        else
            hipLaunchKernelGGL(k_gal<g>, dim3(blocks_for((long long)nc * g)), dim3(kBlock), 0, s, 1, nc, rp, ci, v,
                               agg, p, mem2, nullptr, crp, cci, cv, gF, gU, lmin);
    });
}

void launch_compose(hipStream_t s, int n, int nc_new, const int *agg_prev, const double *p_prev,
                    const int *mem_prev, int stride_prev, const int *agg_s, const double *p_s,
                    const int *mem_s, int *agg_out, double *p_out, int *mem_out) {
    hipLaunchKernelGGL(k_compose_rows, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, agg_prev, p_prev, agg_s, p_s,
                       agg_out, p_out);
    hipLaunchKernelGGL(k_compose_members, dim3(blocks_for(nc_new)), dim3(kBlock), 0, s, nc_new, mem_prev,
                       stride_prev, mem_s, mem_out);
}

void launch_diag_l1(hipStream_t s, int G, int n, const int *rp, const double *v, double *dinv,
                    float *dinv32, float *v32, const LongRows &lr, const double *part) {
    with_G(G, [&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hipLaunchKernelGGL(k_diag_l1<g>, dim3(blocks_for((long long)n * g)), dim3(kBlock), 0, s, n, rp, v, dinv,
                           dinv32, v32, lr, part);
    });
}

void launch_sell_width(hipStream_t s, int n, const int *rp, const int *ci, const double *v, int *cnt, int *uni,
                       int *maxoff, int *inexact, int *mixed) {
    const int ns = (n + kSlice - 1) / kSlice;
    const int nb = std::min(blocks_for((long long)ns * kSlice), 512);
    hipLaunchKernelGGL(k_sell_width, dim3(nb), dim3(kBlock), 0, s, n, rp, ci, v, cnt, uni, maxoff, inexact, mixed);
}

void launch_sell_fill(hipStream_t s, int n, const int *rp, const int *ci, const double *v, const int *sp,
                      const int *uni, int *su, int *sc, short *sd, double *sv, float *sv32) {
    hipLaunchKernelGGL(k_sell_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, rp, ci, v, sp, uni, su, sc, sd, sv,
                       sv32);
}

void launch_sell_scale_cols(hipStream_t s, int n, int nslices, const int *sp, const int *uni, const int *su,
                            const int *sc, const short *sd, const float *sv32, const float *dinv32, float *svd) {
    hipLaunchKernelGGL(k_sell_scale_cols, dim3(blocks_for((long long)nslices * kSlice)), dim3(kBlock), 0, s, n,
                       nslices, sp, uni, su, sc, sd, sv32, dinv32, svd);
}

void launch_cast(hipStream_t s, size_t n, const double *src, float *dst) {
    hipLaunchKernelGGL(k_cast, dim3(stream_grid(n)), dim3(kBlock), 0, s, n, src, dst);
}

void launch_copy_f64(hipStream_t s, size_t n, const double *src, double *dst) {
    hipLaunchKernelGGL(k_copy_f64, dim3(stream_grid(n)), dim3(kBlock), 0, s, n, src, dst);
}

void launch_fill_i32(hipStream_t s, size_t n, int *dst, int val) {
    hipLaunchKernelGGL(k_fill_i32, dim3(stream_grid(n)), dim3(kBlock), 0, s, n, dst, val);
}

void launch_fill_u64(hipStream_t s, size_t n, unsigned long long *dst, unsigned long long val) {
    hipLaunchKernelGGL(k_fill_u64, dim3(stream_grid(n)), dim3(kBlock), 0, s, n, dst, val);
}

// Grid of the grid-stride long-segment kernels (their counts are on the device).
constexpr int kSegGrid = 1024;

void launch_find_long(hipStream_t s, int n, const int *rp, int lmin, const SegList &seg, int *idx) {
    hipLaunchKernelGGL(k_find_long, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, rp, lmin, seg, idx);
}

void launch_find_long_gal(hipStream_t s, int nc, const int *mem2, const int *rp, int lmin, const SegList &seg) {
    hipLaunchKernelGGL(k_find_long_gal, dim3(blocks_for(nc)), dim3(kBlock), 0, s, nc, mem2, rp, lmin, seg);
}

void launch_seg_fix(hipStream_t s, const SegList &seg) {
    hipLaunchKernelGGL(k_seg_fix, dim3(1), dim3(kSegBlock), 0, s, seg);
}

void launch_long_validate(hipStream_t s, int n, int nnz, const int *rp, const int *ci, const double *v,
                          int check_sym, const SegList &seg, int *flags) {
    hipLaunchKernelGGL(k_long_validate, dim3(kSegGrid), dim3(kBlock), 0, s, n, nnz, rp, ci, v, check_sym, seg, flags);
}

void launch_long_weights(hipStream_t s, const SegList &seg, const int *rp, const int *ci, const double *v,
                         const double *diag, const double *w, double *c) {
    hipLaunchKernelGGL(k_long_weights, dim3(kSegGrid), dim3(kBlock), 0, s, seg, rp, ci, v, diag, w, c);
}

namespace {
// Chunk sort, then merge passes until runs cover maxlen; returns the buffer
// holding the sorted segments (k0 or k1).
template <typename Key>
unsigned long long *seg_sort(hipStream_t s, const SegList &seg, int maxlen, Key key, unsigned long long *k0,
                             unsigned long long *k1) {
    hipLaunchKernelGGL((k_seg_sort_chunks<Key>), dim3(kSegGrid), dim3(kSortThreads), 0, s, seg, key, k0);
    for (long long run = kSegChunk; run < maxlen; run *= 2) {
        hipLaunchKernelGGL(k_seg_merge, dim3(kSegGrid), dim3(kBlock), 0, s, seg, (int)run, k0, k1);
        std::swap(k0, k1);
    }
    return k0;
}
}  // namespace

void launch_long_ranks(hipStream_t s, const SegList &seg, int maxlen, const int *rp, const double *c,
                       unsigned *rk, unsigned long long *k0, unsigned long long *k1) {
    unsigned long long *sorted = seg_sort(s, seg, maxlen, KeyRank{rp, c}, k0, k1);
    hipLaunchKernelGGL(k_long_rank, dim3(kSegGrid), dim3(kBlock), 0, s, seg, sorted, rp, c, rk);
}

void launch_long_candidates(hipStream_t s, const SegList &seg, int maxlen, const int *rp, const int *ci,
                            const double *c, const unsigned *rk, int lmin, bool direct, unsigned long long *cand,
                            unsigned long long *k0, unsigned long long *k1) {
    unsigned long long *sorted = seg_sort(s, seg, maxlen, KeyCand{rp, ci, c, rk}, k0, k1);
    hipLaunchKernelGGL(k_long_cand, dim3(kSegGrid), dim3(kBlock), 0, s, seg, sorted, rp, ci, c, rk, lmin,
                       direct ? 1 : 0, cand);
}

void launch_gal_long_sort(hipStream_t s, const SegList &seg, int maxlen, const int *rp, const int *ci,
                          const int *agg, const int *mem2, unsigned long long *k0, unsigned long long *k1,
                          unsigned long long **sorted) {
    *sorted = seg_sort(s, seg, maxlen, KeyGal{rp, ci, agg, mem2}, k0, k1);
}

void launch_gal_long(hipStream_t s, int pass, const SegList &seg, const unsigned long long *sorted, const int *rp,
                     const int *ci, const double *v, const int *agg, const double *p, const int *mem2, int *cnt,
                     int *cc, const int *crp, int *cci, double *cv) {
    hipLaunchKernelGGL(k_gal_long, dim3(kSegGrid), dim3(kSegBlock), 0, s, pass, seg, sorted, rp, ci, v, agg, p, mem2,
                       cnt, cc, crp, cci, cv);
}

void launch_long_abs(hipStream_t s, const LongRows &lr, const int *rp, const double *v, double *part, float *v32) {
    if (lr.nchunks > 0)
        hipLaunchKernelGGL(k_long_abs, dim3(lr.nchunks), dim3(kBlock), 0, s, lr, rp, v, part, v32);
}

}  // namespace bcm
