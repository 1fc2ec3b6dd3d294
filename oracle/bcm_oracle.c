/*
 * bcm_oracle.c -- serial FP64 CPU reference ("oracle") for AMG based on
 * compatible weighted matching used inside flexible CG
 * (Bernaschi, D'Ambra, Pasquini, arXiv 1810.04221).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares
 * no code, header, table or helper with it; the two meet only through the
 * seeded problem generators that feed both.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no fast-math, no
 * FMA contraction), so every floating-point operation below is one IEEE
 * binary64 operation with round-to-nearest in the order written.
 *
 * Each step follows a passage of the paper; where the paper is silent the
 * reading used is stated in the comment of the step:
 *   - edge weights C(A, w): Section 2.2 states only that they are positive and
 *     computed in linear time from A and w.  Reading: the compatible weighted
 *     matching weight c_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2).
 *   - maximum weight matching: Section 2.2 defines it; Section 3.1 replaces it
 *     by the half-approximate Suitor matching, whose result equals the greedy
 *     matching under a strict edge order.  Reading: the order is weight
 *     descending, then larger endpoint, then smaller endpoint, both descending.
 *   - pairwise aggregation: Algorithm 2 with "pick i in U" = smallest index.
 *   - prolongator: Section 2.2, orthonormal projection of w on each aggregate;
 *     coarse w = restriction of w = the aggregate's norm of w.
 *   - Galerkin product A_c = P^T A P (Section 2.1) with the terms of each
 *     coarse entry summed in a fixed canonical order.
 *   - double pairwise aggregation: two matching sweeps composed per level
 *     (Section 5, experimental settings).
 *   - l1-Jacobi smoother (Section 3.2): d_i = sum_j |a_ij|, x += (b - A x) / d.
 *   - V-cycle: Algorithm 1, one pre- and one post-smoothing sweep, a fixed
 *     number of l1-Jacobi sweeps from zero at the coarsest level.
 *   - W- and K-cycles (Section 2.1 names both beside Algorithm 1): the W-cycle
 *     solves each coarse problem by two cycles, the second on the coarse
 *     residual; the K-cycle by two iterations of the flexible CG below,
 *     preconditioned by the coarse level's cycle (Krylov-based cycle of Notay
 *     and Vassilevski, the reason Section 3.2 gives for the flexible CG).
 *   - flexible CG: Algorithm 3 with its sign and index typos read as
 *     r <- r - (alpha/rho) q and d, q updated with gamma_i / rho_{i-1}.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_MAXLEV 64

typedef struct {
    int n, nnz;
    int *rp, *ci;
    double *v;
} ocsr;

typedef struct {
    ocsr A;
    double *w;    /* smooth vector on this level */
    double *dinv; /* 1 / (l1 row norm) */
    /* prolongator to the next level (one nonzero per row): column agg[i], value p[i] */
    int nc;
    int *agg;
    double *p;
    double *b, *x, *r, *xc_tmp; /* cycle work vectors */
} olevel;

typedef struct {
    int nl;
    int coarse_sweeps;
    int cycle;   /* 1 = V-cycle, 2 = W-cycle, 3 = K-cycle */
    int klevels; /* K-cycle: levels k < klevels accelerate their coarse solve (0: all) */
    olevel lv[ORA_MAXLEV];
    /* per-level statistics of the last setup */
    int npairs[ORA_MAXLEV][8];
} ohier;

static void *xmalloc(size_t s) { return malloc(s ? s : 1); }

static void csr_free(ocsr *A) {
    free(A->rp); free(A->ci); free(A->v);
    memset(A, 0, sizeof(*A));
}

static void csr_copy(ocsr *dst, int n, const int *rp, const int *ci, const double *v) {
    int nnz = rp[n];
    dst->n = n; dst->nnz = nnz;
    dst->rp = xmalloc(sizeof(int) * (size_t)(n + 1));
    dst->ci = xmalloc(sizeof(int) * (size_t)nnz);
    dst->v = xmalloc(sizeof(double) * (size_t)nnz);
    memcpy(dst->rp, rp, sizeof(int) * (size_t)(n + 1));
    memcpy(dst->ci, ci, sizeof(int) * (size_t)nnz);
    memcpy(dst->v, v, sizeof(double) * (size_t)nnz);
}

/* ------------------------------------------------------------------ */
/* Edge weights C(A, w) (Section 2.2).                                  */
/*   c_ij = 1 - 2 a_ij w_i w_j / (a_ii w_i^2 + a_jj w_j^2)              */
/* Evaluated with m = min(i,j), M = max(i,j) so that both ends of an    */
/* edge produce the same double:                                        */
/*   num = ((2 a) w_m) w_M ; den = (a_mm w_m) w_m + (a_MM w_M) w_M      */
/* Diagonal positions get 0 (not an edge).                              */
/* ------------------------------------------------------------------ */
int ora_weights(int n, const int *rp, const int *ci, const double *v,
                const double *w, double *c) {
    double *dg = xmalloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; i++) {
        dg[i] = NAN;
        for (int q = rp[i]; q < rp[i + 1]; q++)
            if (ci[q] == i) dg[i] = v[q];
    }
    for (int i = 0; i < n; i++) {
        for (int q = rp[i]; q < rp[i + 1]; q++) {
            int j = ci[q];
            if (j == i) { c[q] = 0.0; continue; }
            int m = i < j ? i : j, M = i < j ? j : i;
            double a = v[q];
            double num = ((2.0 * a) * w[m]) * w[M];
            double den = (dg[m] * w[m]) * w[m] + (dg[M] * w[M]) * w[M];
            c[q] = 1.0 - num / den;
        }
    }
    free(dg);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Greedy matching, equal to Suitor's result under the strict order     */
/* (c desc, M desc, m desc).  Only positive finite weights are edges.   */
/* ------------------------------------------------------------------ */
typedef struct { double c; int m, M; } oedge;

static int edge_cmp(const void *pa, const void *pb) {
    const oedge *a = pa, *b = pb;
    if (a->c > b->c) return -1;
    if (a->c < b->c) return 1;
    if (a->M > b->M) return -1;
    if (a->M < b->M) return 1;
    if (a->m > b->m) return -1;
    if (a->m < b->m) return 1;
    return 0;
}

int ora_match(int n, const int *rp, const int *ci, const double *c, int *mate) {
    size_t ne = 0;
    for (int i = 0; i < n; i++)
        for (int q = rp[i]; q < rp[i + 1]; q++)
            if (ci[q] > i && isfinite(c[q]) && c[q] > 0.0) ne++;
    oedge *E = xmalloc(sizeof(oedge) * ne);
    ne = 0;
    for (int i = 0; i < n; i++)
        for (int q = rp[i]; q < rp[i + 1]; q++)
            if (ci[q] > i && isfinite(c[q]) && c[q] > 0.0) {
                E[ne].c = c[q]; E[ne].m = i; E[ne].M = ci[q]; ne++;
            }
    qsort(E, ne, sizeof(oedge), edge_cmp);
    for (int i = 0; i < n; i++) mate[i] = -1;
    int np = 0;
    for (size_t e = 0; e < ne; e++) {
        if (mate[E[e].m] < 0 && mate[E[e].M] < 0) {
            mate[E[e].m] = E[e].M;
            mate[E[e].M] = E[e].m;
            np++;
        }
    }
    free(E);
    return np;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2: pairwise aggregation from a matching.  U holds the      */
/* unaggregated indices; the index picked is the smallest one left.     */
/* Returns n_c; writes agg[i] in 0..n_c-1 and the counts n_p, n_s.      */
/* ------------------------------------------------------------------ */
int ora_aggregate(int n, const int *mate, int *agg, int *np_out, int *ns_out) {
    char *inU = xmalloc((size_t)n);
    memset(inU, 1, (size_t)n);
    int nc = 0, np = 0, ns = 0;
    for (int i = 0; i < n; i++) {
        if (!inU[i]) continue;
        int j = mate[i];
        if (j >= 0 && j != i && inU[j]) {
            np++;
            agg[i] = nc; agg[j] = nc; nc++;
            inU[i] = 0; inU[j] = 0;
        } else {
            ns++;
            agg[i] = nc; nc++;
            inU[i] = 0;
        }
    }
    free(inU);
    if (np_out) *np_out = np;
    if (ns_out) *ns_out = ns;
    return nc;
}

/* ------------------------------------------------------------------ */
/* Prolongator: orthonormal projection of w on each aggregate.          */
/* Pair {i<j}: s = sqrt(w_i*w_i + w_j*w_j), p_i = w_i/s, p_j = w_j/s.   */
/* Singleton {i}: s = |w_i|, p_i = w_i/s.  Coarse w_c[e] = s (= P^T w). */
/* ------------------------------------------------------------------ */
int ora_prolong(int n, const int *agg, int nc, const double *w, double *p, double *wc) {
    int *first = xmalloc(sizeof(int) * (size_t)nc), *second = xmalloc(sizeof(int) * (size_t)nc);
    for (int e = 0; e < nc; e++) { first[e] = -1; second[e] = -1; }
    for (int i = 0; i < n; i++) {
        int e = agg[i];
        if (first[e] < 0) first[e] = i;
        else if (second[e] < 0) second[e] = i;
        else { free(first); free(second); return -1; } /* not pairwise */
    }
    for (int e = 0; e < nc; e++) {
        int i = first[e], j = second[e];
        if (j >= 0) {
            double s = sqrt(w[i] * w[i] + w[j] * w[j]);
            p[i] = w[i] / s; p[j] = w[j] / s; wc[e] = s;
        } else {
            double s = fabs(w[i]);
            p[i] = w[i] / s; wc[e] = s;
        }
    }
    free(first); free(second);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Galerkin product A_c = P^T A P for P with one nonzero per row        */
/* (column agg[i], value p[i]) (Section 2.1).                           */
/*   (A_c)_EF = sum over stored (i, j) with agg i = E, agg j = F of     */
/*              (p_m * a_ij) * p_M,   m = min(i,j), M = max(i,j)        */
/* Terms of one entry are summed left to right, starting from the first */
/* term, in ascending (m, M, i).  No entry is dropped.                  */
/* ------------------------------------------------------------------ */
typedef struct { int F, m, M, i; double t; } oterm;

static int term_cmp(const void *pa, const void *pb) {
    const oterm *a = pa, *b = pb;
    if (a->F != b->F) return a->F < b->F ? -1 : 1;
    if (a->m != b->m) return a->m < b->m ? -1 : 1;
    if (a->M != b->M) return a->M < b->M ? -1 : 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    return 0;
}

static void galerkin(const ocsr *A, const int *agg, const double *p, int nc, ocsr *Ac) {
    int n = A->n;
    /* members of each aggregate, ascending (counting sort) */
    int *mp = calloc((size_t)nc + 1, sizeof(int));
    int *mem = xmalloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; i++) mp[agg[i] + 1]++;
    for (int e = 0; e < nc; e++) mp[e + 1] += mp[e];
    int *fill = xmalloc(sizeof(int) * (size_t)nc);
    for (int e = 0; e < nc; e++) fill[e] = mp[e];
    for (int i = 0; i < n; i++) mem[fill[agg[i]]++] = i;
    free(fill);

    size_t cap = 16;
    oterm *T = xmalloc(sizeof(oterm) * cap);
    int *crp = xmalloc(sizeof(int) * (size_t)(nc + 1));
    size_t ccap = (size_t)A->nnz + 16, cnnz = 0;
    int *cci = xmalloc(sizeof(int) * ccap);
    double *cv = xmalloc(sizeof(double) * ccap);
    crp[0] = 0;
    for (int E = 0; E < nc; E++) {
        size_t nt = 0;
        for (int t = mp[E]; t < mp[E + 1]; t++) {
            int i = mem[t];
            for (int q = A->rp[i]; q < A->rp[i + 1]; q++) {
                if (nt == cap) { cap *= 2; T = realloc(T, sizeof(oterm) * cap); }
                int j = A->ci[q];
                int m = i < j ? i : j, M = i < j ? j : i;
                T[nt].F = agg[j]; T[nt].m = m; T[nt].M = M; T[nt].i = i;
                T[nt].t = (p[m] * A->v[q]) * p[M];
                nt++;
            }
        }
        qsort(T, nt, sizeof(oterm), term_cmp);
        size_t k = 0;
        while (k < nt) {
            int F = T[k].F;
            double s = T[k].t;
            size_t l = k + 1;
            while (l < nt && T[l].F == F) { s = s + T[l].t; l++; }
            if (cnnz == ccap) {
                ccap *= 2;
                cci = realloc(cci, sizeof(int) * ccap);
                cv = realloc(cv, sizeof(double) * ccap);
            }
            cci[cnnz] = F; cv[cnnz] = s; cnnz++;
            k = l;
        }
        crp[E + 1] = (int)cnnz;
    }
    free(T); free(mp); free(mem);
    Ac->n = nc; Ac->nnz = (int)cnnz; Ac->rp = crp; Ac->ci = cci; Ac->v = cv;
}

/* Stand-alone Galerkin product: two-call protocol.  First call with
 * ci_out == NULL returns nnz of A_c; second call fills rp/ci/v. */
int ora_galerkin(int n, const int *rp, const int *ci, const double *v,
                 const int *agg, const double *p, int nc,
                 int *rp_out, int *ci_out, double *v_out) {
    ocsr A = { n, rp[n], (int *)rp, (int *)ci, (double *)v };
    ocsr Ac;
    galerkin(&A, agg, p, nc, &Ac);
    int nnz = Ac.nnz;
    if (ci_out) {
        memcpy(rp_out, Ac.rp, sizeof(int) * (size_t)(nc + 1));
        memcpy(ci_out, Ac.ci, sizeof(int) * (size_t)nnz);
        memcpy(v_out, Ac.v, sizeof(double) * (size_t)nnz);
    }
    csr_free(&Ac);
    return nnz;
}

/* l1-Jacobi (Section 3.2): d_i = sum_j |a_ij| left to right, dinv = 1/d. */
static void l1_dinv(const ocsr *A, double *dinv) {
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int q = A->rp[i]; q < A->rp[i + 1]; q++) s = s + fabs(A->v[q]);
        dinv[i] = 1.0 / s;
    }
}

int ora_l1_dinv(int n, const int *rp, const int *ci, const double *v, double *dinv) {
    ocsr A = { n, rp[n], (int *)rp, (int *)ci, (double *)v };
    l1_dinv(&A, dinv);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Hierarchy setup (Section 2.1, 2.2, Section 5 settings).              */
/* ------------------------------------------------------------------ */
static void level_alloc_vectors(olevel *L) {
    int n = L->A.n;
    L->b = calloc((size_t)n, sizeof(double));
    L->x = calloc((size_t)n, sizeof(double));
    L->r = calloc((size_t)n, sizeof(double));
    L->xc_tmp = calloc((size_t)n, sizeof(double));
    L->dinv = xmalloc(sizeof(double) * (size_t)n);
    l1_dinv(&L->A, L->dinv);
}

void ora_free(void *hv) {
    ohier *h = hv;
    if (!h) return;
    for (int k = 0; k < h->nl; k++) {
        olevel *L = &h->lv[k];
        csr_free(&L->A);
        free(L->w); free(L->dinv); free(L->agg); free(L->p);
        free(L->b); free(L->x); free(L->r); free(L->xc_tmp);
    }
    free(h);
}

/*
 * Builds the hierarchy.  Section 5 (experimental settings) stops the
 * coarsening at a coarsest matrix of at most maxcoarseset * n^(1/3) rows and
 * at 40 levels: level k is the coarsest when n_k <= max_coarse, or
 * k + 1 == max_levels, or its coarsening left the size unchanged (no pair
 * formed: every later sweep would form none either).  min_ratio > 1 adds a
 * rule that is not the paper's: a level formed with a size ratio
 * n_{k-1} / n_k below min_ratio is the coarsest (coarsening that has stalled);
 * min_ratio <= 1 leaves it out.  Each coarsening composes `sweeps` pairwise
 * sweeps; a sweep that forms no pair is skipped.  Returns NULL on invalid
 * input (status < 0).
 */
void *ora_setup(int n, const int *rp, const int *ci, const double *v, const double *w,
                int max_levels, int max_coarse, int sweeps, int coarse_sweeps, int cycle,
                int klevels, double min_ratio, int *status) {
    *status = 0;
    if (max_levels < 1 || max_levels > ORA_MAXLEV || sweeps < 1 || sweeps > 8 || cycle < 1 || cycle > 3 ||
        klevels < 0) {
        *status = -1;
        return NULL;
    }
    for (int i = 0; i < n; i++) {
        if (!(isfinite(w[i]) && w[i] != 0.0)) { *status = -1; return NULL; }
        int hasd = 0;
        for (int q = rp[i]; q < rp[i + 1]; q++) {
            if (!isfinite(v[q])) { *status = -1; return NULL; }
            if (ci[q] == i) { hasd = 1; if (!(v[q] > 0.0)) { *status = -1; return NULL; } }
        }
        if (!hasd) { *status = -1; return NULL; }
    }
    const double rmin = min_ratio > 1.0 ? min_ratio : 1.0;
    ohier *h = calloc(1, sizeof(ohier));
    h->coarse_sweeps = coarse_sweeps;
    h->cycle = cycle;
    h->klevels = klevels;
    csr_copy(&h->lv[0].A, n, rp, ci, v);
    h->lv[0].w = xmalloc(sizeof(double) * (size_t)n);
    memcpy(h->lv[0].w, w, sizeof(double) * (size_t)n);
    int k = 0;
    for (;;) {
        olevel *L = &h->lv[k];
        int nk = L->A.n;
        if (nk <= max_coarse || k + 1 >= max_levels) break;
        /* composed prolongator of this level, starting from the identity */
        int *agg = xmalloc(sizeof(int) * (size_t)nk);
        double *p = xmalloc(sizeof(double) * (size_t)nk);
        for (int i = 0; i < nk; i++) { agg[i] = i; p[i] = 1.0; }
        ocsr Acur = L->A;          /* borrowed for the first sweep */
        int own = 0;
        double *wcur = L->w;
        int own_w = 0;
        for (int s = 0; s < sweeps; s++) {
            int m = Acur.n;
            double *c = xmalloc(sizeof(double) * (size_t)Acur.nnz);
            int *mate = xmalloc(sizeof(int) * (size_t)m);
            int *ag = xmalloc(sizeof(int) * (size_t)m);
            ora_weights(m, Acur.rp, Acur.ci, Acur.v, wcur, c);
            int np = ora_match(m, Acur.rp, Acur.ci, c, mate);
            int nps, nss;
            int nc = ora_aggregate(m, mate, ag, &nps, &nss);
            h->npairs[k][s] = np;
            free(c); free(mate);
            if (nc == m) { free(ag); break; } /* no pair: sweep contributes nothing */
            double *ps = xmalloc(sizeof(double) * (size_t)m);
            double *wc = xmalloc(sizeof(double) * (size_t)nc);
            ora_prolong(m, ag, nc, wcur, ps, wc);
            ocsr Ac;
            galerkin(&Acur, ag, ps, nc, &Ac);
            /* compose: agg <- ag[agg], p <- p * ps[agg] */
            for (int i = 0; i < nk; i++) {
                int a = agg[i];
                p[i] = p[i] * ps[a];
                agg[i] = ag[a];
            }
            free(ag); free(ps);
            if (own) csr_free(&Acur);
            Acur = Ac; own = 1;
            if (own_w) free(wcur);
            wcur = wc; own_w = 1;
        }
        if (!own || Acur.n == nk) { /* stagnation: level k is the coarsest */
            if (own) csr_free(&Acur);
            if (own_w) free(wcur);
            free(agg); free(p);
            break;
        }
        L->nc = Acur.n; L->agg = agg; L->p = p;
        h->lv[k + 1].A = Acur;
        h->lv[k + 1].w = wcur;
        k++;
        /* min_ratio > 1 only: coarsening has stalled, the new level is the coarsest */
        if (rmin > 1.0 && (double)nk < rmin * (double)Acur.n) break;
    }
    h->nl = k + 1;
    for (int l = 0; l < h->nl; l++) level_alloc_vectors(&h->lv[l]);
    return h;
}

int ora_nlevels(void *hv) { return ((ohier *)hv)->nl; }
int ora_level_n(void *hv, int k) { return ((ohier *)hv)->lv[k].A.n; }
int ora_level_nnz(void *hv, int k) { return ((ohier *)hv)->lv[k].A.nnz; }
int ora_level_npairs(void *hv, int k, int s) { return ((ohier *)hv)->npairs[k][s]; }

/* Copies level k out (NULL pointers are skipped).  agg/p describe P^k and
 * exist only for k < nl - 1. */
int ora_level_get(void *hv, int k, int *rp, int *ci, double *v, double *w, double *dinv,
                  int *agg, double *p) {
    ohier *h = hv;
    if (k < 0 || k >= h->nl) return -1;
    olevel *L = &h->lv[k];
    int n = L->A.n, nnz = L->A.nnz;
    if (rp) memcpy(rp, L->A.rp, sizeof(int) * (size_t)(n + 1));
    if (ci) memcpy(ci, L->A.ci, sizeof(int) * (size_t)nnz);
    if (v) memcpy(v, L->A.v, sizeof(double) * (size_t)nnz);
    if (w) memcpy(w, L->w, sizeof(double) * (size_t)n);
    if (dinv) memcpy(dinv, L->dinv, sizeof(double) * (size_t)n);
    if (k < h->nl - 1) {
        if (agg) memcpy(agg, L->agg, sizeof(int) * (size_t)n);
        if (p) memcpy(p, L->p, sizeof(double) * (size_t)n);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Preconditioner application: Algorithm 1.                             */
/* ------------------------------------------------------------------ */
static void spmv(const ocsr *A, const double *x, double *y) {
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int q = A->rp[i]; q < A->rp[i + 1]; q++) s = s + A->v[q] * x[A->ci[q]];
        y[i] = s;
    }
}

/* x <- x + D^{-1} (b - A x), one l1-Jacobi sweep */
static void jacobi_sweep(const olevel *L, const double *b, double *x, double *r) {
    spmv(&L->A, x, r);
    for (int i = 0; i < L->A.n; i++) r[i] = b[i] - r[i];
    for (int i = 0; i < L->A.n; i++) x[i] = x[i] + L->dinv[i] * r[i];
}

static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

static void cycle(ohier *h, int k);

/*
 * K-cycle coarse solve at level k: x_c ~ (A^{k+1})^{-1} b_c by two iterations
 * of the flexible CG of Algorithm 3 (same reading as ora_fcg) from x_c = 0,
 * preconditioned by cycle(k + 1).  If rho is not positive and finite (b_c = 0,
 * or a second direction parallel to the first) the iteration stops and x_c
 * keeps what it has.
 */
static void kcycle_coarse(ohier *h, int k, const double *bc, double *xc) {
    olevel *C = &h->lv[k + 1];
    int n = C->A.n;
    size_t bytes = sizeof(double) * (size_t)n;
    double *r = xmalloc(bytes), *w = xmalloc(bytes), *v = xmalloc(bytes);
    double *d = calloc((size_t)n, sizeof(double)), *q = calloc((size_t)n, sizeof(double));
    memcpy(r, bc, bytes);
    memset(xc, 0, bytes);
    double rho = 0.0;
    for (int it = 0; it < 2; it++) {
        memcpy(C->b, r, bytes);
        cycle(h, k + 1);
        memcpy(w, C->x, bytes);
        spmv(&C->A, w, v);
        double alpha = dot(n, w, r);
        double beta = dot(n, w, v);
        double rho_new = beta, g = 0.0;
        if (it > 0) {
            double gamma = dot(n, w, q);
            rho_new = beta - gamma * gamma / rho;
            g = gamma / rho;
        }
        if (!(rho_new > 0.0) || !isfinite(rho_new)) break;
        double an = alpha / rho_new;
        for (int i = 0; i < n; i++) d[i] = w[i] - g * d[i];
        for (int i = 0; i < n; i++) xc[i] = xc[i] + an * d[i];
        for (int i = 0; i < n; i++) q[i] = v[i] - g * q[i];
        for (int i = 0; i < n; i++) r[i] = r[i] - an * q[i];
        rho = rho_new;
    }
    free(r); free(w); free(v); free(d); free(q);
}

/*
 * cycle(k) (Algorithm 1): on entry L->b holds the right-hand side; on exit
 * L->x holds the result, from a zero initial guess.  The coarse problem
 * A^{k+1} x_c = P^T r is solved by one cycle of level k + 1 (V), by two
 * successive cycles x_c = cycle(b_c), x_c = x_c + cycle(b_c - A^{k+1} x_c) (W),
 * or by kcycle_coarse on the K-accelerated levels (K).
 */
static void cycle(ohier *h, int k) {
    olevel *L = &h->lv[k];
    int n = L->A.n;
    memset(L->x, 0, sizeof(double) * (size_t)n);
    if (k == h->nl - 1) {
        for (int t = 0; t < h->coarse_sweeps; t++) jacobi_sweep(L, L->b, L->x, L->r);
        return;
    }
    olevel *C = &h->lv[k + 1];
    int nc = C->A.n;
    /* pre-smoothing */
    jacobi_sweep(L, L->b, L->x, L->r);
    /* restriction of the residual: b_c = P^T (b - A x) */
    spmv(&L->A, L->x, L->r);
    for (int i = 0; i < n; i++) L->r[i] = L->b[i] - L->r[i];
    double *bc = xmalloc(sizeof(double) * (size_t)nc), *xc = xmalloc(sizeof(double) * (size_t)nc);
    for (int e = 0; e < nc; e++) bc[e] = 0.0;
    for (int i = 0; i < n; i++) bc[L->agg[i]] = bc[L->agg[i]] + L->p[i] * L->r[i];
    if (h->cycle == 3 && (h->klevels == 0 || k < h->klevels)) {
        kcycle_coarse(h, k, bc, xc);
    } else {
        memcpy(C->b, bc, sizeof(double) * (size_t)nc);
        cycle(h, k + 1);
        memcpy(xc, C->x, sizeof(double) * (size_t)nc);
        if (h->cycle == 2) {
            spmv(&C->A, xc, C->b);
            for (int e = 0; e < nc; e++) C->b[e] = bc[e] - C->b[e];
            cycle(h, k + 1);
            for (int e = 0; e < nc; e++) xc[e] = xc[e] + C->x[e];
        }
    }
    /* prolongation: x = x + P x_c */
    for (int i = 0; i < n; i++) L->x[i] = L->x[i] + L->p[i] * xc[L->agg[i]];
    free(bc); free(xc);
    /* post-smoothing (M^{-T} = M^{-1} for a diagonal M) */
    jacobi_sweep(L, L->b, L->x, L->r);
}

/* x = B(b): one cycle from a zero initial guess */
int ora_vcycle(void *hv, const double *b, double *x) {
    ohier *h = hv;
    olevel *L = &h->lv[0];
    memcpy(L->b, b, sizeof(double) * (size_t)L->A.n);
    cycle(h, 0);
    memcpy(x, L->x, sizeof(double) * (size_t)L->A.n);
    return 0;
}

/* preconditioner: 0 identity, 1 multigrid cycle, 2 one l1-Jacobi step from zero */
static void precond(ohier *h, int mode, const double *r, double *z) {
    int n = h->lv[0].A.n;
    if (mode == 0) memcpy(z, r, sizeof(double) * (size_t)n);
    else if (mode == 1) ora_vcycle(h, r, z);
    else for (int i = 0; i < n; i++) z[i] = h->lv[0].dinv[i] * r[i];
}

/* ------------------------------------------------------------------ */
/* Flexible preconditioned CG: Algorithm 3, read with                   */
/*   r_{i+1} = r_i - (alpha_i/rho_i) q_i   and                          */
/*   d_i = w_i - (gamma_i/rho_{i-1}) d_{i-1}, q_i = v_i - (...) q_{i-1} */
/* Stops when ||r_i|| / ||b|| <= tol on the recurrence residual, or     */
/* after itmax preconditioner applications.  At exit the true residual  */
/* b - A u is recomputed; if it misses tol the iteration restarts from  */
/* u (at most 3 times).  Returns 0 converged, 1 itmax reached,          */
/* -2 breakdown (rho <= 0 or not finite).                               */
/* ------------------------------------------------------------------ */
int ora_fcg(void *hv, int mode, const double *b, double *u, double tol, int itmax,
            int *iters_out, double *relres_out) {
    ohier *h = hv;
    olevel *L = &h->lv[0];
    int n = L->A.n;
    double *r = xmalloc(sizeof(double) * (size_t)n), *w = xmalloc(sizeof(double) * (size_t)n);
    double *d = xmalloc(sizeof(double) * (size_t)n), *v = xmalloc(sizeof(double) * (size_t)n);
    double *q = xmalloc(sizeof(double) * (size_t)n);
    double bn = sqrt(dot(n, b, b));
    int it = 0, status = 0;
    double relres = 0.0;
    if (bn == 0.0) {
        memset(u, 0, sizeof(double) * (size_t)n);
        goto done;
    }
    for (int restart = 0; restart < 4; restart++) {
        spmv(&L->A, u, r);
        for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
        relres = sqrt(dot(n, r, r)) / bn;
        if (relres <= tol) { status = 0; goto done; }
        if (restart > 0 && it >= itmax) { status = 1; goto done; }
        if (it >= itmax) { status = 1; goto done; }
        /* first step */
        precond(h, mode, r, w);
        spmv(&L->A, w, v);
        double alpha = dot(n, w, r);
        double beta = dot(n, w, v);
        double rho = beta;
        if (!(rho > 0.0) || !isfinite(rho)) { status = -2; goto done; }
        for (int i = 0; i < n; i++) { d[i] = w[i]; q[i] = v[i]; }
        double a = alpha / rho;
        for (int i = 0; i < n; i++) u[i] = u[i] + a * d[i];
        for (int i = 0; i < n; i++) r[i] = r[i] - a * q[i];
        it++;
        relres = sqrt(dot(n, r, r)) / bn;
        while (relres > tol && it < itmax) {
            precond(h, mode, r, w);
            spmv(&L->A, w, v);
            alpha = dot(n, w, r);
            beta = dot(n, w, v);
            double gamma = dot(n, w, q);
            double rho_new = beta - gamma * gamma / rho;
            if (!(rho_new > 0.0) || !isfinite(rho_new)) { status = -2; goto done; }
            double g = gamma / rho;
            double an = alpha / rho_new;
            for (int i = 0; i < n; i++) d[i] = w[i] - g * d[i];
            for (int i = 0; i < n; i++) u[i] = u[i] + an * d[i];
            for (int i = 0; i < n; i++) q[i] = v[i] - g * q[i];
            for (int i = 0; i < n; i++) r[i] = r[i] - an * q[i];
            rho = rho_new;
            it++;
            relres = sqrt(dot(n, r, r)) / bn;
        }
        /* true residual */
        spmv(&L->A, u, r);
        for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
        relres = sqrt(dot(n, r, r)) / bn;
        if (relres <= tol) { status = 0; goto done; }
        if (it >= itmax) { status = 1; goto done; }
    }
    status = 1;
done:
    free(r); free(w); free(d); free(v); free(q);
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = relres;
    return status;
}

/* ------------------------------------------------------------------ */
/* Gradient of a loss L(x) with x = A^{-1} b, given g = dL/dx:          */
/*   lambda = A^{-1} g (adjoint solve; A symmetric), dL/db = lambda,    */
/*   dL/da_ij = -lambda_i x_j on the stored pattern of A.               */
/* ------------------------------------------------------------------ */
int ora_sampled_outer(int n, const int *rp, const int *ci, const double *lam,
                      const double *x, double *G) {
    for (int i = 0; i < n; i++)
        for (int q = rp[i]; q < rp[i + 1]; q++) G[q] = -(lam[i] * x[ci[q]]);
    return 0;
}

int ora_spmv(int n, const int *rp, const int *ci, const double *v, const double *x, double *y) {
    ocsr A = { n, rp[n], (int *)rp, (int *)ci, (double *)v };
    spmv(&A, x, y);
    return 0;
}
