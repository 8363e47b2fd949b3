/*
 * DDLR oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the domain-decomposition low-rank
 * (DDLR) preconditioner of Li & Saad, "Low-rank correction methods for
 * algebraic domain decomposition preconditioners".  It exists to check the HIP
 * library against; nothing in the library includes, links or calls it, and it
 * shares no code with the library.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it.
 *
 * Every step follows the paper in its own order and notation:
 *   - classification of unknowns into interior / interface (Sec. 2.1, edge
 *     separator: interface = coupled to an unknown of another subdomain),
 *   - global reordering into the form of eq. (Bmat): interiors of subdomain
 *     1..p, then all interface unknowns (Sec. 2.2),
 *   - splitting A = A0 - E E^T with E = [alpha^{-1} Ehat ; -alpha I] and
 *     A0 = blockdiag(B + alpha^{-2} Ehat Ehat^T, C + alpha^2 I)
 *     (eqs. splitA, EF, splitA1, split; Proposition on the locality of
 *     Ehat Ehat^T),
 *   - local solvers: incomplete LDL^T with the matrix's own pattern, one per
 *     B_{i,alpha} and one for C_alpha (Sec. 5: "incomplete Cholesky or LDL"),
 *     or exact dense LDL^T per block for the identity tests; alternatively
 *     C_alpha is solved by a sparse approximate inverse X built with the
 *     self-preconditioned global MR iteration with dropping (Sec. 4.3 (sec:csolve),
 *     Algorithm alg:mr), applied as a product with X, or by 5 preconditioned
 *     Chebyshev iterations with the block-Jacobi matrix D_alpha of the local
 *     blocks C_i and spectrum estimates from Lanczos on (C_alpha, D_alpha),
 *   - Lanczos on E^T A0^{-1} E (DDLR-1) or E^T A0^{-2} E (DDLR-2) with full
 *     reorthogonalisation (Sec. 4.4 (sec:Lan)), Ritz pairs of T_m by cyclic Jacobi,
 *   - G_{k,theta}^{-1} of eq. (gkt) with theta = lambda_{k+1}, applied through
 *     the five steps of the DDLR-1 preconditioning algorithm (Sec. 4.2), or
 *     M^{-1} = A0^{-1} + U_k H_k U_k^T, H_k = (I - U_k^T E V_k)^{-1}
 *     (eq. Form2a, Lemma on H_k) for DDLR-2,
 *   - preconditioned CG and right-preconditioned GMRES(restart) with the
 *     paper's stopping rule (residual reduced by 6 orders, at most 500 steps).
 *
 * Readings where the paper is silent (ordering inside blocks, C_alpha solver,
 * colouring, breakdown thresholds) are listed in the design document and in
 * the comments at each step.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID -1
#define ORC_E_NOT_SYMMETRIC -2
#define ORC_E_BREAKDOWN -3
#define ORC_E_NOT_SPD -4
#define ORC_E_NO_CONVERGENCE -5
#define ORC_E_LANCZOS -6

typedef struct {
    int64_t n;
    int64_t *rp;
    int32_t *ci;
    double *v;
} csr_t;

typedef struct {
    /* problem */
    int64_t n;
    int32_t p;
    double alpha;
    int corder;  /* 0 multicolour, 1 natural */
    int factor;  /* 0 IC (positive pivots), 1 indefinite LDL (nonzero pivots), 2 exact dense */
    csr_t A;     /* user order */
    /* ordering */
    int32_t *part;
    int32_t *iface;   /* user row -> 1 if interface */
    int32_t *perm;    /* internal position -> user row */
    int32_t *iperm;   /* user row -> internal position */
    int32_t *colour;  /* internal interface index (0..s-1) -> colour */
    int32_t ncolours;
    int64_t m, s;
    int64_t *boff;    /* p+2 offsets: block b = [boff[b], boff[b+1]), block p = interface */
    /* splitting, internal order */
    csr_t Ap;     /* P A P^T */
    csr_t A0;     /* blockdiag(B_alpha, C_alpha) */
    csr_t Et;     /* E^T, s x n */
    csr_t E;      /* E, n x s */
    /* local factors: L strictly lower (internal indices), D */
    csr_t L;
    double *D;
    int64_t breakdown_row;  /* internal row of a failed pivot, -1 if none */
    /* low rank */
    int variant;  /* 0 none, 1 DDLR-1, 2 DDLR-2 */
    int spd;      /* 1 if the low-rank build certifies an SPD preconditioner */
    int k;
    double *U;    /* DDLR-1: s x k (column-major); DDLR-2: n x k */
    double *lam;  /* DDLR-1 Ritz values lambda_1..lambda_k */
    double theta, c0;
    double *dvec; /* DDLR-1: 1/(1-lambda_j) - c0 */
    double *Hk;   /* DDLR-2: k x k */
    /* Lanczos record */
    int msteps;
    double *ta, *tb;  /* alpha_1..alpha_m, beta_1..beta_m */
    double *ritz;     /* descending, length msteps */
    double *Q;        /* s x (msteps + 1): q_1..q_m and q_{m+1} */
    int qcap;         /* columns allocated in Q, ta, tb */
    int lvariant;     /* operator of the stored run (1 or 2), 0 if none */
    int broke;        /* the stored run ended in an invariant subspace */
    double amax;      /* max |alpha_i| so far */
    /* reorthogonalisation: 0 full (classical Gram-Schmidt twice, every step),
     * 1 partial (Simon's omega recurrence), 2 none (tests only) */
    int reorth;
    double *om_prev, *om_cur;  /* omega estimates of q_i^T q_{j-1} and q_i^T q_j, length qcap + 1 */
    double tnorm;              /* running estimate of ||T_j|| in the omega recurrence */
    int force_next;            /* the step after a partial reorthogonalisation is reorthogonalised too */
    int *rsteps;               /* 1 for the steps whose new vector was reorthogonalised */
    int nreorth;
    /* C_alpha approximate inverse (csolve = 1) */
    int csolve;       /* 0: factor of C_alpha, 1: X ~ C_alpha^{-1} */
    csr_t X;          /* s x s, symmetric, interface indices */
    int x_iters;      /* MR steps taken */
    double *x_res;    /* ||I - C X_j||_F for j = 0..x_iters */
    double x_rinf;    /* ||I - C X||_inf (largest absolute row sum) of the final X */
    int x_spd;        /* 1 if ||I - C X||_inf < 1: then C^{1/2} X C^{1/2} has its eigenvalues in (0, 2), so X is SPD */
    /* csolve = 2: Chebyshev on C_alpha with D_alpha = blockdiag(C_i) (factored in L, D) */
    int ch_nu;            /* iterations per solve */
    double ch_lo, ch_hi;  /* safeguarded spectrum interval of D_alpha^{-1} C_alpha */
    double ch_rlo, ch_rhi;/* extreme Ritz values of the estimate */
} orc_t;

static void *xcalloc(size_t n, size_t sz) {
    void *p = calloc(n ? n : 1, sz ? sz : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

static void csr_free(csr_t *a) {
    free(a->rp); free(a->ci); free(a->v);
    a->rp = NULL; a->ci = NULL; a->v = NULL;
}

/* ---------------------------------------------------------------- dense helpers */

static double dot(const double *a, const double *b, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double nrm2(const double *a, int64_t n) { return sqrt(dot(a, a, n)); }

/* y = A x for an internal-order CSR */
static void csr_mv(const csr_t *a, int64_t nrows, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        double s = 0.0;
        for (int64_t t = a->rp[i]; t < a->rp[i + 1]; ++t) s += a->v[t] * x[a->ci[t]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------- ordering (Sec. 2) */

/* Interface unknowns are those coupled to an unknown of another subdomain
 * (edge separator, Sec. 2.1). Interior unknowns of subdomain i come first, in
 * ascending original index, subdomain by subdomain; then the interface unknowns,
 * subdomain by subdomain, ascending (the form of eq. Bmat).  With multicolour
 * ordering the interface block is then reordered by (greedy colour, position). */
static int build_ordering(orc_t *o) {
    const int64_t n = o->n;
    const int32_t p = o->p;
    o->iface = xcalloc(n, sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        if (o->part[i] < 0 || o->part[i] >= p) return ORC_E_INVALID;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = o->A.rp[i]; t < o->A.rp[i + 1]; ++t) {
            int32_t j = o->A.ci[t];
            if (j != i && o->part[j] != o->part[i]) { o->iface[i] = 1; break; }
        }
    o->perm = xcalloc(n, sizeof(int32_t));
    o->iperm = xcalloc(n, sizeof(int32_t));
    o->boff = xcalloc(p + 2, sizeof(int64_t));
    int64_t pos = 0;
    for (int32_t b = 0; b < p; ++b) {
        o->boff[b] = pos;
        for (int64_t i = 0; i < n; ++i)
            if (o->part[i] == b && !o->iface[i]) o->perm[pos++] = (int32_t)i;
    }
    o->m = pos;
    o->boff[p] = pos;
    for (int32_t b = 0; b < p; ++b)
        for (int64_t i = 0; i < n; ++i)
            if (o->part[i] == b && o->iface[i]) o->perm[pos++] = (int32_t)i;
    o->boff[p + 1] = pos;
    o->s = n - o->m;
    /* colouring of the interface graph */
    const int64_t s = o->s, m = o->m;
    o->colour = xcalloc(s > 0 ? s : 1, sizeof(int32_t));
    o->ncolours = s > 0 ? 1 : 0;
    if (o->corder == 0 && s > 0) {
        for (int64_t i = 0; i < n; ++i) o->iperm[o->perm[i]] = (int32_t)i;
        int32_t *used = xcalloc(s + 1, sizeof(int32_t));
        for (int64_t y = 0; y < s; ++y) o->colour[y] = -1;
        int32_t ncol = 0;
        for (int64_t y = 0; y < s; ++y) {
            int32_t u = o->perm[m + y];
            /* mark colours of already coloured interface neighbours */
            for (int64_t t = o->A.rp[u]; t < o->A.rp[u + 1]; ++t) {
                int32_t v = o->A.ci[t];
                if (v == u || !o->iface[v]) continue;
                int64_t yv = o->iperm[v] - m;
                if (o->colour[yv] >= 0) used[o->colour[yv]] = (int32_t)(y + 1);
            }
            int32_t c = 0;
            while (used[c] == y + 1) ++c;
            o->colour[y] = c;
            if (c + 1 > ncol) ncol = c + 1;
        }
        free(used);
        o->ncolours = ncol;
        /* stable reorder of the interface block by colour */
        int32_t *newp = xcalloc(s, sizeof(int32_t));
        int32_t *newc = xcalloc(s, sizeof(int32_t));
        int64_t q = 0;
        for (int32_t c = 0; c < ncol; ++c)
            for (int64_t y = 0; y < s; ++y)
                if (o->colour[y] == c) { newp[q] = o->perm[m + y]; newc[q] = c; ++q; }
        memcpy(o->perm + m, newp, s * sizeof(int32_t));
        memcpy(o->colour, newc, s * sizeof(int32_t));
        free(newp); free(newc);
    }
    for (int64_t i = 0; i < n; ++i) o->iperm[o->perm[i]] = (int32_t)i;
    return ORC_OK;
}

/* ----------------------------------------------------- splitting (Sec. 3.1) */

typedef struct { int32_t c; double v; } ent_t;

static int ent_cmp(const void *a, const void *b) {
    const ent_t *x = a, *y = b;
    return (x->c > y->c) - (x->c < y->c);
}

/* Builds P A P^T, A0 = blockdiag(B + alpha^{-2} Ehat Ehat^T, C + alpha^2 I),
 * E = [alpha^{-1} Ehat; -alpha I] (n x s) and E^T.  The pattern of
 * B_{i,alpha} is the structural union of B_i and E_i E_i^T. */
static void build_split(orc_t *o) {
    const int64_t n = o->n, m = o->m, s = o->s;
    const double a = o->alpha, ia = 1.0 / o->alpha;
    /* P A P^T */
    o->Ap.rp = xcalloc(n + 1, sizeof(int64_t));
    int64_t nnz = o->A.rp[n];
    o->Ap.ci = xcalloc(nnz, sizeof(int32_t));
    o->Ap.v = xcalloc(nnz, sizeof(double));
    for (int64_t r = 0; r < n; ++r) {
        int32_t u = o->perm[r];
        int64_t cnt = o->A.rp[u + 1] - o->A.rp[u];
        o->Ap.rp[r + 1] = o->Ap.rp[r] + cnt;
        ent_t *row = xcalloc(cnt, sizeof(ent_t));
        for (int64_t t = 0; t < cnt; ++t) {
            row[t].c = o->iperm[o->A.ci[o->A.rp[u] + t]];
            row[t].v = o->A.v[o->A.rp[u] + t];
        }
        qsort(row, cnt, sizeof(ent_t), ent_cmp);
        for (int64_t t = 0; t < cnt; ++t) {
            o->Ap.ci[o->Ap.rp[r] + t] = row[t].c;
            o->Ap.v[o->Ap.rp[r] + t] = row[t].v;
        }
        free(row);
    }
    /* A0: rows of B blocks get B_i + alpha^{-2} E_i E_i^T, rows of C get C + alpha^2 I */
    double *acc = xcalloc(n, sizeof(double));
    char *mark = xcalloc(n, 1);
    int32_t *list = xcalloc(n, sizeof(int32_t));
    int64_t cap = nnz * 2 + n, used = 0;
    o->A0.rp = xcalloc(n + 1, sizeof(int64_t));
    o->A0.ci = xcalloc(cap, sizeof(int32_t));
    o->A0.v = xcalloc(cap, sizeof(double));
    for (int64_t r = 0; r < n; ++r) {
        int64_t cnt = 0;
        if (r < m) {
            for (int64_t t = o->Ap.rp[r]; t < o->Ap.rp[r + 1]; ++t) {
                int32_t c = o->Ap.ci[t];
                if (c < m) {
                    if (!mark[c]) { mark[c] = 1; acc[c] = 0.0; list[cnt++] = c; }
                    acc[c] += o->Ap.v[t];
                }
            }
            /* (Ehat Ehat^T)_{rj} = sum over interface c of Ehat_{rc} Ehat_{jc};
             * Ehat_{jc} = A_{cj} by symmetry.  Ascending interface index c. */
            for (int64_t t = o->Ap.rp[r]; t < o->Ap.rp[r + 1]; ++t) {
                int32_t c = o->Ap.ci[t];
                if (c < m) continue;
                double erc = o->Ap.v[t];
                for (int64_t t2 = o->Ap.rp[c]; t2 < o->Ap.rp[c + 1]; ++t2) {
                    int32_t j = o->Ap.ci[t2];
                    if (j >= m) continue;
                    if (!mark[j]) { mark[j] = 1; acc[j] = 0.0; list[cnt++] = j; }
                    acc[j] += ia * ia * erc * o->Ap.v[t2];
                }
            }
        } else {
            for (int64_t t = o->Ap.rp[r]; t < o->Ap.rp[r + 1]; ++t) {
                int32_t c = o->Ap.ci[t];
                if (c >= m) {
                    if (!mark[c]) { mark[c] = 1; acc[c] = 0.0; list[cnt++] = c; }
                    acc[c] += o->Ap.v[t];
                }
            }
            if (!mark[r]) { mark[r] = 1; acc[r] = 0.0; list[cnt++] = (int32_t)r; }
            acc[r] += a * a;
        }
        if (used + cnt > cap) {
            cap = 2 * (used + cnt);
            o->A0.ci = realloc(o->A0.ci, cap * sizeof(int32_t));
            o->A0.v = realloc(o->A0.v, cap * sizeof(double));
        }
        ent_t *row = xcalloc(cnt, sizeof(ent_t));
        for (int64_t t = 0; t < cnt; ++t) { row[t].c = list[t]; row[t].v = acc[list[t]]; mark[list[t]] = 0; }
        qsort(row, cnt, sizeof(ent_t), ent_cmp);
        for (int64_t t = 0; t < cnt; ++t) { o->A0.ci[used + t] = row[t].c; o->A0.v[used + t] = row[t].v; }
        free(row);
        used += cnt;
        o->A0.rp[r + 1] = used;
    }
    free(acc); free(mark); free(list);
    /* E (n x s): interior rows alpha^{-1} Ehat, interface row m+j has -alpha at column j */
    o->E.rp = xcalloc(n + 1, sizeof(int64_t));
    o->E.ci = xcalloc(nnz + s, sizeof(int32_t));
    o->E.v = xcalloc(nnz + s, sizeof(double));
    used = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (r < m) {
            for (int64_t t = o->Ap.rp[r]; t < o->Ap.rp[r + 1]; ++t)
                if (o->Ap.ci[t] >= m) {
                    o->E.ci[used] = (int32_t)(o->Ap.ci[t] - m);
                    o->E.v[used] = ia * o->Ap.v[t];
                    ++used;
                }
        } else {
            o->E.ci[used] = (int32_t)(r - m);
            o->E.v[used] = -a;
            ++used;
        }
        o->E.rp[r + 1] = used;
    }
    /* E^T (s x n) by transposition */
    o->Et.rp = xcalloc(s + 1, sizeof(int64_t));
    o->Et.ci = xcalloc(used, sizeof(int32_t));
    o->Et.v = xcalloc(used, sizeof(double));
    for (int64_t t = 0; t < used; ++t) o->Et.rp[o->E.ci[t] + 1]++;
    for (int64_t j = 0; j < s; ++j) o->Et.rp[j + 1] += o->Et.rp[j];
    int64_t *fill = xcalloc(s, sizeof(int64_t));
    for (int64_t r = 0; r < n; ++r)
        for (int64_t t = o->E.rp[r]; t < o->E.rp[r + 1]; ++t) {
            int32_t j = o->E.ci[t];
            int64_t q = o->Et.rp[j] + fill[j]++;
            o->Et.ci[q] = (int32_t)r;
            o->Et.v[q] = o->E.v[t];
        }
    free(fill);
}

/* ------------------------------------------------ local factorisation (Sec. 5) */

static int block_of(const orc_t *o, int64_t r) {
    int lo = 0, hi = o->p + 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (o->boff[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

/* Incomplete LDL^T on each diagonal block of A0, row by row, restricted to the
 * block's lower pattern (or the full lower triangle of the block in exact mode):
 *   L_ij = (a_ij - sum_{t<j} L_it D_t L_jt) / D_j   for j in pattern(i), j < i,
 *   D_i  = a_ii - sum_{t<i} L_it^2 D_t,
 * all sums over t ascending, restricted to positions present in both rows. */
/* with the Chebyshev C_alpha solver the interface block is factored as
 * D_alpha = blockdiag(C_i): only couplings inside one subdomain's interface */
static int in_pattern(const orc_t *o, int b, int64_t i, int64_t j) {
    if (o->csolve != 2 || b != o->p) return 1;
    return o->part[o->perm[i]] == o->part[o->perm[j]];
}

/* Factors rows from..n-1 (from = 0: everything; from = m: the interface
 * block again, keeping the B factors). */
static int factor_from(orc_t *o, int64_t from) {
    const int64_t n = o->n;
    int64_t cap, used;
    if (from == 0) {
        cap = o->A0.rp[n] + 16;
        used = 0;
        o->L.rp = xcalloc(n + 1, sizeof(int64_t));
        o->L.ci = xcalloc(cap, sizeof(int32_t));
        o->L.v = xcalloc(cap, sizeof(double));
        o->D = xcalloc(n, sizeof(double));
    } else {
        used = o->L.rp[from];
        cap = used + (o->A0.rp[n] - o->A0.rp[from]) + 16;
        o->L.ci = realloc(o->L.ci, cap * sizeof(int32_t));
        o->L.v = realloc(o->L.v, cap * sizeof(double));
    }
    o->breakdown_row = -1;
    double *w = xcalloc(n, sizeof(double));
    char *inrow = xcalloc(n, 1);
    for (int64_t i = from; i < n; ++i) {
        int b = block_of(o, i);
        int64_t lo = o->boff[b];
        /* pattern of row i strictly below the diagonal, inside block b */
        double aii = 0.0;
        int64_t cnt = 0;
        if (o->factor == 2) {
            cnt = i - lo;
            for (int64_t j = lo; j < i; ++j) w[j] = 0.0;
        }
        for (int64_t t = o->A0.rp[i]; t < o->A0.rp[i + 1]; ++t) {
            int32_t j = o->A0.ci[t];
            if (j == i) aii = o->A0.v[t];
            else if (j < i && j >= lo && in_pattern(o, b, i, j)) {
                if (o->factor != 2) ++cnt;
                w[j] = o->A0.v[t];
            }
        }
        if (used + cnt > cap) {
            cap = 2 * (used + cnt);
            o->L.ci = realloc(o->L.ci, cap * sizeof(int32_t));
            o->L.v = realloc(o->L.v, cap * sizeof(double));
        }
        int64_t start = used;
        if (o->factor == 2) {
            for (int64_t j = lo; j < i; ++j) o->L.ci[used++] = (int32_t)j;
        } else {
            for (int64_t t = o->A0.rp[i]; t < o->A0.rp[i + 1]; ++t) {
                int32_t j = o->A0.ci[t];
                if (j < i && j >= lo && in_pattern(o, b, i, j)) o->L.ci[used++] = j;
            }
        }
        for (int64_t q = start; q < used; ++q) inrow[o->L.ci[q]] = 1;
        /* ascending j: L_ij needs L_it for t < j, already final in w */
        for (int64_t q = start; q < used; ++q) {
            int32_t j = o->L.ci[q];
            double s = w[j];
            for (int64_t t2 = o->L.rp[j]; t2 < o->L.rp[j + 1]; ++t2) {
                int32_t t = o->L.ci[t2];
                if (inrow[t]) s -= w[t] * o->D[t] * o->L.v[t2];
            }
            w[j] = s / o->D[j];
        }
        double d = aii;
        for (int64_t q = start; q < used; ++q) {
            int32_t j = o->L.ci[q];
            o->L.v[q] = w[j];
            d -= w[j] * w[j] * o->D[j];
            inrow[j] = 0;
        }
        o->L.rp[i + 1] = used;
        o->D[i] = d;
        int bad = (o->factor == 1) ? (fabs(d) < 1e-14 * fabs(aii) || d == 0.0) : !(d > 0.0);
        if (bad) {
            o->breakdown_row = i;
            free(w); free(inrow);
            return ORC_E_BREAKDOWN;
        }
    }
    free(w); free(inrow);
    return ORC_OK;
}

static int build_factor(orc_t *o) { return factor_from(o, 0); }

static void cheb_solve(const orc_t *o, const double *x, double *z);

/* z = A0^{-1} x (internal order) with the local factors: per block
 * L y = x (unit lower), w = D^{-1} y, L^T z = w; with csolve the interface
 * block instead takes z_C = X x_C.  Blocks are independent. */
static void block_solve(const orc_t *o, int b, const double *x, double *z);

static void a0_solve(const orc_t *o, const double *x, double *z) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b <= o->p; ++b) {
        int64_t lo = o->boff[b];
        if (b == o->p && o->csolve == 1) {  /* z_C = X x_C */
            csr_mv(&o->X, o->s, x + lo, z + lo);
            continue;
        }
        if (b == o->p && o->csolve == 2) {
            cheb_solve(o, x, z);
            continue;
        }
        block_solve(o, b, x, z);
    }
}

/* L y = x, w = D^{-1} y, L^T z = w on the rows of block b (full-length vectors) */
static void block_solve(const orc_t *o, int b, const double *x, double *z) {
    {
        int64_t lo = o->boff[b], hi = o->boff[b + 1];
        for (int64_t i = lo; i < hi; ++i) {
            double s = x[i];
            for (int64_t t = o->L.rp[i]; t < o->L.rp[i + 1]; ++t) s -= o->L.v[t] * z[o->L.ci[t]];
            z[i] = s;
        }
        for (int64_t i = lo; i < hi; ++i) z[i] /= o->D[i];
        for (int64_t i = hi - 1; i >= lo; --i) {
            double zi = z[i];
            for (int64_t t = o->L.rp[i]; t < o->L.rp[i + 1]; ++t) z[o->L.ci[t]] -= o->L.v[t] * zi;
        }
    }
}

/* --------------------------------------- C_alpha approximate inverse (Sec. 4.3 (sec:csolve))
 *
 * X ~ C_alpha^{-1} by the self-preconditioned global minimal residual
 * iteration with numerical dropping (Algorithm alg:mr), X_0 = diag(C_alpha)^{-1}:
 *   R = I - C X;  Z = X R;  drop in Z;  beta = tr(R^T C Z) / ||C Z||_F^2;
 *   X = X + beta Z.
 * The paper does not state the dropping constants; the reading used here:
 *   - Z is symmetrised, z_ij := (z_ij + z_ji) / 2 (X R is symmetric in exact
 *     arithmetic when X is), so that X stays symmetric for CG;
 *   - dual threshold per column j: off-diagonal entries with
 *     |z_ij| < tol * ||z_:j||_2 are dropped, of the others the lfil largest in
 *     magnitude are kept (ties: lower row first); the diagonal is always kept;
 *     an entry survives only if it survives in its column and in its row's
 *     column (symmetric pattern);
 *   - the loop stops early if C Z = 0.
 * Arithmetic order (fixed so that any implementation can reproduce X
 * exactly): every entry of a sparse product sum_k a_ik b_kj is accumulated
 * from 0.0 by adding the terms in ascending k; tr(R^T W) and ||W||_F^2
 * (W = C Z) are single running sums over the stored entries of W in row-major
 * order with ascending columns; ||z_:j||^2 runs over column j in ascending
 * row order.  Matrices are CSR with ascending columns; symmetric ones serve
 * as their own CSC. */

/* c = a b (Gustavson, rows of a times rows of b) */
static void sp_mul(const csr_t *a, const csr_t *b, int64_t nrows, int64_t ncols, csr_t *c) {
    double *acc = xcalloc(ncols, sizeof(double));
    char *mark = xcalloc(ncols, 1);
    int32_t *list = xcalloc(ncols, sizeof(int32_t));
    int64_t cap = a->rp[nrows] + 16, used = 0;
    c->rp = xcalloc(nrows + 1, sizeof(int64_t));
    c->ci = xcalloc(cap, sizeof(int32_t));
    c->v = xcalloc(cap, sizeof(double));
    for (int64_t i = 0; i < nrows; ++i) {
        int64_t cnt = 0;
        for (int64_t t = a->rp[i]; t < a->rp[i + 1]; ++t) {
            const int32_t k = a->ci[t];
            const double aik = a->v[t];
            for (int64_t t2 = b->rp[k]; t2 < b->rp[k + 1]; ++t2) {
                const int32_t j = b->ci[t2];
                if (!mark[j]) { mark[j] = 1; acc[j] = 0.0; list[cnt++] = j; }
                acc[j] += aik * b->v[t2];
            }
        }
        if (used + cnt > cap) {
            cap = 2 * (used + cnt);
            c->ci = realloc(c->ci, cap * sizeof(int32_t));
            c->v = realloc(c->v, cap * sizeof(double));
        }
        ent_t *row = xcalloc(cnt > 0 ? cnt : 1, sizeof(ent_t));
        for (int64_t q = 0; q < cnt; ++q) { row[q].c = list[q]; row[q].v = acc[list[q]]; mark[list[q]] = 0; }
        qsort(row, cnt, sizeof(ent_t), ent_cmp);
        for (int64_t q = 0; q < cnt; ++q) { c->ci[used + q] = row[q].c; c->v[used + q] = row[q].v; }
        free(row);
        used += cnt;
        c->rp[i + 1] = used;
    }
    free(acc); free(mark); free(list);
}

/* value of entry (i, j) of a, 0 if not stored */
static double sp_get(const csr_t *a, int64_t i, int32_t j) {
    int64_t lo = a->rp[i], hi = a->rp[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (a->ci[mid] == j) return a->v[mid];
        if (a->ci[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}

static double frob(const csr_t *a, int64_t nrows) {
    double t = 0.0;
    for (int64_t q = 0; q < a->rp[nrows]; ++q) t += a->v[q] * a->v[q];
    return sqrt(t);
}

typedef struct { int32_t i; double a; } cand_t;

static int cand_cmp(const void *x, const void *y) {
    const cand_t *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? 1 : -1;  /* larger magnitude first */
    return (p->i > q->i) - (p->i < q->i);
}

/* R = I - W (W = C X) */
static void sp_i_minus(const csr_t *w, int64_t s, csr_t *r) {
    r->rp = xcalloc(s + 1, sizeof(int64_t));
    r->ci = xcalloc(w->rp[s] + s, sizeof(int32_t));
    r->v = xcalloc(w->rp[s] + s, sizeof(double));
    int64_t used = 0;
    for (int64_t i = 0; i < s; ++i) {
        int diag = 0;
        for (int64_t t = w->rp[i]; t < w->rp[i + 1]; ++t) {
            const int32_t j = w->ci[t];
            if (!diag && j > i) { r->ci[used] = (int32_t)i; r->v[used++] = 1.0; diag = 1; }
            if (j == i) { r->ci[used] = j; r->v[used++] = 1.0 - w->v[t]; diag = 1; }
            else { r->ci[used] = j; r->v[used++] = -w->v[t]; }
        }
        if (!diag) { r->ci[used] = (int32_t)i; r->v[used++] = 1.0; }
        r->rp[i + 1] = used;
    }
}

/* Builds X (Algorithm alg:mr) from C_alpha = A0[m:n, m:n]. */
static int build_cinv(orc_t *o, int nit, double tol, int lfil) {
    const int64_t s = o->s, m = o->m;
    csr_t C = {0}, X = {0};
    /* C_alpha with interface indices */
    C.rp = xcalloc(s + 1, sizeof(int64_t));
    int64_t cnt = 0;
    for (int64_t y = 0; y < s; ++y)
        for (int64_t t = o->A0.rp[m + y]; t < o->A0.rp[m + y + 1]; ++t) ++cnt;
    C.ci = xcalloc(cnt > 0 ? cnt : 1, sizeof(int32_t));
    C.v = xcalloc(cnt > 0 ? cnt : 1, sizeof(double));
    cnt = 0;
    for (int64_t y = 0; y < s; ++y) {
        for (int64_t t = o->A0.rp[m + y]; t < o->A0.rp[m + y + 1]; ++t) {
            C.ci[cnt] = (int32_t)(o->A0.ci[t] - m);
            C.v[cnt++] = o->A0.v[t];
        }
        C.rp[y + 1] = cnt;
    }
    /* X_0 = diag(C)^{-1} */
    X.rp = xcalloc(s + 1, sizeof(int64_t));
    X.ci = xcalloc(s > 0 ? s : 1, sizeof(int32_t));
    X.v = xcalloc(s > 0 ? s : 1, sizeof(double));
    for (int64_t y = 0; y < s; ++y) {
        const double d = sp_get(&C, y, (int32_t)y);
        if (!(d > 0.0)) { csr_free(&C); csr_free(&X); return ORC_E_BREAKDOWN; }
        X.ci[y] = (int32_t)y;
        X.v[y] = 1.0 / d;
        X.rp[y + 1] = y + 1;
    }
    free(o->x_res);
    o->x_res = xcalloc(nit + 1, sizeof(double));
    o->x_iters = 0;
    for (int it = 0; it <= nit; ++it) {
        csr_t W = {0}, R = {0};
        sp_mul(&C, &X, s, s, &W);
        sp_i_minus(&W, s, &R);
        csr_free(&W);
        o->x_res[it] = frob(&R, s);
        o->x_rinf = 0.0;
        for (int64_t i = 0; i < s; ++i) {
            double rs = 0.0;
            for (int64_t t = R.rp[i]; t < R.rp[i + 1]; ++t) rs += fabs(R.v[t]);
            if (rs > o->x_rinf) o->x_rinf = rs;
        }
        if (it == nit) { csr_free(&R); break; }
        /* Z = X R, symmetrised */
        csr_t Zh = {0};
        sp_mul(&X, &R, s, s, &Zh);
        csr_t Z = {0};
        Z.rp = xcalloc(s + 1, sizeof(int64_t));
        /* pattern of Zh + Zh^T: union of row i of Zh and column i of Zh */
        csr_t Zt = {0};
        {
            Zt.rp = xcalloc(s + 1, sizeof(int64_t));
            Zt.ci = xcalloc(Zh.rp[s] > 0 ? Zh.rp[s] : 1, sizeof(int32_t));
            Zt.v = xcalloc(Zh.rp[s] > 0 ? Zh.rp[s] : 1, sizeof(double));
            for (int64_t q = 0; q < Zh.rp[s]; ++q) Zt.rp[Zh.ci[q] + 1]++;
            for (int64_t y = 0; y < s; ++y) Zt.rp[y + 1] += Zt.rp[y];
            int64_t *fill = xcalloc(s > 0 ? s : 1, sizeof(int64_t));
            for (int64_t i = 0; i < s; ++i)
                for (int64_t t = Zh.rp[i]; t < Zh.rp[i + 1]; ++t) {
                    const int32_t j = Zh.ci[t];
                    const int64_t q = Zt.rp[j] + fill[j]++;
                    Zt.ci[q] = (int32_t)i;
                    Zt.v[q] = Zh.v[t];
                }
            free(fill);
        }
        int64_t cap = 2 * Zh.rp[s] + 1, used = 0;
        Z.ci = xcalloc(cap, sizeof(int32_t));
        Z.v = xcalloc(cap, sizeof(double));
        for (int64_t i = 0; i < s; ++i) {
            int64_t a = Zh.rp[i], ae = Zh.rp[i + 1], b = Zt.rp[i], be = Zt.rp[i + 1];
            while (a < ae || b < be) {
                int32_t j;
                double u = 0.0, w = 0.0;
                if (b >= be || (a < ae && Zh.ci[a] < Zt.ci[b])) { j = Zh.ci[a]; u = Zh.v[a++]; }
                else if (a >= ae || Zt.ci[b] < Zh.ci[a]) { j = Zt.ci[b]; w = Zt.v[b++]; }
                else { j = Zh.ci[a]; u = Zh.v[a++]; w = Zt.v[b++]; }
                Z.ci[used] = j;
                Z.v[used++] = 0.5 * (u + w);
            }
            Z.rp[i + 1] = used;
        }
        csr_free(&Zh); csr_free(&Zt);
        /* dual-threshold choice per column (= row, Z symmetric) */
        char *keep = xcalloc(Z.rp[s] > 0 ? Z.rp[s] : 1, 1);
        cand_t *cd = xcalloc(s > 0 ? s : 1, sizeof(cand_t));
        for (int64_t j = 0; j < s; ++j) {
            double nn = 0.0;
            for (int64_t t = Z.rp[j]; t < Z.rp[j + 1]; ++t) nn += Z.v[t] * Z.v[t];
            const double thr = tol * sqrt(nn);
            int64_t nc = 0;
            for (int64_t t = Z.rp[j]; t < Z.rp[j + 1]; ++t) {
                if (Z.ci[t] == j) { keep[t] = 1; continue; }
                if (fabs(Z.v[t]) < thr) continue;
                cd[nc].i = (int32_t)t;  /* position; ties broken by row = ascending position */
                cd[nc].a = fabs(Z.v[t]);
                ++nc;
            }
            qsort(cd, nc, sizeof(cand_t), cand_cmp);
            for (int64_t q = 0; q < nc && q < lfil; ++q) keep[cd[q].i] = 1;
        }
        free(cd);
        /* symmetric survivors: (i,j) kept in column j and (j,i) kept in column i */
        csr_t Zd = {0};
        Zd.rp = xcalloc(s + 1, sizeof(int64_t));
        Zd.ci = xcalloc(Z.rp[s] > 0 ? Z.rp[s] : 1, sizeof(int32_t));
        Zd.v = xcalloc(Z.rp[s] > 0 ? Z.rp[s] : 1, sizeof(double));
        used = 0;
        for (int64_t i = 0; i < s; ++i) {
            for (int64_t t = Z.rp[i]; t < Z.rp[i + 1]; ++t) {
                const int32_t j = Z.ci[t];
                if (!keep[t]) continue;
                /* position of (j, i) */
                int64_t lo = Z.rp[j], hi = Z.rp[j + 1] - 1, hit = -1;
                while (lo <= hi) {
                    int64_t mid = (lo + hi) / 2;
                    if (Z.ci[mid] == i) { hit = mid; break; }
                    if (Z.ci[mid] < i) lo = mid + 1; else hi = mid - 1;
                }
                if (hit < 0 || !keep[hit]) continue;
                Zd.ci[used] = j;
                Zd.v[used++] = Z.v[t];
            }
            Zd.rp[i + 1] = used;
        }
        free(keep);
        csr_free(&Z);
        /* beta = tr(R^T C Z) / ||C Z||_F^2 */
        csr_t CZ = {0};
        sp_mul(&C, &Zd, s, s, &CZ);
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < s; ++i)
            for (int64_t t = CZ.rp[i]; t < CZ.rp[i + 1]; ++t) {
                const double w = CZ.v[t];
                num += sp_get(&R, i, CZ.ci[t]) * w;
                den += w * w;
            }
        csr_free(&CZ); csr_free(&R);
        if (!(den > 0.0)) { csr_free(&Zd); break; }
        const double beta = num / den;
        /* X = X + beta Z (pattern union) */
        csr_t Xn = {0};
        Xn.rp = xcalloc(s + 1, sizeof(int64_t));
        Xn.ci = xcalloc(X.rp[s] + Zd.rp[s] + 1, sizeof(int32_t));
        Xn.v = xcalloc(X.rp[s] + Zd.rp[s] + 1, sizeof(double));
        used = 0;
        for (int64_t i = 0; i < s; ++i) {
            int64_t a = X.rp[i], ae = X.rp[i + 1], b = Zd.rp[i], be = Zd.rp[i + 1];
            while (a < ae || b < be) {
                if (b >= be || (a < ae && X.ci[a] < Zd.ci[b])) { Xn.ci[used] = X.ci[a]; Xn.v[used++] = X.v[a++]; }
                else if (a >= ae || Zd.ci[b] < X.ci[a]) { Xn.ci[used] = Zd.ci[b]; Xn.v[used++] = beta * Zd.v[b++]; }
                else { Xn.ci[used] = X.ci[a]; Xn.v[used++] = X.v[a++] + beta * Zd.v[b++]; }
            }
            Xn.rp[i + 1] = used;
        }
        csr_free(&Zd); csr_free(&X);
        X = Xn;
        o->x_iters = it + 1;
    }
    csr_free(&C);
    /* SPD certificate: I - C X is similar to I - C^{1/2} X C^{1/2}, whose
     * spectral radius is at most any induced norm of I - C X */
    o->x_spd = o->x_rinf < 1.0;
    csr_free(&o->X);
    o->X = X;
    o->csolve = 1;
    return ORC_OK;
}

/* ------------------------- C_alpha by preconditioned Chebyshev (Sec. 4.3 (sec:csolve))
 *
 * D_alpha = blockdiag(C_i), C_i the coupling of subdomain i's interface
 * unknowns, factored by incomplete LDL^T (the interface block of L, D).  The
 * spectrum of D_alpha^{-1} C_alpha is estimated by mc Lanczos steps on the
 * pencil (C_alpha, D_alpha) from the vector of ones, in the D_alpha inner
 * product; each extreme Ritz value is widened by its residual bound
 * beta_mc |s_mc| (the safeguard; a non-positive lower end becomes half the
 * smallest Ritz value).  A solve is nu steps of Chebyshev acceleration
 * (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1) from 0 on
 * [lo, hi]: theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta,
 * rho_0 = 1/sigma, d_0 = D^{-1} r_0 / theta, x_{k+1} = x_k + d_k,
 * r_{k+1} = r_k - C d_k, rho_{k+1} = 1/(2 sigma - rho_k),
 * d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) D^{-1} r_{k+1}. */

/* y_C = C_alpha x_C (full-length vectors, interface rows) */
static void c_mul(const orc_t *o, const double *x, double *y) {
    for (int64_t i = o->m; i < o->n; ++i) {
        double acc = 0.0;
        for (int64_t t = o->A0.rp[i]; t < o->A0.rp[i + 1]; ++t) acc += o->A0.v[t] * x[o->A0.ci[t]];
        y[i] = acc;
    }
}

static double c_dot(const orc_t *o, const double *a, const double *b) {
    double t = 0.0;
    for (int64_t i = o->m; i < o->n; ++i) t += a[i] * b[i];
    return t;
}

static void jacobi_eig(int m, double *T, double *ev, double *V);

static void cheb_solve(const orc_t *o, const double *x, double *z) {
    const int64_t m = o->m, n = o->n;
    const double th = 0.5 * (o->ch_hi + o->ch_lo), de = 0.5 * (o->ch_hi - o->ch_lo), sg = th / de;
    double *r = xcalloc(n, sizeof(double)), *d = xcalloc(n, sizeof(double)), *t = xcalloc(n, sizeof(double));
    double *cd = xcalloc(n, sizeof(double));
    for (int64_t i = m; i < n; ++i) r[i] = x[i];
    block_solve(o, o->p, r, t);
    for (int64_t i = m; i < n; ++i) { d[i] = t[i] / th; z[i] = d[i]; }
    double rho = 1.0 / sg;
    for (int k = 1; k < o->ch_nu; ++k) {
        c_mul(o, d, cd);
        for (int64_t i = m; i < n; ++i) r[i] -= cd[i];
        const double rn = 1.0 / (2.0 * sg - rho);
        block_solve(o, o->p, r, t);
        for (int64_t i = m; i < n; ++i) {
            d[i] = rn * rho * d[i] + (2.0 * rn / de) * t[i];
            z[i] += d[i];
        }
        rho = rn;
    }
    free(r); free(d); free(t); free(cd);
}

static void cheb_bounds(orc_t *o, int mc) {
    const int64_t m = o->m, n = o->n;
    double *r = xcalloc(n, sizeof(double)), *zz = xcalloc(n, sizeof(double));
    double *v = xcalloc(n, sizeof(double)), *y = xcalloc(n, sizeof(double));
    double *vp = xcalloc(n, sizeof(double)), *yp = xcalloc(n, sizeof(double)), *w = xcalloc(n, sizeof(double));
    double *al = xcalloc(mc, sizeof(double)), *be = xcalloc(mc, sizeof(double));
    for (int64_t i = m; i < n; ++i) r[i] = 1.0;
    block_solve(o, o->p, r, zz);
    const double b0 = sqrt(c_dot(o, r, zz));
    for (int64_t i = m; i < n; ++i) { v[i] = zz[i] / b0; y[i] = r[i] / b0; }
    double bprev = 0.0;
    int mm = 0;
    for (int j = 0; j < mc; ++j) {
        c_mul(o, v, w);
        al[j] = c_dot(o, v, w);
        for (int64_t i = m; i < n; ++i) w[i] -= al[j] * y[i] + bprev * yp[i];
        block_solve(o, o->p, w, zz);
        const double wz = c_dot(o, w, zz);
        mm = j + 1;
        be[j] = wz > 0.0 ? sqrt(wz) : 0.0;
        if (!(be[j] > 1e-14 * fabs(al[0]))) { be[j] = 0.0; break; }
        for (int64_t i = m; i < n; ++i) {
            vp[i] = v[i]; yp[i] = y[i];
            v[i] = zz[i] / be[j]; y[i] = w[i] / be[j];
        }
        bprev = be[j];
    }
    double *T = xcalloc((int64_t)mm * mm, sizeof(double)), *S = xcalloc((int64_t)mm * mm, sizeof(double));
    double *ev = xcalloc(mm, sizeof(double));
    for (int i = 0; i < mm; ++i) {
        T[i + i * mm] = al[i];
        if (i + 1 < mm) T[i + 1 + i * mm] = T[i + (i + 1) * mm] = be[i];
    }
    jacobi_eig(mm, T, ev, S);
    int imax = 0, imin = 0;
    for (int i = 1; i < mm; ++i) {
        if (ev[i] > ev[imax]) imax = i;
        if (ev[i] < ev[imin]) imin = i;
    }
    const double bl = be[mm - 1];
    o->ch_rhi = ev[imax];
    o->ch_rlo = ev[imin];
    o->ch_hi = ev[imax] + bl * fabs(S[(mm - 1) + (int64_t)imax * mm]);
    o->ch_lo = ev[imin] - bl * fabs(S[(mm - 1) + (int64_t)imin * mm]);
    if (!(o->ch_lo > 0.0)) o->ch_lo = 0.5 * ev[imin];
    free(r); free(zz); free(v); free(y); free(vp); free(yp); free(w); free(al); free(be); free(T); free(S); free(ev);
}

/* ---------------------------------------------------------- E and E^T products */

static void e_mul(const orc_t *o, const double *w, double *v) { csr_mv(&o->E, o->n, w, v); }
static void et_mul(const orc_t *o, const double *z, double *y) { csr_mv(&o->Et, o->s, z, y); }

/* Lanczos operator: DDLR-1 q -> E^T A0^{-1} E q ; DDLR-2 q -> E^T A0^{-1} A0^{-1} E q */
static void lanczos_op(const orc_t *o, int variant, const double *q, double *out, double *t1, double *t2) {
    e_mul(o, q, t1);
    a0_solve(o, t1, t2);
    if (variant == 2) {
        a0_solve(o, t2, t1);
        et_mul(o, t1, out);
    } else {
        et_mul(o, t2, out);
    }
}

/* ------------------------------------------- symmetric eigensolver (cyclic Jacobi) */

/* Eigen-decomposition of a dense symmetric m x m matrix T (column-major) by the
 * cyclic Jacobi method with the textbook rotation (Golub & Van Loan, Sec. 8.5).
 * On return ev holds eigenvalues, V (column-major) eigenvectors. */
static void jacobi_eig(int m, double *T, double *ev, double *V) {
    for (int i = 0; i < m * m; ++i) V[i] = 0.0;
    for (int i = 0; i < m; ++i) V[i + i * m] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
                double t = T[i + j * m] * T[i + j * m];
                tot += t;
                if (i != j) off += t;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int pp = 0; pp < m - 1; ++pp)
            for (int q = pp + 1; q < m; ++q) {
                double apq = T[pp + q * m];
                if (apq == 0.0) continue;
                double app = T[pp + pp * m], aqq = T[q + q * m];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* T <- J^T T J with J the rotation in plane (pp, q) */
                for (int r = 0; r < m; ++r) {
                    double trp = T[r + pp * m], trq = T[r + q * m];
                    T[r + pp * m] = c * trp - s * trq;
                    T[r + q * m] = s * trp + c * trq;
                }
                for (int r = 0; r < m; ++r) {
                    double tpr = T[pp + r * m], tqr = T[q + r * m];
                    T[pp + r * m] = c * tpr - s * tqr;
                    T[q + r * m] = s * tpr + c * tqr;
                }
                for (int r = 0; r < m; ++r) {
                    double vrp = V[r + pp * m], vrq = V[r + q * m];
                    V[r + pp * m] = c * vrp - s * vrq;
                    V[r + q * m] = s * vrp + c * vrq;
                }
            }
    }
    for (int i = 0; i < m; ++i) ev[i] = T[i + i * m];
}

/* ---------------------------------------------------------- Lanczos (Sec. 4.4 (sec:Lan)) */

/* m steps of Lanczos with full reorthogonalisation (classical Gram-Schmidt,
 * applied twice) on the s x s operator; start vector v0 (length s, internal
 * interface order).  Stops early on breakdown (beta_j <= 1e-12 max|alpha|).
 * Returns the number of steps taken. */
/* Sum of the k largest eigenvalues of the leading j x j block of T_m
 * (the sigma of the convergence test, eq. converge); cyclic Jacobi. */
static double ritz_top_sum(const orc_t *o, int j, int k) {
    double *T = xcalloc((int64_t)j * j, sizeof(double));
    double *V = xcalloc((int64_t)j * j, sizeof(double));
    double *ev = xcalloc(j, sizeof(double));
    for (int i = 0; i < j; ++i) {
        T[i + i * j] = o->ta[i];
        if (i + 1 < j) { T[i + 1 + i * j] = o->tb[i]; T[i + (i + 1) * j] = o->tb[i]; }
    }
    jacobi_eig(j, T, ev, V);
    /* k largest by repeated selection */
    double sum = 0.0;
    for (int c = 0; c < k && c < j; ++c) {
        int best = -1;
        for (int i = 0; i < j; ++i)
            if (ev[i] == ev[i] && (best < 0 || ev[i] > ev[best])) best = i;
        sum += ev[best];
        ev[best] = NAN;
    }
    free(T); free(V); free(ev);
    return sum;
}

/* Make room for m_max Lanczos steps (q_1..q_{m_max+1}), keeping the run so far. */
static void lanczos_reserve(orc_t *o, int m_max) {
    if (m_max + 1 <= o->qcap) return;
    const int64_t s = o->s;
    double *Q = xcalloc(s * (int64_t)(m_max + 1), sizeof(double));
    double *ta = xcalloc(m_max + 1, sizeof(double)), *tb = xcalloc(m_max + 1, sizeof(double));
    double *op = xcalloc(m_max + 2, sizeof(double)), *oc = xcalloc(m_max + 2, sizeof(double));
    int *rs = xcalloc(m_max + 1, sizeof(int));
    if (o->Q) memcpy(Q, o->Q, s * (int64_t)(o->msteps + 1) * sizeof(double));
    if (o->ta) memcpy(ta, o->ta, o->msteps * sizeof(double));
    if (o->tb) memcpy(tb, o->tb, o->msteps * sizeof(double));
    if (o->om_prev) memcpy(op, o->om_prev, (o->msteps + 1) * sizeof(double));
    if (o->om_cur) memcpy(oc, o->om_cur, (o->msteps + 1) * sizeof(double));
    if (o->rsteps) memcpy(rs, o->rsteps, o->msteps * sizeof(int));
    free(o->Q); free(o->ta); free(o->tb); free(o->om_prev); free(o->om_cur); free(o->rsteps);
    o->Q = Q; o->ta = ta; o->tb = tb; o->om_prev = op; o->om_cur = oc; o->rsteps = rs;
    o->qcap = m_max + 1;
}

/* Classical Gram-Schmidt applied twice: w loses its components along q_0..q_j. */
static void cgs2(const orc_t *o, int j, double *w, double *c) {
    const int64_t s = o->s;
    for (int pass = 0; pass < 2; ++pass) {
        for (int l = 0; l <= j; ++l) c[l] = dot(o->Q + s * (int64_t)l, w, s);
        for (int l = 0; l <= j; ++l) {
            const double *ql = o->Q + s * (int64_t)l;
            for (int64_t i = 0; i < s; ++i) w[i] -= c[l] * ql[i];
        }
    }
}

/* Partial reorthogonalisation (Simon, "The Lanczos algorithm with partial
 * reorthogonalization", Math. Comp. 42, 1984), the scheme the paper uses.
 * omega_i estimates q_i^T q of the Lanczos vectors; for the new vector j+1
 * (before normalisation, norm b0) Simon's recurrence gives, for i < j,
 *   b0 om_new_i = beta_i om_cur_{i+1} + (alpha_i - alpha_j) om_cur_i
 *                 + beta_{i-1} om_cur_{i-1} - beta_{j-1} om_prev_i + theta,
 * theta = 2 eps ||T||_est with the sign of the rest (the rounding term, eps =
 * 2^-52, ||T||_est the running max of |alpha_i| + beta_i + beta_{i-1});
 * om_new_j = eps sqrt(s) (the local rounding level) and om_new_{j+1} = 1.
 * When some |om_new_i| (i <= j) exceeds sqrt(eps) -- or when the previous
 * step was reorthogonalised, as Simon requires for the next vector too --
 * the new vector is orthogonalised against q_0..q_j (classical Gram-Schmidt
 * twice) and its estimates reset to eps.  Returns 1 if it did so. */
static int pro_step(orc_t *o, int j, double aj, double b0, double *w, double *c) {
    const double eps = 2.220446049250313e-16;
    const double bprev = j > 0 ? o->tb[j - 1] : 0.0;
    const double tn = fabs(aj) + b0 + bprev;
    if (tn > o->tnorm) o->tnorm = tn;
    double *on = xcalloc(j + 2, sizeof(double));
    double big = 0.0;
    for (int i = 0; i < j; ++i) {
        double t = o->tb[i] * o->om_cur[i + 1] + (o->ta[i] - aj) * o->om_cur[i];
        if (i > 0) t += o->tb[i - 1] * o->om_cur[i - 1];
        t -= bprev * o->om_prev[i];
        t += (t >= 0.0 ? 1.0 : -1.0) * 2.0 * eps * o->tnorm;
        on[i] = t / b0;
        if (fabs(on[i]) > big) big = fabs(on[i]);
    }
    on[j] = eps * sqrt((double)o->s);
    if (on[j] > big) big = on[j];
    on[j + 1] = 1.0;
    const int forced = o->force_next;
    const int need = forced || big > sqrt(eps);
    if (need) {
        cgs2(o, j, w, c);
        for (int i = 0; i <= j; ++i) on[i] = eps;
        o->force_next = forced ? 0 : 1;
        o->nreorth++;
    } else {
        o->force_next = 0;
    }
    memcpy(o->om_prev, o->om_cur, (j + 1) * sizeof(double));
    memcpy(o->om_cur, on, (j + 2) * sizeof(double));
    free(on);
    return need;
}

/* Lanczos on E^T A0^{-1} E (DDLR-1) or E^T A0^{-2} E (DDLR-2), Sec. 4.4 (sec:Lan), with
 * full reorthogonalisation (classical Gram-Schmidt applied twice), or with
 * partial reorthogonalisation (pro_step) as the paper does.  Continues
 * the stored run from step msteps up to m_max steps.  With check > 0 it stops
 * early at the first step m that is a multiple of check, with m >= k + 1,
 * where the sums of the k largest Ritz values of T_{m-1} and T_m satisfy
 * |sigma_m - sigma_{m-1}| / |sigma_{m-1}| < eps (eq. converge). */
static int lanczos_run(orc_t *o, int m_max, int check, double eps, int k) {
    const int64_t s = o->s, n = o->n;
    const int variant = o->lvariant;
    lanczos_reserve(o, m_max);
    double *w = xcalloc(s, sizeof(double));
    double *c = xcalloc(m_max + 1, sizeof(double));
    double *t1 = xcalloc(n, sizeof(double)), *t2 = xcalloc(n, sizeof(double));
    int j;
    for (j = o->msteps; j < m_max && !o->broke; ++j) {
        double *qj = o->Q + s * (int64_t)j;
        lanczos_op(o, variant, qj, w, t1, t2);
        double aj = dot(qj, w, s);
        o->ta[j] = aj;
        if (fabs(aj) > o->amax) o->amax = fabs(aj);
        for (int64_t i = 0; i < s; ++i) w[i] -= aj * qj[i];
        if (j > 0) {
            double *qp = o->Q + s * (int64_t)(j - 1);
            for (int64_t i = 0; i < s; ++i) w[i] -= o->tb[j - 1] * qp[i];
        }
        double bj;
        o->rsteps[j] = 0;
        if (o->reorth == 0) {
            cgs2(o, j, w, c);
            bj = nrm2(w, s);
        } else {
            bj = nrm2(w, s);
            if (o->reorth == 1 && bj > 1e-12 * o->amax) {
                o->rsteps[j] = pro_step(o, j, aj, bj, w, c);
                if (o->rsteps[j]) bj = nrm2(w, s);
            }
        }
        o->tb[j] = bj;
        o->msteps = j + 1;
        if (bj <= 1e-12 * o->amax) { o->broke = 1; break; }  /* invariant subspace found */
        double *qn = o->Q + s * (int64_t)(j + 1);  /* q_{j+1}, kept also after the last step */
        for (int64_t i = 0; i < s; ++i) qn[i] = w[i] / bj;
        const int m = j + 1;
        if (check > 0 && m % check == 0 && m >= k + 1) {
            const double sp = ritz_top_sum(o, m - 1, k), sm = ritz_top_sum(o, m, k);
            if (fabs((sm - sp) / sp) < eps) break;
        }
    }
    free(w); free(c); free(t1); free(t2);
    return o->msteps;
}

/* Start a new run from v0 (interface order, not normalised). */
static void lanczos_start(orc_t *o, int variant, const double *v0) {
    const int64_t s = o->s;
    o->msteps = 0;
    o->broke = 0;
    o->amax = 0.0;
    o->lvariant = variant;
    o->tnorm = 0.0;
    o->force_next = 0;
    o->nreorth = 0;
    lanczos_reserve(o, 1);
    o->om_cur[0] = 1.0;  /* q_0^T q_0 */
    double nv = nrm2(v0, s);
    for (int64_t i = 0; i < s; ++i) o->Q[i] = v0[i] / nv;
}

/* Ritz pairs of T_m (descending, stable by index); each eigenvector's
 * largest-magnitude entry (lowest index on ties) is made positive. */
static void ritz(orc_t *o, double *Y) {
    int m = o->msteps;
    double *T = xcalloc((int64_t)m * m, sizeof(double));
    double *V = xcalloc((int64_t)m * m, sizeof(double));
    double *ev = xcalloc(m, sizeof(double));
    for (int i = 0; i < m; ++i) {
        T[i + i * m] = o->ta[i];
        if (i + 1 < m) { T[i + 1 + i * m] = o->tb[i]; T[i + (i + 1) * m] = o->tb[i]; }
    }
    jacobi_eig(m, T, ev, V);
    int *idx = xcalloc(m, sizeof(int));
    for (int i = 0; i < m; ++i) idx[i] = i;
    for (int i = 1; i < m; ++i) {  /* insertion sort, descending, stable */
        int v = idx[i], q = i;
        while (q > 0 && ev[idx[q - 1]] < ev[v]) { idx[q] = idx[q - 1]; --q; }
        idx[q] = v;
    }
    free(o->ritz);
    o->ritz = xcalloc(m, sizeof(double));
    for (int i = 0; i < m; ++i) {
        o->ritz[i] = ev[idx[i]];
        const double *src = V + (int64_t)idx[i] * m;
        int big = 0;
        for (int r = 1; r < m; ++r) if (fabs(src[r]) > fabs(src[big])) big = r;
        double sg = src[big] < 0 ? -1.0 : 1.0;
        for (int r = 0; r < m; ++r) Y[r + (int64_t)i * m] = sg * src[r];
    }
    free(T); free(V); free(ev); free(idx);
}

/* Cholesky of a dense SPD k x k (column-major, lower), returns 0 on success */
static int dense_chol(int k, double *a) {
    for (int j = 0; j < k; ++j) {
        double d = a[j + j * k];
        for (int t = 0; t < j; ++t) d -= a[j + t * k] * a[j + t * k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        a[j + j * k] = d;
        for (int i = j + 1; i < k; ++i) {
            double v = a[i + j * k];
            for (int t = 0; t < j; ++t) v -= a[i + t * k] * a[j + t * k];
            a[i + j * k] = v / d;
        }
    }
    return 0;
}

/* The SPD results (Propositions on SPD-ness of DDLR-1 and DDLR-2) assume A0
 * SPD; with an indefinite local factor the preconditioner is not SPD. */
static int pivots_positive(const orc_t *o) {
    const int64_t last = o->csolve == 1 ? o->m : o->n;
    for (int64_t i = 0; i < last; ++i)
        if (!(o->D[i] > 0.0)) return 0;
    if (o->csolve == 1) return o->x_spd;
    if (o->csolve == 2) return o->ch_rlo > 0.0;  /* the polynomial is positive on the safeguarded interval */
    return 1;
}

static int ddlr2_hk(orc_t *o, int k, const double *EV);

/* Low-rank part of the preconditioner from the Lanczos run (Sec. 3.2 / 3.3). */
static int build_lowrank(orc_t *o, int variant, int k, int thetamode) {
    const int m = o->msteps;
    const int64_t s = o->s, n = o->n;
    if (k < 1 || k + 1 > m) return ORC_E_LANCZOS;
    double *Y = xcalloc((int64_t)m * m, sizeof(double));
    ritz(o, Y);
    free(o->U); free(o->lam); free(o->dvec); free(o->Hk);
    o->U = NULL; o->lam = NULL; o->dvec = NULL; o->Hk = NULL;
    o->variant = variant;
    o->k = k;
    /* Q_m Y_k */
    double *QY = xcalloc(s * (int64_t)k, sizeof(double));
    for (int j = 0; j < k; ++j)
        for (int l = 0; l < m; ++l) {
            double y = Y[l + (int64_t)j * m];
            const double *ql = o->Q + s * (int64_t)l;
            double *dst = QY + s * (int64_t)j;
            for (int64_t i = 0; i < s; ++i) dst[i] += y * ql[i];
        }
    free(Y);
    int st = ORC_OK;
    if (variant == 1) {
        o->U = QY;
        o->lam = xcalloc(k, sizeof(double));
        for (int j = 0; j < k; ++j) o->lam[j] = o->ritz[j];
        o->theta = thetamode == 1 ? 0.0 : o->ritz[k];
        /* G_{k,theta}^{-1} needs theta < 1 and lambda_j != 1 (eq. gkt); the
         * preconditioner is SPD only if also lambda_1 < 1 (Sec. 5), which is
         * recorded in spd and left to the caller (CG needs it, GMRES does not). */
        if (!(o->theta < 1.0)) st = ORC_E_NOT_SPD;
        o->c0 = 1.0 / (1.0 - o->theta);
        o->dvec = xcalloc(k, sizeof(double));
        for (int j = 0; j < k; ++j) {
            if (o->lam[j] == 1.0) st = ORC_E_NOT_SPD;
            o->dvec[j] = 1.0 / (1.0 - o->lam[j]) - o->c0;
        }
        o->spd = (o->lam[0] < 1.0) && st == ORC_OK && pivots_positive(o);
    } else {
        /* V_k = Q_m Y_k, U_k = A0^{-1} E V_k, H_k = (I - U_k^T E V_k)^{-1} */
        double *EV = xcalloc(n * (int64_t)k, sizeof(double));
        o->U = xcalloc(n * (int64_t)k, sizeof(double));
        for (int j = 0; j < k; ++j) {
            e_mul(o, QY + s * (int64_t)j, EV + n * (int64_t)j);
            a0_solve(o, EV + n * (int64_t)j, o->U + n * (int64_t)j);
        }
        free(QY);
        st = ddlr2_hk(o, k, EV);
        free(EV);
    }
    return st;
}

/* H_k = (I - U_k^T E V_k)^{-1} from o->U and EV = E V_k (both n x k), the
 * product symmetrised; the preconditioner of eq. (Form2a) is SPD only if
 * I - sym(K) is (Lemma on H_k). */
static int ddlr2_hk(orc_t *o, int k, const double *EV) {
    const int64_t n = o->n;
    int st = ORC_OK;
    {
        double *K = xcalloc((int64_t)k * k, sizeof(double));
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i) K[i + j * k] = dot(o->U + n * (int64_t)i, EV + n * (int64_t)j, n);
        double *Mx = xcalloc((int64_t)k * k, sizeof(double));
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i)
                Mx[i + j * k] = (i == j ? 1.0 : 0.0) - 0.5 * (K[i + j * k] + K[j + i * k]);
        if (dense_chol(k, Mx) != 0) {
            st = ORC_E_NOT_SPD;
        } else {
            /* H_k = (L L^T)^{-1}, column by column */
            o->Hk = xcalloc((int64_t)k * k, sizeof(double));
            for (int c = 0; c < k; ++c) {
                double *h = o->Hk + (int64_t)c * k;
                for (int i = 0; i < k; ++i) {
                    double v = (i == c) ? 1.0 : 0.0;
                    for (int t = 0; t < i; ++t) v -= Mx[i + t * k] * h[t];
                    h[i] = v / Mx[i + i * k];
                }
                for (int i = k - 1; i >= 0; --i) {
                    double v = h[i];
                    for (int t = i + 1; t < k; ++t) v -= Mx[t + i * k] * h[t];
                    h[i] = v / Mx[i + i * k];
                }
            }
        }
        free(K); free(Mx);
        o->spd = (st == ORC_OK) && pivots_positive(o);
        o->theta = 0.0;
        o->c0 = 0.0;
    }
    return st;
}

/* ---------------------------------------------- preconditioner application (Sec. 4.2) */

/* u = M^{-1} x, internal order.  DDLR-1 evaluates eq. (Mprec) as written:
 * M^{-1} = A0^{-1} + (A0^{-1} E) G_{k,theta}^{-1} (A0^{-1} E)^T, with
 * G_{k,theta}^{-1} = c0 I + U_k diag(d) U_k^T from eq. (gkt), i.e.
 * u = z + A0^{-1} E G^{-1} E^T z with z = A0^{-1} x (A0 symmetric). */
static void apply_internal(const orc_t *o, const double *x, double *u) {
    const int64_t n = o->n, s = o->s;
    const int k = o->k;
    if (o->variant == 1) {
        double *z = xcalloc(n, sizeof(double)), *y = xcalloc(s, sizeof(double));
        double *g = xcalloc(s, sizeof(double)), *t = xcalloc(n, sizeof(double));
        double *c = xcalloc(k, sizeof(double)), *corr = xcalloc(n, sizeof(double));
        a0_solve(o, x, z);                        /* z = A0^{-1} x */
        et_mul(o, z, y);                          /* y = (A0^{-1} E)^T x = E^T z */
        for (int j = 0; j < k; ++j) c[j] = o->dvec[j] * dot(o->U + s * (int64_t)j, y, s);
        for (int64_t i = 0; i < s; ++i) {         /* g = G_{k,theta}^{-1} y, eq. (gkt) */
            double a = o->c0 * y[i];
            for (int j = 0; j < k; ++j) a += o->U[i + s * (int64_t)j] * c[j];
            g[i] = a;
        }
        e_mul(o, g, t);                           /* t = E g */
        a0_solve(o, t, corr);                     /* corr = (A0^{-1} E) g */
        for (int64_t i = 0; i < n; ++i) u[i] = z[i] + corr[i];
        free(z); free(y); free(g); free(t); free(c); free(corr);
    } else if (o->variant == 2) {
        a0_solve(o, x, u);
        double *c = xcalloc(k, sizeof(double)), *h = xcalloc(k, sizeof(double));
        for (int j = 0; j < k; ++j) c[j] = dot(o->U + n * (int64_t)j, x, n);
        for (int i = 0; i < k; ++i) {
            double t = 0.0;
            for (int j = 0; j < k; ++j) t += o->Hk[i + (int64_t)j * k] * c[j];
            h[i] = t;
        }
        for (int j = 0; j < k; ++j) {
            const double *uj = o->U + n * (int64_t)j;
            for (int64_t i = 0; i < n; ++i) u[i] += uj[i] * h[j];
        }
        free(c); free(h);
    } else {
        a0_solve(o, x, u);
    }
}

static void to_internal(const orc_t *o, const double *xu, double *xi) {
    for (int64_t i = 0; i < o->n; ++i) xi[i] = xu[o->perm[i]];
}
static void to_user(const orc_t *o, const double *xi, double *xu) {
    for (int64_t i = 0; i < o->n; ++i) xu[o->perm[i]] = xi[i];
}

/* ================================================================ public API */

void orc_free(orc_t *o) {
    if (!o) return;
    csr_free(&o->A); csr_free(&o->Ap); csr_free(&o->A0); csr_free(&o->E); csr_free(&o->Et); csr_free(&o->L);
    free(o->om_prev); free(o->om_cur); free(o->rsteps);
    free(o->part); free(o->iface); free(o->perm); free(o->iperm); free(o->colour); free(o->boff);
    free(o->D); free(o->U); free(o->lam); free(o->dvec); free(o->Hk);
    free(o->ta); free(o->tb); free(o->ritz); free(o->Q);
    csr_free(&o->X); free(o->x_res);
    free(o);
}

/* Setup up to and including the local factorisation. */
orc_t *orc_create(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const int32_t *part,
                  int32_t p, double alpha, int corder, int factor, int *status) {
    orc_t *o = xcalloc(1, sizeof(orc_t));
    o->n = n; o->p = p; o->alpha = alpha; o->corder = corder; o->factor = factor;
    o->A.rp = xcalloc(n + 1, sizeof(int64_t));
    memcpy(o->A.rp, rp, (n + 1) * sizeof(int64_t));
    o->A.ci = xcalloc(rp[n], sizeof(int32_t));
    memcpy(o->A.ci, ci, rp[n] * sizeof(int32_t));
    o->A.v = xcalloc(rp[n], sizeof(double));
    memcpy(o->A.v, v, rp[n] * sizeof(double));
    o->part = xcalloc(n, sizeof(int32_t));
    memcpy(o->part, part, n * sizeof(int32_t));
    *status = ORC_OK;
    if (p < 1 || !(alpha > 0.0)) { *status = ORC_E_INVALID; return o; }
    /* the method is for symmetric A: check sorted in-range columns and a_ij == a_ji */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
            int32_t j = ci[t];
            if (j < 0 || j >= n || (t > rp[i] && ci[t - 1] >= j)) { *status = ORC_E_INVALID; return o; }
            int64_t lo = rp[j], hi = rp[j + 1] - 1, hit = -1;
            while (lo <= hi) {
                int64_t mid = (lo + hi) / 2;
                if (ci[mid] == i) { hit = mid; break; }
                if (ci[mid] < i) lo = mid + 1; else hi = mid - 1;
            }
            if (hit < 0 || v[hit] != v[t]) { *status = ORC_E_NOT_SYMMETRIC; return o; }
        }
    int st = build_ordering(o);
    if (st != ORC_OK) { *status = st; return o; }
    build_split(o);
    *status = build_factor(o);
    return o;
}

int64_t orc_size(const orc_t *o, int what) {
    switch (what) {
    case 0: return o->n;
    case 1: return o->m;
    case 2: return o->s;
    case 3: return o->L.rp[o->n];
    case 4: return o->A0.rp[o->n];
    case 5: return o->E.rp[o->n];
    case 6: return o->ncolours;
    case 7: return o->msteps;
    case 8: return o->breakdown_row;
    case 9: return o->k;
    case 10: return o->spd;
    case 11: return o->csolve == 1 ? o->X.rp[o->s] : 0;
    case 12: return o->x_iters;
    case 13: return o->x_spd;
    default: return -1;
    }
}

void orc_ordering(const orc_t *o, int32_t *perm, int32_t *iface, int32_t *colour, int64_t *boff) {
    memcpy(perm, o->perm, o->n * sizeof(int32_t));
    memcpy(iface, o->iface, o->n * sizeof(int32_t));
    if (o->s > 0) memcpy(colour, o->colour, o->s * sizeof(int32_t));
    memcpy(boff, o->boff, (o->p + 2) * sizeof(int64_t));
}

/* which: 0 = P A P^T, 1 = A0, 2 = E, 3 = L (strict lower); internal indices */
void orc_csr(const orc_t *o, int which, int64_t *rp, int32_t *ci, double *v) {
    const csr_t *a = which == 0 ? &o->Ap : which == 1 ? &o->A0 : which == 2 ? &o->E : &o->L;
    memcpy(rp, a->rp, (o->n + 1) * sizeof(int64_t));
    memcpy(ci, a->ci, a->rp[o->n] * sizeof(int32_t));
    memcpy(v, a->v, a->rp[o->n] * sizeof(double));
}

void orc_diag(const orc_t *o, double *D) { memcpy(D, o->D, o->n * sizeof(double)); }

/* Switches the C_alpha solve to the MR approximate inverse (nit steps, drop
 * tolerance tol, at most lfil kept off-diagonal entries per column); a
 * breakdown of the C_alpha factor no longer matters.  Call before the
 * low-rank build. */
int orc_use_cinv(orc_t *o, int nit, double tol, int lfil) {
    if (nit < 0 || !(tol >= 0.0) || lfil < 0 || o->s < 1) return ORC_E_INVALID;
    if (o->breakdown_row >= 0 && o->breakdown_row < o->m) return ORC_E_BREAKDOWN;
    const int st = build_cinv(o, nit, tol, lfil);
    if (st == ORC_OK && o->breakdown_row >= o->m) o->breakdown_row = -1;
    return st;
}

/* Switches the C_alpha solve to nu preconditioned Chebyshev steps with the
 * block-Jacobi D_alpha (the interface block is factored again on the
 * subdomains' own couplings) and a spectrum estimate from mc Lanczos steps
 * on (C_alpha, D_alpha).  Call before the low-rank build. */
int orc_use_cheb(orc_t *o, int nu, int mc) {
    if (nu < 1 || mc < 2 || o->s < 2 || o->factor == 2) return ORC_E_INVALID;
    if (o->breakdown_row >= 0 && o->breakdown_row < o->m) return ORC_E_BREAKDOWN;
    o->csolve = 2;
    const int st = factor_from(o, o->m);
    if (st != ORC_OK) return st;
    cheb_bounds(o, mc);
    o->ch_nu = nu;
    return ORC_OK;
}

/* lo, hi (safeguarded interval), smallest and largest Ritz value */
void orc_cheb(const orc_t *o, double *out) {
    out[0] = o->ch_lo; out[1] = o->ch_hi; out[2] = o->ch_rlo; out[3] = o->ch_rhi;
}

/* X (s x s CSR, interface indices), nnz via orc_size(o, 11); res: the
 * residual norms ||I - C X_j||_F, j = 0..x_iters (orc_size(o, 12)), then
 * ||I - C X||_inf of the final X */
void orc_cinv(const orc_t *o, int64_t *rp, int32_t *ci, double *v, double *res) {
    memcpy(rp, o->X.rp, (o->s + 1) * sizeof(int64_t));
    memcpy(ci, o->X.ci, o->X.rp[o->s] * sizeof(int32_t));
    memcpy(v, o->X.v, o->X.rp[o->s] * sizeof(double));
    memcpy(res, o->x_res, (o->x_iters + 1) * sizeof(double));
    res[o->x_iters + 1] = o->x_rinf;
}

/* z = A0^{-1} x, user order, nrhs columns with leading dimension n */
void orc_a0_solve(const orc_t *o, int nrhs, const double *x, double *z) {
    double *a = xcalloc(o->n, sizeof(double)), *b = xcalloc(o->n, sizeof(double));
    for (int r = 0; r < nrhs; ++r) {
        to_internal(o, x + o->n * (int64_t)r, a);
        a0_solve(o, a, b);
        to_user(o, b, z + o->n * (int64_t)r);
    }
    free(a); free(b);
}

/* Lanczos + low-rank build. v0: length n, user order (interface entries used). */
/* Low-rank build from a Lanczos run of m steps (check = 0), or of up to m
 * steps stopped by eq. (converge) tested every check steps with tolerance eps
 * (Sec. 5: every 10 steps, eps = 1e-4, at most 5k steps). */
int orc_lowrank_ctl(orc_t *o, int variant, int k, int m, int check, double eps, int thetamode, const double *v0) {
    if (variant != 1 && variant != 2) return ORC_E_INVALID;
    if (k < 1 || k + 1 > o->s || m < k + 1 || check < 0) return ORC_E_INVALID;
    if (m > o->s) m = (int)o->s;
    double *q = xcalloc(o->s, sizeof(double));
    for (int64_t y = 0; y < o->s; ++y) q[y] = v0[o->perm[o->m + y]];
    lanczos_start(o, variant, q);
    free(q);
    lanczos_run(o, m, check, eps, k);
    if (o->msteps < k + 1) return ORC_E_LANCZOS;
    return build_lowrank(o, variant, k, thetamode);
}

/* DDLR-2 with U_k and V_k from the Lanczos (Golub-Kahan) bidiagonalisation of
 * B = A0^{-1} E (n x s), the alternative build named in Sec. 4.4 (sec:Lan) (Golub & Van
 * Loan, Sec. 10.4).  From a unit q_1 (the interface entries of v0):
 *   p_j = (B q_j - beta_{j-1} p_{j-1}) / alpha_j,
 *   q_{j+1} = (B^T p_j - alpha_j q_j) / beta_j,   B^T = E^T A0^{-1},
 * with alpha_j, beta_j the norms and full reorthogonalisation of p_j against
 * p_1..p_{j-1} and of q_{j+1} against q_1..q_j (classical Gram-Schmidt
 * twice), so B Q_m = P_m B_m with B_m upper bidiagonal (alpha on the
 * diagonal, beta above).  The right singular vectors Z of B_m are the
 * eigenvectors of B_m^T B_m (cyclic Jacobi; eigenvalues sigma^2 descending,
 * largest-|.| entry of each vector positive); then V_k = Q_m Z_k and
 * U_k = P_m B_m Z_k (= B V_k), and H_k as in the Lanczos route.  Two A0
 * solves per step and none afterwards.  The run stops early when alpha_j or
 * beta_j <= 1e-12 times the largest alpha so far.  The record keeps alpha,
 * beta and the sigma^2 (Ritz values of E^T A0^{-2} E). */
int orc_lowrank_gk(orc_t *o, int k, int m, const double *v0) {
    const int64_t s = o->s, n = o->n;
    if (k < 1 || k + 1 > s || m < k + 1) return ORC_E_INVALID;
    if (m > s) m = (int)s;
    double *Q = xcalloc(s * (int64_t)(m + 1), sizeof(double));
    double *P = xcalloc(n * (int64_t)m, sizeof(double));
    double *al = xcalloc(m, sizeof(double)), *be = xcalloc(m, sizeof(double));
    double *c = xcalloc(m + 1, sizeof(double));
    double *t = xcalloc(n, sizeof(double)), *w = xcalloc(s, sizeof(double));
    for (int64_t y = 0; y < s; ++y) Q[y] = v0[o->perm[o->m + y]];
    const double nq = nrm2(Q, s);
    for (int64_t y = 0; y < s; ++y) Q[y] /= nq;
    double amax = 0.0;
    int meff = 0;
    for (int j = 0; j < m; ++j) {
        double *pj = P + n * (int64_t)j;
        const double *qj = Q + s * (int64_t)j;
        e_mul(o, qj, t);
        a0_solve(o, t, pj);  /* B q_j */
        if (j > 0) {
            const double *pp = P + n * (int64_t)(j - 1);
            for (int64_t i = 0; i < n; ++i) pj[i] -= be[j - 1] * pp[i];
        }
        for (int pass = 0; pass < 2; ++pass) {
            for (int l = 0; l < j; ++l) c[l] = dot(P + n * (int64_t)l, pj, n);
            for (int l = 0; l < j; ++l) {
                const double *pl = P + n * (int64_t)l;
                for (int64_t i = 0; i < n; ++i) pj[i] -= c[l] * pl[i];
            }
        }
        al[j] = nrm2(pj, n);
        if (al[j] > amax) amax = al[j];
        if (!(al[j] > 1e-12 * amax)) break;
        for (int64_t i = 0; i < n; ++i) pj[i] /= al[j];
        a0_solve(o, pj, t);
        et_mul(o, t, w);  /* B^T p_j */
        for (int64_t i = 0; i < s; ++i) w[i] -= al[j] * qj[i];
        for (int pass = 0; pass < 2; ++pass) {
            for (int l = 0; l <= j; ++l) c[l] = dot(Q + s * (int64_t)l, w, s);
            for (int l = 0; l <= j; ++l) {
                const double *ql = Q + s * (int64_t)l;
                for (int64_t i = 0; i < s; ++i) w[i] -= c[l] * ql[i];
            }
        }
        be[j] = nrm2(w, s);
        meff = j + 1;
        if (!(be[j] > 1e-12 * amax)) break;
        double *qn = Q + s * (int64_t)(j + 1);
        for (int64_t i = 0; i < s; ++i) qn[i] = w[i] / be[j];
    }
    free(c); free(t); free(w);
    int st = ORC_OK;
    if (meff < k + 1) st = ORC_E_LANCZOS;
    if (st == ORC_OK) {
        /* B_m^T B_m: diagonal alpha_j^2 + beta_{j-1}^2, off-diagonal alpha_j beta_j */
        const int mm = meff;
        double *T = xcalloc((int64_t)mm * mm, sizeof(double));
        double *V = xcalloc((int64_t)mm * mm, sizeof(double));
        double *ev = xcalloc(mm, sizeof(double));
        for (int i = 0; i < mm; ++i) {
            T[i + i * mm] = al[i] * al[i] + (i > 0 ? be[i - 1] * be[i - 1] : 0.0);
            if (i + 1 < mm) T[i + 1 + i * mm] = T[i + (i + 1) * mm] = al[i] * be[i];
        }
        jacobi_eig(mm, T, ev, V);
        int *idx = xcalloc(mm, sizeof(int));
        for (int i = 0; i < mm; ++i) idx[i] = i;
        for (int i = 1; i < mm; ++i) {  /* insertion sort, descending, stable */
            int v = idx[i], q = i;
            while (q > 0 && ev[idx[q - 1]] < ev[v]) { idx[q] = idx[q - 1]; --q; }
            idx[q] = v;
        }
        double *Z = xcalloc((int64_t)mm * k, sizeof(double));
        for (int c2 = 0; c2 < k; ++c2) {
            const double *src = V + (int64_t)idx[c2] * mm;
            int big = 0;
            for (int r = 1; r < mm; ++r) if (fabs(src[r]) > fabs(src[big])) big = r;
            const double sg = src[big] < 0 ? -1.0 : 1.0;
            for (int r = 0; r < mm; ++r) Z[r + (int64_t)c2 * mm] = sg * src[r];
        }
        /* record: alpha, beta, sigma^2 */
        free(o->ta); free(o->tb); free(o->ritz);
        o->ta = xcalloc(mm, sizeof(double));
        o->tb = xcalloc(mm, sizeof(double));
        o->ritz = xcalloc(mm, sizeof(double));
        memcpy(o->ta, al, mm * sizeof(double));
        memcpy(o->tb, be, mm * sizeof(double));
        for (int i = 0; i < mm; ++i) o->ritz[i] = ev[idx[i]];
        o->msteps = mm;
        o->qcap = 0;
        free(o->Q);
        o->Q = NULL;
        o->lvariant = 0;  /* the stored run cannot be continued by orc_extend */
        /* V_k = Q_m Z_k; W = B_m Z_k (m x k); U_k = P_m W */
        double *Vk = xcalloc(s * (int64_t)k, sizeof(double));
        double *W = xcalloc((int64_t)mm * k, sizeof(double));
        for (int c2 = 0; c2 < k; ++c2) {
            for (int l = 0; l < mm; ++l) {
                const double zl = Z[l + (int64_t)c2 * mm];
                const double *ql = Q + s * (int64_t)l;
                double *dst = Vk + s * (int64_t)c2;
                for (int64_t i = 0; i < s; ++i) dst[i] += zl * ql[i];
            }
            for (int r = 0; r < mm; ++r)
                W[r + (int64_t)c2 * mm] = al[r] * Z[r + (int64_t)c2 * mm] +
                                          (r + 1 < mm ? be[r] * Z[r + 1 + (int64_t)c2 * mm] : 0.0);
        }
        free(o->U); free(o->lam); free(o->dvec); free(o->Hk);
        o->lam = NULL; o->dvec = NULL; o->Hk = NULL;
        o->U = xcalloc(n * (int64_t)k, sizeof(double));
        for (int c2 = 0; c2 < k; ++c2)
            for (int l = 0; l < mm; ++l) {
                const double wl = W[l + (int64_t)c2 * mm];
                const double *pl = P + n * (int64_t)l;
                double *dst = o->U + n * (int64_t)c2;
                for (int64_t i = 0; i < n; ++i) dst[i] += wl * pl[i];
            }
        o->variant = 2;
        o->k = k;
        double *EV = xcalloc(n * (int64_t)k, sizeof(double));
        for (int c2 = 0; c2 < k; ++c2) e_mul(o, Vk + s * (int64_t)c2, EV + n * (int64_t)c2);
        st = ddlr2_hk(o, k, EV);
        free(EV); free(Vk); free(W); free(Z); free(idx); free(T); free(V); free(ev);
    }
    free(Q); free(P); free(al); free(be);
    return st;
}

int orc_lowrank(orc_t *o, int variant, int k, int m, int thetamode, const double *v0) {
    return orc_lowrank_ctl(o, variant, k, m, 0, 0.0, thetamode, v0);
}

/* Improving a given preconditioner (Sec. on improving): continue the stored
 * Lanczos run by `more` steps (check = 0) or until eq. (converge) holds
 * within `more` steps, then rebuild the low-rank part with rank k. */
int orc_extend(orc_t *o, int k, int more, int check, double eps, int thetamode) {
    if (o->lvariant == 0 || more < 0 || check < 0 || k < 1 || k + 1 > o->s) return ORC_E_INVALID;
    int m = o->msteps + more;
    if (m > o->s) m = (int)o->s;
    if (!o->broke) lanczos_run(o, m, check, eps, k);
    if (o->msteps < k + 1) return ORC_E_LANCZOS;
    return build_lowrank(o, o->lvariant, k, thetamode);
}

void orc_lanczos_record(const orc_t *o, double *ta, double *tb, double *ritzv) {
    memcpy(ta, o->ta, o->msteps * sizeof(double));
    memcpy(tb, o->tb, o->msteps * sizeof(double));
    memcpy(ritzv, o->ritz, o->msteps * sizeof(double));
}

/* Q_m (s x m, internal interface order) */
void orc_lanczos_basis(const orc_t *o, double *Q) {
    if (o->Q) memcpy(Q, o->Q, o->s * (int64_t)o->msteps * sizeof(double));  /* none after a bidiagonalisation build */
}

/* Low-rank data in user order: DDLR-1 U is n x k with zero interior rows and
 * aux = lambda (k) then theta; DDLR-2 U is n x k and aux = H_k (k x k). */
void orc_get_lowrank(const orc_t *o, double *U, double *aux) {
    const int64_t n = o->n, s = o->s, m = o->m;
    const int k = o->k;
    memset(U, 0, n * (int64_t)k * sizeof(double));
    for (int j = 0; j < k; ++j) {
        if (o->variant == 1)
            for (int64_t y = 0; y < s; ++y) U[o->perm[m + y] + n * (int64_t)j] = o->U[y + s * (int64_t)j];
        else
            for (int64_t i = 0; i < n; ++i) U[o->perm[i] + n * (int64_t)j] = o->U[i + n * (int64_t)j];
    }
    if (o->variant == 1) {
        for (int j = 0; j < k; ++j) aux[j] = o->lam[j];
        aux[k] = o->theta;
    } else {
        memcpy(aux, o->Hk, (int64_t)k * k * sizeof(double));
    }
}

/* Installs externally given low-rank data (same layout as orc_get_lowrank). */
void orc_set_lowrank(orc_t *o, int variant, int k, const double *U, const double *aux) {
    const int64_t n = o->n, s = o->s, m = o->m;
    free(o->U); free(o->lam); free(o->dvec); free(o->Hk);
    o->U = NULL; o->lam = NULL; o->dvec = NULL; o->Hk = NULL;
    o->variant = variant;
    o->k = k;
    if (variant == 1) {
        o->U = xcalloc(s * (int64_t)k, sizeof(double));
        for (int j = 0; j < k; ++j)
            for (int64_t y = 0; y < s; ++y) o->U[y + s * (int64_t)j] = U[o->perm[m + y] + n * (int64_t)j];
        o->lam = xcalloc(k, sizeof(double));
        o->dvec = xcalloc(k, sizeof(double));
        for (int j = 0; j < k; ++j) o->lam[j] = aux[j];
        o->theta = aux[k];
        o->c0 = 1.0 / (1.0 - o->theta);
        for (int j = 0; j < k; ++j) o->dvec[j] = 1.0 / (1.0 - o->lam[j]) - o->c0;
    } else {
        o->U = xcalloc(n * (int64_t)k, sizeof(double));
        for (int j = 0; j < k; ++j)
            for (int64_t i = 0; i < n; ++i) o->U[i + n * (int64_t)j] = U[o->perm[i] + n * (int64_t)j];
        o->Hk = xcalloc((int64_t)k * k, sizeof(double));
        memcpy(o->Hk, aux, (int64_t)k * k * sizeof(double));
    }
}

/* y = M^{-1} x, user order, nrhs columns (leading dimension n). */
void orc_apply(const orc_t *o, int nrhs, const double *x, double *y) {
    double *a = xcalloc(o->n, sizeof(double)), *b = xcalloc(o->n, sizeof(double));
    for (int r = 0; r < nrhs; ++r) {
        to_internal(o, x + o->n * (int64_t)r, a);
        apply_internal(o, a, b);
        to_user(o, b, y + o->n * (int64_t)r);
    }
    free(a); free(b);
}

/* Preconditioned CG (Hestenes-Stiefel with M^{-1}), x0 = 0, stop when the
 * recursive residual satisfies ||r|| <= rtol ||b|| or after maxit steps.
 * Per right-hand side: its[r], relres[2r] = recursive, relres[2r+1] = true. */
int orc_pcg(const orc_t *o, int nrhs, const double *b, double *x, double rtol, int maxit, int *its, double *relres) {
    const int64_t n = o->n;
    double *r = xcalloc(n, sizeof(double)), *z = xcalloc(n, sizeof(double));
    double *pv = xcalloc(n, sizeof(double)), *q = xcalloc(n, sizeof(double));
    double *xi = xcalloc(n, sizeof(double)), *t = xcalloc(n, sizeof(double));
    int st = ORC_OK;
    for (int c = 0; c < nrhs; ++c) {
        to_internal(o, b + n * (int64_t)c, r);
        double bn = nrm2(r, n);
        memset(xi, 0, n * sizeof(double));
        int it = 0;
        double rn = bn;
        if (bn > 0.0) {
            apply_internal(o, r, z);
            memcpy(pv, z, n * sizeof(double));
            double rz = dot(r, z, n);
            while (1) {
                csr_mv(&o->Ap, n, pv, q);
                double a = rz / dot(pv, q, n);
                for (int64_t i = 0; i < n; ++i) { xi[i] += a * pv[i]; r[i] -= a * q[i]; }
                ++it;
                rn = nrm2(r, n);
                if (rn <= rtol * bn || it >= maxit) break;
                apply_internal(o, r, z);
                double rz2 = dot(r, z, n);
                double beta = rz2 / rz;
                rz = rz2;
                for (int64_t i = 0; i < n; ++i) pv[i] = z[i] + beta * pv[i];
            }
        }
        to_user(o, xi, x + n * (int64_t)c);
        /* true residual in user order */
        to_internal(o, b + n * (int64_t)c, t);
        csr_mv(&o->Ap, n, xi, q);
        for (int64_t i = 0; i < n; ++i) t[i] -= q[i];
        its[c] = it;
        relres[2 * c] = bn > 0 ? rn / bn : 0.0;
        relres[2 * c + 1] = bn > 0 ? nrm2(t, n) / bn : 0.0;
        if (bn > 0 && !(rn <= rtol * bn)) st = ORC_E_NO_CONVERGENCE;
    }
    free(r); free(z); free(pv); free(q); free(xi); free(t);
    return st;
}

/* Right-preconditioned restarted GMRES: A M^{-1} u = b, x = M^{-1} u, x0 = 0.
 * Arnoldi by classical Gram-Schmidt applied twice; Givens rotations for the
 * least-squares problem.  Stops when the residual estimate <= rtol ||b|| or
 * after maxit total inner steps. */
int orc_gmres(const orc_t *o, int nrhs, const double *b, double *x, int restart, double rtol, int maxit,
              int *its, double *relres) {
    const int64_t n = o->n;
    const int R = restart;
    double *V = xcalloc(n * (int64_t)(R + 1), sizeof(double));
    double *Hm = xcalloc((int64_t)(R + 1) * R, sizeof(double));
    double *cs = xcalloc(R, sizeof(double)), *sn = xcalloc(R, sizeof(double));
    double *g = xcalloc(R + 1, sizeof(double)), *yv = xcalloc(R, sizeof(double));
    double *xi = xcalloc(n, sizeof(double)), *r = xcalloc(n, sizeof(double));
    double *z = xcalloc(n, sizeof(double)), *w = xcalloc(n, sizeof(double));
    double *bi = xcalloc(n, sizeof(double)), *h = xcalloc(R + 1, sizeof(double));
    int st = ORC_OK;
    for (int c = 0; c < nrhs; ++c) {
        to_internal(o, b + n * (int64_t)c, bi);
        double bn = nrm2(bi, n);
        memset(xi, 0, n * sizeof(double));
        int it = 0;
        double est = bn;
        int conv = (bn == 0.0);
        while (!conv && it < maxit) {
            /* r = b - A x */
            csr_mv(&o->Ap, n, xi, r);
            for (int64_t i = 0; i < n; ++i) r[i] = bi[i] - r[i];
            double beta = nrm2(r, n);
            if (beta <= rtol * bn) { est = beta; conv = 1; break; }
            for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
            memset(g, 0, (R + 1) * sizeof(double));
            g[0] = beta;
            int j;
            for (j = 0; j < R && it < maxit; ++j) {
                apply_internal(o, V + n * (int64_t)j, z);
                csr_mv(&o->Ap, n, z, w);
                for (int l = 0; l <= j + 1; ++l) h[l] = 0.0;
                for (int pass = 0; pass < 2; ++pass) {
                    double cc[64 + 1];
                    double *cp = (j + 1 <= 64) ? cc : xcalloc(j + 1, sizeof(double));
                    for (int l = 0; l <= j; ++l) cp[l] = dot(V + n * (int64_t)l, w, n);
                    for (int l = 0; l <= j; ++l) {
                        const double *vl = V + n * (int64_t)l;
                        for (int64_t i = 0; i < n; ++i) w[i] -= cp[l] * vl[i];
                        h[l] += cp[l];
                    }
                    if (cp != cc) free(cp);
                }
                h[j + 1] = nrm2(w, n);
                if (h[j + 1] > 0.0)
                    for (int64_t i = 0; i < n; ++i) V[i + n * (int64_t)(j + 1)] = w[i] / h[j + 1];
                /* apply previous rotations, then a new one */
                for (int l = 0; l < j; ++l) {
                    double t0 = cs[l] * h[l] + sn[l] * h[l + 1];
                    double t1 = -sn[l] * h[l] + cs[l] * h[l + 1];
                    h[l] = t0; h[l + 1] = t1;
                }
                double den = sqrt(h[j] * h[j] + h[j + 1] * h[j + 1]);
                cs[j] = den > 0 ? h[j] / den : 1.0;
                sn[j] = den > 0 ? h[j + 1] / den : 0.0;
                h[j] = den;
                h[j + 1] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                for (int l = 0; l <= j; ++l) Hm[l + (int64_t)j * (R + 1)] = h[l];
                ++it;
                est = fabs(g[j + 1]);
                if (est <= rtol * bn) { conv = 1; ++j; break; }
            }
            /* solve the triangular system and update x = x + M^{-1} V y */
            for (int i = j - 1; i >= 0; --i) {
                double v = g[i];
                for (int l = i + 1; l < j; ++l) v -= Hm[i + (int64_t)l * (R + 1)] * yv[l];
                yv[i] = v / Hm[i + (int64_t)i * (R + 1)];
            }
            memset(w, 0, n * sizeof(double));
            for (int l = 0; l < j; ++l) {
                const double *vl = V + n * (int64_t)l;
                for (int64_t i = 0; i < n; ++i) w[i] += yv[l] * vl[i];
            }
            apply_internal(o, w, z);
            for (int64_t i = 0; i < n; ++i) xi[i] += z[i];
        }
        to_user(o, xi, x + n * (int64_t)c);
        csr_mv(&o->Ap, n, xi, r);
        for (int64_t i = 0; i < n; ++i) r[i] = bi[i] - r[i];
        its[c] = it;
        relres[2 * c] = bn > 0 ? est / bn : 0.0;
        relres[2 * c + 1] = bn > 0 ? nrm2(r, n) / bn : 0.0;
        if (!conv) st = ORC_E_NO_CONVERGENCE;
    }
    free(V); free(Hm); free(cs); free(sn); free(g); free(yv); free(xi); free(r); free(z); free(w); free(bi); free(h);
    return st;
}

/* y = A x in user order (used by tests for residuals) */
void orc_matvec(const orc_t *o, const double *x, double *y) { csr_mv(&o->A, o->n, x, y); }

/* Reorthogonalisation of the next Lanczos runs: 0 full, 1 partial, 2 none
 * (tests only).  Returns 0, or -1 for another value. */
int orc_set_reorth(orc_t *o, int mode) {
    if (mode < 0 || mode > 2) return -1;
    o->reorth = mode;
    return 0;
}

/* Steps of the stored run whose new vector was reorthogonalised (partial
 * reorthogonalisation): flags[0..msteps-1]; returns their count. */
int orc_reorth_steps(const orc_t *o, int32_t *flags) {
    int cnt = 0;
    for (int j = 0; j < o->msteps; ++j) {
        const int f = o->rsteps ? o->rsteps[j] : 0;
        if (flags) flags[j] = f;
        cnt += f;
    }
    return cnt;
}

/* sets the number of OpenMP threads of the parallel loops */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* number of OpenMP threads the parallel loops above run with */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
