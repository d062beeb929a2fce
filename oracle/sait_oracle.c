/*
 * SAIT CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 reference for everything the GPU
 * library computes.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library; the product
 * (the HIP library and its Python binding) never links, imports or calls
 * it, and shares no code with it.
 *
 * Paper: Z. Lu, "A sparse approximate inverse for triangular matrices based
 * on Jacobi iteration" (arXiv 2106.12836).  Each function names the passage
 * it follows.  Compiled with -ffp-contract=off: every a*b+c below is two
 * roundings, exactly as written.
 *
 * Conventions: square CSR matrices, int32 row pointers and column indices
 * (columns sorted, unique per row), double values.  Functions that produce
 * a matrix allocate its three arrays with malloc and hand them back through
 * out-pointers; the caller releases them with or_free().
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *   - the SAIT loop count m is the highest power of the iteration matrix
 *     kept (Eq. M_m; Alg. 1 runs m passes of M <- T~ M + I);
 *   - threshold dropping keeps an entry iff |M_ij| > tau (Appendix A's
 *     mask), applied to M before the final column scaling M <- M D^-1;
 *     exact zeros are never stored;
 *   - T~ = I - D^-1 T has a structurally zero diagonal (Sec. 2 defines it
 *     as strictly triangular), off-diagonal T~_ij = -(fl(1/d_i) * T_ij);
 *   - the optional per-row cap K (not in the paper) keeps the diagonal and
 *     the K-1 largest magnitudes, ties to the smaller column;
 *   - ILU(0) is Doolittle (unit lower L stored with its diagonal), IKJ order
 *     (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 10.4);
 *   - ILUT(tau, p) is Saad's dual-threshold ILUT (Alg. 10.6) with
 *     tau_i = tau * ||a_i,*||_2, drop on |w_k| < tau_i, keep the p largest in
 *     each of L and U (ties to the smaller column), exact zeros dropped;
 *   - GMRES is right-preconditioned restarted GMRES with modified
 *     Gram-Schmidt and Givens rotations (Saad Alg. 9.5 / 6.9); FGMRES stores
 *     the preconditioned vectors (Saad Alg. 9.6).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_E_INVALID -1
#define OR_E_ZERO_PIVOT -2
#define OR_E_NONFINITE -3
#define OR_E_NOMEM -4

void or_free(void *p) { free(p); }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n, cap, nnz;
    int32_t *rp, *ci;
    double *v;
} or_builder; /* row-by-row CSR builder */

static int bld_init(or_builder *b, int64_t n, int64_t cap) {
    b->n = n;
    b->cap = cap > 16 ? cap : 16;
    b->nnz = 0;
    b->rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    b->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)b->cap);
    b->v = (double *)malloc(sizeof(double) * (size_t)b->cap);
    if (!b->rp || !b->ci || !b->v) return OR_E_NOMEM;
    b->rp[0] = 0;
    return OR_OK;
}

static int bld_push(or_builder *b, int32_t col, double val) {
    if (b->nnz == b->cap) {
        int64_t nc = b->cap * 2;
        int32_t *nci = (int32_t *)realloc(b->ci, sizeof(int32_t) * (size_t)nc);
        if (!nci) return OR_E_NOMEM;
        b->ci = nci;
        double *nv = (double *)realloc(b->v, sizeof(double) * (size_t)nc);
        if (!nv) return OR_E_NOMEM;
        b->v = nv;
        b->cap = nc;
    }
    if (b->nnz >= INT32_MAX) return OR_E_INVALID;
    b->ci[b->nnz] = col;
    b->v[b->nnz] = val;
    b->nnz++;
    return OR_OK;
}

static void bld_end_row(or_builder *b, int64_t i) { b->rp[i + 1] = (int32_t)b->nnz; }

static void bld_free(or_builder *b) {
    free(b->rp);
    free(b->ci);
    free(b->v);
    b->rp = NULL;
    b->ci = NULL;
    b->v = NULL;
}

static void bld_give(or_builder *b, int32_t **rp, int32_t **ci, double **v) {
    *rp = b->rp;
    *ci = b->ci;
    *v = b->v;
    b->rp = NULL;
    b->ci = NULL;
    b->v = NULL;
}

static int cmp_int32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Entry used when ranking by magnitude: larger |val| first, then smaller col. */
typedef struct {
    int32_t col;
    double val;
} or_entry;

static int cmp_mag_desc(const void *a, const void *b) {
    const or_entry *x = (const or_entry *)a, *y = (const or_entry *)b;
    double ax = fabs(x->val), ay = fabs(y->val);
    if (ax > ay) return -1;
    if (ax < ay) return 1;
    return (x->col > y->col) - (x->col < y->col);
}

static int cmp_col_asc(const void *a, const void *b) {
    const or_entry *x = (const or_entry *)a, *y = (const or_entry *)b;
    return (x->col > y->col) - (x->col < y->col);
}

/* ------------------------------------------------------------------ */
/* ILU(0): Saad Alg. 10.4 (IKJ), pattern of A; "level-0 ILU" of Sec. 4. */
/* ------------------------------------------------------------------ */
int or_ilu0(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
            int32_t **Lrp, int32_t **Lci, double **Lv,
            int32_t **Urp, int32_t **Uci, double **Uv) {
    int64_t nnz = rp[n];
    double *a = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *dpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!a || !dpos || !where) { free(a); free(dpos); free(where); return OR_E_NOMEM; }
    memcpy(a, v, sizeof(double) * (size_t)nnz);
    for (int64_t j = 0; j < n; j++) where[j] = -1;
    int st = OR_OK;
    for (int64_t i = 0; i < n && st == OR_OK; i++) {
        dpos[i] = -1;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            where[ci[p]] = p;
            if (ci[p] == i) dpos[i] = p;
        }
        if (dpos[i] < 0) { st = OR_E_ZERO_PIVOT; }
        for (int64_t p = rp[i]; p < rp[i + 1] && st == OR_OK; p++) {
            int64_t k = ci[p];
            if (k >= i) break; /* columns sorted: the L part comes first */
            double piv = a[dpos[k]];
            a[p] = a[p] / piv;              /* a_ik <- a_ik / a_kk */
            for (int64_t q = dpos[k] + 1; q < rp[k + 1]; q++) {
                int64_t j = ci[q];          /* a_kj, j > k */
                if (where[j] >= 0) a[where[j]] = a[where[j]] - a[p] * a[q];
            }
        }
        if (st == OR_OK) {
            double d = a[dpos[i]];
            if (d == 0.0) st = OR_E_ZERO_PIVOT;
            else if (!isfinite(d)) st = OR_E_NONFINITE;
        }
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) where[ci[p]] = -1;
    }
    if (st != OR_OK) { free(a); free(dpos); free(where); return st; }
    or_builder L, U;
    memset(&L, 0, sizeof(L));
    memset(&U, 0, sizeof(U));
    int64_t nl = 0;
    for (int64_t i = 0; i < n; i++) nl += dpos[i] - rp[i];
    if (bld_init(&L, n, nl + n) || bld_init(&U, n, nnz - nl)) {
        bld_free(&L); bld_free(&U); free(a); free(dpos); free(where); return OR_E_NOMEM;
    }
    for (int64_t i = 0; i < n; i++) {
        for (int64_t p = rp[i]; p < dpos[i]; p++) bld_push(&L, ci[p], a[p]);
        bld_push(&L, (int32_t)i, 1.0);
        bld_end_row(&L, i);
        for (int64_t p = dpos[i]; p < rp[i + 1]; p++) bld_push(&U, ci[p], a[p]);
        bld_end_row(&U, i);
    }
    bld_give(&L, Lrp, Lci, Lv);
    bld_give(&U, Urp, Uci, Uv);
    free(a); free(dpos); free(where);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* ILU(p) by levels of fill ("level-1 ILU" of Sec. 4; Saad, ILU(p)):    */
/* lev(a_ij) = 0 on the pattern of A; eliminating a_ik (k < i, in       */
/* increasing k) creates (i, j) for every j > k of row k of U with      */
/* level lev_ik + lev_kj + 1, kept when <= p.  The factors are the      */
/* ILU(0) elimination on that pattern (A's values, zeros at the fill).  */
/* ------------------------------------------------------------------ */
static void heap_push(int32_t *h, int64_t *cnt, int32_t x) {
    int64_t i = (*cnt)++;
    h[i] = x;
    while (i > 0 && h[(i - 1) / 2] > h[i]) {
        int32_t t = h[i]; h[i] = h[(i - 1) / 2]; h[(i - 1) / 2] = t;
        i = (i - 1) / 2;
    }
}

static int32_t heap_pop(int32_t *h, int64_t *cnt) {
    int32_t top = h[0];
    h[0] = h[--(*cnt)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *cnt && h[l] < h[m]) m = l;
        if (r < *cnt && h[r] < h[m]) m = r;
        if (m == i) break;
        int32_t t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
    return top;
}

/* The level-p pattern of A (the extended matrix E: A's values, 0 at the
 * kept fill); or_iluk factors E by ILU(0), or_parilu iterates on it. */
int or_iluk_pattern(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, int p,
                    int32_t **Erp, int32_t **Eci, double **Ev) {
    if (p < 0) return OR_E_INVALID;
    const int INF = 0x7fffffff;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int *lev = (int *)malloc(sizeof(int) * nn);
    int32_t *heap = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *act = (int32_t *)malloc(sizeof(int32_t) * nn);
    /* levels of the U part (columns > i) of every finished row */
    int64_t ucap = rp[n] + 16, ucnt = 0;
    int64_t *uptr = (int64_t *)malloc(sizeof(int64_t) * (nn + 1));
    int32_t *ucol = (int32_t *)malloc(sizeof(int32_t) * (size_t)ucap);
    int *ulev = (int *)malloc(sizeof(int) * (size_t)ucap);
    /* extended pattern */
    int64_t ecap = rp[n] + 16, ecnt = 0;
    int32_t *erp = (int32_t *)malloc(sizeof(int32_t) * (nn + 1));
    int32_t *eci = (int32_t *)malloc(sizeof(int32_t) * (size_t)ecap);
    double *ev = (double *)malloc(sizeof(double) * (size_t)ecap);
    double *wv = (double *)calloc(nn, sizeof(double));
    int st = OR_OK;
    if (!lev || !heap || !act || !uptr || !ucol || !ulev || !erp || !eci || !ev || !wv) { st = OR_E_NOMEM; goto out; }
    for (int64_t j = 0; j < n; j++) lev[j] = INF;
    uptr[0] = 0;
    erp[0] = 0;
    for (int64_t i = 0; i < n && st == OR_OK; i++) {
        int64_t na = 0, nh = 0;
        for (int64_t q = rp[i]; q < rp[i + 1]; q++) {
            int32_t j = ci[q];
            lev[j] = 0;
            wv[j] = v[q];
            act[na++] = j;
            if (j < i) heap_push(heap, &nh, j);
        }
        while (nh > 0) {
            int32_t k = heap_pop(heap, &nh);
            for (int64_t q = uptr[k]; q < uptr[k + 1]; q++) {
                int32_t j = ucol[q];
                int nl = lev[k] + ulev[q] + 1;
                if (nl > p) continue;
                if (lev[j] == INF) {
                    lev[j] = nl;
                    wv[j] = 0.0;
                    act[na++] = j;
                    if (j < i) heap_push(heap, &nh, j);
                } else if (nl < lev[j]) {
                    lev[j] = nl;
                }
            }
        }
        /* sort the row's columns (insertion sort: rows are short) */
        for (int64_t a = 1; a < na; a++) {
            int32_t x = act[a];
            int64_t b = a - 1;
            while (b >= 0 && act[b] > x) { act[b + 1] = act[b]; b--; }
            act[b + 1] = x;
        }
        if (ecnt + na > ecap || ucnt + na > ucap) {
            int64_t nc = 2 * (ecap > ucap ? ecap : ucap) + na;
            int32_t *t1 = (int32_t *)realloc(eci, sizeof(int32_t) * (size_t)nc);
            double *t2 = (double *)realloc(ev, sizeof(double) * (size_t)nc);
            int32_t *t3 = (int32_t *)realloc(ucol, sizeof(int32_t) * (size_t)nc);
            int *t4 = (int *)realloc(ulev, sizeof(int) * (size_t)nc);
            if (t1) eci = t1;
            if (t2) ev = t2;
            if (t3) ucol = t3;
            if (t4) ulev = t4;
            if (!t1 || !t2 || !t3 || !t4) { st = OR_E_NOMEM; break; }
            ecap = ucap = nc;
        }
        for (int64_t a = 0; a < na; a++) {
            int32_t j = act[a];
            eci[ecnt] = j;
            ev[ecnt] = wv[j];
            ecnt++;
            if (j > i) {
                ucol[ucnt] = j;
                ulev[ucnt] = lev[j];
                ucnt++;
            }
            lev[j] = INF;
            wv[j] = 0.0;
        }
        erp[i + 1] = (int32_t)ecnt;
        uptr[i + 1] = ucnt;
    }
out:
    free(lev); free(heap); free(act); free(uptr); free(ucol); free(ulev); free(wv);
    if (st == OR_OK) {
        *Erp = erp; *Eci = eci; *Ev = ev;
    } else {
        free(erp); free(eci); free(ev);
    }
    return st;
}

int or_iluk(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, int p,
            int32_t **Lrp, int32_t **Lci, double **Lv,
            int32_t **Urp, int32_t **Uci, double **Uv) {
    int32_t *erp = NULL, *eci = NULL;
    double *ev = NULL;
    int st = or_iluk_pattern(n, rp, ci, v, p, &erp, &eci, &ev);
    if (st == OR_OK) st = or_ilu0(n, erp, eci, ev, Lrp, Lci, Lv, Urp, Uci, Uv);
    free(erp); free(eci); free(ev);
    return st;
}

/* ------------------------------------------------------------------ */
/* Fine-grained parallel ILU (Chow and Patel, SIAM J. Sci. Comput. 37    */
/* (2015); cited in the introduction), synchronous form.                */
/* ------------------------------------------------------------------ */

/* Position of column j in the sorted row [b, e) of ci, or -1. */
static int64_t find_col(const int32_t *ci, int64_t b, int64_t e, int32_t j) {
    while (b < e) {
        int64_t m = (b + e) / 2;
        if (ci[m] == j) return m;
        if (ci[m] < j) b = m + 1;
        else e = m;
    }
    return -1;
}

/*
 * ILU factors on the pattern S of the given matrix (values a_ij, explicit
 * zeros at fill) as the fixed point of
 *     u_ij = a_ij - sum_{k < i} l_ik u_kj                 (i <= j)
 *     l_ij = (a_ij - sum_{k < j} l_ik u_kj) / u_jj        (i > j)
 * with all k such that (i,k) and (k,j) lie in S.  Each sweep recomputes
 * every entry from the previous sweep's L and U (Jacobi-like), subtracting
 * the products in increasing k with separate roundings.  Start: l_ij =
 * a_ij / a_jj, u_ij = a_ij.  With enough sweeps (the depth of the
 * dependency graph) the result is the ILU factorisation of S itself.
 * L is returned unit lower triangular with its diagonal stored.
 */
int or_parilu(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, int sweeps,
              int32_t **Lrp, int32_t **Lci, double **Lv,
              int32_t **Urp, int32_t **Uci, double **Uv) {
    if (sweeps < 0) return OR_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t nl = 0, nu = 0;
    for (int64_t i = 0; i < n; i++) {
        int diag = 0;
        for (int64_t q = rp[i]; q < rp[i + 1]; q++) {
            if (ci[q] < i) nl++;
            else nu++;
            if (ci[q] == i) diag = (v[q] != 0.0);
        }
        if (!diag) return OR_E_ZERO_PIVOT;
    }
    int32_t *lrp = (int32_t *)malloc(sizeof(int32_t) * (nn + 1));
    int32_t *lci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nl + n + 1));
    double *la = (double *)malloc(sizeof(double) * (size_t)(nl + 1));
    double *l0 = (double *)malloc(sizeof(double) * (size_t)(nl + 1));
    double *l1 = (double *)malloc(sizeof(double) * (size_t)(nl + 1));
    int32_t *urp = (int32_t *)malloc(sizeof(int32_t) * (nn + 1));
    int32_t *uci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nu + 1));
    double *ua = (double *)malloc(sizeof(double) * (size_t)(nu + 1));
    double *u0 = (double *)malloc(sizeof(double) * (size_t)(nu + 1));
    double *u1 = (double *)malloc(sizeof(double) * (size_t)(nu + 1));
    int st = OR_OK;
    if (!lrp || !lci || !la || !l0 || !l1 || !urp || !uci || !ua || !u0 || !u1) { st = OR_E_NOMEM; goto out; }
    /* strictly lower part (the unit diagonal is added at the end) and upper part */
    {
        int64_t a = 0, b = 0;
        lrp[0] = 0;
        urp[0] = 0;
        for (int64_t i = 0; i < n; i++) {
            for (int64_t q = rp[i]; q < rp[i + 1]; q++) {
                if (ci[q] < i) { lci[a] = ci[q]; la[a] = v[q]; a++; }
                else { uci[b] = ci[q]; ua[b] = v[q]; b++; }
            }
            lrp[i + 1] = (int32_t)a;
            urp[i + 1] = (int32_t)b;
        }
    }
    for (int64_t e = 0; e < nu; e++) u0[e] = ua[e];
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = lrp[i]; e < lrp[i + 1]; e++) l0[e] = la[e] / ua[urp[lci[e]]];  /* a_ij / a_jj */
    for (int s = 0; s < sweeps; s++) {
        for (int64_t i = 0; i < n; i++) {
            /* L entries (i, j), j < i */
            for (int64_t e = lrp[i]; e < lrp[i + 1]; e++) {
                int32_t j = lci[e];
                double t = la[e];
                for (int64_t q = lrp[i]; q < lrp[i + 1] && lci[q] < j; q++) {
                    int32_t k = lci[q];
                    int64_t f = find_col(uci, urp[k], urp[k + 1], j);
                    if (f >= 0) t = t - l0[q] * u0[f];
                }
                l1[e] = t / u0[urp[j]];
            }
            /* U entries (i, j), j >= i */
            for (int64_t e = urp[i]; e < urp[i + 1]; e++) {
                int32_t j = uci[e];
                double t = ua[e];
                for (int64_t q = lrp[i]; q < lrp[i + 1]; q++) {
                    int32_t k = lci[q];
                    int64_t f = find_col(uci, urp[k], urp[k + 1], j);
                    if (f >= 0) t = t - l0[q] * u0[f];
                }
                u1[e] = t;
            }
        }
        double *tl = l0; l0 = l1; l1 = tl;
        double *tu = u0; u0 = u1; u1 = tu;
    }
    for (int64_t e = 0; e < nl; e++) if (!isfinite(l0[e])) st = OR_E_NONFINITE;
    for (int64_t e = 0; e < nu; e++) if (!isfinite(u0[e])) st = OR_E_NONFINITE;
    if (st != OR_OK) goto out;
    /* outputs: L with its unit diagonal, U as computed */
    {
        or_builder Lb, Ub;
        st = bld_init(&Lb, n, nl + n);
        if (st == OR_OK) st = bld_init(&Ub, n, nu);
        if (st != OR_OK) goto out;
        for (int64_t i = 0; i < n; i++) {
            for (int64_t e = lrp[i]; e < lrp[i + 1]; e++) bld_push(&Lb, lci[e], l0[e]);
            bld_push(&Lb, (int32_t)i, 1.0);
            bld_end_row(&Lb, i);
            for (int64_t e = urp[i]; e < urp[i + 1]; e++) bld_push(&Ub, uci[e], u0[e]);
            bld_end_row(&Ub, i);
        }
        bld_give(&Lb, Lrp, Lci, Lv);
        bld_give(&Ub, Urp, Uci, Uv);
    }
out:
    free(lrp); free(lci); free(la); free(l0); free(l1);
    free(urp); free(uci); free(ua); free(u0); free(u1);
    return st;
}

/*
 * Symmetric (incomplete Cholesky) form of the same iteration, for a
 * symmetric A (only its upper triangle is read): the unknowns are the
 * u_ij, i <= j, on the upper pattern, and l_ki = u_ik / u_ii throughout, so
 *     u_ij = a_ij - sum_{k < i} (u_ki / u_kk) u_kj
 * over k with (k,i) and (k,j) in the pattern.  Every sweep recomputes all
 * u_ij from the previous sweep's U (each product formed as
 * fl(fl(u_ki / u_kk) * u_kj), subtracted in increasing k); the start is
 * u_ij = a_ij.  L is taken from the final U (l_ji = u_ij / u_ii, unit
 * diagonal), so U = D L^T up to that division's rounding after any number
 * of sweeps.
 */
int or_paric(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, int sweeps,
             int32_t **Lrp, int32_t **Lci, double **Lv,
             int32_t **Urp, int32_t **Uci, double **Uv) {
    if (sweeps < 0) return OR_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t nu = 0;
    for (int64_t i = 0; i < n; i++) {
        int diag = 0;
        for (int64_t q = rp[i]; q < rp[i + 1]; q++) {
            if (ci[q] >= i) nu++;
            if (ci[q] == i) diag = (v[q] != 0.0);
        }
        if (!diag) return OR_E_ZERO_PIVOT;
    }
    int32_t *urp = (int32_t *)malloc(sizeof(int32_t) * (nn + 1));
    int32_t *uci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nu + 1));
    double *ua = (double *)malloc(sizeof(double) * (size_t)(nu + 1));
    double *u0 = (double *)malloc(sizeof(double) * (size_t)(nu + 1));
    double *u1 = (double *)malloc(sizeof(double) * (size_t)(nu + 1));
    /* column lists of U (rows k < i holding column i), as (k, position) */
    int32_t *ccnt = (int32_t *)calloc(nn + 1, sizeof(int32_t));
    int32_t *crow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nu + 1));
    int64_t *cpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nu + 1));
    int32_t *cfill = (int32_t *)calloc(nn, sizeof(int32_t));
    int st = OR_OK;
    if (!urp || !uci || !ua || !u0 || !u1 || !ccnt || !crow || !cpos || !cfill) { st = OR_E_NOMEM; goto out; }
    {
        int64_t b = 0;
        urp[0] = 0;
        for (int64_t i = 0; i < n; i++) {
            for (int64_t q = rp[i]; q < rp[i + 1]; q++)
                if (ci[q] >= i) { uci[b] = ci[q]; ua[b] = v[q]; b++; }
            urp[i + 1] = (int32_t)b;
        }
    }
    /* strictly upper entries (k, i), k < i, grouped by column i, rows ascending */
    for (int64_t k = 0; k < n; k++)
        for (int64_t e = urp[k] + 1; e < urp[k + 1]; e++) ccnt[uci[e] + 1]++;
    for (int64_t i = 0; i < n; i++) ccnt[i + 1] += ccnt[i];
    for (int64_t k = 0; k < n; k++)
        for (int64_t e = urp[k] + 1; e < urp[k + 1]; e++) {
            int32_t i = uci[e];
            int64_t o = ccnt[i] + cfill[i]++;
            crow[o] = (int32_t)k;
            cpos[o] = e;
        }
    for (int64_t e = 0; e < nu; e++) u0[e] = ua[e];
    for (int s = 0; s < sweeps; s++) {
        for (int64_t i = 0; i < n; i++)
            for (int64_t e = urp[i]; e < urp[i + 1]; e++) {
                int32_t j = uci[e];
                double t = ua[e];
                for (int64_t q = ccnt[i]; q < ccnt[i + 1]; q++) {
                    int32_t k = crow[q];
                    int64_t f = find_col(uci, urp[k], urp[k + 1], j);
                    if (f >= 0) t = t - (u0[cpos[q]] / u0[urp[k]]) * u0[f];
                }
                u1[e] = t;
            }
        double *tu = u0; u0 = u1; u1 = tu;
    }
    for (int64_t e = 0; e < nu; e++) if (!isfinite(u0[e])) st = OR_E_NONFINITE;
    if (st != OR_OK) goto out;
    {
        or_builder Lb, Ub;
        st = bld_init(&Lb, n, nu);
        if (st == OR_OK) st = bld_init(&Ub, n, nu);
        if (st != OR_OK) goto out;
        for (int64_t i = 0; i < n; i++) {
            for (int64_t q = ccnt[i]; q < ccnt[i + 1]; q++) {
                int32_t k = crow[q];
                bld_push(&Lb, k, u0[cpos[q]] / u0[urp[k]]);   /* l_ik = u_ki / u_kk */
            }
            bld_push(&Lb, (int32_t)i, 1.0);
            bld_end_row(&Lb, i);
            for (int64_t e = urp[i]; e < urp[i + 1]; e++) bld_push(&Ub, uci[e], u0[e]);
            bld_end_row(&Ub, i);
        }
        bld_give(&Lb, Lrp, Lci, Lv);
        bld_give(&Ub, Urp, Uci, Uv);
    }
out:
    free(urp); free(uci); free(ua); free(u0); free(u1);
    free(ccnt); free(crow); free(cpos); free(cfill);
    return st;
}

/* ------------------------------------------------------------------ */
/* ILUT(tau, p): Saad Alg. 10.6 (dual threshold).                       */
/* ------------------------------------------------------------------ */
int or_ilut(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
            double tau, int p,
            int32_t **Lrp, int32_t **Lci, double **Lv,
            int32_t **Urp, int32_t **Uci, double **Uv) {
    if (p < 0 || !(tau >= 0.0)) return OR_E_INVALID;
    double *w = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    char *present = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    or_entry *sel = (or_entry *)malloc(sizeof(or_entry) * (size_t)(n > 0 ? n : 1));
    double *udiag = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    or_builder L, U;
    memset(&L, 0, sizeof(L));
    memset(&U, 0, sizeof(U));
    int st = OR_OK;
    if (!w || !present || !cols || !sel || !udiag) st = OR_E_NOMEM;
    if (st == OR_OK && (bld_init(&L, n, rp[n] + n) || bld_init(&U, n, rp[n] + n))) st = OR_E_NOMEM;
    for (int64_t i = 0; i < n && st == OR_OK; i++) {
        int64_t ncols = 0;
        double nrm2 = 0.0;
        for (int64_t q = rp[i]; q < rp[i + 1]; q++) {
            int32_t j = ci[q];
            w[j] = v[q];
            present[j] = 1;
            cols[ncols++] = j;
            nrm2 = nrm2 + v[q] * v[q];
        }
        double tau_i = tau * sqrt(nrm2);
        /* eliminate in increasing k over the (growing) set of columns < i */
        int64_t kprev = -1;
        for (;;) {
            int64_t k = -1;
            for (int64_t t = 0; t < ncols; t++) {
                int64_t c = cols[t];
                if (c < i && c > kprev && (k < 0 || c < k)) k = c;
            }
            if (k < 0) break;
            kprev = k;
            if (w[k] == 0.0) continue;
            w[k] = w[k] / udiag[k];
            if (fabs(w[k]) < tau_i) { w[k] = 0.0; continue; }
            for (int64_t q = U.rp[k]; q < U.rp[k + 1]; q++) {
                int32_t j = U.ci[q];
                if (j <= k) continue; /* the diagonal of row k */
                if (!present[j]) { present[j] = 1; w[j] = 0.0; cols[ncols++] = j; }
                w[j] = w[j] - w[k] * U.v[q];
            }
        }
        /* L part: j < i */
        int64_t ns = 0;
        for (int64_t t = 0; t < ncols; t++) {
            int32_t j = cols[t];
            if (j < i && w[j] != 0.0 && !(fabs(w[j]) < tau_i)) { sel[ns].col = j; sel[ns].val = w[j]; ns++; }
        }
        qsort(sel, (size_t)ns, sizeof(or_entry), cmp_mag_desc);
        if (ns > p) ns = p;
        qsort(sel, (size_t)ns, sizeof(or_entry), cmp_col_asc);
        for (int64_t t = 0; t < ns; t++) bld_push(&L, sel[t].col, sel[t].val);
        bld_push(&L, (int32_t)i, 1.0);
        bld_end_row(&L, i);
        /* diagonal */
        double d = present[i] ? w[i] : 0.0;
        if (d == 0.0) st = OR_E_ZERO_PIVOT;
        else if (!isfinite(d)) st = OR_E_NONFINITE;
        udiag[i] = d;
        /* U part: j > i */
        ns = 0;
        for (int64_t t = 0; t < ncols; t++) {
            int32_t j = cols[t];
            if (j > i && w[j] != 0.0 && !(fabs(w[j]) < tau_i)) { sel[ns].col = j; sel[ns].val = w[j]; ns++; }
        }
        qsort(sel, (size_t)ns, sizeof(or_entry), cmp_mag_desc);
        if (ns > p) ns = p;
        qsort(sel, (size_t)ns, sizeof(or_entry), cmp_col_asc);
        bld_push(&U, (int32_t)i, d);
        for (int64_t t = 0; t < ns; t++) bld_push(&U, sel[t].col, sel[t].val);
        bld_end_row(&U, i);
        for (int64_t t = 0; t < ncols; t++) { w[cols[t]] = 0.0; present[cols[t]] = 0; }
    }
    free(w); free(present); free(cols); free(sel); free(udiag);
    if (st != OR_OK) { bld_free(&L); bld_free(&U); return st; }
    bld_give(&L, Lrp, Lci, Lv);
    bld_give(&U, Urp, Uci, Uv);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Exact substitution (Sec. 1: forward / backward substitution).        */
/* ------------------------------------------------------------------ */
int or_lower_solve(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                   const double *b, double *x) {
    for (int64_t i = 0; i < n; i++) {
        double s = b[i], d = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] < i) s = s - v[p] * x[ci[p]];
            else if (ci[p] == i) d = v[p];
        }
        if (d == 0.0) return OR_E_ZERO_PIVOT;
        x[i] = s / d;
    }
    return OR_OK;
}

int or_upper_solve(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                   const double *b, double *x) {
    for (int64_t i = n - 1; i >= 0; i--) {
        double s = b[i], d = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] > i) s = s - v[p] * x[ci[p]];
            else if (ci[p] == i) d = v[p];
        }
        if (d == 0.0) return OR_E_ZERO_PIVOT;
        x[i] = s / d;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* SAIT (Sec. 2-3; Alg. 1, 2, 3; Appendix A)                            */
/* ------------------------------------------------------------------ */

/* d_i and fl(1/d_i) of a triangular T; rejects missing, zero or
 * non-finite diagonals (D^-1 must exist, Eq. Jacobi_iter). */
static int sait_dinv(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *dinv) {
    for (int64_t i = 0; i < n; i++) {
        double d = 0.0;
        int found = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] == i) { d = v[p]; found = 1; }
        if (!found || d == 0.0) return OR_E_ZERO_PIVOT;
        if (!isfinite(d)) return OR_E_NONFINITE;
        dinv[i] = 1.0 / d;
    }
    return OR_OK;
}

/*
 * One pass of the Horner recursion (Eq. Recursive) with dropping:
 *     W = T~ * Mprev + I   (right == 0, Alg. 1 step 3 as printed), or
 *     W = Mprev * T~ + I   (right == 1),   T~ = I - D^-1 T
 * (diagonal of T~ structurally zero).  Both sides give the same truncated
 * Neumann sum when nothing is dropped, since the polynomial in T~ commutes
 * with T~; with dropping they differ.  Multiplying from the right for the
 * upper factor U of a symmetric A (U = D L^T, so T~_U = T~_L^T) makes the
 * upper factor the transpose of the lower one, M_U = M_L^T D^-1, and
 * M_U M_L symmetric positive definite, as the PCG experiments of Sec. 4
 * need.  Then keep (i,j) iff |W_ij| > tau (Alg. 2 / Appendix A mask) -- or
 * iff (i,j) lies in the pattern S when S is given (Alg. 3) -- and finally,
 * if cap > 0, keep the diagonal plus the cap-1 largest |W_ij|.
 * Row i of W is formed the Gustavson way into a dense accumulator:
 *   left:  for each l in T~ row i in increasing column order, add
 *          T~_il * M_l,*;
 *   right: for each l in M row i in increasing column order, add
 *          M_il * T~_l,*.
 * Either way every W_ij sums its products in increasing l, then adds the
 * identity.  Pattern mode (S != NULL): keep iff W_ij != 0 and (i,j) in S.
 */
static int sait_pass(int64_t n, const int32_t *Trp, const int32_t *Tci, const double *Tv,
                     const double *dinv, int right,
                     const int32_t *Mrp, const int32_t *Mci, const double *Mv,
                     double tau, int cap,
                     const int32_t *Srp, const int32_t *Sci,
                     double *acc, char *touched, int32_t *list, char *inS, or_entry *ent,
                     or_builder *out) {
    for (int64_t i = 0; i < n; i++) {
        int64_t nl = 0;
        if (!right) {
            for (int64_t p = Trp[i]; p < Trp[i + 1]; p++) {
                int64_t l = Tci[p];
                if (l == i) continue;                       /* T~_ii = 0 */
                double tl = -(dinv[i] * Tv[p]);             /* T~_il */
                for (int64_t q = Mrp[l]; q < Mrp[l + 1]; q++) {
                    int32_t j = Mci[q];
                    if (!touched[j]) { touched[j] = 1; acc[j] = 0.0; list[nl++] = j; }
                    acc[j] = acc[j] + tl * Mv[q];
                }
            }
        } else {
            for (int64_t p = Mrp[i]; p < Mrp[i + 1]; p++) {
                int64_t l = Mci[p];
                double ml = Mv[p];                          /* M_il */
                for (int64_t q = Trp[l]; q < Trp[l + 1]; q++) {
                    int32_t j = Tci[q];
                    if (j == l) continue;                   /* T~_ll = 0 */
                    double tlj = -(dinv[l] * Tv[q]);        /* T~_lj */
                    if (!touched[j]) { touched[j] = 1; acc[j] = 0.0; list[nl++] = j; }
                    acc[j] = acc[j] + ml * tlj;
                }
            }
        }
        /* + I */
        if (!touched[i]) { touched[i] = 1; acc[i] = 0.0; list[nl++] = (int32_t)i; }
        acc[i] = acc[i] + 1.0;
        qsort(list, (size_t)nl, sizeof(int32_t), cmp_int32);
        if (Srp) for (int64_t q = Srp[i]; q < Srp[i + 1]; q++) inS[Sci[q]] = 1;
        int64_t ne = 0;
        double wdiag = 0.0;
        for (int64_t t = 0; t < nl; t++) {
            int32_t j = list[t];
            double w = acc[j];
            int keep = Srp ? (inS[j] && w != 0.0) : (fabs(w) > tau);
            if (j == i) { wdiag = w; continue; }         /* diagonal handled below */
            if (keep) { ent[ne].col = j; ent[ne].val = w; ne++; }
        }
        if (Srp) for (int64_t q = Srp[i]; q < Srp[i + 1]; q++) inS[Sci[q]] = 0;
        for (int64_t t = 0; t < nl; t++) touched[list[t]] = 0;
        if (cap > 0 && ne > cap - 1) {
            qsort(ent, (size_t)ne, sizeof(or_entry), cmp_mag_desc);
            ne = cap - 1;
            qsort(ent, (size_t)ne, sizeof(or_entry), cmp_col_asc);
        }
        /* emit in column order with the diagonal in its place */
        int placed = 0;
        for (int64_t t = 0; t <= ne; t++) {
            if (!placed && (t == ne || ent[t].col > i)) {
                if (bld_push(out, (int32_t)i, wdiag)) return OR_E_NOMEM;
                placed = 1;
            }
            if (t < ne && bld_push(out, ent[t].col, ent[t].val)) return OR_E_NOMEM;
        }
        bld_end_row(out, i);
    }
    return OR_OK;
}

typedef struct {
    double *acc;
    char *touched, *inS;
    int32_t *list;
    or_entry *ent;
    double *dinv;
} sait_ws;

static int ws_init(sait_ws *w, int64_t n) {
    size_t m = (size_t)(n > 0 ? n : 1);
    w->acc = (double *)malloc(sizeof(double) * m);
    w->touched = (char *)calloc(m, 1);
    w->inS = (char *)calloc(m, 1);
    w->list = (int32_t *)malloc(sizeof(int32_t) * m);
    w->ent = (or_entry *)malloc(sizeof(or_entry) * m);
    w->dinv = (double *)malloc(sizeof(double) * m);
    return (w->acc && w->touched && w->inS && w->list && w->ent && w->dinv) ? OR_OK : OR_E_NOMEM;
}

static void ws_free(sait_ws *w) {
    free(w->acc); free(w->touched); free(w->inS); free(w->list); free(w->ent); free(w->dinv);
}

/* One unscaled pass, exported for step-by-step comparison:
 * Mnext = drop(T~ * Mprev + I), or drop(Mprev * T~ + I) when right != 0. */
int or_sait_step(int64_t n, const int32_t *Trp, const int32_t *Tci, const double *Tv,
                 const int32_t *Mrp, const int32_t *Mci, const double *Mv,
                 double tau, int cap, int right,
                 int32_t **Orp, int32_t **Oci, double **Ov) {
    if (!(tau >= 0.0 && tau < 1.0) || cap < 0) return OR_E_INVALID;
    sait_ws w;
    or_builder out;
    int st = ws_init(&w, n);
    if (st == OR_OK) st = sait_dinv(n, Trp, Tci, Tv, w.dinv);
    if (st == OR_OK) st = bld_init(&out, n, Mrp[n] + n);
    if (st == OR_OK) {
        st = sait_pass(n, Trp, Tci, Tv, w.dinv, right, Mrp, Mci, Mv, tau, cap, NULL, NULL,
                       w.acc, w.touched, w.list, w.inS, w.ent, &out);
        if (st == OR_OK) bld_give(&out, Orp, Oci, Ov);
        else bld_free(&out);
    }
    ws_free(&w);
    return st;
}

/* Common driver for Alg. 2 (S == NULL after p passes: threshold) and Alg. 3. */
static int sait_run(int64_t n, const int32_t *Trp, const int32_t *Tci, const double *Tv,
                    double tau, int m, int cap, int p_pattern, int right,
                    int32_t **Orp, int32_t **Oci, double **Ov) {
    sait_ws w;
    int st = ws_init(&w, n);
    if (st == OR_OK) st = sait_dinv(n, Trp, Tci, Tv, w.dinv);
    /* M = I */
    or_builder cur;
    if (st == OR_OK) st = bld_init(&cur, n, n);
    if (st != OR_OK) { ws_free(&w); return st; }
    for (int64_t i = 0; i < n; i++) { bld_push(&cur, (int32_t)i, 1.0); bld_end_row(&cur, i); }
    int32_t *Srp = NULL, *Sci = NULL;
    /* Alg. 3 steps 2-4: p unrestricted passes, then S = pattern(M) */
    for (int k = 0; k < p_pattern && st == OR_OK; k++) {
        or_builder nxt;
        st = bld_init(&nxt, n, cur.nnz + n);
        if (st == OR_OK) st = sait_pass(n, Trp, Tci, Tv, w.dinv, right, cur.rp, cur.ci, cur.v, 0.0, 0,
                                        NULL, NULL, w.acc, w.touched, w.list, w.inS, w.ent, &nxt);
        bld_free(&cur);
        cur = nxt;
    }
    if (st == OR_OK && p_pattern >= 0) {
        Srp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        Sci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cur.nnz > 0 ? cur.nnz : 1));
        if (!Srp || !Sci) st = OR_E_NOMEM;
        else {
            memcpy(Srp, cur.rp, sizeof(int32_t) * (size_t)(n + 1));
            memcpy(Sci, cur.ci, sizeof(int32_t) * (size_t)cur.nnz);
        }
    }
    /* Alg. 2 steps 2-5 / Alg. 3 steps 5-8: m passes with dropping */
    for (int k = 0; k < m && st == OR_OK; k++) {
        or_builder nxt;
        st = bld_init(&nxt, n, cur.nnz + n);
        if (st == OR_OK) st = sait_pass(n, Trp, Tci, Tv, w.dinv, right, cur.rp, cur.ci, cur.v, tau, cap,
                                        Srp, Sci, w.acc, w.touched, w.list, w.inS, w.ent, &nxt);
        bld_free(&cur);
        cur = nxt;
    }
    /* final step: M = M D^-1  (column j scaled by fl(1/d_j)) */
    if (st == OR_OK) {
        for (int64_t q = 0; q < cur.nnz; q++) cur.v[q] = cur.v[q] * w.dinv[cur.ci[q]];
        bld_give(&cur, Orp, Oci, Ov);
    } else {
        bld_free(&cur);
    }
    free(Srp); free(Sci);
    ws_free(&w);
    return st;
}

/* SAIT_Thr(tau, m) with optional per-row cap (Alg. 2; Appendix A);
 * right != 0 multiplies T~ from the right in every pass. */
int or_sait_thr(int64_t n, const int32_t *Trp, const int32_t *Tci, const double *Tv,
                double tau, int m, int cap, int right,
                int32_t **Orp, int32_t **Oci, double **Ov) {
    if (!(tau >= 0.0 && tau < 1.0) || m < 0 || cap < 0) return OR_E_INVALID;
    return sait_run(n, Trp, Tci, Tv, tau, m, cap, -1, right, Orp, Oci, Ov);
}

/* SAIT_Pat(p, m) (Alg. 3): p passes without dropping fix the pattern S of
 * T^p (= pattern of M_{p+1} in Eq. M_poly), m further passes masked to S. */
int or_sait_pat(int64_t n, const int32_t *Trp, const int32_t *Tci, const double *Tv,
                int p, int m, int right,
                int32_t **Orp, int32_t **Oci, double **Ov) {
    if (p < 0 || m < 0) return OR_E_INVALID;
    return sait_run(n, Trp, Tci, Tv, 0.0, m, 0, p, right, Orp, Oci, Ov);
}

/* ------------------------------------------------------------------ */
/* Apply (Sec. 3.1: U(Lx) = y replaced by x = M_U (M_L y))              */
/* ------------------------------------------------------------------ */

void or_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
             const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) s = s + v[p] * x[ci[p]];
        y[i] = s;
    }
}

/* z = second * (first * r): (first, second) = (M_L, M_U) for the
 * preconditioner, (M_U^T, M_L^T) for its transpose. */
int or_apply(int64_t n,
             const int32_t *Arp, const int32_t *Aci, const double *Av,
             const int32_t *Brp, const int32_t *Bci, const double *Bv,
             const double *r, double *z) {
    double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!y) return OR_E_NOMEM;
    or_spmv(n, Arp, Aci, Av, r, y);
    or_spmv(n, Brp, Bci, Bv, y, z);
    free(y);
    return OR_OK;
}

/* Storage roundings of the factor values: binary32 by round-to-nearest-
 * even, and bfloat16 as the round-to-nearest-even of that binary32 value
 * (upper 16 bits of the binary32 encoding). */
void or_round_f32(int64_t n, const double *in, float *out) {
    for (int64_t i = 0; i < n; i++) out[i] = (float)in[i];
}

static uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u); /* quiet NaN */
    uint32_t lsb = (u >> 16) & 1u;
    u = u + 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

void or_round_bf16(int64_t n, const double *in, uint16_t *out) {
    for (int64_t i = 0; i < n; i++) out[i] = f32_to_bf16_rne((float)in[i]);
}

void or_bf16_to_f32(int64_t n, const uint16_t *in, float *out) {
    for (int64_t i = 0; i < n; i++) {
        uint32_t u = ((uint32_t)in[i]) << 16;
        memcpy(&out[i], &u, 4);
    }
}

/* Mixed apply with binary32 accumulation: r32 = fl32(r), y32 = A32 r32,
 * z = (double)(B32 y32), each row summed in column order in binary32. */
int or_apply_f32acc(int64_t n,
                    const int32_t *Arp, const int32_t *Aci, const float *Av,
                    const int32_t *Brp, const int32_t *Bci, const float *Bv,
                    const double *r, double *z) {
    float *r32 = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    float *y32 = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    if (!r32 || !y32) { free(r32); free(y32); return OR_E_NOMEM; }
    for (int64_t i = 0; i < n; i++) r32[i] = (float)r[i];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        float s = 0.0f;
        for (int64_t p = Arp[i]; p < Arp[i + 1]; p++) s = s + Av[p] * r32[Aci[p]];
        y32[i] = s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        float s = 0.0f;
        for (int64_t p = Brp[i]; p < Brp[i + 1]; p++) s = s + Bv[p] * y32[Bci[p]];
        z[i] = (double)s;
    }
    free(r32); free(y32);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Transpose and the adjoint gradient                                   */
/* ------------------------------------------------------------------ */
int or_transpose(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                 int32_t **Orp, int32_t **Oci, double **Ov) {
    int64_t nnz = rp[n];
    int32_t *orp = (int32_t *)calloc((size_t)(n + 1), sizeof(int32_t));
    int32_t *oci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *ov = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!orp || !oci || !ov || !fill) { free(orp); free(oci); free(ov); free(fill); return OR_E_NOMEM; }
    for (int64_t p = 0; p < nnz; p++) orp[ci[p] + 1]++;
    for (int64_t j = 0; j < n; j++) orp[j + 1] += orp[j];
    for (int64_t j = 0; j < n; j++) fill[j] = orp[j];
    for (int64_t i = 0; i < n; i++)         /* rows in increasing order: output rows sorted */
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int32_t j = ci[p];
            oci[fill[j]] = (int32_t)i;
            ov[fill[j]] = v[p];
            fill[j]++;
        }
    free(fill);
    *Orp = orp; *Oci = oci; *Ov = ov;
    return OR_OK;
}

/* Gradient of a loss through x = A^-1 b with respect to the stored
 * entries of A, given the adjoint lambda = A^-T dloss/dx:
 * dloss/dA_ij = -lambda_i x_j on the pattern of A. */
void or_grad_values(int64_t n, const int32_t *rp, const int32_t *ci,
                    const double *lambda, const double *x, double *grad) {
    for (int64_t i = 0; i < n; i++)
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) grad[p] = -(lambda[i] * x[ci[p]]);
}

/* ------------------------------------------------------------------ */
/* Restarted GMRES / FGMRES, right preconditioned                       */
/* ------------------------------------------------------------------ */

/* Preconditioner kinds. */
#define OR_PREC_NONE 0
#define OR_PREC_SAIT64 1   /* z = M2 (M1 r), FP64 values */
#define OR_PREC_SAIT32 2   /* z = (double)(M2_32 (M1_32 fl32(r))), binary32 */
#define OR_PREC_EXACT 3    /* z = U^-1 (L^-1 r): M1 = L (lower), M2 = U (upper) */
#define OR_PREC_JACOBI 4   /* z = J_U^s (J_L^s r): s Jacobi sweeps on each factor */

typedef struct {
    int kind;
    const int32_t *rp1, *ci1;
    const double *v1;
    const float *f1;
    const int32_t *rp2, *ci2;
    const double *v2;
    const float *f2;
    int sweeps;
} or_prec;

/*
 * s Jacobi sweeps for a triangular system T y = r from y = 0 (Sec. 2: the
 * Jacobi iteration the SAIT series is built from): every sweep computes
 * y_new_i = (r_i - sum_{j != i} T_ij y_old_j) / T_ii from the previous
 * iterate.  One sweep gives r / diag(T); with s sweeps the result is the
 * truncated series of SAIT_Thr(0, s - 1).  Works for lower and upper T.
 */
static int jacobi_sweeps(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                         const double *r, int s, double *y) {
    if (s < 1) return OR_E_INVALID;
    double *old = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!old) return OR_E_NOMEM;
    for (int64_t i = 0; i < n; i++) y[i] = 0.0;
    int st = OR_OK;
    for (int k = 0; k < s && st == OR_OK; k++) {
        memcpy(old, y, sizeof(double) * (size_t)n);
        int bad = 0;
        /* rows are independent within a sweep: the result does not depend on the threads */
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t i = 0; i < n; i++) {
            double acc = r[i], d = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
                if (ci[p] == i) d = v[p];
                else acc = acc - v[p] * old[ci[p]];
            }
            if (d == 0.0) bad = 1;
            else y[i] = acc / d;
        }
        if (bad) st = OR_E_ZERO_PIVOT;
    }
    free(old);
    return st;
}

int or_jacobi_sweeps(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     const double *r, int s, double *y) {
    return jacobi_sweeps(n, rp, ci, v, r, s, y);
}

static int prec_apply(int64_t n, const or_prec *P, const double *r, double *z, double *tmp) {
    switch (P ? P->kind : OR_PREC_NONE) {
    case OR_PREC_NONE:
        memcpy(z, r, sizeof(double) * (size_t)n);
        return OR_OK;
    case OR_PREC_SAIT64:
        or_spmv(n, P->rp1, P->ci1, P->v1, r, tmp);
        or_spmv(n, P->rp2, P->ci2, P->v2, tmp, z);
        return OR_OK;
    case OR_PREC_SAIT32:
        return or_apply_f32acc(n, P->rp1, P->ci1, P->f1, P->rp2, P->ci2, P->f2, r, z);
    case OR_PREC_EXACT: {
        int st = or_lower_solve(n, P->rp1, P->ci1, P->v1, r, tmp);
        if (st) return st;
        return or_upper_solve(n, P->rp2, P->ci2, P->v2, tmp, z);
    }
    case OR_PREC_JACOBI: {
        int st = jacobi_sweeps(n, P->rp1, P->ci1, P->v1, r, P->sweeps, tmp);
        if (st) return st;
        return jacobi_sweeps(n, P->rp2, P->ci2, P->v2, tmp, P->sweeps, z);
    }
    default:
        return OR_E_INVALID;
    }
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

/*
 * x (in: x0, out: solution).  Stops on the true relative residual
 * ||b - A x|| / ||b|| <= rtol checked at the end of every cycle; a cycle
 * ends after `restart` inner steps, when the Arnoldi residual estimate
 * |g_{j+1}| / ||b|| <= rtol, on breakdown (h_{j+1,j} == 0) or at maxit.
 * iters = total inner steps.  hist (may be NULL, length maxit) receives
 * the estimate after every inner step.
 */
int or_gmres(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
             const or_prec *P, const double *b, double *x,
             int restart, int maxit, double rtol, int flexible,
             int *iters_out, int *restarts_out, double *relres_out, double *est_out, double *hist) {
    if (restart < 1 || maxit < 0 || !(rtol >= 0.0)) return OR_E_INVALID;
    int k = restart;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *V = (double *)malloc(sizeof(double) * nn * (size_t)(k + 1));
    double *Z = flexible ? (double *)malloc(sizeof(double) * nn * (size_t)k) : NULL;
    double *H = (double *)calloc((size_t)(k + 1) * (size_t)k, sizeof(double)); /* H[i*k + j] */
    double *cs = (double *)malloc(sizeof(double) * (size_t)k);
    double *sn = (double *)malloc(sizeof(double) * (size_t)k);
    double *g = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)k);
    double *r = (double *)malloc(sizeof(double) * nn);
    double *w = (double *)malloc(sizeof(double) * nn);
    double *z = (double *)malloc(sizeof(double) * nn);
    double *tmp = (double *)malloc(sizeof(double) * nn);
    int st = OR_OK;
    if (!V || (flexible && !Z) || !H || !cs || !sn || !g || !y || !r || !w || !z || !tmp) st = OR_E_NOMEM;
    double nb = st == OR_OK ? sqrt(dot(n, b, b)) : 0.0;
    int iters = 0, restarts = 0;
    double relres = 0.0, est = 0.0;
    if (st == OR_OK && nb == 0.0) {
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    } else if (st == OR_OK) {
        for (;;) {
            or_spmv(n, rp, ci, v, x, r);
            for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
            double beta = sqrt(dot(n, r, r));
            relres = beta / nb;
            if (relres <= rtol) { st = OR_OK; break; }
            if (iters >= maxit) { st = OR_NOT_CONVERGED; break; }
            for (int64_t i = 0; i < n; i++) V[i] = r[i] / beta;
            for (int i = 0; i <= k; i++) g[i] = 0.0;
            g[0] = beta;
            int jend = 0;
            for (int j = 0; j < k; j++) {
                double *vj = V + (size_t)j * nn;
                double *zj = flexible ? Z + (size_t)j * nn : z;
                st = prec_apply(n, P, vj, zj, tmp);
                if (st) break;
                or_spmv(n, rp, ci, v, zj, w);
                for (int i = 0; i <= j; i++) {            /* modified Gram-Schmidt */
                    double *vi = V + (size_t)i * nn;
                    double h = dot(n, w, vi);
                    H[i * k + j] = h;
                    for (int64_t t = 0; t < n; t++) w[t] = w[t] - h * vi[t];
                }
                double hn = sqrt(dot(n, w, w));
                H[(j + 1) * k + j] = hn;
                for (int i = 0; i < j; i++) {              /* previous rotations */
                    double a = H[i * k + j], c = H[(i + 1) * k + j];
                    H[i * k + j] = cs[i] * a + sn[i] * c;
                    H[(i + 1) * k + j] = -sn[i] * a + cs[i] * c;
                }
                double a = H[j * k + j], c = H[(j + 1) * k + j];
                double den = hypot(a, c);
                if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
                else { cs[j] = a / den; sn[j] = c / den; }
                H[j * k + j] = den;
                H[(j + 1) * k + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                iters++;
                jend = j + 1;
                est = fabs(g[j + 1]) / nb;
                if (hist && iters <= maxit) hist[iters - 1] = est;
                if (hn == 0.0) break;                      /* lucky breakdown */
                double *vn = V + (size_t)(j + 1) * nn;
                for (int64_t t = 0; t < n; t++) vn[t] = w[t] / hn;
                if (est <= rtol || iters >= maxit) break;
            }
            if (st) break;
            /* y = R^-1 g (upper triangular back substitution) */
            for (int i = jend - 1; i >= 0; i--) {
                double s = g[i];
                for (int t = i + 1; t < jend; t++) s = s - H[i * k + t] * y[t];
                y[i] = H[i * k + i] != 0.0 ? s / H[i * k + i] : 0.0;
            }
            if (flexible) {
                for (int i = 0; i < jend; i++) {
                    double *zi = Z + (size_t)i * nn;
                    for (int64_t t = 0; t < n; t++) x[t] = x[t] + y[i] * zi[t];
                }
            } else {
                for (int64_t t = 0; t < n; t++) w[t] = 0.0;
                for (int i = 0; i < jend; i++) {
                    double *vi = V + (size_t)i * nn;
                    for (int64_t t = 0; t < n; t++) w[t] = w[t] + y[i] * vi[t];
                }
                st = prec_apply(n, P, w, z, tmp);
                if (st) break;
                for (int64_t t = 0; t < n; t++) x[t] = x[t] + z[t];
            }
            restarts++;
        }
    }
    if (iters_out) *iters_out = iters;
    if (restarts_out) *restarts_out = restarts;
    if (relres_out) *relres_out = relres;
    if (est_out) *est_out = est;
    free(V); free(Z); free(H); free(cs); free(sn); free(g); free(y); free(r); free(w); free(z); free(tmp);
    return st;
}

/* ------------------------------------------------------------------ */
/* Preconditioned conjugate gradients (Sec. 4: the solver of the paper's */
/* experiments), textbook form (Saad, Alg. 9.1)                         */
/* ------------------------------------------------------------------ */
/*
 * r = b - A x, z = M r, p = z; per iteration: q = A p, alpha = (r, z) / (p, q),
 * x += alpha p, r -= alpha q, stop once ||r|| / ||b|| <= rtol (the recursively
 * updated residual), z = M r, beta = (r, z)_new / (r, z)_old, p = z + beta p.
 * iters = number of x updates; relres = the true ||b - A x|| / ||b|| at the
 * end; hist (may be NULL, length maxit) receives ||r|| / ||b|| after every
 * update.  Returns OR_OK, OR_NOT_CONVERGED (maxit) or OR_E_INVALID when
 * (p, q) = 0 before convergence.
 */
int or_pcg(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
           const or_prec *P, const double *b, double *x, int maxit, double rtol,
           int *iters_out, double *relres_out, double *hist) {
    if (maxit < 0 || !(rtol >= 0.0)) return OR_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(sizeof(double) * nn), *z = (double *)malloc(sizeof(double) * nn);
    double *p = (double *)malloc(sizeof(double) * nn), *q = (double *)malloc(sizeof(double) * nn);
    double *tmp = (double *)malloc(sizeof(double) * nn);
    int st = OR_OK, it = 0;
    if (!r || !z || !p || !q || !tmp) {
        st = OR_E_NOMEM;
        goto done;
    }
    or_spmv(n, rp, ci, v, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    double nb = sqrt(dot(n, b, b));
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
        goto done;
    }
    if (sqrt(dot(n, r, r)) / nb <= rtol) goto done;
    st = prec_apply(n, P, r, z, tmp);
    if (st) goto done;
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rz = dot(n, r, z);
    st = OR_NOT_CONVERGED;
    while (it < maxit) {
        or_spmv(n, rp, ci, v, p, q);
        double pq = dot(n, p, q);
        if (pq == 0.0) {
            st = OR_E_INVALID;
            break;
        }
        double alpha = rz / pq;
        for (int64_t i = 0; i < n; i++) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        it++;
        double rel = sqrt(dot(n, r, r)) / nb;
        if (hist) hist[it - 1] = rel;
        if (rel <= rtol) {
            st = OR_OK;
            break;
        }
        int s2 = prec_apply(n, P, r, z, tmp);
        if (s2) {
            st = s2;
            break;
        }
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
done:
    if (st >= 0 && relres_out) {
        or_spmv(n, rp, ci, v, x, q);
        double nb2 = sqrt(dot(n, b, b)), rr = 0.0;
        for (int64_t i = 0; i < n; i++) rr += (b[i] - q[i]) * (b[i] - q[i]);
        *relres_out = nb2 > 0.0 ? sqrt(rr) / nb2 : 0.0;
    }
    if (iters_out) *iters_out = it;
    free(r);
    free(z);
    free(p);
    free(q);
    free(tmp);
    return st;
}
