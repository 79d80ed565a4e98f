/*
 * Plain FP64 CPU oracle for repeated sparse LU refactorization of same-pattern KKT systems.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct definition that the
 * GPU library is checked against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it; the product path never calls it.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * What it computes (the refactorization strategy of Section III, Algorithm 1, and the
 * three-stage direct solver of Section II):
 *   O0 validate the CSR pattern (square, sorted, unique, in range, full diagonal);
 *   O1 exact minimum-degree column order on pattern(A + A^T) in the elimination-graph
 *      model, ties broken by the lowest original index (one vertex at a time);
 *   O2 power-of-two row-then-column max equilibration ("the system is equilibrated" in
 *      the analysis stage, Section II);
 *   O3 left-looking Gilbert-Peierls LU of the scaled first system with threshold
 *      pivoting that prefers the diagonal (the diagonal is kept when it is a nonzero
 *      candidate with |x_diag| >= tau * max|x_cand|; tau = 0 is static diagonal
 *      pivoting), which fixes the row order and the structural L/U pattern
 *      (Algorithm 1, first system factored on the CPU);
 *   O4 canonical symbolic products: combined L+U in CSC in permuted index space,
 *      elimination tree, refactor / forward / backward level sets, structural
 *      supernodes and the scatter map of each input entry into L+U (Algorithm 1,
 *      extraction and conversion of the factor structure);
 *   O5 refactorization of a later system with rows, columns and pattern fixed, tiny
 *      pivots replaced by +-eps*||A~||_inf and counted (Algorithm 1, refactor without
 *      pivoting);
 *   O6 permuted, scaled forward/backward triangular solve;
 *   O7 FP64 residual r = b - A x with the original A and the normwise backward error
 *      ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf);
 *   O8 right-preconditioned flexible GMRES(m) with classical Gram-Schmidt applied twice,
 *      preconditioned by O6, stopped on the true backward error (Algorithm 1: the solve
 *      is always followed by iterative refinement; Section V asks for a configurable one);
 *   O9 approximate triangular solves by Jacobi or block Gauss-Seidel sweeps (Section V).
 *
 * Arithmetic rules: every update of a factor entry is t = l*x (rounded), x = x - t
 * (rounded), applied in ascending pivot step; division is a true division; build with
 * -ffp-contract=off so no operation is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_WARN_PERTURBED 1
#define ORC_WARN_NOT_CONVERGED 2
#define ORC_ERR_ARG (-1)
#define ORC_ERR_PATTERN (-2)
#define ORC_ERR_SINGULAR (-3)
#define ORC_ERR_NONFINITE (-4)
#define ORC_ERR_NOMEM (-6)

typedef struct {
    int32_t n;
    int64_t nnz_a;
    /* copy of the input pattern (CSR) and its column view */
    int64_t *a_rowptr;
    int32_t *a_colind;
    int64_t *a_colptr;   /* CSC of A: column j holds entries a_cidx[..] (CSR positions) */
    int64_t *a_cpos;     /* CSR position of each CSC slot, rows ascending within a column */
    int32_t *a_crow;     /* row index of each CSC slot */
    /* permutations: row k of PAQ is row P[k] of A, column k is column Q[k] */
    int32_t *P, *Q, *pinv, *qinv;
    /* combined L+U in CSC, permuted index space */
    int64_t nnz_lu;
    int64_t *lu_colptr;
    int32_t *lu_rowidx;
    double *lu_k1;       /* numeric factors of the analysed system */
    int32_t *parent, *lev_f, *lev_l, *lev_u;
    int32_t nsn;
    int32_t *sn_start;
    int64_t *map;        /* CSR entry -> L+U slot */
} orc_sym;

/* ------------------------------------------------------------------ small helpers */

static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* 2^-floor(log2 m), via frexp; m = 0 gives 1.  The exponent is clamped to +-1020. */
static double pow2_inv_floor_log2(double m) {
    int e;
    if (!(m > 0.0)) return 1.0;
    frexp(m, &e);          /* m = f 2^e, f in [0.5, 1): floor(log2 m) = e - 1 */
    e = e - 1;
    if (e > 1020) e = 1020;
    if (e < -1020) e = -1020;
    return ldexp(1.0, -e);
}

/* ------------------------------------------------------------------ O0 validation */

int orc_validate(int32_t n, const int64_t *rowptr, const int32_t *colind) {
    if (n <= 0 || !rowptr || !colind) return ORC_ERR_ARG;
    if (rowptr[0] != 0) return ORC_ERR_PATTERN;
    for (int32_t i = 0; i < n; i++) {
        int has_diag = 0;
        if (rowptr[i + 1] < rowptr[i]) return ORC_ERR_PATTERN;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            int32_t j = colind[p];
            if (j < 0 || j >= n) return ORC_ERR_PATTERN;
            if (p > rowptr[i] && colind[p - 1] >= j) return ORC_ERR_PATTERN;
            if (j == i) has_diag = 1;
        }
        if (!has_diag) return ORC_ERR_PATTERN;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ O1 minimum degree */

/* Binary min-heap of (degree, vertex) keys with lazy deletion. */
typedef struct { int64_t key; } hitem;
typedef struct { hitem *a; int64_t size, cap; } heap_t;

static int heap_push(heap_t *h, int64_t key) {
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hitem *na = realloc(h->a, (size_t)nc * sizeof(hitem));
        if (!na) return -1;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->size++;
    h->a[i].key = key;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].key <= h->a[i].key) break;
        hitem t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t;
        i = p;
    }
    return 0;
}

static int64_t heap_pop(heap_t *h) {
    int64_t top = h->a[0].key;
    h->a[0] = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->size && h->a[l].key < h->a[m].key) m = l;
        if (r < h->size && h->a[r].key < h->a[m].key) m = r;
        if (m == i) break;
        hitem t = h->a[m]; h->a[m] = h->a[i]; h->a[i] = t;
        i = m;
    }
    return top;
}

/*
 * Exact minimum degree in the elimination-graph model.  adj[v] is the sorted neighbour
 * list of uneliminated vertex v in the current elimination graph; eliminating v joins its
 * neighbours into a clique and removes v.  The degree of v is |adj[v]|, which equals the
 * number of uneliminated vertices reachable from v through eliminated ones.  The next
 * vertex is argmin (degree, original index).
 */
int orc_min_degree(int32_t n, const int64_t *rowptr, const int32_t *colind, int32_t *order) {
    int32_t **adj = xcalloc((size_t)n, sizeof(int32_t *));
    int32_t *deg = xcalloc((size_t)n, sizeof(int32_t));
    int32_t *cap = xcalloc((size_t)n, sizeof(int32_t));
    char *gone = xcalloc((size_t)n, 1);
    int32_t *tmp = NULL;
    int64_t tmpcap = 0;
    heap_t h = {0};
    int rc = ORC_OK;
    if (!adj || !deg || !cap || !gone) { rc = ORC_ERR_NOMEM; goto done; }
    /* symmetric pattern without the diagonal */
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
            if (colind[p] != i) { deg[i]++; deg[colind[p]]++; }
    for (int32_t i = 0; i < n; i++) {
        cap[i] = deg[i] > 0 ? deg[i] : 1;
        adj[i] = malloc((size_t)cap[i] * sizeof(int32_t));
        if (!adj[i]) { rc = ORC_ERR_NOMEM; goto done; }
        deg[i] = 0;
    }
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            int32_t j = colind[p];
            if (j != i) { adj[i][deg[i]++] = j; adj[j][deg[j]++] = i; }
        }
    for (int32_t i = 0; i < n; i++) {
        qsort(adj[i], (size_t)deg[i], sizeof(int32_t), cmp_i32);
        int32_t m = 0;
        for (int32_t t = 0; t < deg[i]; t++)
            if (m == 0 || adj[i][m - 1] != adj[i][t]) adj[i][m++] = adj[i][t];
        deg[i] = m;
        if (heap_push(&h, (int64_t)deg[i] * n + i)) { rc = ORC_ERR_NOMEM; goto done; }
    }
    for (int32_t k = 0; k < n; k++) {
        int32_t v;
        for (;;) {
            int64_t key = heap_pop(&h);
            v = (int32_t)(key % n);
            if (!gone[v] && key / n == deg[v]) break;
        }
        order[k] = v;
        gone[v] = 1;
        /* each neighbour u: adj[u] <- (adj[u] U adj[v]) \ {u, v} */
        for (int32_t t = 0; t < deg[v]; t++) {
            int32_t u = adj[v][t];
            int64_t need = (int64_t)deg[u] + deg[v];
            if (need > tmpcap) {
                int32_t *nt = realloc(tmp, (size_t)need * sizeof(int32_t));
                if (!nt) { rc = ORC_ERR_NOMEM; goto done; }
                tmp = nt;
                tmpcap = need;
            }
            int32_t a = 0, b = 0, m = 0;
            const int32_t *A = adj[u], *B = adj[v];
            while (a < deg[u] || b < deg[v]) {
                int32_t w;
                if (b >= deg[v] || (a < deg[u] && A[a] < B[b])) w = A[a++];
                else if (a >= deg[u] || B[b] < A[a]) w = B[b++];
                else { w = A[a++]; b++; }
                if (w != u && w != v) tmp[m++] = w;
            }
            if (m > cap[u]) {
                int32_t *na = realloc(adj[u], (size_t)m * sizeof(int32_t));
                if (!na) { rc = ORC_ERR_NOMEM; goto done; }
                adj[u] = na;
                cap[u] = m;
            }
            memcpy(adj[u], tmp, (size_t)m * sizeof(int32_t));
            deg[u] = m;
            if (heap_push(&h, (int64_t)deg[u] * n + u)) { rc = ORC_ERR_NOMEM; goto done; }
        }
        free(adj[v]);
        adj[v] = NULL;
        deg[v] = 0;
    }
done:
    if (adj) for (int32_t i = 0; i < n; i++) free(adj[i]);
    free(adj); free(deg); free(cap); free(gone); free(tmp); free(h.a);
    return rc;
}

/* ------------------------------------------------------------------ O2 equilibration */

/* r_i = 2^-floor(log2 max_j |a_ij|), then c_j from the row-scaled matrix the same way. */
int orc_equilibrate(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                    int do_scale, double *r, double *c) {
    for (int32_t i = 0; i < n; i++) { r[i] = 1.0; c[i] = 1.0; }
    for (int64_t p = 0; p < rowptr[n]; p++)
        if (!isfinite(val[p])) return ORC_ERR_NONFINITE;
    if (!do_scale) return ORC_OK;
    for (int32_t i = 0; i < n; i++) {
        double m = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
            if (fabs(val[p]) > m) m = fabs(val[p]);
        r[i] = pow2_inv_floor_log2(m);
    }
    double *cm = xcalloc((size_t)n, sizeof(double));
    if (!cm) return ORC_ERR_NOMEM;
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            double a = fabs(r[i] * val[p]);
            if (a > cm[colind[p]]) cm[colind[p]] = a;
        }
    for (int32_t j = 0; j < n; j++) c[j] = pow2_inv_floor_log2(cm[j]);
    free(cm);
    return ORC_OK;
}

/* ------------------------------------------------------------------ analyze (O3, O4) */

void orc_free(orc_sym *s) {
    if (!s) return;
    free(s->a_rowptr); free(s->a_colind); free(s->a_colptr); free(s->a_cpos); free(s->a_crow);
    free(s->P); free(s->Q); free(s->pinv); free(s->qinv);
    free(s->lu_colptr); free(s->lu_rowidx); free(s->lu_k1);
    free(s->parent); free(s->lev_f); free(s->lev_l); free(s->lev_u);
    free(s->sn_start); free(s->map);
    free(s);
}

/* growable column store used while the factor pattern is being discovered */
typedef struct { int32_t *idx; double *val; int32_t len, cap; } col_t;

static int col_push(col_t *c, int32_t i, double v) {
    if (c->len == c->cap) {
        int32_t nc = c->cap ? 2 * c->cap : 4;
        int32_t *ni = realloc(c->idx, (size_t)nc * sizeof(int32_t));
        if (!ni) return -1;
        c->idx = ni;
        double *nv = realloc(c->val, (size_t)nc * sizeof(double));
        if (!nv) return -1;
        c->val = nv;
        c->cap = nc;
    }
    c->idx[c->len] = i;
    c->val[c->len] = v;
    c->len++;
    return 0;
}

typedef struct { int32_t row; double v; } rv_t;
static int cmp_rv(const void *a, const void *b) {
    int32_t x = ((const rv_t *)a)->row, y = ((const rv_t *)b)->row;
    return (x > y) - (x < y);
}

/*
 * Analyze: validate, order (unless fixed_q), scale the first system, factor it with
 * threshold pivoting (unless fixed_p), and build the canonical symbolic products.
 * On ORC_ERR_SINGULAR, *err_col holds the pivot step that had no usable candidate.
 */
int orc_analyze(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                double tau, int32_t sn_max, int do_scale,
                const int32_t *fixed_p, const int32_t *fixed_q,
                orc_sym **out, int32_t *err_col) {
    int rc;
    *out = NULL;
    if (err_col) *err_col = -1;
    if (!val || sn_max < 1 || !(tau >= 0.0 && tau <= 1.0)) return ORC_ERR_ARG;
    if (fixed_p && !fixed_q) return ORC_ERR_ARG;
    rc = orc_validate(n, rowptr, colind);
    if (rc) return rc;
    int64_t nnz = rowptr[n];
    orc_sym *s = xcalloc(1, sizeof(orc_sym));
    if (!s) return ORC_ERR_NOMEM;
    s->n = n;
    s->nnz_a = nnz;
    s->a_rowptr = malloc((size_t)(n + 1) * sizeof(int64_t));
    s->a_colind = malloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
    s->a_colptr = xcalloc((size_t)n + 1, sizeof(int64_t));
    s->a_cpos = xcalloc((size_t)nnz, sizeof(int64_t));
    s->a_crow = xcalloc((size_t)nnz, sizeof(int32_t));
    s->P = malloc((size_t)n * sizeof(int32_t));
    s->Q = malloc((size_t)n * sizeof(int32_t));
    s->pinv = malloc((size_t)n * sizeof(int32_t));
    s->qinv = malloc((size_t)n * sizeof(int32_t));
    double *r = malloc((size_t)n * sizeof(double)), *c = malloc((size_t)n * sizeof(double));
    double *x = xcalloc((size_t)n, sizeof(double));
    char *mark = xcalloc((size_t)n, 1);
    int32_t *stack = malloc((size_t)n * sizeof(int32_t)), *reach = malloc((size_t)n * sizeof(int32_t));
    int32_t *piv_steps = malloc((size_t)n * sizeof(int32_t));
    col_t *Lc = xcalloc((size_t)n, sizeof(col_t)), *Uc = xcalloc((size_t)n, sizeof(col_t));
    double *ukk = malloc((size_t)n * sizeof(double));
    if (!s->a_rowptr || !s->a_colind || !s->a_colptr || !s->a_cpos || !s->a_crow || !s->P || !s->Q || !s->pinv ||
        !s->qinv || !r || !c || !x || !mark || !stack || !reach || !piv_steps || !Lc || !Uc || !ukk) {
        rc = ORC_ERR_NOMEM;
        goto fail;
    }
    memcpy(s->a_rowptr, rowptr, (size_t)(n + 1) * sizeof(int64_t));
    memcpy(s->a_colind, colind, (size_t)nnz * sizeof(int32_t));
    /* column view of A (rows ascending within each column) */
    for (int64_t p = 0; p < nnz; p++) s->a_colptr[colind[p] + 1]++;
    for (int32_t j = 0; j < n; j++) s->a_colptr[j + 1] += s->a_colptr[j];
    {
        int64_t *fill = malloc((size_t)n * sizeof(int64_t));
        if (!fill) { rc = ORC_ERR_NOMEM; goto fail; }
        memcpy(fill, s->a_colptr, (size_t)n * sizeof(int64_t));
        for (int32_t i = 0; i < n; i++)
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
                s->a_crow[fill[colind[p]]] = i;
                s->a_cpos[fill[colind[p]]++] = p;
            }
        free(fill);
    }
    /* O1 */
    if (fixed_q) {
        for (int32_t k = 0; k < n; k++) s->qinv[k] = -1;
        for (int32_t k = 0; k < n; k++) {
            if (fixed_q[k] < 0 || fixed_q[k] >= n || s->qinv[fixed_q[k]] >= 0) { rc = ORC_ERR_ARG; goto fail; }
            s->qinv[fixed_q[k]] = k;
            s->Q[k] = fixed_q[k];
        }
    } else {
        rc = orc_min_degree(n, rowptr, colind, s->Q);
        if (rc) goto fail;
        for (int32_t k = 0; k < n; k++) s->qinv[s->Q[k]] = k;
    }
    if (fixed_p) {
        /* check that fixed_p is a permutation; pinv is then rebuilt step by step */
        for (int32_t k = 0; k < n; k++) s->pinv[k] = -1;
        for (int32_t k = 0; k < n; k++) {
            if (fixed_p[k] < 0 || fixed_p[k] >= n || s->pinv[fixed_p[k]] >= 0) { rc = ORC_ERR_ARG; goto fail; }
            s->pinv[fixed_p[k]] = k;
        }
    }
    for (int32_t k = 0; k < n; k++) s->pinv[k] = -1;
    /* O2 */
    rc = orc_equilibrate(n, rowptr, colind, val, do_scale, r, c);
    if (rc) goto fail;
    /* O3: left-looking LU, column k = column Q[k] of the scaled matrix */
    for (int32_t k = 0; k < n; k++) {
        int32_t col = s->Q[k], nr = 0, top;
        /* reach of the column's rows through the graph of the computed L columns */
        for (int64_t t = s->a_colptr[col]; t < s->a_colptr[col + 1]; t++) {
            int32_t i0 = s->a_crow[t];
            if (mark[i0]) continue;
            top = 0;
            stack[top++] = i0;
            mark[i0] = 1;
            while (top > 0) {
                int32_t i = stack[--top];
                reach[nr++] = i;
                int32_t j = s->pinv[i];
                if (j < 0) continue;
                for (int32_t q = 0; q < Lc[j].len; q++) {
                    int32_t i2 = Lc[j].idx[q];
                    if (!mark[i2]) { mark[i2] = 1; stack[top++] = i2; }
                }
            }
        }
        for (int32_t t = 0; t < nr; t++) mark[reach[t]] = 0;
        /* numeric: x = scaled column, then updates from pivotal rows in ascending step */
        for (int64_t t = s->a_colptr[col]; t < s->a_colptr[col + 1]; t++) {
            int32_t i = s->a_crow[t];
            x[i] = (r[i] * val[s->a_cpos[t]]) * c[col];
        }
        int32_t np = 0;
        for (int32_t t = 0; t < nr; t++)
            if (s->pinv[reach[t]] >= 0) piv_steps[np++] = s->pinv[reach[t]];
        qsort(piv_steps, (size_t)np, sizeof(int32_t), cmp_i32);
        for (int32_t t = 0; t < np; t++) {
            int32_t j = piv_steps[t];
            double xj = x[s->P[j]];
            for (int32_t q = 0; q < Lc[j].len; q++) {
                double tprod = Lc[j].val[q] * xj;
                x[Lc[j].idx[q]] = x[Lc[j].idx[q]] - tprod;
            }
            if (col_push(&Uc[k], j, xj)) { rc = ORC_ERR_NOMEM; goto fail; }
        }
        /* pivot choice among the non-pivotal rows of the reach */
        int32_t piv = -1;
        if (fixed_p) {
            piv = fixed_p[k];
            int found = 0;
            for (int32_t t = 0; t < nr; t++) if (reach[t] == piv && s->pinv[piv] < 0) found = 1;
            if (!found) { rc = ORC_ERR_SINGULAR; if (err_col) *err_col = k; goto fail; }
        } else {
            double m = 0.0;
            int diag_cand = 0;
            for (int32_t t = 0; t < nr; t++) {
                int32_t i = reach[t];
                if (s->pinv[i] >= 0) continue;
                if (fabs(x[i]) > m) m = fabs(x[i]);
                if (i == col) diag_cand = 1;
            }
            if (!(m > 0.0)) { rc = ORC_ERR_SINGULAR; if (err_col) *err_col = k; goto fail; }
            if (diag_cand && x[col] != 0.0 && fabs(x[col]) >= tau * m) {
                piv = col;
            } else {
                for (int32_t t = 0; t < nr; t++) {
                    int32_t i = reach[t];
                    if (s->pinv[i] >= 0) continue;
                    if (fabs(x[i]) == m && (piv < 0 || i < piv)) piv = i;
                }
            }
        }
        s->P[k] = piv;
        s->pinv[piv] = k;
        ukk[k] = x[piv];
        for (int32_t t = 0; t < nr; t++) {
            int32_t i = reach[t];
            if (s->pinv[i] >= 0) continue;       /* pivotal rows, including piv itself */
            if (col_push(&Lc[k], i, x[i] / ukk[k])) { rc = ORC_ERR_NOMEM; goto fail; }
        }
        for (int32_t t = 0; t < nr; t++) x[reach[t]] = 0.0;
    }
    /* O4: canonical L+U CSC in permuted index space */
    s->lu_colptr = xcalloc((size_t)n + 1, sizeof(int64_t));
    if (!s->lu_colptr) { rc = ORC_ERR_NOMEM; goto fail; }
    for (int32_t k = 0; k < n; k++) s->lu_colptr[k + 1] = s->lu_colptr[k] + Uc[k].len + 1 + Lc[k].len;
    s->nnz_lu = s->lu_colptr[n];
    s->lu_rowidx = malloc((size_t)s->nnz_lu * sizeof(int32_t));
    s->lu_k1 = malloc((size_t)s->nnz_lu * sizeof(double));
    if (!s->lu_rowidx || !s->lu_k1) { rc = ORC_ERR_NOMEM; goto fail; }
    {
        int32_t maxl = 1;
        for (int32_t k = 0; k < n; k++) if (Lc[k].len > maxl) maxl = Lc[k].len;
        rv_t *buf = malloc((size_t)maxl * sizeof(rv_t));
        if (!buf) { rc = ORC_ERR_NOMEM; goto fail; }
        for (int32_t k = 0; k < n; k++) {
            int64_t p = s->lu_colptr[k];
            for (int32_t q = 0; q < Uc[k].len; q++) {      /* already ascending in step */
                s->lu_rowidx[p] = Uc[k].idx[q];
                s->lu_k1[p++] = Uc[k].val[q];
            }
            s->lu_rowidx[p] = k;
            s->lu_k1[p++] = ukk[k];
            for (int32_t q = 0; q < Lc[k].len; q++) { buf[q].row = s->pinv[Lc[k].idx[q]]; buf[q].v = Lc[k].val[q]; }
            qsort(buf, (size_t)Lc[k].len, sizeof(rv_t), cmp_rv);
            for (int32_t q = 0; q < Lc[k].len; q++) { s->lu_rowidx[p] = buf[q].row; s->lu_k1[p++] = buf[q].v; }
        }
        free(buf);
    }
    /* elimination tree, levels */
    s->parent = malloc((size_t)n * sizeof(int32_t));
    s->lev_f = xcalloc((size_t)n, sizeof(int32_t));
    s->lev_l = xcalloc((size_t)n, sizeof(int32_t));
    s->lev_u = xcalloc((size_t)n, sizeof(int32_t));
    s->sn_start = malloc((size_t)(n + 1) * sizeof(int32_t));
    s->map = malloc((size_t)(nnz ? nnz : 1) * sizeof(int64_t));
    if (!s->parent || !s->lev_f || !s->lev_l || !s->lev_u || !s->sn_start || !s->map) { rc = ORC_ERR_NOMEM; goto fail; }
    for (int32_t k = 0; k < n; k++) {
        s->parent[k] = -1;
        for (int64_t p = s->lu_colptr[k]; p < s->lu_colptr[k + 1]; p++) {
            int32_t i = s->lu_rowidx[p];
            if (i < k) {                       /* U(i,k): refactor dependency */
                if (s->lev_f[i] + 1 > s->lev_f[k]) s->lev_f[k] = s->lev_f[i] + 1;
            } else if (i > k) {                /* L(i,k) */
                if (s->parent[k] < 0) s->parent[k] = i;   /* rows ascending: first is min */
                if (s->lev_l[k] + 1 > s->lev_l[i]) s->lev_l[i] = s->lev_l[k] + 1;
            }
        }
    }
    for (int32_t k = n - 1; k >= 0; k--)
        for (int64_t p = s->lu_colptr[k]; p < s->lu_colptr[k + 1]; p++) {
            int32_t i = s->lu_rowidx[p];
            if (i < k && s->lev_u[k] + 1 > s->lev_u[i]) s->lev_u[i] = s->lev_u[k] + 1;
        }
    /* structural supernodes: needs rows of U; build the strictly-upper CSR */
    {
        int64_t *urp = xcalloc((size_t)n + 1, sizeof(int64_t));
        int64_t nu = 0;
        for (int32_t k = 0; k < n; k++)
            for (int64_t p = s->lu_colptr[k]; p < s->lu_colptr[k + 1]; p++)
                if (s->lu_rowidx[p] < k) { urp[s->lu_rowidx[p] + 1]++; nu++; }
        for (int32_t i = 0; i < n; i++) urp[i + 1] += urp[i];
        int32_t *uci = malloc((size_t)(nu ? nu : 1) * sizeof(int32_t));
        int64_t *fill = malloc((size_t)n * sizeof(int64_t));
        if (!urp || !uci || !fill) { free(urp); free(uci); free(fill); rc = ORC_ERR_NOMEM; goto fail; }
        memcpy(fill, urp, (size_t)n * sizeof(int64_t));
        for (int32_t k = 0; k < n; k++)           /* columns ascending: rows of U sorted */
            for (int64_t p = s->lu_colptr[k]; p < s->lu_colptr[k + 1]; p++)
                if (s->lu_rowidx[p] < k) uci[fill[s->lu_rowidx[p]]++] = k;
        int32_t ns = 0, width = 1;
        s->sn_start[ns++] = 0;
        for (int32_t j = 1; j < n; j++) {
            int join = width < sn_max;
            /* L(j, j-1) != 0: column j-1's first L row is j */
            int64_t l0 = s->lu_colptr[j - 1], l1 = s->lu_colptr[j];
            int64_t dj1 = -1;
            for (int64_t p = l0; p < l1; p++) if (s->lu_rowidx[p] == j - 1) dj1 = p;
            int64_t la = dj1 + 1;                  /* L rows of column j-1 */
            if (join && !(la < l1 && s->lu_rowidx[la] == j)) join = 0;
            /* U(j-1, j) != 0: row j-1 of U contains column j */
            if (join && !(urp[j] > urp[j - 1] && uci[urp[j - 1]] == j)) join = 0;
            if (join) {   /* struct L(j+1:, j-1) == struct L(j+1:, j) */
                int64_t dj = -1;
                for (int64_t p = s->lu_colptr[j]; p < s->lu_colptr[j + 1]; p++) if (s->lu_rowidx[p] == j) dj = p;
                int64_t lb = dj + 1;
                int64_t na = l1 - (la + 1), nb = s->lu_colptr[j + 1] - lb;
                if (na != nb) join = 0;
                for (int64_t q = 0; join && q < na; q++)
                    if (s->lu_rowidx[la + 1 + q] != s->lu_rowidx[lb + q]) join = 0;
            }
            if (join) {   /* struct U(j-1, j+1:) == struct U(j, j+1:) */
                int64_t na = (urp[j] - urp[j - 1]) - 1, nb = urp[j + 1] - urp[j];
                if (na != nb) join = 0;
                for (int64_t q = 0; join && q < na; q++)
                    if (uci[urp[j - 1] + 1 + q] != uci[urp[j] + q]) join = 0;
            }
            if (join) width++;
            else { s->sn_start[ns++] = j; width = 1; }
        }
        s->sn_start[ns] = n;
        s->nsn = ns;
        free(urp); free(uci); free(fill);
    }
    /* scatter map: input entry (i, j) -> slot of (pinv[i], qinv[j]) in L+U */
    for (int32_t i = 0; i < n; i++)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            int32_t pr = s->pinv[i], pc = s->qinv[colind[p]];
            int64_t slot = -1;
            for (int64_t q = s->lu_colptr[pc]; q < s->lu_colptr[pc + 1]; q++)
                if (s->lu_rowidx[q] == pr) { slot = q; break; }
            if (slot < 0) { rc = ORC_ERR_PATTERN; goto fail; }   /* cannot happen */
            s->map[p] = slot;
        }
    rc = ORC_OK;
    *out = s;
    s = NULL;
fail:
    if (Lc) for (int32_t k = 0; k < n; k++) { free(Lc[k].idx); free(Lc[k].val); }
    if (Uc) for (int32_t k = 0; k < n; k++) { free(Uc[k].idx); free(Uc[k].val); }
    free(Lc); free(Uc); free(ukk);
    free(r); free(c); free(x); free(mark); free(stack); free(reach); free(piv_steps);
    orc_free(s);
    return rc;
}

/* ------------------------------------------------------------------ accessors */

void orc_sizes(const orc_sym *s, int32_t *n, int64_t *nnz_a, int64_t *nnz_lu, int32_t *nsn) {
    *n = s->n; *nnz_a = s->nnz_a; *nnz_lu = s->nnz_lu; *nsn = s->nsn;
}

void orc_export(const orc_sym *s, int32_t *P, int32_t *Q, int64_t *colptr, int32_t *rowidx,
                int32_t *parent, int32_t *lev_f, int32_t *lev_l, int32_t *lev_u,
                int32_t *sn_start, int64_t *map, double *lu_k1) {
    int32_t n = s->n;
    memcpy(P, s->P, (size_t)n * sizeof(int32_t));
    memcpy(Q, s->Q, (size_t)n * sizeof(int32_t));
    memcpy(colptr, s->lu_colptr, (size_t)(n + 1) * sizeof(int64_t));
    memcpy(rowidx, s->lu_rowidx, (size_t)s->nnz_lu * sizeof(int32_t));
    memcpy(parent, s->parent, (size_t)n * sizeof(int32_t));
    memcpy(lev_f, s->lev_f, (size_t)n * sizeof(int32_t));
    memcpy(lev_l, s->lev_l, (size_t)n * sizeof(int32_t));
    memcpy(lev_u, s->lev_u, (size_t)n * sizeof(int32_t));
    memcpy(sn_start, s->sn_start, (size_t)(s->nsn + 1) * sizeof(int32_t));
    memcpy(map, s->map, (size_t)s->nnz_a * sizeof(int64_t));
    memcpy(lu_k1, s->lu_k1, (size_t)s->nnz_lu * sizeof(double));
}

/* ------------------------------------------------------------------ O5 refactor */

/*
 * Refactor the system with values val (same CSR pattern) keeping P, Q and the L+U
 * pattern.  lu receives the canonical L+U values, r and c the scale factors.  A pivot with
 * |u_kk| < eps * ||A~||_inf is replaced by copysign(eps * ||A~||_inf, u_kk) (zero of either
 * sign counts as positive) and counted in *nperturbed.
 */
int orc_refactor(const orc_sym *s, const double *val, double eps, int do_scale,
                 double *lu, double *r, double *c, int64_t *nperturbed) {
    int32_t n = s->n;
    int rc = orc_equilibrate(n, s->a_rowptr, s->a_colind, val, do_scale, r, c);
    if (rc) return rc;
    /* ||A~||_inf: maximum over rows of the row sum of |r_i a_ij c_j| in CSR order */
    double anorm = 0.0;
    for (int32_t i = 0; i < n; i++) {
        double sum = 0.0;
        for (int64_t p = s->a_rowptr[i]; p < s->a_rowptr[i + 1]; p++)
            sum = sum + fabs((r[i] * val[p]) * c[s->a_colind[p]]);
        if (sum > anorm) anorm = sum;
    }
    double thresh = eps * anorm;
    double *x = xcalloc((size_t)n, sizeof(double));
    if (!x) return ORC_ERR_NOMEM;
    int64_t npert = 0;
    for (int32_t k = 0; k < n; k++) {
        int32_t col = s->Q[k];
        int64_t c0 = s->lu_colptr[k], c1 = s->lu_colptr[k + 1];
        /* x = column k of P A~ Q, in permuted row index */
        for (int64_t t = s->a_colptr[col]; t < s->a_colptr[col + 1]; t++) {
            int32_t i = s->a_crow[t];
            x[s->pinv[i]] = (r[i] * val[s->a_cpos[t]]) * c[col];
        }
        /* U part in ascending row: updates from columns j = row of U(j,k) */
        int64_t p = c0;
        for (; p < c1 && s->lu_rowidx[p] < k; p++) {
            int32_t j = s->lu_rowidx[p];
            double xj = x[j];
            int64_t q = s->lu_colptr[j];
            while (s->lu_rowidx[q] <= j) q++;   /* skip U part and diagonal of column j */
            for (; q < s->lu_colptr[j + 1]; q++) {
                double tprod = lu[q] * xj;
                x[s->lu_rowidx[q]] = x[s->lu_rowidx[q]] - tprod;
            }
            lu[p] = xj;
        }
        double u = x[k];
        if (!isfinite(u)) { free(x); return ORC_ERR_NONFINITE; }
        if (fabs(u) < thresh) {
            u = (u < 0.0) ? -thresh : thresh;
            npert++;
        }
        lu[p++] = u;
        for (; p < c1; p++) lu[p] = x[s->lu_rowidx[p]] / u;
        for (int64_t q = c0; q < c1; q++) {
            if (!isfinite(lu[q])) { free(x); return ORC_ERR_NONFINITE; }
            x[s->lu_rowidx[q]] = 0.0;
        }
    }
    free(x);
    *nperturbed = npert;
    return npert ? ORC_WARN_PERTURBED : ORC_OK;
}

/* ------------------------------------------------------------------ O6 solve */

/* x = Q C (LU)^-1 P R b, with L unit lower and U upper stored in the canonical CSC. */
void orc_solve(const orc_sym *s, const double *lu, const double *r, const double *c,
               const double *b, double *x, double *work) {
    int32_t n = s->n;
    double *y = work;
    for (int32_t k = 0; k < n; k++) y[k] = r[s->P[k]] * b[s->P[k]];
    for (int32_t j = 0; j < n; j++)              /* forward, unit L, column oriented */
        for (int64_t p = s->lu_colptr[j]; p < s->lu_colptr[j + 1]; p++) {
            int32_t i = s->lu_rowidx[p];
            if (i > j) { double t = lu[p] * y[j]; y[i] = y[i] - t; }
        }
    for (int32_t j = n - 1; j >= 0; j--) {       /* backward, U, column oriented */
        int64_t p = s->lu_colptr[j];
        while (s->lu_rowidx[p] != j) p++;
        y[j] = y[j] / lu[p];
        for (int64_t q = s->lu_colptr[j]; q < p; q++) {
            double t = lu[q] * y[j];
            y[s->lu_rowidx[q]] = y[s->lu_rowidx[q]] - t;
        }
    }
    for (int32_t k = 0; k < n; k++) x[s->Q[k]] = c[s->Q[k]] * y[k];
}

/* ------------------------------------------------------------------ O9 approximate solves */

/*
 * One approximate application of the preconditioner (Section V: the triangular solves may
 * be approximated by Jacobi or Gauss-Seidel iterations).  With y~ = P R b (permuted,
 * scaled right-hand side), `sweeps` sweeps on L y = y~ from y = 0, then `sweeps` sweeps on
 * U x~ = y from x~ = 0, and x = Q C x~.
 *   kind 0, Jacobi: every row of a sweep reads the previous iterate only,
 *       y'_i = y~_i - sum_{j<i} L_ij y_j,     x'_i = (y_i - sum_{j>i} U_ij x_j) / U_ii;
 *   kind 1, block Gauss-Seidel: the rows are cut into consecutive chunks of `chunk` rows of
 *       the permuted order; inside its chunk a row is taken after the rows before it
 *       (ascending for L, descending for U) and reads the values of its own chunk from the
 *       current sweep, every other value from the previous iterate (Jacobi between chunks).
 * Each sum runs over the row's entries in ascending column order, one rounded product and
 * one rounded addition at a time.  work: 3n doubles.
 */
int orc_approx_solve(const orc_sym *s, const double *lu, const double *r, const double *c,
                     const double *b, int32_t sweeps, int32_t kind, int32_t chunk, double *x,
                     double *work) {
    int32_t n = s->n;
    if (sweeps < 1 || (kind != 0 && kind != 1) || chunk < 1) return ORC_ERR_ARG;
    /* row-wise view of L+U: entries of row i with their columns, ascending columns */
    int64_t *rp = xcalloc((size_t)n + 1, sizeof(int64_t));
    int32_t *rc = malloc((size_t)(s->nnz_lu ? s->nnz_lu : 1) * sizeof(int32_t));
    double *rv = malloc((size_t)(s->nnz_lu ? s->nnz_lu : 1) * sizeof(double));
    int64_t *nx = malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    if (!rp || !rc || !rv || !nx) { free(rp); free(rc); free(rv); free(nx); return ORC_ERR_NOMEM; }
    for (int64_t p = 0; p < s->nnz_lu; p++) rp[s->lu_rowidx[p] + 1]++;
    for (int32_t i = 0; i < n; i++) rp[i + 1] += rp[i];
    for (int32_t i = 0; i < n; i++) nx[i] = rp[i];
    for (int32_t j = 0; j < n; j++)          /* columns ascending: rows list columns ascending */
        for (int64_t p = s->lu_colptr[j]; p < s->lu_colptr[j + 1]; p++) {
            int32_t i = s->lu_rowidx[p];
            rc[nx[i]] = j;
            rv[nx[i]] = lu[p];
            nx[i]++;
        }
    double *bt = work, *cur = work + n, *nxt = work + 2 * (size_t)n;
    for (int32_t k = 0; k < n; k++) bt[k] = r[s->P[k]] * b[s->P[k]];
    /* forward: L y = bt */
    for (int32_t i = 0; i < n; i++) cur[i] = 0.0;
    for (int32_t t = 0; t < sweeps; t++) {
        for (int32_t c0 = 0; c0 < n; c0 += chunk) {
            int32_t c1 = c0 + chunk < n ? c0 + chunk : n;
            for (int32_t i = c0; i < c1; i++) {
                double sum = 0.0;
                for (int64_t p = rp[i]; p < rp[i + 1] && rc[p] < i; p++) {
                    int32_t j = rc[p];
                    double v = (kind == 1 && j >= c0) ? nxt[j] : cur[j];
                    sum = sum + rv[p] * v;
                }
                nxt[i] = bt[i] - sum;
            }
        }
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    /* cur holds y; backward: U x~ = y, into bt (no longer needed) from zero */
    double *y = cur, *xo = bt, *xn = nxt;
    for (int32_t i = 0; i < n; i++) xo[i] = 0.0;
    for (int32_t t = 0; t < sweeps; t++) {
        for (int32_t c0 = 0; c0 < n; c0 += chunk) {
            int32_t c1 = c0 + chunk < n ? c0 + chunk : n;
            for (int32_t i = c1 - 1; i >= c0; i--) {
                double sum = 0.0, d = 0.0;
                for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
                    int32_t j = rc[p];
                    if (j < i) continue;
                    if (j == i) { d = rv[p]; continue; }
                    double v = (kind == 1 && j < c1) ? xn[j] : xo[j];
                    sum = sum + rv[p] * v;
                }
                xn[i] = (y[i] - sum) / d;
            }
        }
        double *tmp = xo; xo = xn; xn = tmp;
    }
    for (int32_t k = 0; k < n; k++) x[s->Q[k]] = c[s->Q[k]] * xo[k];
    free(rp); free(rc); free(rv); free(nx);
    return ORC_OK;
}

/* ------------------------------------------------------------------ O7 residual */

/* r = b - A x (original A), returns the normwise backward error. */
double orc_residual(int32_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                    const double *x, const double *b, double *res) {
    double anorm = 0.0, xnorm = 0.0, bnorm = 0.0, rnorm = 0.0;
    for (int32_t i = 0; i < n; i++) {
        double sum = 0.0, asum = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            sum = sum + val[p] * x[colind[p]];
            asum = asum + fabs(val[p]);
        }
        double ri = b[i] - sum;
        if (res) res[i] = ri;
        if (fabs(ri) > rnorm || isnan(ri)) rnorm = isnan(ri) ? NAN : fabs(ri);
        if (asum > anorm) anorm = asum;
        if (fabs(x[i]) > xnorm || isnan(x[i])) xnorm = isnan(x[i]) ? NAN : fabs(x[i]);
        if (fabs(b[i]) > bnorm) bnorm = fabs(b[i]);
    }
    double den = anorm * xnorm + bnorm;
    if (den == 0.0) return rnorm == 0.0 ? 0.0 : INFINITY;
    return rnorm / den;
}

/* ------------------------------------------------------------------ O8 FGMRES */

static double dot(int32_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int32_t i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

/*
 * Flexible GMRES(m), right-preconditioned by the solve above, starting from x = solve(b).
 * Stops when the true backward error is <= tol (checked at every restart and whenever the
 * Arnoldi residual estimate falls below tol * (||A|| ||x|| + ||b||)), or after max_it
 * Arnoldi steps.  Returns ORC_OK or ORC_WARN_NOT_CONVERGED; *iters and *berr report.
 */
int orc_fgmres(const orc_sym *s, const double *val, const double *lu, const double *r,
               const double *c, const double *b, double *x, int32_t m, int32_t max_it,
               double tol, int32_t *iters, double *berr_out) {
    int32_t n = s->n;
    if (m < 1) return ORC_ERR_ARG;
    double *V = malloc((size_t)n * (m + 1) * sizeof(double));
    double *Z = malloc((size_t)n * m * sizeof(double));
    double *w = malloc((size_t)n * sizeof(double)), *res = malloc((size_t)n * sizeof(double));
    double *work = malloc((size_t)n * sizeof(double));
    double *H = xcalloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc((size_t)m * sizeof(double)), *sn = malloc((size_t)m * sizeof(double));
    double *g = malloc((size_t)(m + 1) * sizeof(double)), *h = malloc((size_t)(m + 1) * sizeof(double));
    double *yv = malloc((size_t)m * sizeof(double));
    int rc = ORC_OK;
    if (!V || !Z || !w || !res || !work || !H || !cs || !sn || !g || !h || !yv) { rc = ORC_ERR_NOMEM; goto out; }
    double anorm = 0.0, bnorm = 0.0;
    for (int32_t i = 0; i < n; i++) {
        double a = 0.0;
        for (int64_t p = s->a_rowptr[i]; p < s->a_rowptr[i + 1]; p++) a = a + fabs(val[p]);
        if (a > anorm) anorm = a;
        if (fabs(b[i]) > bnorm) bnorm = fabs(b[i]);
    }
    orc_solve(s, lu, r, c, b, x, work);
    int32_t it = 0;
    double berr;
    for (;;) {
        berr = orc_residual(n, s->a_rowptr, s->a_colind, val, x, b, res);
        if (berr <= tol) { rc = ORC_OK; break; }
        if (it >= max_it || !isfinite(berr)) { rc = ORC_WARN_NOT_CONVERGED; break; }
        double xnorm = 0.0;
        for (int32_t i = 0; i < n; i++) if (fabs(x[i]) > xnorm) xnorm = fabs(x[i]);
        double target = tol * (anorm * xnorm + bnorm);
        double beta = sqrt(dot(n, res, res));
        for (int32_t i = 0; i < n; i++) V[i] = res[i] / beta;
        for (int32_t i = 0; i <= m; i++) g[i] = 0.0;
        g[0] = beta;
        int32_t jend = -1;
        for (int32_t j = 0; j < m; j++) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            orc_solve(s, lu, r, c, vj, zj, work);
            for (int32_t i = 0; i < n; i++) {           /* w = A z_j */
                double sum = 0.0;
                for (int64_t p = s->a_rowptr[i]; p < s->a_rowptr[i + 1]; p++)
                    sum = sum + val[p] * zj[s->a_colind[p]];
                w[i] = sum;
            }
            for (int32_t pass = 0; pass < 2; pass++) {   /* classical Gram-Schmidt, twice */
                for (int32_t i = 0; i <= j; i++) h[i] = dot(n, V + (size_t)i * n, w);
                for (int32_t i = 0; i <= j; i++) {
                    const double *vi = V + (size_t)i * n;
                    for (int32_t q = 0; q < n; q++) w[q] = w[q] - h[i] * vi[q];
                }
                for (int32_t i = 0; i <= j; i++)
                    H[(size_t)i * m + j] = (pass == 0) ? h[i] : H[(size_t)i * m + j] + h[i];
            }
            double hn = sqrt(dot(n, w, w));
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0)
                for (int32_t q = 0; q < n; q++) V[(size_t)(j + 1) * n + q] = w[q] / hn;
            for (int32_t i = 0; i < j; i++) {           /* previous rotations */
                double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            {
                double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
                double rr = hypot(a, bb);
                cs[j] = rr > 0.0 ? a / rr : 1.0;
                sn[j] = rr > 0.0 ? bb / rr : 0.0;
                H[(size_t)j * m + j] = rr;
                H[(size_t)(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
            }
            it++;
            jend = j;
            if (fabs(g[j + 1]) <= target || it >= max_it || hn == 0.0) break;
        }
        for (int32_t i = jend; i >= 0; i--) {            /* H y = g */
            double t = g[i];
            for (int32_t q = i + 1; q <= jend; q++) t = t - H[(size_t)i * m + q] * yv[q];
            yv[i] = H[(size_t)i * m + i] != 0.0 ? t / H[(size_t)i * m + i] : 0.0;
        }
        for (int32_t i = 0; i <= jend; i++) {
            const double *zi = Z + (size_t)i * n;
            for (int32_t q = 0; q < n; q++) x[q] = x[q] + yv[i] * zi[q];
        }
    }
    *iters = it;
    *berr_out = berr;
out:
    free(V); free(Z); free(w); free(res); free(work); free(H); free(cs); free(sn); free(g); free(h); free(yv);
    return rc;
}
