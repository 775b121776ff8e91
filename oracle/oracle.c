/*
 * oracle.c -- plain, slow, FP64 CPU reference for the symbolic and numeric
 * phases of sparse Cholesky factorization and sparse triangular solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may link,
 * load or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header or table with
 * the GPU library.
 *
 * Every routine works on a matrix that is already permuted (C = P A P^T) and
 * is given as its lower triangle in compressed sparse column form:
 * Cp int64[n+1], Ci int32[nnz] (row >= column), Cx double[nnz].  A factor L
 * is returned in the same form with the diagonal entry first in each column
 * and the rows of each column in increasing order.
 *
 * Paper passages followed (Cheshmi et al., "Sympiler", 2017):
 *   - dependence graph DG_L and reach set:          Section 1.1 (motivating
 *     scenario), Gilbert-Peierls theorem; Section 3.1 (DFS inspector)
 *   - elimination tree parent[j] = min{i > j : L_ij != 0}: Section 3.2
 *   - column pattern L_j = A_j u {j} u (u_{children s} L_s \ {s}): Eq. (1)
 *   - left-looking column Cholesky, update phase then column factorization:
 *     Section 3.2 (the left-looking Cholesky pseudo-code figure)
 *   - forward substitution over all columns, and over the reach set only:
 *     Section 1.1 (the forward-substitution and decoupled-code figures)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* O1: dense boolean elimination (the elimination game on a bitset).        */
/* ------------------------------------------------------------------------ */

/* Eliminating vertex k joins all of its higher-numbered neighbours into a
 * clique; after all eliminations, column j of L holds every i >= j that is
 * adjacent to j.  B is kept symmetric and row-major as 64-bit words.
 * Writes Lp[n+1] always and Li[] when cap >= nnz(L); returns nnz(L), or -1
 * when memory is exhausted. */
int64_t orc_bool_elim(int32_t n, const int64_t *Cp, const int32_t *Ci,
                      int64_t *Lp, int32_t *Li, int64_t cap)
{
    int64_t words = ((int64_t)n + 63) / 64;
    uint64_t *B = (uint64_t *)calloc((size_t)(n > 0 ? n : 1) * (size_t)(words > 0 ? words : 1),
                                     sizeof(uint64_t));
    if (!B) return -1;
#define BIT_SET(r, c) (B[(int64_t)(r) * words + ((c) >> 6)] |= (1ull << ((c) & 63)))
#define BIT_GET(r, c) ((B[(int64_t)(r) * words + ((c) >> 6)] >> ((c) & 63)) & 1ull)
    for (int32_t j = 0; j < n; ++j) {
        BIT_SET(j, j);
        for (int64_t p = Cp[j]; p < Cp[j + 1]; ++p) {
            int32_t i = Ci[p];
            BIT_SET(i, j);
            BIT_SET(j, i);
        }
    }
    for (int32_t k = 0; k < n; ++k) {
        const uint64_t *rk = B + (int64_t)k * words;
        for (int32_t i = k + 1; i < n; ++i) {
            if (!BIT_GET(k, i)) continue;
            uint64_t *ri = B + (int64_t)i * words;
            /* row i gains every neighbour of k above k */
            int64_t w0 = (k + 1) >> 6;
            uint64_t first_mask = ((k + 1) & 63) ? ~((1ull << ((k + 1) & 63)) - 1ull) : ~0ull;
            ri[w0] |= rk[w0] & first_mask;
            for (int64_t w = w0 + 1; w < words; ++w) ri[w] |= rk[w];
        }
    }
    int64_t nnz = 0;
    Lp[0] = 0;
    for (int32_t j = 0; j < n; ++j) {
        for (int32_t i = j; i < n; ++i) {
            if (BIT_GET(j, i)) {
                if (nnz < cap) Li[nnz] = i;
                ++nnz;
            }
        }
        Lp[j + 1] = nnz;
    }
#undef BIT_SET
#undef BIT_GET
    free(B);
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* O2: column patterns by Eq. (1), with explicit sorted sets.               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    int64_t nnz;
    int64_t *Lp;
    int32_t *Li;
    int32_t *parent;
} orc_pattern;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Columns in increasing order: L_j = C_j u {j} u (union over children s of
 * j in the elimination tree of L_s \ {s}); parent[j] = min(L_j \ {j}), or -1
 * for a root.  Returns NULL when memory is exhausted. */
orc_pattern *orc_symbolic_eq1(int32_t n, const int64_t *Cp, const int32_t *Ci)
{
    orc_pattern *P = (orc_pattern *)calloc(1, sizeof(orc_pattern));
    if (!P) return NULL;
    P->n = n;
    P->Lp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    P->parent = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *child_head = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *child_next = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int64_t cap = 16 + 4 * (n > 0 ? Cp[n] : 0);
    P->Li = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    if (!P->Lp || !P->parent || !child_head || !child_next || !mark || !buf || !P->Li) goto fail;
    for (int32_t j = 0; j < n; ++j) { child_head[j] = -1; mark[j] = -1; }
    P->Lp[0] = 0;
    for (int32_t j = 0; j < n; ++j) {
        int32_t cnt = 0;
        mark[j] = j;
        buf[cnt++] = j;
        for (int64_t p = Cp[j]; p < Cp[j + 1]; ++p) {
            int32_t i = Ci[p];
            if (mark[i] != j) { mark[i] = j; buf[cnt++] = i; }
        }
        for (int32_t s = child_head[j]; s != -1; s = child_next[s]) {
            for (int64_t p = P->Lp[s]; p < P->Lp[s + 1]; ++p) {
                int32_t i = P->Li[p];
                if (i == s) continue;
                if (mark[i] != j) { mark[i] = j; buf[cnt++] = i; }
            }
        }
        qsort(buf, (size_t)cnt, sizeof(int32_t), cmp_i32);
        if (P->Lp[j] + cnt > cap) {
            while (P->Lp[j] + cnt > cap) cap *= 2;
            int32_t *nl = (int32_t *)realloc(P->Li, sizeof(int32_t) * (size_t)cap);
            if (!nl) goto fail;
            P->Li = nl;
        }
        memcpy(P->Li + P->Lp[j], buf, sizeof(int32_t) * (size_t)cnt);
        P->Lp[j + 1] = P->Lp[j] + cnt;
        int32_t par = cnt > 1 ? buf[1] : -1;
        P->parent[j] = par;
        if (par >= 0) { child_next[j] = child_head[par]; child_head[par] = j; }
    }
    P->nnz = n > 0 ? P->Lp[n] : 0;
    free(child_head); free(child_next); free(mark); free(buf);
    return P;
fail:
    free(child_head); free(child_next); free(mark); free(buf);
    free(P->Lp); free(P->Li); free(P->parent); free(P);
    return NULL;
}

int64_t orc_pattern_nnz(const orc_pattern *P) { return P->nnz; }

void orc_pattern_copy(const orc_pattern *P, int64_t *Lp, int32_t *Li, int32_t *parent)
{
    memcpy(Lp, P->Lp, sizeof(int64_t) * ((size_t)P->n + 1));
    if (P->nnz) memcpy(Li, P->Li, sizeof(int32_t) * (size_t)P->nnz);
    if (P->n) memcpy(parent, P->parent, sizeof(int32_t) * (size_t)P->n);
}

void orc_pattern_free(orc_pattern *P)
{
    if (!P) return;
    free(P->Lp); free(P->Li); free(P->parent); free(P);
}

/* ------------------------------------------------------------------------ */
/* Fundamental supernodes (Section 3.2, the rule after Eq. (1)).            */
/* ------------------------------------------------------------------------ */

/* Column j-1 joins column j's supernode when j-1's only parent is j, j has
 * exactly one child, and the counts agree once j-1's diagonal is dropped.
 * Writes super_ptr (first column of each supernode, then n) and returns the
 * number of supernodes. */
int32_t orc_supernodes(int32_t n, const int32_t *parent, const int64_t *colcount,
                       int32_t *super_ptr)
{
    int32_t *nchild = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!nchild) return -1;
    for (int32_t j = 0; j < n; ++j)
        if (parent[j] >= 0) nchild[parent[j]]++;
    int32_t ns = 0;
    for (int32_t j = 0; j < n; ++j) {
        int merge = j > 0 && parent[j - 1] == j && nchild[j] == 1 &&
                    colcount[j - 1] - 1 == colcount[j];
        if (!merge) super_ptr[ns++] = j;
    }
    super_ptr[ns] = n;
    free(nchild);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* O3: left-looking column Cholesky (update phase, then column phase).      */
/* ------------------------------------------------------------------------ */

/* L's pattern (Lp, Li) must be the filled pattern of C with the diagonal
 * first in each column.  For each column j: scatter C(:, j) into a dense
 * work vector w; for every earlier column k with L_jk != 0 subtract
 * L_ik * L_jk from w_i for all i >= j in column k; then L_jj = sqrt(w_j) and
 * L_ij = w_i / L_jj.  Returns 0, or 1 + j for the first column j whose pivot
 * w_j is not positive (the factorization stops there).  *flops counts one
 * flop per multiply, subtract, divide and square root. */
int64_t orc_chol_column(int32_t n, const int64_t *Cp, const int32_t *Ci, const double *Cx,
                        const int64_t *Lp, const int32_t *Li, double *Lx, double *flops)
{
    double fl = 0.0;
    int64_t info = 0;
    double *w = (double *)calloc((size_t)n + 1, sizeof(double));
    int64_t *rowptr = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
    int64_t nnzL = n > 0 ? Lp[n] : 0;
    int64_t noff = nnzL - n;
    int32_t *rowk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(noff > 0 ? noff : 1));
    int64_t *rowpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(noff > 0 ? noff : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!w || !rowptr || !rowk || !rowpos || !fill) { info = -1; goto done; }
    /* row pattern of L: for every row i, the columns k < i with L_ik != 0 */
    for (int32_t k = 0; k < n; ++k)
        for (int64_t p = Lp[k] + 1; p < Lp[k + 1]; ++p) rowptr[Li[p] + 1]++;
    for (int32_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
    for (int32_t i = 0; i < n; ++i) fill[i] = rowptr[i];
    for (int32_t k = 0; k < n; ++k)
        for (int64_t p = Lp[k] + 1; p < Lp[k + 1]; ++p) {
            int32_t i = Li[p];
            rowk[fill[i]] = k;
            rowpos[fill[i]] = p;
            fill[i]++;
        }
    for (int32_t j = 0; j < n; ++j) {
        /* update phase */
        for (int64_t p = Cp[j]; p < Cp[j + 1]; ++p) w[Ci[p]] += Cx[p];
        for (int64_t r = rowptr[j]; r < rowptr[j + 1]; ++r) {
            int32_t k = rowk[r];
            int64_t pj = rowpos[r];            /* position of L_jk in column k */
            double ljk = Lx[pj];
            for (int64_t q = pj; q < Lp[k + 1]; ++q) {
                w[Li[q]] -= Lx[q] * ljk;
                fl += 2.0;
            }
        }
        /* column factorization */
        double d = w[j];
        if (!(d > 0.0)) { info = (int64_t)j + 1; goto done; }
        double ljj = sqrt(d);
        fl += 1.0;
        Lx[Lp[j]] = ljj;
        w[j] = 0.0;
        for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) {
            Lx[p] = w[Li[p]] / ljj;
            w[Li[p]] = 0.0;
            fl += 1.0;
        }
    }
done:
    if (flops) *flops = fl;
    free(w); free(rowptr); free(rowk); free(rowpos); free(fill);
    return info;
}

/* ------------------------------------------------------------------------ */
/* O4: substitution.                                                        */
/* ------------------------------------------------------------------------ */

/* Forward substitution over every column: x_j /= L_jj, then x_i -= L_ij x_j
 * for the rows i > j of column j.  x holds b on entry, the solution on exit. */
void orc_fwd(int32_t n, const int64_t *Lp, const int32_t *Li, const double *Lx, double *x)
{
    for (int32_t j = 0; j < n; ++j) {
        x[j] /= Lx[Lp[j]];
        double xj = x[j];
        for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) x[Li[p]] -= Lx[p] * xj;
    }
}

/* Backward substitution with L^T: columns in decreasing order,
 * x_j = (x_j - sum_{i > j} L_ij x_i) / L_jj. */
void orc_bwd(int32_t n, const int64_t *Lp, const int32_t *Li, const double *Lx, double *x)
{
    for (int32_t j = n - 1; j >= 0; --j) {
        double s = x[j];
        for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) s -= Lx[p] * x[Li[p]];
        x[j] = s / Lx[Lp[j]];
    }
}

/* Reach set of beta in DG_L (edge j -> i for every L_ij != 0, i != j), by
 * depth-first search.  Writes the reached columns into out[] in increasing
 * order (a topological order for a lower-triangular L) and returns their
 * count, or -1 when memory is exhausted. */
int64_t orc_reach(int32_t n, const int64_t *Lp, const int32_t *Li,
                  const int32_t *beta, int64_t nb, int32_t *out)
{
    uint8_t *seen = (uint8_t *)calloc((size_t)n + 1, 1);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!seen || !stack) { free(seen); free(stack); return -1; }
    int64_t top = 0;
    for (int64_t t = 0; t < nb; ++t) {
        int32_t s = beta[t];
        if (seen[s]) continue;
        seen[s] = 1;
        stack[top++] = s;
        while (top > 0) {
            int32_t j = stack[--top];
            for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) {
                int32_t i = Li[p];
                if (!seen[i]) { seen[i] = 1; stack[top++] = i; }
            }
        }
    }
    int64_t cnt = 0;
    for (int32_t j = 0; j < n; ++j)
        if (seen[j]) out[cnt++] = j;
    free(seen);
    free(stack);
    return cnt;
}

/* Forward substitution restricted to the given columns (which must be the
 * reach set of b's nonzeros, in a topological order).  Entries of x outside
 * the set are neither read nor written. */
void orc_fwd_pruned(int32_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
                    const int32_t *cols, int64_t ncols, double *x)
{
    (void)n;
    for (int64_t t = 0; t < ncols; ++t) {
        int32_t j = cols[t];
        x[j] /= Lx[Lp[j]];
        double xj = x[j];
        for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) x[Li[p]] -= Lx[p] * xj;
    }
}

/* ------------------------------------------------------------------------ */
/* O5: invariants.                                                          */
/* ------------------------------------------------------------------------ */

static int64_t find_row(const int32_t *Li, int64_t lo, int64_t hi, int32_t row)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (Li[mid] < row) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* ||L L^T - C||_F / ||C||_F over the full symmetric matrices.  L L^T is
 * formed on the pattern of L (every column pattern is a clique of the filled
 * graph, so L L^T has no entry outside it).  Returns -1 when memory is
 * exhausted and -2 when C has an entry outside L's pattern. */
double orc_llt_residual(int32_t n, const int64_t *Cp, const int32_t *Ci, const double *Cx,
                        const int64_t *Lp, const int32_t *Li, const double *Lx)
{
    int64_t nnzL = n > 0 ? Lp[n] : 0;
    double *M = (double *)calloc((size_t)(nnzL > 0 ? nnzL : 1), sizeof(double));
    if (!M) return -1.0;
    for (int32_t k = 0; k < n; ++k) {
        for (int64_t a = Lp[k]; a < Lp[k + 1]; ++a) {
            int32_t j = Li[a];
            for (int64_t b = a; b < Lp[k + 1]; ++b) {
                int32_t i = Li[b];
                int64_t q = find_row(Li, Lp[j], Lp[j + 1], i);
                M[q] += Lx[a] * Lx[b];
            }
        }
    }
    double num = 0.0, den = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        for (int64_t p = Cp[j]; p < Cp[j + 1]; ++p) {
            int32_t i = Ci[p];
            int64_t q = find_row(Li, Lp[j], Lp[j + 1], i);
            if (q >= Lp[j + 1] || Li[q] != i) { free(M); return -2.0; }
            M[q] -= Cx[p];
            den += (i == j ? 1.0 : 2.0) * Cx[p] * Cx[p];
        }
    }
    for (int32_t j = 0; j < n; ++j)
        for (int64_t q = Lp[j]; q < Lp[j + 1]; ++q)
            num += (Li[q] == j ? 1.0 : 2.0) * M[q] * M[q];
    free(M);
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/* y = C x for the symmetric matrix whose lower triangle is (Cp, Ci, Cx). */
void orc_symv_lower(int32_t n, const int64_t *Cp, const int32_t *Ci, const double *Cx,
                    const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = Cp[j]; p < Cp[j + 1]; ++p) {
            int32_t i = Ci[p];
            y[i] += Cx[p] * x[j];
            if (i != j) y[j] += Cx[p] * x[i];
        }
}

/* y = L x and y = L^T x. */
void orc_lmul(int32_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
              const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = Lp[j]; p < Lp[j + 1]; ++p) y[Li[p]] += Lx[p] * x[j];
}

void orc_ltmul(int32_t n, const int64_t *Lp, const int32_t *Li, const double *Lx,
               const double *x, double *y)
{
    for (int32_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t p = Lp[j]; p < Lp[j + 1]; ++p) s += Lx[p] * x[Li[p]];
        y[j] = s;
    }
}
