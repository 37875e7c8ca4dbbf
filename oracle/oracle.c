/*
 * CPU FP64 oracle for the domain-decomposed ILU0 path of
 * "Mapping Sparse Triangular Solves to GPUs via Fine-grained Domain
 * Decomposition" (arXiv 2508.04917).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * table with the GPU library and includes nothing from it.
 *
 * Every routine is a direct, sequential statement of the operation it names:
 * loops in natural order, no blocking, no reordering beyond what the
 * definition states.  Blocks are bs x bs (bs = 1 or 3), stored row-major;
 * BSR arrays are (ptr[n+1], col[nnzb], val[nnzb*bs*bs]).
 *
 * Return codes: 0 ok, -1 invalid argument, -2 grid not divisible by the
 * subdomain extents, -4 zero (or numerically singular) pivot block,
 * -5 BiCGSTAB breakdown, -6 no convergence within maxit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_OK 0
#define O_EINVAL (-1)
#define O_ENOTDIV (-2)
#define O_EZEROPIVOT (-4)
#define O_EBREAKDOWN (-5)
#define O_ENOCONV (-6)

/* ------------------------------------------------------------------ */
/* small dense block helpers (bs x bs, row-major)                      */
/* ------------------------------------------------------------------ */

/* C = A * B */
static void blk_mul(int bs, const double *A, const double *B, double *C) {
    for (int i = 0; i < bs; ++i)
        for (int j = 0; j < bs; ++j) {
            double s = 0.0;
            for (int k = 0; k < bs; ++k) s += A[i * bs + k] * B[k * bs + j];
            C[i * bs + j] = s;
        }
}

/* y -= A x */
static void blk_matvec_sub(int bs, const double *A, const double *x, double *y) {
    for (int i = 0; i < bs; ++i) {
        double s = 0.0;
        for (int k = 0; k < bs; ++k) s += A[i * bs + k] * x[k];
        y[i] -= s;
    }
}

/* y = A x */
static void blk_matvec(int bs, const double *A, const double *x, double *y) {
    for (int i = 0; i < bs; ++i) {
        double s = 0.0;
        for (int k = 0; k < bs; ++k) s += A[i * bs + k] * x[k];
        y[i] = s;
    }
}

static double blk_norm1(int bs, const double *A) {
    double m = 0.0;
    for (int j = 0; j < bs; ++j) {
        double s = 0.0;
        for (int i = 0; i < bs; ++i) s += fabs(A[i * bs + j]);
        if (s > m) m = s;
    }
    return m;
}

/* Inverse by Gauss-Jordan elimination with partial pivoting.
 * Returns 0, or -4 when a pivot is zero/non-finite or cond_1 > 1e14. */
int o_block_inverse(int bs, const double *A, double *Ainv) {
    double a[9], inv[9];
    if (bs < 1 || bs > 3) return O_EINVAL;
    memcpy(a, A, sizeof(double) * bs * bs);
    for (int i = 0; i < bs * bs; ++i) inv[i] = 0.0;
    for (int i = 0; i < bs; ++i) inv[i * bs + i] = 1.0;
    for (int c = 0; c < bs; ++c) {
        int p = c;
        for (int r = c + 1; r < bs; ++r)
            if (fabs(a[r * bs + c]) > fabs(a[p * bs + c])) p = r;
        double piv = a[p * bs + c];
        if (!(fabs(piv) > 0.0) || !isfinite(piv)) return O_EZEROPIVOT;
        if (p != c)
            for (int k = 0; k < bs; ++k) {
                double t = a[c * bs + k]; a[c * bs + k] = a[p * bs + k]; a[p * bs + k] = t;
                t = inv[c * bs + k]; inv[c * bs + k] = inv[p * bs + k]; inv[p * bs + k] = t;
            }
        for (int k = 0; k < bs; ++k) { a[c * bs + k] /= piv; inv[c * bs + k] /= piv; }
        for (int r = 0; r < bs; ++r) {
            if (r == c) continue;
            double f = a[r * bs + c];
            for (int k = 0; k < bs; ++k) {
                a[r * bs + k] -= f * a[c * bs + k];
                inv[r * bs + k] -= f * inv[c * bs + k];
            }
        }
    }
    double cond = blk_norm1(bs, A) * blk_norm1(bs, inv);
    if (!isfinite(cond) || cond > 1e14) return O_EZEROPIVOT;
    memcpy(Ainv, inv, sizeof(double) * bs * bs);
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Section 3, Algorithm 2: partition labels by geometric cuts          */
/* ------------------------------------------------------------------ */
/* (sx, sy, sz) are subdomain EXTENTS in cells; the grid must divide evenly. */
int o_partition(int nx, int ny, int nz, int sx, int sy, int sz, int32_t *part_id) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || sx <= 0 || sy <= 0 || sz <= 0) return O_EINVAL;
    if (nx % sx || ny % sy || nz % sz) return O_ENOTDIV;
    int bx = nx / sx, by = ny / sy;
    for (int i = 0; i < nx; ++i) {
        int ibx = i / sx;
        for (int j = 0; j < ny; ++j) {
            int jby = j / sy;
            for (int k = 0; k < nz; ++k) {
                int kbz = k / sz;
                int64_t gidx = (int64_t)i + (int64_t)nx * ((int64_t)j + (int64_t)ny * k);
                part_id[gidx] = ibx + bx * (jby + by * kbz);
            }
        }
    }
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Section 3 (graph-based labels) and Section 5.3 (uniform part sizes): */
/* partition a matrix graph without geometry into parts of exactly S    */
/* vertices.  The paper uses METIS and then balances the parts to one   */
/* size by hand; METIS is not available, so this is a stated reading:   */
/* recursive BFS bisection.  A segment of k parts (k*S vertices, all     */
/* labelled with its first part number b) is split, if k > 1, as        */
/* follows: BFS inside the segment (edges to vertices of other segments */
/* are ignored) from its smallest vertex; the reached vertex of largest */
/* distance, smallest index on ties, is the start v0 of a second BFS;   */
/* the segment's vertices ordered by (distance from v0, index), with    */
/* unreached vertices last, give their first k0*S (k0 = floor(k/2)) to  */
/* label b and the rest to label b + k0.  All segments of one depth are */
/* independent.  Edges are the off-diagonal blocks of the pattern;      */
/* the pattern need not be symmetric (a vertex reaches the columns of   */
/* its row).                                                            */
/* ------------------------------------------------------------------ */
static void seg_bfs(const int32_t *ptr, const int32_t *col, const int32_t *label, int32_t lab,
                    int32_t src, int64_t *dist, int32_t *queue) {
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t v = queue[head++];
        for (int32_t q = ptr[v]; q < ptr[v + 1]; ++q) {
            int32_t u = col[q];
            if (label[u] == lab && dist[u] < 0) {
                dist[u] = dist[v] + 1;
                queue[tail++] = u;
            }
        }
    }
}

typedef struct { int64_t d; int32_t v; } o_dv;

static int cmp_dv(const void *a, const void *b) {
    const o_dv *x = (const o_dv *)a, *y = (const o_dv *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return (x->v > y->v) - (x->v < y->v);
}

int o_graph_partition(int64_t n, const int32_t *ptr, const int32_t *col, int32_t S, int32_t *part_id) {
    if (n <= 0 || S <= 0 || n % S) return O_ENOTDIV;
    const int32_t nparts = (int32_t)(n / S);
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *segk = (int32_t *)calloc((size_t)nparts, sizeof(int32_t));
    int32_t *members = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    o_dv *ord = (o_dv *)malloc(sizeof(o_dv) * (size_t)n);
    if (!dist || !queue || !segk || !members || !ord) {
        free(dist); free(queue); free(segk); free(members); free(ord);
        return O_EINVAL;
    }
    for (int64_t v = 0; v < n; ++v) part_id[v] = 0;
    segk[0] = nparts;
    for (int round = 0; ; ++round) {
        int any = 0;
        for (int32_t b = 0; b < nparts; ++b) {
            int32_t k = segk[b];
            if (k <= 1) continue;
            any = 1;
            /* the segment's vertices in ascending index */
            int64_t m = 0;
            for (int64_t v = 0; v < n; ++v)
                if (part_id[v] == b) members[m++] = (int32_t)v;
            for (int64_t i = 0; i < m; ++i) dist[members[i]] = -1;
            seg_bfs(ptr, col, part_id, b, members[0], dist, queue);
            int32_t v0 = members[0];
            int64_t dmax = -1;
            for (int64_t i = 0; i < m; ++i) {
                int32_t v = members[i];
                if (dist[v] > dmax) { dmax = dist[v]; v0 = v; }
            }
            for (int64_t i = 0; i < m; ++i) dist[members[i]] = -1;
            seg_bfs(ptr, col, part_id, b, v0, dist, queue);
            for (int64_t i = 0; i < m; ++i) {
                int32_t v = members[i];
                ord[i].d = dist[v] < 0 ? INT64_MAX : dist[v];
                ord[i].v = v;
            }
            qsort(ord, (size_t)m, sizeof(o_dv), cmp_dv);
            int32_t k0 = k / 2;
            for (int64_t i = 0; i < m; ++i) part_id[ord[i].v] = i < (int64_t)k0 * S ? b : b + k0;
        }
        if (!any) break;
        /* children of every split segment (after all labels of this depth are final) */
        int32_t *next = (int32_t *)calloc((size_t)nparts, sizeof(int32_t));
        if (!next) { free(dist); free(queue); free(segk); free(members); free(ord); return O_EINVAL; }
        for (int32_t b = 0; b < nparts; ++b) {
            int32_t k = segk[b];
            if (k == 1) next[b] = 1;
            else if (k > 1) { next[b] = k / 2; next[b + k / 2] = k - k / 2; }
        }
        memcpy(segk, next, sizeof(int32_t) * (size_t)nparts);
        free(next);
    }
    free(dist); free(queue); free(segk); free(members); free(ord);
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Section 3.1: renumber vertices by their label (stable in old index) */
/* ------------------------------------------------------------------ */
int o_permutation(int64_t n, int32_t nsub, const int32_t *part_id,
                  int32_t *new2old, int32_t *old2new) {
    int64_t *count = (int64_t *)calloc((size_t)nsub + 1, sizeof(int64_t));
    if (!count) return O_EINVAL;
    for (int64_t g = 0; g < n; ++g) {
        if (part_id[g] < 0 || part_id[g] >= nsub) { free(count); return O_EINVAL; }
        count[part_id[g] + 1]++;
    }
    for (int32_t s = 0; s < nsub; ++s) count[s + 1] += count[s];
    for (int64_t g = 0; g < n; ++g) {
        int64_t pos = count[part_id[g]]++;
        new2old[pos] = (int32_t)g;
        old2new[g] = (int32_t)pos;
    }
    free(count);
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Section 3.1, Algorithm 3 (block rows): reorder by row permutation   */
/* Row i of the result is old row new2old[i]; columns map through      */
/* old2new; each row's (column, block) pairs are sorted by column.     */
/* val/oval may be NULL (pattern only).                                */
/* ------------------------------------------------------------------ */
int o_reorder(int64_t n, int bs, const int32_t *ptr, const int32_t *col, const double *val,
              const int32_t *new2old, const int32_t *old2new,
              int32_t *optr, int32_t *ocol, double *oval) {
    int bb = bs * bs;
    optr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t k = new2old[i];
        optr[i + 1] = ptr[k + 1] - ptr[k];
    }
    for (int64_t i = 0; i < n; ++i) optr[i + 1] += optr[i];
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t src = new2old[i];
        int64_t start = m;
        for (int64_t j = ptr[src]; j < ptr[src + 1]; ++j) {
            ocol[m] = old2new[col[j]];
            if (val) memcpy(oval + m * bb, val + j * bb, sizeof(double) * bb);
            ++m;
        }
        /* insertion sort of the row's (column, block) pairs */
        for (int64_t a = start + 1; a < m; ++a) {
            int32_t c = ocol[a];
            double blk[9];
            if (val) memcpy(blk, oval + a * bb, sizeof(double) * bb);
            int64_t b = a - 1;
            while (b >= start && ocol[b] > c) {
                ocol[b + 1] = ocol[b];
                if (val) memcpy(oval + (b + 1) * bb, oval + b * bb, sizeof(double) * bb);
                --b;
            }
            ocol[b + 1] = c;
            if (val) memcpy(oval + (b + 1) * bb, blk, sizeof(double) * bb);
        }
    }
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Section 3.2: drop every block outside the S x S diagonal windows    */
/* Returns the number of kept blocks.  With optr == NULL it only       */
/* counts.  val/oval may be NULL (pattern only).                       */
/* ------------------------------------------------------------------ */
int64_t o_drop(int64_t n, int bs, int64_t S, const int32_t *ptr, const int32_t *col,
               const double *val, int32_t *optr, int32_t *ocol, double *oval) {
    int bb = bs * bs;
    int64_t m = 0;
    if (optr) optr[0] = 0;
    for (int64_t I = 0; I < n; ++I) {
        for (int64_t j = ptr[I]; j < ptr[I + 1]; ++j) {
            if (col[j] / S == I / S) {
                if (optr) {
                    ocol[m] = col[j];
                    if (val && oval) memcpy(oval + m * bb, val + j * bb, sizeof(double) * bb);
                }
                ++m;
            }
        }
        if (optr) optr[I + 1] = (int32_t)m;
    }
    return m;
}

/* ------------------------------------------------------------------ */
/* Section 4.2.1: level (longest dependency path) of each row.         */
/* which = 0: lower factor, level(I) = 0 if row I has no J < I, else   */
/*            1 + max level(J) over J < I in row I.                    */
/* which = 1: upper factor, the mirror image over K > I.               */
/* Computed sequentially (I ascending for L, descending for U).        */
/* ------------------------------------------------------------------ */
int o_levels(int64_t n, const int32_t *ptr, const int32_t *col, int which, int32_t *lev) {
    if (which == 0) {
        for (int64_t I = 0; I < n; ++I) {
            int32_t l = 0;
            for (int64_t j = ptr[I]; j < ptr[I + 1]; ++j)
                if (col[j] < I && lev[col[j]] + 1 > l) l = lev[col[j]] + 1;
            lev[I] = l;
        }
    } else if (which == 1) {
        for (int64_t I = n - 1; I >= 0; --I) {
            int32_t l = 0;
            for (int64_t j = ptr[I]; j < ptr[I + 1]; ++j)
                if (col[j] > I && lev[col[j]] + 1 > l) l = lev[col[j]] + 1;
            lev[I] = l;
        }
    } else {
        return O_EINVAL;
    }
    return O_OK;
}

/* Per-subdomain level lists (the explicit DAG of Section 4.2.2): for
 * subdomain s, nlev[s] levels; level_ptr holds nlev[s]+1 offsets per
 * subdomain (relative to the subdomain's first row), concatenated over s;
 * level_rows holds the subdomain's local row indices grouped by level,
 * ascending within a level.  level_ptr must have room for n + nsub entries.
 * Returns the number of level_ptr entries written. */
int64_t o_level_lists(int64_t n, int64_t S, const int32_t *lev, int32_t *nlev,
                      int32_t *level_ptr, int32_t *level_rows) {
    if (S <= 0 || n % S) return O_EINVAL;
    int64_t nsub = n / S, w = 0;
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(S + 1));
    if (!cnt) return O_EINVAL;
    for (int64_t s = 0; s < nsub; ++s) {
        const int32_t *L = lev + s * S;
        int32_t maxl = -1;
        for (int64_t i = 0; i < S; ++i) if (L[i] > maxl) maxl = L[i];
        int32_t nl = maxl + 1;
        nlev[s] = nl;
        for (int32_t l = 0; l <= nl; ++l) cnt[l] = 0;
        for (int64_t i = 0; i < S; ++i) cnt[L[i] + 1]++;
        for (int32_t l = 0; l < nl; ++l) cnt[l + 1] += cnt[l];
        for (int32_t l = 0; l <= nl; ++l) level_ptr[w + l] = cnt[l];
        for (int64_t i = 0; i < S; ++i) level_rows[s * S + cnt[L[i]]++] = (int32_t)i;
        w += nl + 1;
    }
    free(cnt);
    return w;
}

/* ------------------------------------------------------------------ */
/* Section 4.3, Algorithm 5 (block form): ILU0 in IKJ order.           */
/* In place on the values of a matrix whose pattern has every diagonal */
/* block: afterwards the strictly lower blocks hold L (unit block      */
/* diagonal implied) and the diagonal and upper blocks hold U.         */
/* For each row I, for each J < I in row I (ascending):                */
/*   L_IJ = U_IJ * U_JJ^{-1};                                          */
/*   U_IK -= L_IJ * U_JK for every K > J present in both rows I and J. */
/* (The listing's inner loop also visits K = J, which only cancels U's */
/* copy of the lower entry; here that slot stores L_IJ instead.)       */
/* ------------------------------------------------------------------ */
static int64_t find_col(const int32_t *ptr, const int32_t *col, int64_t row, int32_t c) {
    for (int64_t j = ptr[row]; j < ptr[row + 1]; ++j)
        if (col[j] == c) return j;
    return -1;
}

int o_bilu0(int64_t n, int bs, const int32_t *ptr, const int32_t *col, double *val,
            int64_t *bad_row) {
    int bb = bs * bs;
    double inv[9], Lij[9], tmp[9];
    for (int64_t I = 0; I < n; ++I) {
        if (find_col(ptr, col, I, (int32_t)I) < 0) { if (bad_row) *bad_row = I; return O_EZEROPIVOT; }
    }
    for (int64_t I = 0; I < n; ++I) {
        for (int64_t pj = ptr[I]; pj < ptr[I + 1]; ++pj) {
            int32_t J = col[pj];
            if (J >= I) continue;
            int64_t djj = find_col(ptr, col, J, J);
            if (o_block_inverse(bs, val + djj * bb, inv) != O_OK) {
                if (bad_row) *bad_row = J;
                return O_EZEROPIVOT;
            }
            blk_mul(bs, val + pj * bb, inv, Lij);
            memcpy(val + pj * bb, Lij, sizeof(double) * bb);
            for (int64_t pk = ptr[I]; pk < ptr[I + 1]; ++pk) {
                int32_t K = col[pk];
                if (K <= J) continue;
                int64_t pjk = find_col(ptr, col, J, K);
                if (pjk < 0) continue;
                blk_mul(bs, Lij, val + pjk * bb, tmp);
                for (int e = 0; e < bb; ++e) val[pk * bb + e] -= tmp[e];
            }
        }
    }
    /* the last pivots are never inverted above: check every diagonal block */
    for (int64_t I = 0; I < n; ++I) {
        if (o_block_inverse(bs, val + find_col(ptr, col, I, (int32_t)I) * bb, inv) != O_OK) {
            if (bad_row) *bad_row = I;
            return O_EZEROPIVOT;
        }
    }
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Section 4.3, ILDU0 post-pass: inv_D_I = U_II^{-1}, and the strictly */
/* upper blocks are scaled from the left, Uhat_IK = inv_D_I U_IK, so   */
/* U = D Uhat with unit block diagonal.  In place: the diagonal slot   */
/* receives inv_D_I.                                                   */
/* ------------------------------------------------------------------ */
int o_ildu0(int64_t n, int bs, const int32_t *ptr, const int32_t *col, double *val,
            int64_t *bad_row) {
    int bb = bs * bs;
    double inv[9], tmp[9];
    for (int64_t I = 0; I < n; ++I) {
        int64_t d = find_col(ptr, col, I, (int32_t)I);
        if (d < 0 || o_block_inverse(bs, val + d * bb, inv) != O_OK) {
            if (bad_row) *bad_row = I;
            return O_EZEROPIVOT;
        }
        memcpy(val + d * bb, inv, sizeof(double) * bb);
        for (int64_t pk = ptr[I]; pk < ptr[I + 1]; ++pk) {
            if (col[pk] <= I) continue;
            blk_mul(bs, inv, val + pk * bb, tmp);
            memcpy(val + pk * bb, tmp, sizeof(double) * bb);
        }
    }
    return O_OK;
}

/* ------------------------------------------------------------------ */
/* Section 4.2.2 (Algorithm 7) and 4.4: apply M^{-1} = (L D Uhat)^{-1} */
/* f holds L (strictly lower), inv_D (diagonal) and Uhat (strictly     */
/* upper) in one pattern.  Forward y_I = r_I - sum_{J<I} L_IJ y_J (I   */
/* ascending), scale w_I = inv_D_I y_I, backward z_I = w_I -           */
/* sum_{K>I} Uhat_IK z_K (I descending).  Rows sum in ascending        */
/* column order.  r and z may not alias.                               */
/* ------------------------------------------------------------------ */
void o_apply(int64_t n, int bs, const int32_t *ptr, const int32_t *col, const double *f,
             const double *r, double *z) {
    int bb = bs * bs;
    double *y = (double *)malloc(sizeof(double) * (size_t)(n * bs));
    for (int64_t I = 0; I < n; ++I) {
        for (int c = 0; c < bs; ++c) y[I * bs + c] = r[I * bs + c];
        for (int64_t p = ptr[I]; p < ptr[I + 1]; ++p)
            if (col[p] < I) blk_matvec_sub(bs, f + p * bb, y + (int64_t)col[p] * bs, y + I * bs);
    }
    for (int64_t I = 0; I < n; ++I) {
        int64_t d = find_col(ptr, col, I, (int32_t)I);
        blk_matvec(bs, f + d * bb, y + I * bs, z + I * bs);
    }
    for (int64_t I = n - 1; I >= 0; --I) {
        for (int64_t p = ptr[I]; p < ptr[I + 1]; ++p)
            if (col[p] > I) blk_matvec_sub(bs, f + p * bb, z + (int64_t)col[p] * bs, z + I * bs);
    }
    free(y);
}

/* ILU0 form of the same apply (Algorithm 7 with the division inside the
 * row): f holds L and U (not the ILDU0 form); backward step
 * z_I = U_II^{-1} (y_I - sum_{K>I} U_IK z_K).  Used to pin the ILDU0 pass. */
int o_apply_ilu0(int64_t n, int bs, const int32_t *ptr, const int32_t *col, const double *f,
                 const double *r, double *z) {
    int bb = bs * bs;
    double inv[9], t[3];
    double *y = (double *)malloc(sizeof(double) * (size_t)(n * bs));
    for (int64_t I = 0; I < n; ++I) {
        for (int c = 0; c < bs; ++c) y[I * bs + c] = r[I * bs + c];
        for (int64_t p = ptr[I]; p < ptr[I + 1]; ++p)
            if (col[p] < I) blk_matvec_sub(bs, f + p * bb, y + (int64_t)col[p] * bs, y + I * bs);
    }
    for (int64_t I = n - 1; I >= 0; --I) {
        for (int c = 0; c < bs; ++c) t[c] = y[I * bs + c];
        int64_t d = -1;
        for (int64_t p = ptr[I]; p < ptr[I + 1]; ++p) {
            if (col[p] > I) blk_matvec_sub(bs, f + p * bb, z + (int64_t)col[p] * bs, t);
            if (col[p] == I) d = p;
        }
        if (d < 0 || o_block_inverse(bs, f + d * bb, inv) != O_OK) { free(y); return O_EZEROPIVOT; }
        blk_matvec(bs, inv, t, z + I * bs);
    }
    free(y);
    return O_OK;
}

/* Adjoint apply z = M^{-T} r, with M^{-T} = L^{-T} inv_D^T Uhat^{-T}:
 * solve Uhat^T a = r (unit lower: a_I = r_I - sum_{K<I} Uhat_KI^T a_K,
 * I ascending), then w = inv_D^T a, then solve L^T z = w (unit upper:
 * z_I = w_I - sum_{J>I} L_JI^T z_J, I descending).  The stored rows are
 * read column-wise: once a_K (resp. z_J) is final it is pushed into the
 * rows it couples. */
void o_apply_transpose(int64_t n, int bs, const int32_t *ptr, const int32_t *col,
                       const double *f, const double *r, double *z) {
    int bb = bs * bs;
    double *a = (double *)malloc(sizeof(double) * (size_t)(n * bs));
    memcpy(a, r, sizeof(double) * (size_t)(n * bs));
    /* Uhat^T a = r: a_I is final once every row K < I has pushed its
     * contribution; push a_K into the rows I > K that Uhat_KI couples. */
    for (int64_t K = 0; K < n; ++K) {
        for (int64_t p = ptr[K]; p < ptr[K + 1]; ++p) {
            int32_t I = col[p];
            if (I <= K) continue;
            for (int c = 0; c < bs; ++c) {
                double s = 0.0;
                for (int d = 0; d < bs; ++d) s += f[p * bb + d * bs + c] * a[K * bs + d];
                a[(int64_t)I * bs + c] -= s;
            }
        }
    }
    for (int64_t I = 0; I < n; ++I) {
        int64_t d = find_col(ptr, col, I, (int32_t)I);
        for (int c = 0; c < bs; ++c) {
            double s = 0.0;
            for (int e = 0; e < bs; ++e) s += f[d * bb + e * bs + c] * a[I * bs + e];
            z[I * bs + c] = s;
        }
    }
    /* L^T z = w: backward, push z_J into rows I < J coupled by L_JI */
    for (int64_t J = n - 1; J >= 0; --J) {
        for (int64_t p = ptr[J]; p < ptr[J + 1]; ++p) {
            int32_t I = col[p];
            if (I >= J) continue;
            for (int c = 0; c < bs; ++c) {
                double s = 0.0;
                for (int d = 0; d < bs; ++d) s += f[p * bb + d * bs + c] * z[J * bs + d];
                z[(int64_t)I * bs + c] -= s;
            }
        }
    }
    free(a);
}

/* ------------------------------------------------------------------ */
/* BSR sparse matrix-vector product y = A x                            */
/* ------------------------------------------------------------------ */
void o_spmv(int64_t n, int bs, const int32_t *ptr, const int32_t *col, const double *val,
            const double *x, double *y) {
    int bb = bs * bs;
    for (int64_t I = 0; I < n; ++I) {
        for (int c = 0; c < bs; ++c) y[I * bs + c] = 0.0;
        for (int64_t p = ptr[I]; p < ptr[I + 1]; ++p)
            for (int c = 0; c < bs; ++c) {
                double s = 0.0;
                for (int d = 0; d < bs; ++d) s += val[p * bb + c * bs + d] * x[(int64_t)col[p] * bs + d];
                y[I * bs + c] += s;
            }
    }
}

static double dot(int64_t m, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* Section 2, Algorithm 1 with K1 = I and K2 = M (right               */
/* preconditioning), relative stop ||r|| <= rtol ||b||, x0 given.      */
/* Because x = K2^{-1} y and K2^{-1} is linear, x is advanced by       */
/* alpha*M^{-1}p + omega*M^{-1}s with the same preconditioned vectors  */
/* that enter A; an exit after the half step (||s|| small) is added.   */
/* history (may be NULL) receives ||r_j||/||b|| after each iteration   */
/* (maxit+1 entries, entry 0 = initial).                               */
/* iters counts loop trips started.                                    */
/* ------------------------------------------------------------------ */
int o_bicgstab(int64_t n, int bs, const int32_t *aptr, const int32_t *acol, const double *aval,
               const int32_t *fptr, const int32_t *fcol, const double *fval,
               const double *b, double *x, double rtol, int32_t maxit,
               int32_t *iters, double *relres, double *history) {
    int64_t m = n * bs;
    size_t sz = sizeof(double) * (size_t)m;
    double *r = malloc(sz), *r0 = malloc(sz), *p = malloc(sz), *ph = malloc(sz), *v = malloc(sz);
    double *s = malloc(sz), *sh = malloc(sz), *t = malloc(sz);
    int status = O_ENOCONV;
    double bnorm = sqrt(dot(m, b, b));
    if (bnorm == 0.0) bnorm = 1.0;
    o_spmv(n, bs, aptr, acol, aval, x, t);
    for (int64_t i = 0; i < m; ++i) { r[i] = b[i] - t[i]; r0[i] = r[i]; p[i] = r[i]; }
    double rho = dot(m, r0, r);
    double res = sqrt(dot(m, r, r)) / bnorm;
    if (history) history[0] = res;
    int32_t it = 0;
    if (res <= rtol) { status = O_OK; goto done; }
    for (it = 1; it <= maxit; ++it) {
        o_apply(n, bs, fptr, fcol, fval, p, ph);
        o_spmv(n, bs, aptr, acol, aval, ph, v);
        double r0v = dot(m, r0, v);
        if (r0v == 0.0 || !isfinite(r0v) || rho == 0.0) { status = O_EBREAKDOWN; break; }
        double alpha = rho / r0v;
        for (int64_t i = 0; i < m; ++i) s[i] = r[i] - alpha * v[i];
        double snorm = sqrt(dot(m, s, s)) / bnorm;
        if (snorm <= rtol) {
            for (int64_t i = 0; i < m; ++i) x[i] += alpha * ph[i];
            res = snorm;
            if (history) history[it] = res;
            status = O_OK;
            break;
        }
        o_apply(n, bs, fptr, fcol, fval, s, sh);
        o_spmv(n, bs, aptr, acol, aval, sh, t);
        double ts = dot(m, t, s), tt = dot(m, t, t);
        if (tt == 0.0 || !isfinite(tt)) { status = O_EBREAKDOWN; break; }
        double omega = ts / tt;
        for (int64_t i = 0; i < m; ++i) {
            x[i] += alpha * ph[i] + omega * sh[i];
            r[i] = s[i] - omega * t[i];
        }
        res = sqrt(dot(m, r, r)) / bnorm;
        if (history) history[it] = res;
        if (!isfinite(res)) { status = O_EBREAKDOWN; break; }
        if (res <= rtol) { status = O_OK; break; }
        if (omega == 0.0) { status = O_EBREAKDOWN; break; }
        double rho_new = dot(m, r0, r);
        double beta = (rho_new / rho) * (alpha / omega);
        rho = rho_new;
        for (int64_t i = 0; i < m; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    }
    if (it > maxit) it = maxit;
done:
    *iters = it;
    *relres = res;
    free(r); free(r0); free(p); free(ph); free(v); free(s); free(sh); free(t);
    return status;
}

/* ================================================================== */
/* Learned interface correction (an addition to the paper's method;   */
/* the paper has no learned component).                               */
/*                                                                    */
/* Faces are the directed cut pairs (I, J): the blocks A_IJ of the     */
/* full reordered matrix whose row and column lie in different         */
/* subdomains, i.e. exactly the blocks the drop of Section 3.2         */
/* removes, listed in CSR order.  Each face gets a 3x3 coefficient     */
/* C_f from a small MLP, and the preconditioner becomes                */
/* z = M_DD^{-1} (r + C r) with (C r)_I = sum_{f=(I,J)} C_f r_J: still */
/* a fixed linear operator once C is set.                              */
/* ================================================================== */

#define LIC_IN 27
#define LIC_H 64
#define LIC_OUT 9
/* parameter layout: W1[64][27] b1[64] W2[64][64] b2[64] W3[9][64] b3[9] */
#define LIC_W1 0
#define LIC_B1 (LIC_W1 + LIC_H * LIC_IN)
#define LIC_W2 (LIC_B1 + LIC_H)
#define LIC_B2 (LIC_W2 + LIC_H * LIC_H)
#define LIC_W3 (LIC_B2 + LIC_H)
#define LIC_B3 (LIC_W3 + LIC_OUT * LIC_H)
#define LIC_NPARAM (LIC_B3 + LIC_OUT)

int64_t o_lic_nparam(void) { return LIC_NPARAM; }

/* Cut faces in CSR order of the full reordered matrix.  With fI == NULL it
 * only counts.  fq[f] is the block's position in (ptr, col, val). */
int64_t o_cut_faces(int64_t n, int64_t S, const int32_t *ptr, const int32_t *col,
                    int32_t *fI, int32_t *fJ, int32_t *fq) {
    int64_t m = 0;
    for (int64_t I = 0; I < n; ++I)
        for (int64_t q = ptr[I]; q < ptr[I + 1]; ++q)
            if (col[q] / S != I / S) {
                if (fI) { fI[m] = (int32_t)I; fJ[m] = col[q]; fq[m] = (int32_t)q; }
                ++m;
            }
    return m;
}

/* Features x_f = [A_II, A_IJ, A_JJ] / sigma_f (three 3x3 blocks, row-major),
 * sigma_f = sqrt(|tr A_II| |tr A_JJ|) / 3. */
void o_lic_features(int64_t nf, const int32_t *ptr, const int32_t *col, const double *val,
                    const int32_t *fI, const int32_t *fJ, const int32_t *fq, double *X) {
    for (int64_t f = 0; f < nf; ++f) {
        int64_t dI = find_col(ptr, col, fI[f], fI[f]);
        int64_t dJ = find_col(ptr, col, fJ[f], fJ[f]);
        const double *Aii = val + dI * 9, *Aij = val + (int64_t)fq[f] * 9, *Ajj = val + dJ * 9;
        double ti = Aii[0] + Aii[4] + Aii[8], tj = Ajj[0] + Ajj[4] + Ajj[8];
        double sigma = sqrt(fabs(ti) * fabs(tj)) / 3.0;
        double *x = X + f * LIC_IN;
        for (int e = 0; e < 9; ++e) {
            x[e] = Aii[e] / sigma;
            x[9 + e] = Aij[e] / sigma;
            x[18 + e] = Ajj[e] / sigma;
        }
    }
}

/* h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), out = W3 h2 + b3 (per face). */
void o_mlp_forward(int64_t nf, const double *P, const double *X, double *H1, double *H2, double *OUT) {
    for (int64_t f = 0; f < nf; ++f) {
        const double *x = X + f * LIC_IN;
        double *h1 = H1 + f * LIC_H, *h2 = H2 + f * LIC_H, *o = OUT + f * LIC_OUT;
        for (int i = 0; i < LIC_H; ++i) {
            double s = P[LIC_B1 + i];
            for (int k = 0; k < LIC_IN; ++k) s += P[LIC_W1 + i * LIC_IN + k] * x[k];
            h1[i] = s > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < LIC_H; ++i) {
            double s = P[LIC_B2 + i];
            for (int k = 0; k < LIC_H; ++k) s += P[LIC_W2 + i * LIC_H + k] * h1[k];
            h2[i] = s > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < LIC_OUT; ++i) {
            double s = P[LIC_B3 + i];
            for (int k = 0; k < LIC_H; ++k) s += P[LIC_W3 + i * LIC_H + k] * h2[k];
            o[i] = s;
        }
    }
}

/* Backpropagation of dOUT (per face) through the MLP, summed over faces
 * into dP (which the caller zeroes).  ReLU'(0) is taken as 0. */
void o_mlp_backward(int64_t nf, const double *P, const double *X, const double *H1, const double *H2,
                    const double *dOUT, double *dP) {
    double g2[LIC_H], g1[LIC_H];
    for (int64_t f = 0; f < nf; ++f) {
        const double *x = X + f * LIC_IN, *h1 = H1 + f * LIC_H, *h2 = H2 + f * LIC_H;
        const double *d = dOUT + f * LIC_OUT;
        for (int i = 0; i < LIC_OUT; ++i) {
            dP[LIC_B3 + i] += d[i];
            for (int k = 0; k < LIC_H; ++k) dP[LIC_W3 + i * LIC_H + k] += d[i] * h2[k];
        }
        for (int k = 0; k < LIC_H; ++k) {
            double s = 0.0;
            for (int i = 0; i < LIC_OUT; ++i) s += P[LIC_W3 + i * LIC_H + k] * d[i];
            g2[k] = h2[k] > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < LIC_H; ++i) {
            dP[LIC_B2 + i] += g2[i];
            for (int k = 0; k < LIC_H; ++k) dP[LIC_W2 + i * LIC_H + k] += g2[i] * h1[k];
        }
        for (int k = 0; k < LIC_H; ++k) {
            double s = 0.0;
            for (int i = 0; i < LIC_H; ++i) s += P[LIC_W2 + i * LIC_H + k] * g2[i];
            g1[k] = h1[k] > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < LIC_H; ++i) {
            dP[LIC_B1 + i] += g1[i];
            for (int k = 0; k < LIC_IN; ++k) dP[LIC_W1 + i * LIC_IN + k] += g1[i] * x[k];
        }
    }
}

/* r~ = r + C r:  r~_I = r_I + sum over faces f = (I, J) of C_f r_J
 * (faces visited in their CSR order). */
void o_lic_correct(int64_t n, int64_t nf, const int32_t *fI, const int32_t *fJ, const double *C,
                   const double *r, double *rt) {
    memcpy(rt, r, sizeof(double) * (size_t)(n * 3));
    for (int64_t f = 0; f < nf; ++f)
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int b = 0; b < 3; ++b) s += C[f * 9 + a * 3 + b] * r[(int64_t)fJ[f] * 3 + b];
            rt[(int64_t)fI[f] * 3 + a] += s;
        }
}

/* dC_f = sum over probes q of a_q[I] r_q[J]^T, with A and R holding nq
 * vectors of length 3n each (probe-major). */
void o_lic_dC(int64_t n, int64_t nf, const int32_t *fI, const int32_t *fJ, int nq, const double *A,
              const double *R, double *dC) {
    for (int64_t f = 0; f < nf; ++f)
        for (int e = 0; e < 9; ++e) dC[f * 9 + e] = 0.0;
    for (int q = 0; q < nq; ++q)
        for (int64_t f = 0; f < nf; ++f)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    dC[f * 9 + a * 3 + b] += A[(int64_t)q * 3 * n + (int64_t)fI[f] * 3 + a] *
                                             R[(int64_t)q * 3 * n + (int64_t)fJ[f] * 3 + b];
}

/* One Adam step (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void o_adam(int64_t np, double *P, const double *G, double *M, double *V, int t, double lr, double b1,
            double b2, double eps) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int64_t i = 0; i < np; ++i) {
        M[i] = b1 * M[i] + (1.0 - b1) * G[i];
        V[i] = b2 * V[i] + (1.0 - b2) * G[i] * G[i];
        P[i] -= lr * (M[i] / c1) / (sqrt(V[i] / c2) + eps);
    }
}
