// Setup kernels: partition labels and permutation (Section 3, Algorithm 2),
// block reorder (Section 3.1, Algorithm 3), inter-subdomain drop (Section
// 3.2), per-subdomain level sets (Section 4.2.1), block ILU0 + ILDU0
// (Section 4.3, Algorithm 5) and the packing of the factors into the
// streaming layout of the apply.
#include <algorithm>

#include "internal.h"

namespace ddilu {

// ------------------------------------------------------------------ scan
constexpr int kScanT = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanT * kScanItems;

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

// Block-wide exclusive scan; sh must hold 65 ints; every thread must call.
__device__ int block_excl_scan(int v, int *sh, int *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    int s = 0, si = 0;
    if (w == 0) {
        s = lane < nw ? sh[lane] : 0;
        si = wave_incl_scan(s);
    }
    __syncthreads();
    if (w == 0) {
        if (lane < nw) sh[lane] = si - s;
        if (lane == 63) sh[64] = si;
    }
    __syncthreads();
    *total = sh[64];
    int res = inc - v + sh[w];
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(kScanT) void k_scan_tiles(const int32_t *in, int64_t n, int32_t *sums) {
    __shared__ int sh[65];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (t0 + k < n) v += in[t0 + k];
    int tot;
    block_excl_scan(v, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanT) void k_scan_sums(int32_t *sums, int64_t m) {
    __shared__ int sh[65];
    int carry = 0;
    for (int64_t base = 0; base < m; base += kScanT) {
        int64_t i = base + threadIdx.x;
        int v = i < m ? sums[i] : 0;
        int tot;
        int ex = block_excl_scan(v, sh, &tot);
        if (i < m) sums[i] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) sums[m] = carry;
}

__global__ __launch_bounds__(kScanT) void k_scan_apply(const int32_t *in, int64_t n, const int32_t *sums,
                                                       int64_t m, int32_t *out) {
    __shared__ int sh[65];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int vals[kScanItems];
    int v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = (t0 + k < n) ? in[t0 + k] : 0;
        v += vals[k];
    }
    int tot;
    int ex = block_excl_scan(v, sh, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (t0 + k < n) out[t0 + k] = ex;
        ex += vals[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[m];
}

hipError_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t st) {
    int64_t m = (n + kScanTile - 1) / kScanTile;
    if (m == 0) {
        return hipMemsetAsync(out, 0, sizeof(int32_t), st);
    }
    k_scan_tiles<<<(unsigned)m, kScanT, 0, st>>>(in, n, tmp);
    k_scan_sums<<<1, kScanT, 0, st>>>(tmp, m);
    k_scan_apply<<<(unsigned)m, kScanT, 0, st>>>(in, n, tmp, m, out);
    return hipGetLastError();
}

// ------------------------------------------------------------- partition
// Algorithm 2 label, and the renumbering of Section 3.1: rows grouped by
// label, stable in the old index.  Inside a box the stable order is the
// local lexicographic order, so the new index has the closed form
// part*S + li + sx*(lj + sy*lk).
__global__ void k_partition(int nx, int ny, int nz, int sx, int sy, int sz, int32_t *part_id,
                            int32_t *old2new, int32_t *new2old) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int i = (int)(g % nx), j = (int)((g / nx) % ny), k = (int)(g / ((int64_t)nx * ny));
    const int bx = nx / sx, by = ny / sy;
    const int p = i / sx + bx * (j / sy + by * (k / sz));
    const int64_t S = (int64_t)sx * sy * sz;
    const int64_t loc = (i % sx) + (int64_t)sx * ((j % sy) + (int64_t)sy * (k % sz));
    const int64_t nw = p * S + loc;
    part_id[g] = p;
    old2new[g] = (int32_t)nw;
    new2old[nw] = (int32_t)g;
}

hipError_t launch_partition(dd_ctx *h, hipStream_t st) {
    const int T = 256;
    k_partition<<<(unsigned)((h->n + T - 1) / T), T, 0, st>>>(h->nx, h->ny, h->nz, h->sx, h->sy, h->sz,
                                                           h->part_id, h->old2new, h->new2old);
    return hipGetLastError();
}

// --------------------------------------------------------------- reorder
__global__ void k_row_len(int64_t n, const int32_t *ptr, const int32_t *new2old, int32_t *len,
                          int32_t *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = new2old[i];
    const int32_t l = ptr[o + 1] - ptr[o];
    len[i] = l;
    if (l < 0 || l > kMaxRowBlocks) atomicMax(&status[0], 1);
}

// One thread per new row: map columns old->new and sort the row's
// (column, source block) pairs by column (insertion sort in place).
__global__ void k_reorder_rows(int64_t n, const int32_t *ptr, const int32_t *col, const int32_t *new2old,
                               const int32_t *old2new, const int32_t *aptr, int32_t *acol,
                               int32_t *src) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = new2old[i];
    const int32_t b0 = ptr[o], len = ptr[o + 1] - b0;
    const int32_t d0 = aptr[i];
    for (int k = 0; k < len; ++k) {
        int32_t c = old2new[col[b0 + k]];
        int32_t s = b0 + k;
        int m = k - 1;
        while (m >= 0 && acol[d0 + m] > c) {
            acol[d0 + m + 1] = acol[d0 + m];
            src[d0 + m + 1] = src[d0 + m];
            --m;
        }
        acol[d0 + m + 1] = c;
        src[d0 + m + 1] = s;
    }
}

__global__ void k_gather_blocks(int64_t nelem, int bb, const int32_t *src, const double *val, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nelem) return;
    const int64_t q = e / bb;
    const int c = (int)(e - q * bb);
    out[e] = val[(int64_t)src[q] * bb + c];
}

// Input check before any kernel indexes through the caller's pattern: every
// row has 0..kMaxRowBlocks blocks inside [0, nnzb) (status[0] |= 1), every
// column is a block row (status[0] |= 2).
__global__ void k_check_rows(int64_t n, int64_t nnzb, const int32_t *ptr, const int32_t *col, int32_t *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b0 = ptr[i], b1 = ptr[i + 1];
    if (b0 < 0 || b1 < b0 || b1 - b0 > kMaxRowBlocks || b1 > nnzb) {
        atomicOr(&status[0], 1);
        return;
    }
    for (int32_t q = b0; q < b1; ++q) {
        const int32_t c = col[q];
        if (c < 0 || c >= n) {
            atomicOr(&status[0], 2);
            return;
        }
    }
}

hipError_t launch_check_rows(int64_t n, int64_t nnzb, const int32_t *ptr, const int32_t *col, int32_t *status,
                             hipStream_t st) {
    const int T = 256;
    k_check_rows<<<(unsigned)((n + T - 1) / T), T, 0, st>>>(n, nnzb, ptr, col, status);
    return hipGetLastError();
}

hipError_t launch_row_len(dd_ctx *h, const int32_t *ptr, int32_t *len, hipStream_t st) {
    const int T = 256;
    k_row_len<<<(unsigned)((h->n + T - 1) / T), T, 0, st>>>(h->n, ptr, h->new2old, len, h->status);
    return hipGetLastError();
}

hipError_t launch_reorder_fill(dd_ctx *h, const int32_t *ptr, const int32_t *col, const double *val,
                               int32_t *src, hipStream_t st) {
    const int T = 256;
    k_reorder_rows<<<(unsigned)((h->n + T - 1) / T), T, 0, st>>>(h->n, ptr, col, h->new2old, h->old2new,
                                                              h->aptr, h->acol, src);
    const int bb = h->bs * h->bs;
    const int64_t ne = h->nnzb * bb;
    k_gather_blocks<<<(unsigned)((ne + T - 1) / T), T, 0, st>>>(ne, bb, src, val, h->aval);
    return hipGetLastError();
}

// ------------------------------------------------------------------ drop
// Columns of a reordered row are sorted and a subdomain is the contiguous
// range [s*S, (s+1)*S), so the kept blocks of a row are one contiguous run.
__global__ void k_drop_count(int64_t n, int S, const int32_t *aptr, const int32_t *acol, int32_t *tbeg,
                             int32_t *tlen, int32_t *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t lo = (i / S) * (int64_t)S, hi = lo + S;
    int32_t b = aptr[i], e = aptr[i + 1];
    while (b < e && acol[b] < lo) ++b;
    int32_t f = b;
    bool diag = false;
    while (f < e && acol[f] < hi) {
        diag |= (acol[f] == i);
        ++f;
    }
    tbeg[i] = b;
    tlen[i] = f - b;
    if (!diag) atomicMin(&status[1], (int32_t)i);  // structurally missing pivot
}

__global__ void k_drop_rows(int64_t n, const int32_t *tbeg, const int32_t *tptr, const int32_t *acol,
                            int32_t *tcol, int32_t *tsrc, int32_t *tdiag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = tbeg[i], d0 = tptr[i], len = tptr[i + 1] - d0;
    for (int k = 0; k < len; ++k) {
        const int32_t c = acol[b + k];
        tcol[d0 + k] = c;
        tsrc[d0 + k] = b + k;
        if (c == i) tdiag[i] = d0 + k;
    }
}

hipError_t launch_drop_count(dd_ctx *h, int32_t *tbeg, int32_t *tlen, hipStream_t st) {
    const int T = 256;
    k_drop_count<<<(unsigned)((h->n + T - 1) / T), T, 0, st>>>(h->n, h->S, h->aptr, h->acol, tbeg, tlen,
                                                            h->status);
    return hipGetLastError();
}

hipError_t launch_gather_blocks(int64_t nblk, int bb, const int32_t *src, const double *val, double *out,
                                hipStream_t st) {
    const int T = 256;
    const int64_t ne = nblk * bb;
    if (ne > 0) k_gather_blocks<<<(unsigned)((ne + T - 1) / T), T, 0, st>>>(ne, bb, src, val, out);
    return hipGetLastError();
}

hipError_t launch_drop_rows(dd_ctx *h, const int32_t *tbeg, int32_t *tsrc, hipStream_t st) {
    const int T = 256;
    k_drop_rows<<<(unsigned)((h->n + T - 1) / T), T, 0, st>>>(h->n, tbeg, h->tptr, h->acol, h->tcol, tsrc,
                                                           h->tdiag);
    const int bb = h->bs * h->bs;
    const int64_t ne = h->nnzt * bb;
    k_gather_blocks<<<(unsigned)((ne + T - 1) / T), T, 0, st>>>(ne, bb, tsrc, h->aval, h->lu);
    return hipGetLastError();
}

// ---------------------------------------------------------------- levels
// Section 4.2.1 (Algorithm 6 semantics): inside one subdomain (one
// workgroup), rows without a dependency get level 0; then, round after
// round, every row whose dependencies all have a level is promoted to
// (round + 1).  A row is promoted in the first round after its last
// dependency got its level, so its level is 1 + the largest level among its
// dependencies: the longest dependency path.  which = 0: dependencies are
// the columns J < I of row I (lower factor); which = 1: columns K > I
// (upper factor).
constexpr int32_t kUnassigned = 0x7fffffff;

__global__ __launch_bounds__(256) void k_levels(int S, int which, const int32_t *tptr, const int32_t *tcol,
                                                int32_t *lev_out, int32_t *nlev_out) {
    extern __shared__ int32_t sm_lev[];
    int32_t *lev = sm_lev;
    uint8_t *mark = reinterpret_cast<uint8_t *>(sm_lev + S);
    __shared__ int added;
    const int64_t base = (int64_t)blockIdx.x * S;
    for (int i = threadIdx.x; i < S; i += blockDim.x) {
        const int64_t gi = base + i;
        bool dep = false;
        for (int32_t q = tptr[gi]; q < tptr[gi + 1]; ++q) {
            const int32_t c = tcol[q];
            if (which == 0 ? (c < gi) : (c > gi)) {
                dep = true;
                break;
            }
        }
        lev[i] = dep ? kUnassigned : 0;
        mark[i] = 0;
    }
    __syncthreads();
    int level = 0;
    while (true) {
        if (threadIdx.x == 0) added = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < S; i += blockDim.x) {
            if (lev[i] != kUnassigned) continue;
            const int64_t gi = base + i;
            bool ok = true;
            for (int32_t q = tptr[gi]; q < tptr[gi + 1]; ++q) {
                const int32_t c = tcol[q];
                if ((which == 0 ? (c < gi) : (c > gi)) && lev[c - base] == kUnassigned) {
                    ok = false;
                    break;
                }
            }
            if (ok) {
                mark[i] = 1;
                added = 1;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < S; i += blockDim.x)
            if (mark[i]) {
                lev[i] = level + 1;
                mark[i] = 0;
            }
        __syncthreads();
        const int a = added;
        __syncthreads();
        if (!a) break;
        ++level;
    }
    for (int i = threadIdx.x; i < S; i += blockDim.x) lev_out[base + i] = lev[i];
    if (threadIdx.x == 0) nlev_out[blockIdx.x] = level + 1;
}

__global__ void k_plus_one(int64_t m, const int32_t *in, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = in[i] + 1;
}

// Explicit DAG (Section 4.2.2): per subdomain, level offsets and the rows
// of each level in ascending local order (a stable counting sort by level,
// done serially by one thread so the order is evident).
__global__ void k_level_lists(int S, const int32_t *lev_g, const int32_t *nlev, const int32_t *off,
                              int32_t *lptr, int32_t *rows) {
    extern __shared__ int32_t sm_ll[];
    int32_t *cnt = sm_ll;                                       // nl + 1
    uint16_t *lv = reinterpret_cast<uint16_t *>(sm_ll + S + 1);  // S
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int nl = nlev[s];
    for (int i = threadIdx.x; i < S; i += blockDim.x) lv[i] = (uint16_t)lev_g[base + i];
    for (int l = threadIdx.x; l <= nl; l += blockDim.x) cnt[l] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < S; ++i) cnt[lv[i] + 1]++;
        for (int l = 0; l < nl; ++l) cnt[l + 1] += cnt[l];
        const int32_t o = off[s];
        for (int l = 0; l <= nl; ++l) lptr[o + l] = cnt[l];
        for (int i = 0; i < S; ++i) rows[base + cnt[lv[i]]++] = i;
    }
}

hipError_t launch_levels(dd_ctx *h, int which, hipStream_t st) {
    Levels &L = h->lev[which];
    const size_t lds = (size_t)h->S * 5;
    k_levels<<<h->nsub, 256, lds, st>>>(h->S, which, h->tptr, h->tcol, L.lev, L.nlev);
    return hipGetLastError();
}

hipError_t launch_plus_one(int64_t m, const int32_t *in, int32_t *out, hipStream_t st) {
    const int T = 256;
    k_plus_one<<<(unsigned)((m + T - 1) / T), T, 0, st>>>(m, in, out);
    return hipGetLastError();
}

hipError_t launch_level_lists(dd_ctx *h, int which, hipStream_t st) {
    Levels &L = h->lev[which];
    const size_t lds = (size_t)(h->S + 1) * 4 + (size_t)h->S * 2;
    k_level_lists<<<h->nsub, 64, lds, st>>>(h->S, L.lev, L.nlev, L.off, L.ptr, L.rows);
    return hipGetLastError();
}

// ------------------------------------------------------------ block math
template <int BS>
__device__ __forceinline__ void blk_mul(const double *A, const double *B, double *C) {
#pragma unroll
    for (int i = 0; i < BS; ++i)
#pragma unroll
        for (int j = 0; j < BS; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < BS; ++k) s += A[i * BS + k] * B[k * BS + j];
            C[i * BS + j] = s;
        }
}

template <int BS>
__device__ __forceinline__ double blk_norm1(const double *A) {
    double m = 0.0;
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < BS; ++i) s += fabs(A[i * BS + j]);
        m = fmax(m, s);
    }
    return m;
}

// Inverse by the adjugate; false when the determinant vanishes, a value is
// not finite, or the 1-norm condition number exceeds 1e14.
template <int BS>
__device__ bool blk_inverse(const double *a, double *inv) {
    if constexpr (BS == 1) {
        if (!(fabs(a[0]) > 0.0) || !isfinite(a[0])) return false;
        inv[0] = 1.0 / a[0];
        return true;
    } else {
        const double c00 = a[4] * a[8] - a[5] * a[7];
        const double c01 = a[5] * a[6] - a[3] * a[8];
        const double c02 = a[3] * a[7] - a[4] * a[6];
        const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
        if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
        const double id = 1.0 / det;
        inv[0] = c00 * id;
        inv[1] = (a[2] * a[7] - a[1] * a[8]) * id;
        inv[2] = (a[1] * a[5] - a[2] * a[4]) * id;
        inv[3] = c01 * id;
        inv[4] = (a[0] * a[8] - a[2] * a[6]) * id;
        inv[5] = (a[2] * a[3] - a[0] * a[5]) * id;
        inv[6] = c02 * id;
        inv[7] = (a[1] * a[6] - a[0] * a[7]) * id;
        inv[8] = (a[0] * a[4] - a[1] * a[3]) * id;
        const double cond = blk_norm1<3>(a) * blk_norm1<3>(inv);
        return cond <= 1e14;
    }
}

// ------------------------------------------------------------------ BILU0
// Section 4.3, Algorithm 5 in block form, IKJ order, one workgroup per
// subdomain.  Rows are processed level by level (L levels): all rows a row
// depends on sit in earlier levels, so rows of one level run in parallel
// and each row performs exactly the sequential IKJ updates:
//   for each J < I in row I (ascending): L_IJ = U_IJ inv(U_JJ);
//     U_IK -= L_IJ U_JK for each K > J in row I that row J also holds.
// When a row is done its pivot inverse inv(U_II) is stored (it is the
// ILDU0 inv_D, and what later rows need).
template <int BS>
__global__ __launch_bounds__(256) void k_bilu0(int S, const int32_t *tptr, const int32_t *tcol,
                                               const int32_t *tdiag, double *lu, double *invd,
                                               const int32_t *nlev, const int32_t *off, const int32_t *lptr,
                                               const int32_t *rows, int32_t *status) {
    constexpr int BB = BS * BS;
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int nl = nlev[s];
    const int32_t o = off[s];
    for (int l = 0; l < nl; ++l) {
        const int32_t p0 = lptr[o + l], p1 = lptr[o + l + 1];
        for (int32_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
            const int64_t gi = base + rows[base + p];
            const int32_t tb = tptr[gi], te = tptr[gi + 1];
            for (int32_t pj = tb; pj < te; ++pj) {
                const int32_t J = tcol[pj];
                if (J >= gi) break;
                double Lij[BB];
                blk_mul<BS>(lu + (int64_t)pj * BB, invd + (int64_t)J * BB, Lij);
#pragma unroll
                for (int e = 0; e < BB; ++e) lu[(int64_t)pj * BB + e] = Lij[e];
                const int32_t jb = tptr[J], je = tptr[J + 1];
                int32_t q = jb;
                for (int32_t pk = pj + 1; pk < te; ++pk) {
                    const int32_t K = tcol[pk];
                    while (q < je && tcol[q] < K) ++q;
                    if (q < je && tcol[q] == K) {
                        double t[BB];
                        blk_mul<BS>(Lij, lu + (int64_t)q * BB, t);
#pragma unroll
                        for (int e = 0; e < BB; ++e) lu[(int64_t)pk * BB + e] -= t[e];
                    }
                }
            }
            double inv[BB];
            const double *piv = lu + (int64_t)tdiag[gi] * BB;
            if (!blk_inverse<BS>(piv, inv)) {
                atomicMin(&status[2], (int32_t)gi);
#pragma unroll
                for (int e = 0; e < BB; ++e) inv[e] = (e % (BS + 1) == 0) ? 1.0 : 0.0;
            }
#pragma unroll
            for (int e = 0; e < BB; ++e) invd[gi * BB + e] = inv[e];
        }
        __syncthreads();
    }
}

hipError_t launch_bilu0(dd_ctx *h, hipStream_t st) {
    const Levels &L = h->lev[0];
    if (h->bs == 3)
        k_bilu0<3><<<h->nsub, 256, 0, st>>>(h->S, h->tptr, h->tcol, h->tdiag, h->lu, h->invd, L.nlev, L.off,
                                            L.ptr, L.rows, h->status);
    else
        k_bilu0<1><<<h->nsub, 256, 0, st>>>(h->S, h->tptr, h->tcol, h->tdiag, h->lu, h->invd, L.nlev, L.off,
                                            L.ptr, L.rows, h->status);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pack
// Per position p of a sweep (subdomain s = p / S, row = rows[p]): the
// number of its factor blocks (lower: J < I; upper: K > I).
__global__ void k_pack_count(int64_t n, int S, int which, const int32_t *tptr, const int32_t *tcol,
                             const int32_t *rows, int32_t *cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t gi = (p / S) * (int64_t)S + rows[p];
    int c = 0;
    for (int32_t q = tptr[gi]; q < tptr[gi + 1]; ++q) c += which == 0 ? (tcol[q] < gi) : (tcol[q] > gi);
    cnt[p] = c;
}

// which 0: L blocks; 1: Uhat = inv_D U blocks and inv_D; 2: the U blocks as
// factored (no scaling; val only, same order as for 1).
template <int BS>
__global__ void k_pack_fill(int64_t n, int S, int which, const int32_t *tptr, const int32_t *tcol,
                            const double *lu, const double *invd, const int32_t *rows, const int32_t *bptr,
                            uint16_t *prow, uint16_t *bcol, double *val, double *dval) {
    constexpr int BB = BS * BS;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t base = (p / S) * (int64_t)S;
    const int64_t gi = base + rows[p];
    if (which != 2) prow[p] = (uint16_t)rows[p];
    int32_t b = bptr[p];
    const double *inv = invd + gi * BB;
    for (int32_t q = tptr[gi]; q < tptr[gi + 1]; ++q) {
        const int32_t c = tcol[q];
        if (which == 0 ? (c < gi) : (c > gi)) {
            if (which != 2) bcol[b] = (uint16_t)(c - base);
            if (which != 1) {
#pragma unroll
                for (int e = 0; e < BB; ++e) val[(int64_t)b * BB + e] = lu[(int64_t)q * BB + e];
            } else {
                double t[BB];
                blk_mul<BS>(inv, lu + (int64_t)q * BB, t);
#pragma unroll
                for (int e = 0; e < BB; ++e) val[(int64_t)b * BB + e] = t[e];
            }
            ++b;
        }
    }
    if (which == 1) {
#pragma unroll
        for (int e = 0; e < BB; ++e) dval[p * BB + e] = inv[e];
    }
}

hipError_t launch_pack_unscaled(dd_ctx *h, hipStream_t st) {
    const int T = 256;
    Sweep &w = h->sw[1];
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    if (h->bs == 3)
        k_pack_fill<3><<<g, T, 0, st>>>(h->n, h->S, 2, h->tptr, h->tcol, h->lu, h->invd, h->lev[1].rows, w.bptr,
                                        nullptr, nullptr, w.uraw, nullptr);
    else
        k_pack_fill<1><<<g, T, 0, st>>>(h->n, h->S, 2, h->tptr, h->tcol, h->lu, h->invd, h->lev[1].rows, w.bptr,
                                        nullptr, nullptr, w.uraw, nullptr);
    return hipGetLastError();
}

hipError_t launch_pack_count(dd_ctx *h, int which, int32_t *cnt, hipStream_t st) {
    const int T = 256;
    k_pack_count<<<(unsigned)((h->n + T - 1) / T), T, 0, st>>>(h->n, h->S, which, h->tptr, h->tcol,
                                                            h->lev[which].rows, cnt);
    return hipGetLastError();
}

hipError_t launch_pack_fill(dd_ctx *h, int which, hipStream_t st) {
    const int T = 256;
    Sweep &w = h->sw[which];
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    if (h->bs == 3)
        k_pack_fill<3><<<g, T, 0, st>>>(h->n, h->S, which, h->tptr, h->tcol, h->lu, h->invd, h->lev[which].rows,
                                        w.bptr, w.prow, w.bcol, w.val64, w.d64);
    else
        k_pack_fill<1><<<g, T, 0, st>>>(h->n, h->S, which, h->tptr, h->tcol, h->lu, h->invd, h->lev[which].rows,
                                        w.bptr, w.prow, w.bcol, w.val64, w.d64);
    return hipGetLastError();
}

// Slot layout of one sweep: position p owns MB block slots; its blocks fill
// the first nb slots in ascending column order, zero blocks the rest.  The
// position's 64-bit descriptor holds its local row in bits 0-15 and the
// local column of slot k in bits 16(k+1)..16(k+1)+15, 0xFFFF for an empty
// slot.
template <int BS>
__global__ void k_pack_slots(int64_t n, int S, int which, int MB, const int32_t *tptr, const int32_t *tcol,
                             const double *lu, const double *invd, const int32_t *rows, uint64_t *desc,
                             double *sval) {
    constexpr int BB = BS * BS;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t base = (p / S) * (int64_t)S;
    const int32_t lr = rows[p];
    const int64_t gi = base + lr;
    const double *inv = invd + gi * BB;
    // lane-contiguous runs: row i of every slot block, then (upper sweep)
    // row i of inv_D, NV values per row i, PS = BS * NV per position
    const int NV = (MB + which) * BS;
    double *o = sval + p * BS * NV;
    uint64_t dsc = (uint64_t)(uint16_t)lr;
    int k = 0;
    for (int32_t q = tptr[gi]; q < tptr[gi + 1] && k < MB; ++q) {
        const int32_t c = tcol[q];
        if (which == 0 ? (c < gi) : (c > gi)) {
            dsc |= (uint64_t)(uint16_t)(c - base) << (16 * (k + 1));
            double t[BB];
            if (which == 0) {
#pragma unroll
                for (int e = 0; e < BB; ++e) t[e] = lu[(int64_t)q * BB + e];
            } else {
                blk_mul<BS>(inv, lu + (int64_t)q * BB, t);
            }
#pragma unroll
            for (int i = 0; i < BS; ++i)
#pragma unroll
                for (int j = 0; j < BS; ++j) o[i * NV + k * BS + j] = t[i * BS + j];
            ++k;
        }
    }
    for (int e = k; e < 3; ++e) dsc |= (uint64_t)0xffffu << (16 * (e + 1));
    for (; k < MB; ++k)
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int j = 0; j < BS; ++j) o[i * NV + k * BS + j] = 0.0;
    if (which == 1)
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int j = 0; j < BS; ++j) o[i * NV + MB * BS + j] = inv[i * BS + j];
    desc[p] = dsc;
}

// Largest per-row block count of a sweep (integer max, order-free).
__global__ void k_max_count(int64_t n, const int32_t *cnt, int32_t *out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) atomicMax(out, cnt[p]);
}

hipError_t launch_max_count(int64_t n, const int32_t *cnt, int32_t *out, hipStream_t st) {
    const int T = 256;
    k_max_count<<<(unsigned)((n + T - 1) / T), T, 0, st>>>(n, cnt, out);
    return hipGetLastError();
}

hipError_t launch_pack_slots(dd_ctx *h, int which, hipStream_t st) {
    const int T = 256;
    Sweep &w = h->sw[which];
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    if (h->bs == 3)
        k_pack_slots<3><<<g, T, 0, st>>>(h->n, h->S, which, h->slots, h->tptr, h->tcol, h->lu, h->invd,
                                         h->lev[which].rows, w.desc, w.sval64);
    else
        k_pack_slots<1><<<g, T, 0, st>>>(h->n, h->S, which, h->slots, h->tptr, h->tcol, h->lu, h->invd,
                                         h->lev[which].rows, w.desc, w.sval64);
    return hipGetLastError();
}

// ------------------------------------------------- segmented slot layout
// For sweeps with rows of more than three blocks.  With MB blocks per
// segment, a lower-sweep row with nb blocks becomes ceil(nb/MB) segments (none
// when nb = 0), an upper-sweep row one segment of MB blocks and inv_D plus
// ceil((nb - MB)/(MB + 1)) continuations of MB + 1 blocks (the extra block
// in the inv_D slot, which a continuation does not need); blocks in column
// order, segments at consecutive positions of one wavefront; the first
// segment (the row's owner) adds the others' partial sums in the apply.  Each level is
// laid out in chunks of at most cw positions (one workgroup pass of the
// apply, rpw positions per wavefront); a group that would straddle a
// wavefront is moved to the next one (the positions skipped are padding), a
// group that would not fit the chunk starts the next chunk of the level.
// Only the last chunk of a level is followed by a barrier in the apply.  One
// thread per subdomain walks its levels (count pass, then fill pass).
// One workgroup per subdomain.  The rows of a level are taken kSegTile at a
// time: every thread loads block counts and computes segment counts, one
// thread places the tile's rows (the placement above, on LDS values only),
// and every thread writes the tile's position map.
constexpr int kSegTile = 1024;

template <bool FILL>
__global__ __launch_bounds__(256) void k_seg_walk(int S, int which, int mb, int cw, int rpw,
                                                  const int32_t *__restrict__ off, const int32_t *__restrict__ lp,
                                                  const int32_t *__restrict__ bptr, int32_t *npos, int32_t *nchk,
                                                  const int32_t *__restrict__ gpos,
                                                  const int32_t *__restrict__ gchk, int2 *pmap, int32_t *chk) {
    __shared__ int m_s[kSegTile], at_s[kSegTile], pad_s[kSegTile];
    __shared__ int32_t pos_s, nc_s, inchunk_s;
    __shared__ bool open_s;
    const int s = blockIdx.x, tid = threadIdx.x;
    const int32_t o = off[s];
    const int nl = off[s + 1] - o - 1;
    const int64_t base = (int64_t)s * S;
    const int32_t pb = FILL ? gpos[s] : 0, cb = FILL ? gchk[s] : 0;
    if (tid == 0) {
        pos_s = 0;
        nc_s = 0;
    }
    for (int l = 0; l < nl; ++l) {
        if (tid == 0) {
            inchunk_s = 0;
            open_s = false;  // a level's first position opens its first chunk
        }
        const int32_t k0 = lp[o + l], k1 = lp[o + l + 1];
        for (int32_t t0 = k0; t0 < k1; t0 += kSegTile) {
            const int cnt = min(kSegTile, k1 - t0);
            for (int i = tid; i < cnt; i += blockDim.x) {
                const int64_t p = base + t0 + i;
                const int32_t nb = bptr[p + 1] - bptr[p];
                // a lower-sweep row without blocks keeps y_I = r_I: no position
                // (a level of such rows, the lower sweep's first, has no chunk)
                m_s[i] = which == 0 ? (nb + mb - 1) / mb : 1 + (max(nb - mb, 0) + mb) / (mb + 1);
            }
            __syncthreads();
            if (tid == 0) {
                int32_t pos = pos_s, nc = nc_s;
                int inchunk = inchunk_s;
                bool open = open_s;
                for (int i = 0; i < cnt; ++i) {
                    const int m = m_s[i];
                    if (m == 0) continue;
                    int pad = (inchunk % rpw) + m > rpw ? rpw - inchunk % rpw : 0;
                    if (!open || inchunk + pad + m > cw) {  // the level's first or next chunk
                        if (FILL) chk[cb + nc] = pos;
                        ++nc;
                        inchunk = 0;
                        pad = 0;
                        open = true;
                    }
                    pad_s[i] = pad;
                    at_s[i] = pos + pad;  // the row's first segment
                    pos += pad + m;
                    inchunk += pad + m;
                }
                pos_s = pos;
                nc_s = nc;
                inchunk_s = inchunk;
                open_s = open;
            }
            __syncthreads();
            if (FILL)
                for (int i = tid; i < cnt; i += blockDim.x) {
                    const int m = m_s[i];
                    if (m == 0) continue;
                    const int32_t at = at_s[i];
                    for (int q = 0; q < pad_s[i]; ++q) pmap[pb + at - pad_s[i] + q] = make_int2(-1, 0);
                    for (int q = 0; q < m; ++q) pmap[pb + at + q] = make_int2((int32_t)(base + t0 + i), q | (m << 8));
                }
            __syncthreads();  // the tile's LDS values are reused by the next tile
        }
        if (FILL && tid == 0 && open_s) chk[cb + nc_s - 1] |= 1 << 30;  // barrier after the level's last chunk
        __syncthreads();
    }
    if (tid != 0) return;
    int32_t nc = nc_s;
    if (nc == 0) {  // no positions: one empty chunk, so the apply's table reads stay inside it
        if (FILL) chk[cb] = 1 << 30;
        ++nc;
    }
    if (FILL) {
        chk[cb + nc] = pos_s;
    } else {
        npos[s] = pos_s;
        nchk[s] = nc + 1;
    }
}

// Position q: its segment's descriptor and values in the lane-run layout of
// k_pack_slots (MB blocks, then inv_D in the upper sweep).  Padding
// positions are continuations of local row 0 with no blocks (they read y_0
// and write nothing).  An upper-sweep continuation holds its (MB+1)-th block
// in the inv_D slot and that block's column in the row field (its own row
// when the slot is empty: a valid LDS entry, times a zero block).  The
// descriptor keeps three 16-bit column fields whatever MB (fields past MB
// empty), so that the bits 15 of fields 1 to 3 hold m - 1 on a row's first
// segment.
template <int BS, int MB>
__global__ void k_seg_pack(int64_t npos, int which, const int2 *__restrict__ pmap, const uint16_t *__restrict__ prow,
                           const int32_t *__restrict__ bptr, const uint16_t *__restrict__ bcol,
                           const double *__restrict__ val, const double *__restrict__ dval, uint64_t *desc,
                           double *sval) {
    constexpr int BB = BS * BS;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npos) return;
    const int NV = (MB + which) * BS;
    double *o = sval + q * BS * NV;
    const int2 e = pmap[q];
    int32_t b0 = 0, b1 = 0, bx = -1;  // segment blocks [b0, b1); bx: a continuation's extra block (upper)
    int k = 0;
    uint64_t d;
    if (e.x < 0) {
        d = 0x8000ull;
        for (int j = 0; j < 3; ++j) d |= 0x7fffull << (16 * (j + 1));
    } else {
        k = e.y & 0xff;
        const int m = e.y >> 8;
        const int32_t rb = bptr[e.x], re = bptr[e.x + 1];
        b0 = rb + (which == 0 || k == 0 ? MB * k : MB + (k - 1) * (MB + 1));
        b1 = min(b0 + MB, re);
        if (which == 1 && k > 0 && b0 + MB < re) bx = b0 + MB;
        d = (uint64_t)(bx >= 0 ? bcol[bx] : prow[e.x]) | (k > 0 ? 0x8000ull : 0ull);
        for (int j = 0; j < 3; ++j) d |= (uint64_t)(j < MB && b0 + j < b1 ? bcol[b0 + j] : 0x7fff) << (16 * (j + 1));
        if (k == 0)
            for (int j = 0; j < 3; ++j)
                if (((m - 1) >> j) & 1) d |= 1ull << (16 * (j + 1) + 15);
    }
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int jj = 0; jj < BS; ++jj)
                o[i * NV + j * BS + jj] = b0 + j < b1 ? val[(int64_t)(b0 + j) * BB + i * BS + jj] : 0.0;
    if (which == 1)
#pragma unroll
        for (int i = 0; i < BS; ++i)
#pragma unroll
            for (int jj = 0; jj < BS; ++jj)
                o[i * NV + MB * BS + jj] = e.x < 0 ? 0.0
                                           : k == 0 ? dval[(int64_t)e.x * BB + i * BS + jj]
                                           : bx >= 0 ? val[(int64_t)bx * BB + i * BS + jj] : 0.0;
    desc[q] = d;
}

hipError_t launch_seg_pack(dd_ctx *h, int which, hipStream_t st) {
    const int T = 256;
    Sweep &w = h->sw[which];
    const unsigned g = (unsigned)((w.snpos + T - 1) / T);
    if (w.snpos == 0) return hipSuccess;
    auto go = [&](auto kern) {
        kern<<<g, T, 0, st>>>(w.snpos, which, w.pmap, w.prow, w.bptr, w.bcol, w.val64, w.d64, w.desc, w.sval64);
    };
    if (h->bs == 3) {
        if (h->seg == 2) go(k_seg_pack<3, 2>); else go(k_seg_pack<3, 3>);
    } else {
        if (h->seg == 2) go(k_seg_pack<1, 2>); else go(k_seg_pack<1, 3>);
    }
    return hipGetLastError();
}

int build_seg_layout(dd_ctx *h, int which, int mb, int cw, int rpw, hipStream_t st) {
    Sweep &w = h->sw[which];
    const Levels &L = h->lev[which];
    const int nsub = h->nsub;
    int32_t *npos = nullptr, *nchk = nullptr;
    int rc = h->alloc(&npos, nsub);
    if (!rc) rc = h->alloc(&nchk, nsub);
    if (!rc && !w.gpos) rc = h->alloc(&w.gpos, nsub + 1);
    if (!rc && !w.gchk) rc = h->alloc(&w.gchk, nsub + 1);
    if (rc) return rc;
    auto drop = [&](void *q) {
        auto it = std::find(h->allocs.begin(), h->allocs.end(), q);
        if (it != h->allocs.end()) {
            (void)hipFree(q);
            h->allocs.erase(it);
        }
    };
    k_seg_walk<false><<<nsub, 256, 0, st>>>(h->S, which, mb, cw, rpw, L.off, L.ptr, w.bptr, npos, nchk, nullptr,
                                        nullptr, nullptr, nullptr);
    hipError_t e = exclusive_scan(npos, w.gpos, nsub, h->scan_tmp, st);
    if (e == hipSuccess) e = exclusive_scan(nchk, w.gchk, nsub, h->scan_tmp, st);
    int32_t tot[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(&tot[0], w.gpos + nsub, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&tot[1], w.gchk + nsub, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "segmented layout: %s", hipGetErrorString(e));
    for (void *q : {(void *)w.pmap, (void *)w.chk, (void *)w.desc, (void *)w.sval64, (void *)w.sval32}) drop(q);
    w.pmap = nullptr; w.chk = nullptr; w.desc = nullptr; w.sval64 = nullptr; w.sval32 = nullptr;
    const int bb = h->bs * h->bs;
    w.snpos = tot[0];
    rc = h->alloc(&w.pmap, tot[0]);
    if (!rc) rc = h->alloc(&w.chk, tot[1]);
    if (!rc) rc = h->alloc(&w.desc, tot[0]);
    if (!rc) rc = h->alloc(&w.sval64, (int64_t)tot[0] * (mb + which) * bb);
    if (rc) return rc;
    k_seg_walk<true><<<nsub, 256, 0, st>>>(h->S, which, mb, cw, rpw, L.off, L.ptr, w.bptr, nullptr, nullptr, w.gpos,
                                       w.gchk, w.pmap, w.chk);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_seg_pack(h, which, st);
    drop(npos);
    drop(nchk);
    if (e != hipSuccess) return h->fail(DD_EHIP, "segmented layout: %s", hipGetErrorString(e));
    return DD_OK;
}

// FP64 -> FP32 copies, round to nearest even.
__global__ void k_cast32(int64_t m, const double *in, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = (float)in[i];
}

hipError_t launch_cast32(dd_ctx *h, hipStream_t st) {
    const int T = 256;
    const int bb = h->bs * h->bs;
    for (int w = 0; w < 2; ++w) {
        Sweep &s = h->sw[w];
        const int64_t m = s.nblk * bb;
        if (m) k_cast32<<<(unsigned)((m + T - 1) / T), T, 0, st>>>(m, s.val64, s.val32);
    }
    const int64_t m = h->n * bb;
    k_cast32<<<(unsigned)((m + T - 1) / T), T, 0, st>>>(m, h->sw[1].d64, h->sw[1].d32);
    if (h->slots || h->seg) {
        const int mb = h->seg ? h->seg : h->slots;
        for (int w = 0; w < 2; ++w) {
            const int64_t ms = h->sw[w].snpos * (mb + w) * bb;  // the upper stream carries inv_D
            if (ms) k_cast32<<<(unsigned)((ms + T - 1) / T), T, 0, st>>>(ms, h->sw[w].sval64, h->sw[w].sval32);
        }
    }
    return hipGetLastError();
}

// L\inv_D\Uhat in the dropped pattern (for inspection).
template <int BS>
__global__ void k_export(int64_t n, const int32_t *tptr, const int32_t *tcol, const double *lu,
                         const double *invd, double *f) {
    constexpr int BB = BS * BS;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *inv = invd + i * BB;
    for (int32_t q = tptr[i]; q < tptr[i + 1]; ++q) {
        const int32_t c = tcol[q];
        double t[BB];
        if (c < i) {
#pragma unroll
            for (int e = 0; e < BB; ++e) t[e] = lu[(int64_t)q * BB + e];
        } else if (c == i) {
#pragma unroll
            for (int e = 0; e < BB; ++e) t[e] = inv[e];
        } else {
            blk_mul<BS>(inv, lu + (int64_t)q * BB, t);
        }
#pragma unroll
        for (int e = 0; e < BB; ++e) f[(int64_t)q * BB + e] = t[e];
    }
}

hipError_t launch_export_factors(dd_ctx *h, double *f, hipStream_t st) {
    const int T = 256;
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    if (h->bs == 3)
        k_export<3><<<g, T, 0, st>>>(h->n, h->tptr, h->tcol, h->lu, h->invd, f);
    else
        k_export<1><<<g, T, 0, st>>>(h->n, h->tptr, h->tcol, h->lu, h->invd, f);
    return hipGetLastError();
}

}  // namespace ddilu
