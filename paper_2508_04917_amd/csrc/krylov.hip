// BSR SpMV, fused FP64 vector kernels and the BiCGSTAB driver
// (Section 2, Algorithm 1, right preconditioned: K1 = I, K2 = M_DD).
//
// Every dot product is reduced deterministically: each workgroup of a fixed
// grid writes one partial sum (fixed in-wave shuffle tree, then waves in
// order), and a one-workgroup kernel sums the partials in a fixed order and
// performs the scalar step of the algorithm on the device.  No floating
// point atomics, so a solve is bit-reproducible and its iteration count does
// not vary from run to run.
//
// The scalars (rho, alpha, omega, beta, norms) and the state word stay on the
// device.  Every kernel of an iteration first reads the state word and
// returns at once when the solve has finished, so the host enqueues a batch
// of iterations and only synchronises once per batch.
#include <chrono>
#include <mutex>

#include "internal.h"
#include "spmv.h"

namespace ddilu {

constexpr int kRedT = 256;        // threads of reducing kernels
constexpr int kMaxGrid = 2048;    // workgroups of grid-stride vector kernels
constexpr int kStride = 8;        // partial-sum slots per reduction (2048 each)

enum : int32_t { ST_RUN = 0, ST_CONV = 1, ST_HALF = 2 };

// Sums NV values over the workgroup in a fixed order and writes them to
// out[k*stride + blockIdx.x].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *out, int stride) {
    __shared__ double sh[NV][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = wave_sum(v[k]);
        if (lane == 0) sh[k][w] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = 0.0;
            for (int i = 0; i < nw; ++i) t += sh[k][i];
            out[k * stride + blockIdx.x] = t;
        }
    }
}

// Sliced ELL copy of the full matrix, for matrices whose rows hold at most
// kUnroll blocks: for each group of RPW consecutive block rows (one
// wavefront's rows) and each position k < kUnroll, the k-th blocks of the
// group's rows one after another (ecol -1 and a zero block past a row's
// end).  In the CSR layout the k-th blocks of a wavefront's rows lie one row
// length apart, so each load instruction touches RPW separate pieces; here
// it reads one contiguous run (measured at 160^3: 441 -> 408 us per SpMV,
// same bits).  One more copy of A's blocks (plus a zero block for each
// position a row leaves empty); the CSR arrays stay for everything else.
// One thread per value of the copy, so that consecutive threads write
// consecutive words (the column of a slot is written by its first value's
// thread).
template <int BS>
__global__ __launch_bounds__(256) void k_ell_fill(int64_t n, const int32_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 int32_t *__restrict__ ecol, double *__restrict__ eval,
                                                 int64_t nslots) {
    constexpr int RPW = kWave / BS, BB = BS * BS;
    const int64_t total = nslots * BB;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / BB, e = t % BB;
        const int64_t r = i % RPW, gk = i / RPW, k = gk % kUnroll, g = gk / kUnroll;
        const int64_t row = g * RPW + r;
        int64_t b = -1;
        if (row < n && ptr[row] + k < ptr[row + 1]) b = ptr[row] + k;
        if (e == 0) ecol[i] = b >= 0 ? col[b] : -1;
        eval[t] = b >= 0 ? val[b * BB + e] : 0.0;
    }
}

// Sliced ELL with per-slice widths (rows of more than kUnroll blocks): one
// workgroup per window of kSellWin slices (the rows of one SpMV workgroup)
// ranks the window's rows by length, longest first (ties by row number),
// and writes the window's row order, the rows' lengths and each slice's
// width (its first, longest row).  Positions past the matrix's last row get
// row -1 and length 0.
constexpr int kSellWin = kRedT / kWave;

template <int BS>
__global__ __launch_bounds__(256) void k_sell_rank(int64_t n, int64_t nslice, const int32_t *__restrict__ ptr,
                                                  int32_t *__restrict__ srow, int32_t *__restrict__ slen,
                                                  int64_t *__restrict__ soff) {
    constexpr int RPW = kWave / BS, WIN = RPW * kSellWin;
    __shared__ int len_s[WIN];
    const int64_t w0 = (int64_t)blockIdx.x * WIN;
    for (int i = threadIdx.x; i < WIN; i += blockDim.x) {
        const int64_t row = w0 + i;
        len_s[i] = row < n ? ptr[row + 1] - ptr[row] : -1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < WIN; i += blockDim.x) {
        const int li = len_s[i];
        int rank = 0;
        for (int p = 0; p < WIN; ++p) {
            const int lp = len_s[p];
            rank += (lp > li || (lp == li && p < i)) ? 1 : 0;
        }
        const int64_t pos = w0 + rank, g = pos / RPW;
        if (g < nslice) {
            srow[pos] = li >= 0 ? (int32_t)(w0 + i) : -1;
            slen[pos] = max(li, 0);
            if (rank % RPW == 0) soff[g] = max(li, 0);
        }
    }
}

// The same ranking with the slices aligned to the parts of a graph
// partition (parts of S rows): part k owns slices k*spp .. k*spp + spp - 1,
// spp = ceil(S / RPW), and a window (kSellWin slices) never crosses a part;
// positions past the part's last row get row -1 and length 0.
template <int BS>
__global__ __launch_bounds__(256) void k_sell_rank_part(int S, int spp, int nwin, const int32_t *__restrict__ ptr,
                                                       int32_t *__restrict__ srow, int32_t *__restrict__ slen,
                                                       int64_t *__restrict__ soff) {
    constexpr int RPW = kWave / BS, WIN = RPW * kSellWin;
    __shared__ int len_s[WIN];
    const int64_t k = blockIdx.x / nwin;
    const int wi = blockIdx.x % nwin;
    const int64_t row0 = k * S;
    const int l0 = wi * WIN;
    for (int i = threadIdx.x; i < WIN; i += blockDim.x) {
        const int lr = l0 + i;
        len_s[i] = lr < S ? ptr[row0 + lr + 1] - ptr[row0 + lr] : -1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < WIN; i += blockDim.x) {
        const int li = len_s[i];
        int rank = 0;
        for (int p = 0; p < WIN; ++p) {
            const int lp = len_s[p];
            rank += (lp > li || (lp == li && p < i)) ? 1 : 0;
        }
        const int ls = wi * kSellWin + rank / RPW, q = rank % RPW;
        if (ls < spp) {
            const int64_t g = k * spp + ls;
            srow[g * RPW + q] = li >= 0 ? (int32_t)(row0 + l0 + i) : -1;
            slen[g * RPW + q] = max(li, 0);
            if (q == 0) soff[g] = max(li, 0);
        }
    }
}

// Exclusive prefix sum of the slice widths in place (soff[0..nslice)), and
// soff[nslice] = the total: one workgroup, each thread a contiguous run.
__global__ __launch_bounds__(1024) void k_sell_scan(int64_t nslice, int64_t *__restrict__ soff) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t run = (nslice + 1023) / 1024, lo = t * run, hi = min(nslice, lo + run);
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += soff[i];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t v = part[i];
            part[i] = acc;
            acc += v;
        }
        soff[nslice] = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t v = soff[i];
        soff[i] = acc;
        acc += v;
    }
}

// Fill (or refill, for new values) the per-slice-width copy: one workgroup
// per slice at a time, consecutive threads writing consecutive words.
template <int BS>
__global__ __launch_bounds__(256) void k_sell_fill(int64_t nslice, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ val,
                                                  const int32_t *__restrict__ srow, const int32_t *__restrict__ slen,
                                                  const int64_t *__restrict__ soff, int32_t *__restrict__ ecol,
                                                  double *__restrict__ eval) {
    constexpr int RPW = kWave / BS, BB = BS * BS;
    for (int64_t g = blockIdx.x; g < nslice; g += gridDim.x) {
        const int64_t base = soff[g] * RPW, cnt = (soff[g + 1] - soff[g]) * RPW * BB;
        for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) {
            const int64_t i = t / BB;
            const int e = (int)(t % BB), k = (int)(i / RPW), q = (int)(i % RPW);
            const int32_t row = srow[g * RPW + q];
            const int64_t b = k < slen[g * RPW + q] ? (int64_t)ptr[row] + k : -1;
            if (e == 0) ecol[base + i] = b >= 0 ? col[b] : -1;
            eval[(base + i) * BB + e] = b >= 0 ? val[b * BB + e] : 0.0;
        }
    }
}

template <int BS>
static void launch_ell_fill(dd_ctx *h, hipStream_t st) {
    const int rpw = kWave / BS, bb = BS * BS;
    const int64_t nslice = (h->n + rpw - 1) / rpw;
    if (h->ell_state == 1 && h->sell_row) {
        const unsigned g = (unsigned)std::min<int64_t>(h->sell_nslice, 1 << 20);
        k_sell_fill<BS><<<g, 256, 0, st>>>(h->sell_nslice, h->aptr, h->acol, h->aval, h->sell_row, h->sell_len,
                                           h->sell_off, h->ell_col, h->ell_val);
        return;
    }
    const int64_t nslots = nslice * kUnroll * rpw;
    const unsigned g = (unsigned)std::min<int64_t>((nslots * bb + 255) / 256, 1 << 20);  // grid-stride beyond
    k_ell_fill<BS><<<g, 256, 0, st>>>(h->n, h->aptr, h->acol, h->aval, h->ell_col, h->ell_val, nslots);
}

// Whether the SpMV of a graph-partitioned matrix runs part by part with the
// part's x in LDS (layout 3): scalar rows (each lane's x_J is an 8-byte
// gather, a cache line of its own in the global-memory form; measured at
// 4,096,000 rows: 233 -> 154 us.  With 3x3 blocks the 24-byte x_J fills
// more of a line and the one-workgroup-per-CU occupancy of the part kernel
// costs more than it saves: 322 against 334 us at 2,048,000 rows), parts of
// at least one ranking window whose x fits the LDS next to the kernel's own
// 1 KB, and one partial sum per part within the Krylov driver's partial-sum
// stride.
constexpr int kPartLds = 163840 - 1024;

static bool part_local_spmv(const dd_ctx *h) {
    const int rpw = kWave / h->bs, rpb = rpw * (kRedT / kWave);
    const int64_t stride = std::max<int64_t>((h->n + rpb - 1) / rpb, kMaxGrid);
    return h->graph && h->bs == 1 && h->S >= rpw * kSellWin && (int64_t)h->S * h->bs * 8 <= kPartLds &&
           h->nsub <= stride;
}

// Build the sliced ELL copy once per handle when the memory is there
// (otherwise the SpMV stays on the CSR arrays): for graph partitions,
// slices aligned to the parts with per-slice widths (the SpMV then runs part
// by part, the part's x in LDS); otherwise fixed width kUnroll when no row
// is longer, per-slice widths with the rows ranked by length when one is.
// Called at the end of the partition step (so its time counts as setup);
// the SpMV entry points call it again, which does nothing once it has run.
void build_spmv_layout(dd_ctx *h, hipStream_t st) {
    if (h->ell_state != 0) return;
    h->ell_state = -1;
    if (h->max_row_a < 1) return;
    const int rpw = kWave / h->bs, bb = h->bs * h->bs;
    const bool parts = part_local_spmv(h);
    const int spp = parts ? (h->S + rpw - 1) / rpw : 0;
    const int64_t nslice = parts ? (int64_t)h->nsub * spp : (h->n + rpw - 1) / rpw;
    h->sell_nslice = nslice;
    h->sell_spp = spp;
    auto grab = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        h->allocs.push_back(p);  // released with the handle, used or not
        return p;
    };
    int64_t nslots = nslice * kUnroll * rpw;
    if (parts || h->max_row_a > kUnroll) {
        h->sell_row = static_cast<int32_t *>(grab((size_t)nslice * rpw * sizeof(int32_t)));
        h->sell_len = static_cast<int32_t *>(grab((size_t)nslice * rpw * sizeof(int32_t)));
        h->sell_off = static_cast<int64_t *>(grab((size_t)(nslice + 1) * sizeof(int64_t)));
        if (!h->sell_row || !h->sell_len || !h->sell_off) {
            h->sell_row = nullptr;
            return;
        }
        if (parts) {
            const int nwin = (spp + kSellWin - 1) / kSellWin;
            const unsigned g = (unsigned)((int64_t)h->nsub * nwin);
            if (h->bs == 3)
                k_sell_rank_part<3><<<g, 256, 0, st>>>(h->S, spp, nwin, h->aptr, h->sell_row, h->sell_len,
                                                       h->sell_off);
            else
                k_sell_rank_part<1><<<g, 256, 0, st>>>(h->S, spp, nwin, h->aptr, h->sell_row, h->sell_len,
                                                       h->sell_off);
        } else {
            const unsigned g = (unsigned)((nslice + kSellWin - 1) / kSellWin);
            if (h->bs == 3)
                k_sell_rank<3><<<g, 256, 0, st>>>(h->n, nslice, h->aptr, h->sell_row, h->sell_len, h->sell_off);
            else
                k_sell_rank<1><<<g, 256, 0, st>>>(h->n, nslice, h->aptr, h->sell_row, h->sell_len, h->sell_off);
        }
        k_sell_scan<<<1, 1024, 0, st>>>(nslice, h->sell_off);
        int64_t total = 0;
        if (hipMemcpyAsync(&total, h->sell_off + nslice, sizeof(total), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            (void)hipGetLastError();
            h->sell_row = nullptr;
            return;
        }
        nslots = total * rpw;
    }
    h->ell_col = static_cast<int32_t *>(grab((size_t)std::max<int64_t>(nslots, 1) * sizeof(int32_t)));
    h->ell_val = static_cast<double *>(grab((size_t)std::max<int64_t>(nslots, 1) * bb * sizeof(double)));
    if (!h->ell_col || !h->ell_val) {
        h->sell_row = nullptr;
        return;
    }
    h->ell_state = 1;
    if (h->bs == 3)
        launch_ell_fill<3>(h, st);
    else
        launch_ell_fill<1>(h, st);
    // later SpMVs may run on other streams: the copy is complete before any
    // of them is enqueued
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        h->ell_state = -1;
        h->sell_row = nullptr;
    }
}

// New values of A on the same pattern: rewrite the sliced ELL copy in place.
hipError_t refresh_spmv_layout(dd_ctx *h, hipStream_t st) {
    if (h->ell_state != 1) return hipSuccess;
    if (h->bs == 3)
        launch_ell_fill<3>(h, st);
    else
        launch_ell_fill<1>(h, st);
    return hipGetLastError();
}

// The matrix as the SpMV kernels read it: CSR arrays, and the sliced ELL
// copy in one of its two forms (layout 1 fixed width, 2 per-slice widths).
struct SpmvMat {
    int64_t n;
    const int32_t *ptr, *col;
    const double *val;
    const int32_t *ecol;
    const double *eval;
    const int32_t *srow, *slen;
    const int64_t *soff;
};

static SpmvMat spmv_mat(const dd_ctx *h) {
    return {h->n, h->aptr, h->acol, h->aval, h->ell_col, h->ell_val, h->sell_row, h->sell_len, h->sell_off};
}

static int spmv_layout(const dd_ctx *h) {
    return h->ell_state == 1 ? (h->sell_row ? (h->sell_spp ? 3 : 2) : 1) : 0;
}

// The block row a lane's wavefront slot (gw, rl) computes (-1: none), and
// its product with x in components c.
template <int BS, int LAYOUT>
__device__ __forceinline__ int64_t slot_row(const SpmvMat &m, int64_t gw, int rl) {
    constexpr int RPW = kWave / BS;
    if (rl >= RPW || gw * RPW >= m.n) return -1;
    if constexpr (LAYOUT == 2) return m.srow[gw * RPW + rl];
    const int64_t row = gw * RPW + rl;
    return row < m.n ? row : -1;
}

template <int BS, int LAYOUT>
__device__ __forceinline__ double row_product(const SpmvMat &m, const double *__restrict__ x, int64_t gw, int rl,
                                              int64_t row, int c) {
    constexpr int RPW = kWave / BS;
    if constexpr (LAYOUT == 2) {
        const int len = m.slen[gw * RPW + rl];
        if (len == 0) return 0.0;
        return sell_row<BS>(m.ecol, m.eval, x, m.soff[gw] * RPW, (int)(m.soff[gw + 1] - m.soff[gw]), rl, len, c);
    } else if constexpr (LAYOUT == 1) {
        return ell_row<BS>(m.ecol, m.eval, x, gw, rl, c);
    } else {
        return bsr_row<BS>(m.ptr, m.col, m.val, x, row, c);
    }
}

template <int BS, int LAYOUT>
__global__ __launch_bounds__(kRedT) void k_spmv(SpmvMat m, const double *__restrict__ x, double *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int c = lane % BS, rl = lane / BS;
    const int64_t row = slot_row<BS, LAYOUT>(m, gw, rl);
    if (row >= 0) y[row * BS + c] = row_product<BS, LAYOUT>(m, x, gw, rl, row, c);
}

// Layout 3 (graph partitions): one workgroup per part.  The part's x is
// staged in LDS (S*BS values, read once), then the wavefronts take the
// part's slices in turn; a column inside the part reads x from LDS.  The
// rows of a part keep their original, unordered numbering inside it, so a
// row's neighbours lie anywhere in the part: in the global-memory form every
// x_J is a cache line of its own.  MODE as in k_spmv_dots, 4 = y = A x only;
// one partial sum per part.
template <int BS, int MODE>
__global__ __launch_bounds__(1024) void k_spmv_part(SpmvMat m, int S, int spp, const double *__restrict__ x,
                                                   double *__restrict__ y, const double *__restrict__ w,
                                                   double *__restrict__ r_out, double *__restrict__ r0_out,
                                                   double *__restrict__ p_out, double *__restrict__ part,
                                                   int part_stride, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != ST_RUN) return;
    constexpr int RPW = kWave / BS;
    constexpr int NV = MODE == 0 ? 1 : (MODE == 3 || MODE == 4 ? 1 : 2);
    extern __shared__ double xs[];
    const int64_t k = blockIdx.x, row0 = k * S;
    {  // eight loads in flight per thread, positions past the end clamped and not stored
        const int m = S * BS, nt = blockDim.x;
        const double *xp = x + row0 * BS;
        for (int i0 = threadIdx.x; i0 < m; i0 += 8 * nt) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = xp[min(i0 + u * nt, m - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u * nt < m) xs[i0 + u * nt] = v[u];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int c = lane % BS, rl = lane / BS;
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    for (int ls = wave; ls < spp; ls += nw) {
        const int64_t g = k * spp + ls;
        if (rl >= RPW) continue;
        const int32_t row = m.srow[g * RPW + rl];
        if (row < 0) continue;
        const int len = m.slen[g * RPW + rl];
        const double t = len == 0 ? 0.0
                                  : sell_row_lds<BS>(m.ecol, m.eval, x, xs, row0, S, m.soff[g] * RPW,
                                                     (int)(m.soff[g + 1] - m.soff[g]), rl, len, c);
        const int64_t e = (int64_t)row * BS + c;
        if constexpr (MODE == 4) {
            y[e] = t;
        } else if constexpr (MODE == 0) {
            y[e] = t;
            acc[0] += w[e] * t;
        } else if constexpr (MODE == 1) {
            y[e] = t;
            acc[0] += t * w[e];
            acc[1] += t * t;
        } else if constexpr (MODE == 2) {
            const double rr = w[e] - t;
            r_out[e] = rr;
            r0_out[e] = rr;
            p_out[e] = rr;
            acc[0] += rr * rr;
            acc[1] += w[e] * w[e];
        } else {
            const double rr = w[e] - t;
            acc[0] += rr * rr;
        }
    }
    if constexpr (MODE != 4) block_partials<NV>(acc, part, part_stride);
}

template <int BS, int MODE>
static void launch_spmv_part(const dd_ctx *h, const double *x, double *y, const double *w, double *r_out,
                             double *r0_out, double *p_out, double *part, int stride, const int32_t *state,
                             hipStream_t st) {
    static bool done = false;
    auto kern = k_spmv_part<BS, MODE>;
    if (!done && hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kPartLds) == hipSuccess)
        done = true;
    const int nt = std::min(1024, h->sell_spp * kWave);
    kern<<<h->nsub, nt, h->S * BS * (int)sizeof(double), st>>>(spmv_mat(h), h->S, h->sell_spp, x, y, w, r_out,
                                                               r0_out, p_out, part, stride, state);
}

// Partial sums one reducing SpMV launch leaves (one per workgroup, or one
// per part for layout 3).
static int spmv_partials(const dd_ctx *h) {
    if (spmv_layout(h) == 3) return h->nsub;
    const int rpb = (kWave / h->bs) * (kRedT / kWave);
    return (int)((h->n + rpb - 1) / rpb);
}

template <int BS>
static void launch_spmv_bs(dd_ctx *h, const double *x, double *y, hipStream_t st) {
    const int rpb = (kWave / BS) * (kRedT / kWave);
    const unsigned g = (unsigned)((h->n + rpb - 1) / rpb);
    const SpmvMat m = spmv_mat(h);
    switch (spmv_layout(h)) {
        case 3:
            launch_spmv_part<BS, 4>(h, x, y, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, st);
            break;
        case 2: k_spmv<BS, 2><<<g, kRedT, 0, st>>>(m, x, y); break;
        case 1: k_spmv<BS, 1><<<g, kRedT, 0, st>>>(m, x, y); break;
        default: k_spmv<BS, 0><<<g, kRedT, 0, st>>>(m, x, y);
    }
}

hipError_t launch_spmv(dd_ctx *h, const double *x, double *y, hipStream_t st) {
    build_spmv_layout(h, st);
    if (h->bs == 3)
        launch_spmv_bs<3>(h, x, y, st);
    else
        launch_spmv_bs<1>(h, x, y, st);
    return hipGetLastError();
}

// y = A x, one wavefront per 64/BS block rows, one workgroup per 4*64/BS
// rows, one partial sum per workgroup and dot product.  mode 0: v = A p^,
// dot r0.v.  mode 1: t = A s^, dots t.s and t.t.  mode 2: t = A x,
// r = b - t (init), dots r.r and b.b.  mode 3: t = A x, dot (b-t).(b-t)
// (true residual).
template <int BS, int MODE, int LAYOUT>
__global__ __launch_bounds__(kRedT) void k_spmv_dots(SpmvMat m, const double *__restrict__ x,
                                                    double *__restrict__ y, const double *__restrict__ w,
                                                    double *__restrict__ r_out, double *__restrict__ r0_out,
                                                    double *__restrict__ p_out, double *__restrict__ part,
                                                    int part_stride, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != ST_RUN) return;
    constexpr int NV = MODE == 0 ? 1 : (MODE == 3 ? 1 : 2);
    const int lane = threadIdx.x & 63;
    const int c = lane % BS, rl = lane / BS;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t row = slot_row<BS, LAYOUT>(m, gw, rl);
    if (row >= 0) {
        const int64_t e = row * BS + c;
        const double t = row_product<BS, LAYOUT>(m, x, gw, rl, row, c);
        if constexpr (MODE == 0) {
            y[e] = t;
            acc[0] += w[e] * t;
        } else if constexpr (MODE == 1) {
            y[e] = t;
            acc[0] += t * w[e];
            acc[1] += t * t;
        } else if constexpr (MODE == 2) {
            const double rr = w[e] - t;
            r_out[e] = rr;
            r0_out[e] = rr;
            p_out[e] = rr;
            acc[0] += rr * rr;
            acc[1] += w[e] * w[e];
        } else {
            const double rr = w[e] - t;
            acc[0] += rr * rr;
        }
    }
    block_partials<NV>(acc, part, part_stride);
}

// Launch k_spmv_dots on the handle's layout.
template <int BS, int MODE>
static void spmv_dots(const dd_ctx *h, int grid, const double *x, double *y, const double *w, double *r_out,
                      double *r0_out, double *p_out, double *part, int stride, const int32_t *state,
                      hipStream_t st) {
    const SpmvMat m = spmv_mat(h);
    switch (spmv_layout(h)) {
        case 3:
            launch_spmv_part<BS, MODE>(h, x, y, w, r_out, r0_out, p_out, part, stride, state, st);
            break;
        case 2:
            k_spmv_dots<BS, MODE, 2><<<grid, kRedT, 0, st>>>(m, x, y, w, r_out, r0_out, p_out, part, stride, state);
            break;
        case 1:
            k_spmv_dots<BS, MODE, 1><<<grid, kRedT, 0, st>>>(m, x, y, w, r_out, r0_out, p_out, part, stride, state);
            break;
        default:
            k_spmv_dots<BS, MODE, 0><<<grid, kRedT, 0, st>>>(m, x, y, w, r_out, r0_out, p_out, part, stride, state);
    }
}

// s = r - alpha v; partial s.s
__global__ __launch_bounds__(kRedT) void k_axpy_s(int64_t m, const double *__restrict__ r,
                                                 const double *__restrict__ v, double *__restrict__ s,
                                                 const KrylovScalars *__restrict__ ks, double *__restrict__ part) {
    if (ks->state != ST_RUN) return;
    const double alpha = ks->alpha;
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const double t = r[i] - alpha * v[i];
        s[i] = t;
        acc[0] += t * t;
    }
    block_partials<1>(acc, part, kMaxGrid);
}

// Zero the completion flags and the ticket counter of the apply + SpMV launch.
__global__ __launch_bounds__(256) void k_fuse_reset(int nsub, uint32_t *__restrict__ flag,
                                                   unsigned long long *__restrict__ ticket) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsub) flag[i] = 0u;
    if (i == 0) *ticket = 0ull;
}

// x += alpha p^ when the half step converged
__global__ __launch_bounds__(kRedT) void k_half(int64_t m, double *__restrict__ x, const double *__restrict__ ph,
                                               KrylovScalars *__restrict__ ks) {
    if (ks->state != ST_HALF) return;
    const double alpha = ks->alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += alpha * ph[i];
}

// x += alpha p^ + omega s^;  r = s - omega t;  partials r.r and r0.r
__global__ __launch_bounds__(kRedT) void k_update(int64_t m, double *__restrict__ x, const double *__restrict__ ph,
                                                 const double *__restrict__ sh, double *__restrict__ r,
                                                 const double *__restrict__ s, const double *__restrict__ t,
                                                 const double *__restrict__ r0, const KrylovScalars *__restrict__ ks,
                                                 double *__restrict__ part) {
    if (ks->state != ST_RUN) return;
    const double alpha = ks->alpha, omega = ks->omega;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * ph[i] + omega * sh[i];
        const double rn = s[i] - omega * t[i];
        r[i] = rn;
        acc[0] += rn * rn;
        acc[1] += r0[i] * rn;
    }
    block_partials<2>(acc, part, kMaxGrid);
}

// p = r + beta (p - omega v).  PAIR: each thread takes pairs of values as
// 16-byte accesses (m even, the vectors 16-byte aligned), the same
// arithmetic per value; there is no reduction, so the result is the same.
template <bool PAIR>
__global__ __launch_bounds__(kRedT) void k_pupdate(int64_t m, double *__restrict__ p, const double *__restrict__ r,
                                                  const double *__restrict__ v, KrylovScalars *__restrict__ ks) {
    const int32_t st0 = ks->state;
    if (st0 != ST_RUN) {
        // The half step converged in this iteration and k_half has added
        // alpha p^ to x: mark the solve converged (every workgroup returns
        // whichever of the two values it reads), so that the batch's later
        // iterations leave x alone.
        if (st0 == ST_HALF && blockIdx.x == 0 && threadIdx.x == 0) ks->state = ST_CONV;
        return;
    }
    const double beta = ks->beta, omega = ks->omega;
    if constexpr (PAIR) {
        double2 *__restrict__ p2 = reinterpret_cast<double2 *>(p);
        const double2 *__restrict__ r2 = reinterpret_cast<const double2 *>(r);
        const double2 *__restrict__ v2 = reinterpret_cast<const double2 *>(v);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m / 2;
             i += (int64_t)gridDim.x * blockDim.x) {
            double2 pp = p2[i];
            const double2 rr = r2[i], vv = v2[i];
            pp.x = rr.x + beta * (pp.x - omega * vv.x);
            pp.y = rr.y + beta * (pp.y - omega * vv.y);
            p2[i] = pp;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = r[i] + beta * (p[i] - omega * v[i]);
    }
}

// Fixed-order sum of nblk partials of slot k.
// Scalar step: one workgroup of kScalT threads sums the partials of one or
// two dot products.  Thread t adds entries t + (j*kScalU + u)*kScalT into
// accumulator u (kScalU x kScalB independent loads in flight per thread), then the
// accumulators, the wavefront and the wavefronts are combined in a fixed
// order, so the result does not depend on timing.
constexpr int kScalT = 1024;
constexpr int kScalU = 4;
constexpr int kScalB = 4;

template <int NS>
__device__ void reduce_slots(const double *part, int nblk, int stride, double (&out)[NS]) {
    __shared__ double sh[2][kScalT / kWave];
    double acc[NS][kScalU];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int u = 0; u < kScalU; ++u) acc[k][u] = 0.0;
    // kScalB passes of that loop have their loads issued together (the
    // additions keep the same order, so the sums do not change)
    for (int i0 = threadIdx.x; i0 < nblk; i0 += kScalT * kScalU * kScalB) {
        double v[kScalB][kScalU][NS];
#pragma unroll
        for (int b = 0; b < kScalB; ++b)
#pragma unroll
            for (int u = 0; u < kScalU; ++u) {
                const int i = i0 + (b * kScalU + u) * kScalT;
#pragma unroll
                for (int k = 0; k < NS; ++k) v[b][u][k] = i < nblk ? part[(int64_t)k * stride + i] : 0.0;
            }
#pragma unroll
        for (int b = 0; b < kScalB; ++b)
#pragma unroll
            for (int u = 0; u < kScalU; ++u)
                if (i0 + (b * kScalU + u) * kScalT < nblk)
#pragma unroll
                    for (int k = 0; k < NS; ++k) acc[k][u] += v[b][u][k];
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double t = acc[k][0];
#pragma unroll
        for (int u = 1; u < kScalU; ++u) t += acc[k][u];
        t = wave_sum(t);
        if (lane == 0) sh[k][w] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double t = 0.0;
        for (int i = 0; i < kScalT / kWave; ++i) t += sh[k][i];
        out[k] = t;
    }
}

constexpr int kMaxRestarts = 4;  // true-residual restarts per solve

enum : int { SC_INIT = 0, SC_ALPHA = 1, SC_S = 2, SC_OMEGA = 3, SC_BETA = 4, SC_TRUE = 5, SC_RESTART = 6 };

// Scalar steps of Algorithm 1 (one workgroup).
__global__ __launch_bounds__(kScalT) void k_scalars(int stage, int it, const double *part, int nblk, int stride,
                                                   KrylovScalars *ks, double *hist, int hist_len) {
    const int32_t st0 = ks->state;
    if (stage != SC_INIT && stage != SC_TRUE && stage != SC_RESTART && st0 != ST_RUN) return;
    double a, b = 0.0;
    if (stage == SC_INIT || stage == SC_OMEGA || stage == SC_BETA) {
        double ab[2];
        reduce_slots<2>(part, nblk, stride, ab);
        a = ab[0];
        b = ab[1];
    } else {
        double a1[1];
        reduce_slots<1>(part, nblk, stride, a1);
        a = a1[0];
    }
    if (threadIdx.x != 0) return;
    switch (stage) {
        case SC_INIT: {  // a = r.r (= r0.r), b = b.b
            double bn = sqrt(b);
            if (bn == 0.0) bn = 1.0;
            ks->bnorm = bn;
            ks->tol = ks->tol * bn;  // tol holds rtol on entry
            ks->rho = a;
            ks->rnorm = sqrt(a);
            ks->iters = 0;
            ks->state = (sqrt(a) <= ks->tol) ? ST_CONV : ST_RUN;
            if (!isfinite(a)) ks->state = DD_EBREAKDOWN;
            if (hist && hist_len > 0) hist[0] = sqrt(a) / bn;
            break;
        }
        case SC_ALPHA: {  // a = r0.v
            ks->iters = it;
            if (a == 0.0 || !isfinite(a) || ks->rho == 0.0) {
                ks->state = DD_EBREAKDOWN;
            } else {
                ks->alpha = ks->rho / a;
            }
            break;
        }
        case SC_S: {  // a = s.s
            const double sn = sqrt(a);
            ks->snorm = sn;
            if (sn <= ks->tol) {
                ks->rnorm = sn;
                ks->state = ST_HALF;
                ks->half = 1;
                if (hist && it < hist_len) hist[it] = sn / ks->bnorm;
            }
            break;
        }
        case SC_OMEGA: {  // a = t.s, b = t.t
            if (b == 0.0 || !isfinite(b)) {
                ks->state = DD_EBREAKDOWN;
            } else {
                ks->omega = a / b;
            }
            break;
        }
        case SC_BETA: {  // a = r.r, b = r0.r
            const double rn = sqrt(a);
            ks->rnorm = rn;
            if (hist && it < hist_len) hist[it] = rn / ks->bnorm;
            if (!isfinite(rn)) {
                ks->state = DD_EBREAKDOWN;
            } else if (rn <= ks->tol) {
                ks->state = ST_CONV;
            } else if (ks->omega == 0.0) {
                ks->state = DD_EBREAKDOWN;
            } else {
                ks->beta = (b / ks->rho) * (ks->alpha / ks->omega);
                ks->rho = b;
                if (it >= ks->maxit) ks->state = DD_ENOCONV;
            }
            break;
        }
        case SC_TRUE: {  // a = ||b - A x||^2
            ks->snorm = sqrt(a);  // reused slot: true residual norm
            break;
        }
        case SC_RESTART: {  // a = r.r of r = b - A x (iteration count, ||b|| and tol kept)
            ks->rho = a;
            ks->rnorm = sqrt(a);
            ks->half = 0;
            ks->state = (sqrt(a) <= ks->tol) ? ST_CONV : ST_RUN;
            if (!isfinite(a)) ks->state = DD_EBREAKDOWN;
            break;
        }
    }
}

// out[i] = in[map[i]] per block row
__global__ void k_permute(int64_t n, int bs, const int32_t *map, const double *in, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * bs) return;
    const int64_t i = e / bs;
    const int c = (int)(e - i * bs);
    out[e] = in[(int64_t)map[i] * bs + c];
}

hipError_t launch_permute(int64_t n, int bs, const int32_t *map, const double *in, double *out, hipStream_t st) {
    const int T = 256;
    k_permute<<<(unsigned)((n * bs + T - 1) / T), T, 0, st>>>(n, bs, map, in, out);
    return hipGetLastError();
}

#define KCHK(x)                                                                             \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) return h->fail(DD_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

template <int BS>
static int run_typed(dd_ctx *h, const KrylovWork &W, const double *b, double *x, double rtol, int32_t maxit,
                     hipStream_t st, dd_solve_info *info) {
    const int64_t n = h->n;
    const int64_t m = n * BS;
    double *V = W.kv;
    double *bp = V + 0 * m, *xp = V + 1 * m, *r = V + 2 * m, *r0 = V + 3 * m, *p = V + 4 * m;
    double *ph = V + 5 * m, *v = V + 6 * m, *s = V + 7 * m, *shat = V + 8 * m, *t = V + 9 * m;
    double *part = W.partials;
    KrylovScalars *ks = W.ks;
    KrylovScalars *ks_host = W.ks_host;
    const int32_t *state = &ks->state;
    // events (solve timing, per-apply profiling) and the fused launch only
    // with the handle's own workspace
    const bool own = W.handle_owned;
    const bool profile = own && h->profile;

    const int gsp = spmv_partials(h);  // SpMV workgroups, and the partial sums they leave
    const int gvec = (int)std::min<int64_t>((m + kRedT - 1) / kRedT, kMaxGrid);
    const bool pair = m % 2 == 0 && ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(r) |
                                      reinterpret_cast<uintptr_t>(v)) & 15) == 0;
    const int sps = W.part_stride;
    // apply + SpMV in one launch (partials one per subdomain) where the
    // handle allows it; the flags and the ticket counter start at zero
    const bool fused = own && h->fuse && !fused_unsupported(h);
    const int gpart = fused ? h->nsub : gsp;
    uint32_t fepoch = 0;
    unsigned long long ftick = 0;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::chrono::steady_clock::time_point h0;
    if (own) {
        KCHK(hipEventCreate(&e0));
        KCHK(hipEventCreate(&e1));
        KCHK(hipEventRecord(e0, st));
    } else {  // host clock from an idle stream to the final synchronisation
        KCHK(hipStreamSynchronize(st));
        h0 = std::chrono::steady_clock::now();
    }

    KrylovScalars init{};
    init.tol = rtol;
    init.maxit = maxit;
    init.state = ST_RUN;
    *ks_host = init;
    KCHK(hipMemcpyAsync(ks, ks_host, sizeof(KrylovScalars), hipMemcpyHostToDevice, st));
    if (fused) k_fuse_reset<<<(h->nsub + 255) / 256, 256, 0, st>>>(h->nsub, h->fflag, h->fticket);
    KCHK(launch_permute(n, BS, h->new2old, b, bp, st));
    KCHK(launch_permute(n, BS, h->new2old, x, xp, st));
    // r = b - A x0, r0 = p = r; rho = r0.r
    spmv_dots<BS, 2>(h, gsp, xp, t, bp, r, r0, p, part, sps, nullptr, st);
    k_scalars<<<1, kScalT, 0, st>>>(SC_INIT, 0, part, gsp, sps, ks, h->hist, h->hist_len);
    KCHK(hipGetLastError());

    const int chunk = 8;
    if (profile && (int)h->events.size() < 4 * chunk) {
        while ((int)h->events.size() < 4 * chunk) {
            hipEvent_t ev;
            // timing only (read after the stream synchronises): no system-scope
            // fence, whose cache writeback and invalidation would slow the
            // kernel after each event and inflate the time it measures
            KCHK(hipEventCreateWithFlags(&ev, hipEventDisableSystemFence));
            h->events.push_back(ev);
        }
    }
    int it = 0, applies = 0, chunk_first = 1, chunk_todo = 0, restarts = 0;
    double apply_ms = 0.0;
    int32_t final_state = ST_RUN;
    for (;;) {  // restarts
        chunk_todo = 0;
        while (true) {
            KCHK(hipMemcpyAsync(ks_host, ks, sizeof(KrylovScalars), hipMemcpyDeviceToHost, st));
            KCHK(hipStreamSynchronize(st));
            final_state = ks_host->state;
            if (profile) {  // applies of the finished chunk that did work
                const KrylovScalars &hk = *ks_host;
                for (int k = 0; k < chunk_todo; ++k) {
                    const int itk = chunk_first + k;
                    if (itk > hk.iters) break;
                    for (int a = 0; a < 2; ++a) {
                        if (a == 1 && itk == hk.iters && final_state != ST_RUN && hk.half) continue;
                        float ms = 0.f;
                        KCHK(hipEventElapsedTime(&ms, h->events[4 * k + 2 * a], h->events[4 * k + 2 * a + 1]));
                        apply_ms += ms;
                        ++applies;
                    }
                }
            }
            if (final_state != ST_RUN || it >= maxit) break;
            const int todo = std::min(chunk, maxit - it);
            chunk_first = it + 1;
            chunk_todo = todo;
            for (int k = 0; k < todo; ++k) {
                ++it;
                if (fused) {  // p^ = M^{-1} p and v = A p^, r0.v in one launch
                    KCHK(launch_apply_spmv(h, 0, p, ph, v, r0, part, sps, ++fepoch, ftick, &ks->state, st));
                    ftick += 2ull * h->nsub;
                } else {
                    KCHK(launch_precond(h, p, ph, state, st, profile ? h->events[4 * k] : nullptr,
                                        profile ? h->events[4 * k + 1] : nullptr));  // p^ = M^{-1} p
                    spmv_dots<BS, 0>(h, gsp, ph, v, r0, nullptr, nullptr, nullptr, part, sps, state,
                                     st);  // v = A p^, r0.v
                }
                k_scalars<<<1, kScalT, 0, st>>>(SC_ALPHA, it, part, gpart, sps, ks, h->hist, h->hist_len);
                k_axpy_s<<<gvec, kRedT, 0, st>>>(m, r, v, s, ks, part);        // s = r - alpha v
                k_scalars<<<1, kScalT, 0, st>>>(SC_S, it, part, gvec, kMaxGrid, ks, h->hist, h->hist_len);
                k_half<<<gvec, kRedT, 0, st>>>(m, xp, ph, ks);
                if (fused) {  // s^ = M^{-1} s and t = A s^, t.s, t.t in one launch
                    KCHK(launch_apply_spmv(h, 1, s, shat, t, s, part, sps, ++fepoch, ftick, &ks->state, st));
                    ftick += 2ull * h->nsub;
                } else {
                    KCHK(launch_precond(h, s, shat, state, st, profile ? h->events[4 * k + 2] : nullptr,
                                        profile ? h->events[4 * k + 3] : nullptr));  // s^ = M^{-1} s
                    spmv_dots<BS, 1>(h, gsp, shat, t, s, nullptr, nullptr, nullptr, part, sps, state,
                                     st);  // t = A s^, t.s, t.t
                }
                k_scalars<<<1, kScalT, 0, st>>>(SC_OMEGA, it, part, gpart, sps, ks, h->hist, h->hist_len);
                k_update<<<gvec, kRedT, 0, st>>>(m, xp, ph, shat, r, s, t, r0, ks, part);
                k_scalars<<<1, kScalT, 0, st>>>(SC_BETA, it, part, gvec, kMaxGrid, ks, h->hist, h->hist_len);
                if (pair)
                    k_pupdate<true><<<gvec, kRedT, 0, st>>>(m, p, r, v, ks);
                else
                    k_pupdate<false><<<gvec, kRedT, 0, st>>>(m, p, r, v, ks);
                KCHK(hipGetLastError());
            }
        }
        // true residual ||b - A x|| / ||b||
        spmv_dots<BS, 3>(h, gsp, xp, t, bp, nullptr, nullptr, nullptr, part, sps, nullptr, st);
        k_scalars<<<1, kScalT, 0, st>>>(SC_TRUE, 0, part, gsp, sps, ks, h->hist, h->hist_len);
        KCHK(hipMemcpyAsync(ks_host, ks, sizeof(KrylovScalars), hipMemcpyDeviceToHost, st));
        KCHK(hipStreamSynchronize(st));
        // The recurrence met the tolerance but the true residual did not (an
        // FP32 trisolve makes the preconditioner slightly inconsistent from one
        // apply to the next): restart from the current iterate.
        {
            const KrylovScalars &hk = *ks_host;
            if (hk.state == ST_CONV && hk.snorm > 2.0 * hk.tol && restarts < kMaxRestarts && it < maxit) {
                ++restarts;
                spmv_dots<BS, 2>(h, gsp, xp, t, bp, r, r0, p, part, sps, nullptr, st);
                k_scalars<<<1, kScalT, 0, st>>>(SC_RESTART, 0, part, gsp, sps, ks, h->hist, h->hist_len);
                KCHK(hipGetLastError());
                continue;
            }
        }
        break;
    }  // restarts
    if (own) KCHK(hipEventRecord(e1, st));
    KCHK(launch_permute(n, BS, h->old2new, xp, x, st));
    KCHK(hipStreamSynchronize(st));
    float ms = 0.f;
    if (own) {
        KCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } else {
        ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - h0).count();
    }
    const KrylovScalars &hk = *ks_host;
    int status = DD_OK;
    if (hk.state == kWaitFailed)
        return h->fail(DD_EHIP, "bicgstab_solve: a wait of the apply + SpMV launch exhausted its bound");
    if (hk.state == ST_CONV) status = hk.snorm > 2.0 * hk.tol ? DD_ENOCONV : DD_OK;  // restarts exhausted
    else if (hk.state == DD_EBREAKDOWN) status = DD_EBREAKDOWN;
    else status = DD_ENOCONV;
    if (info) {
        info->iters = hk.iters;
        info->status = status;
        info->rel_res = hk.rnorm / hk.bnorm;
        info->rel_res_true = hk.snorm / hk.bnorm;
        info->solve_seconds = ms * 1e-3;
        info->applies = applies;
        info->restarts = restarts;
        info->apply_seconds = apply_ms * 1e-3;
        info->fused = fused ? 1 : 0;
        info->fallback = 0;
    }
    if (status == DD_EBREAKDOWN) return h->fail(DD_EBREAKDOWN, "BiCGSTAB breakdown at iteration %d", hk.iters);
    if (status == DD_ENOCONV && hk.state == ST_CONV)
        return h->fail(DD_ENOCONV, "BiCGSTAB true residual %.3e stays above 2 rtol after %d restarts",
                       hk.snorm / hk.bnorm, restarts);
    if (status == DD_ENOCONV)
        return h->fail(DD_ENOCONV, "BiCGSTAB did not reach rtol within %d iterations (rel res %.3e)", maxit,
                       hk.rnorm / hk.bnorm);
    return DD_OK;
}

int krylov_workspace(dd_ctx *h, KrylovWork *w) {
    if (!h->kv) {
        int rc = h->alloc(&h->kv, kKrylovVectors * h->n * h->bs);
        if (rc) return rc;
        const int rpb = (kWave / h->bs) * (kRedT / kWave);
        h->spmv_part_stride = (int)std::max<int64_t>((h->n + rpb - 1) / rpb, kMaxGrid);
        rc = h->alloc(&h->partials, (int64_t)kStride * h->spmv_part_stride);
        if (rc) return rc;
        rc = h->alloc(&h->ks, 1);
        if (rc) return rc;
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&h->ks_host), sizeof(KrylovScalars));
        if (e != hipSuccess) {
            h->ks_host = nullptr;
            h->kv = nullptr;  // the next call tries again (the buffers stay recorded for dd_destroy)
            return h->fail(DD_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        }
    }
    w->kv = h->kv;
    w->partials = h->partials;
    w->part_stride = h->spmv_part_stride;
    w->ks = h->ks;
    w->ks_host = h->ks_host;
    w->handle_owned = true;
    return DD_OK;
}

// The fixed workspace of bicgstab_solve_noalloc: one array per device (each
// device that loads the library holds its own copy until the process ends).
// Kernels never name it: the host takes each device's address of it once,
// with that device current, and passes that address as it passes the
// handle's own workspace.  Every call on a device shares its array, so calls
// that overlap on one device race.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

int noalloc_workspace(dd_ctx *h, KrylovWork *w, KrylovScalars *host) {
    const int rpb = (kWave / h->bs) * (kRedT / kWave);
    const int64_t stride = std::max<int64_t>((h->n + rpb - 1) / rpb, kMaxGrid);
    const int64_t vec_bytes = align256((int64_t)kKrylovVectors * h->n * h->bs * (int64_t)sizeof(double));
    const int64_t part_bytes = align256((int64_t)kStride * stride * (int64_t)sizeof(double));
    const int64_t need = vec_bytes + part_bytes + align256(sizeof(KrylovScalars));
    if (need > kNoallocBytes)
        return h->fail(DD_EINVAL,
                       "bicgstab_solve_noalloc: the problem needs %lld bytes of Krylov workspace, the fixed array "
                       "holds %lld (at most about %lld values of n*bs)",
                       (long long)need, (long long)kNoallocBytes,
                       (long long)((kNoallocBytes - part_bytes - 256) / (kKrylovVectors * (int64_t)sizeof(double))));
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return h->fail(DD_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return h->fail(DD_EINVAL, "bicgstab_solve_noalloc: device %d", dev);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || p == nullptr) {
                (void)hipGetLastError();
                return h->fail(DD_EHIP, "hipGetSymbolAddress of the fixed workspace on device %d: %s", dev,
                               hipGetErrorString(e));
            }
            g_scratch_ptr[dev] = p;
        }
        base = g_scratch_ptr[dev];
    }
    unsigned char *b = static_cast<unsigned char *>(base);
    w->kv = reinterpret_cast<double *>(b);
    w->partials = reinterpret_cast<double *>(b + vec_bytes);
    w->part_stride = (int32_t)stride;
    w->ks = reinterpret_cast<KrylovScalars *>(b + vec_bytes + part_bytes);
    w->ks_host = host;
    w->handle_owned = false;
    return DD_OK;
}

int bicgstab_run(dd_ctx *h, const KrylovWork &w, const double *b, double *x, double rtol, int32_t maxit,
                 hipStream_t st, dd_solve_info *info) {
    if (w.handle_owned) {
        build_spmv_layout(h, st);
        if (h->fuse && !h->fdep && !fused_unsupported(h)) {
            int rc = h->alloc(&h->fdep, 2 * (int64_t)h->nsub);
            if (!rc) rc = h->alloc(&h->fflag, h->nsub);
            if (!rc) rc = h->alloc(&h->fticket, 1);
            if (rc) return rc;
            hipError_t e = launch_dep_range(h, st);
            if (e != hipSuccess) return h->fail(DD_EHIP, "dependency ranges: %s", hipGetErrorString(e));
        }
    }
    return h->bs == 3 ? run_typed<3>(h, w, b, x, rtol, maxit, st, info)
                      : run_typed<1>(h, w, b, x, rtol, maxit, st, info);
}

}  // namespace ddilu
