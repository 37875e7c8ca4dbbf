// Row kernels of the BSR SpMV, shared by the SpMV launches of the Krylov
// driver and by the apply launch that runs the product behind the apply.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ddilu {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// --------------------------------------------------------------- SpMV
// BS lanes of one wavefront per block row, lane c computes component c.
// The first kUnroll blocks of a row (a 7-point stencil row has at most 7)
// are fetched branch-free: column indices and block rows for all of them are
// issued together, positions past the row end re-read the row's last block
// (a valid address, same cache line) and are discarded by a select, so a row
// costs two memory round trips (A and col, then x) rather than one per block.
// Longer rows finish in a loop.
constexpr int kUnroll = 7;

template <int BS>
__device__ __forceinline__ double bsr_row(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                          const double *__restrict__ val, const double *__restrict__ x,
                                          int64_t row, int c) {
    constexpr int BB = BS * BS;
    const int32_t b0 = ptr[row], b1 = ptr[row + 1];
    const int nb = b1 - b0;
    int32_t idx[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) idx[k] = max(min(b0 + k, b1 - 1), 0);  // nnzb >= 1
    int32_t J[kUnroll];
    double v[kUnroll][BS];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) J[k] = col[idx[k]];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        const double *blk = val + (int64_t)idx[k] * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) v[k][d] = blk[d];
    }
    // keep the scheduler from sinking these loads next to their uses
    __builtin_amdgcn_sched_barrier(0);
    double xv[kUnroll][BS];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        const double *xb = x + (int64_t)J[k] * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) xv[k][d] = xb[d];
    }
    __builtin_amdgcn_sched_barrier(0);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        double t = 0.0;
#pragma unroll
        for (int d = 0; d < BS; ++d) t += v[k][d] * xv[k][d];
        acc += k < nb ? t : 0.0;
    }
    for (int32_t b = b0 + kUnroll; b < b1; ++b) {
        const int64_t Jb = col[b];
        const double *blk = val + (int64_t)b * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc += blk[d] * x[Jb * BS + d];
    }
    return acc;
}

// The same row product on the sliced ELL copy: slot (g, k, r) holds the k-th
// block of row g*RPW + r (column -1 and a zero block past the row's end), so
// the lanes of a wavefront read the k-th blocks of its RPW rows as one
// contiguous run.  Blocks are taken in the row's CSR order and an empty slot
// adds 0 exactly as in bsr_row, so both give the same bits.
template <int BS>
__device__ __forceinline__ double ell_row(const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                          const double *__restrict__ x, int64_t g, int r, int c) {
    constexpr int RPW = 64 / BS, BB = BS * BS;
    int32_t J[kUnroll];
    double v[kUnroll][BS];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) J[k] = ecol[(g * kUnroll + k) * RPW + r];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        const double *blk = eval + ((g * kUnroll + k) * RPW + r) * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) v[k][d] = blk[d];
    }
    __builtin_amdgcn_sched_barrier(0);
    double xv[kUnroll][BS];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        const double *xb = x + (int64_t)max(J[k], 0) * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) xv[k][d] = xb[d];
    }
    __builtin_amdgcn_sched_barrier(0);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        double t = 0.0;
#pragma unroll
        for (int d = 0; d < BS; ++d) t += v[k][d] * xv[k][d];
        acc += J[k] >= 0 ? t : 0.0;
    }
    return acc;
}

// Sliced ELL with one width per slice, for rows of more than kUnroll blocks.
// A slice is one wavefront's RPW rows; the rows of each SpMV workgroup (four
// slices) are stored longest first, so a slice's rows have similar lengths,
// and its width w (wavefront-uniform) is its longest row's length.  Slot
// (k, q) of the slice (at base + k*RPW + q) holds the k-th block of its q-th
// row.  Blocks are fetched in chunks of kSellChunk positions and one last
// chunk of w mod kSellChunk, each chunk straight-line code (column indices
// and blocks issued together, then x), so a slice issues loads for exactly w
// positions and waits twice per chunk.  A position past the row's own
// length re-reads the row's last block (a line the lane has just fetched)
// and adds 0.  Blocks are summed in the row's CSR order.  len >= 1.
constexpr int kSellChunk = 8;

template <int BS, int CH>
__device__ __forceinline__ void sell_chunk(const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                           const double *__restrict__ x, int64_t base, int k0, int q, int len,
                                           int c, double &acc) {
    constexpr int RPW = 64 / BS, BB = BS * BS;
    int32_t J[CH];
    double v[CH][BS];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int64_t s = base + (int64_t)min(k0 + j, len - 1) * RPW + q;
        J[j] = ecol[s];
        const double *blk = eval + s * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) v[j][d] = blk[d];
    }
    __builtin_amdgcn_sched_barrier(0);
    double xv[CH][BS];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const double *xb = x + (int64_t)J[j] * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) xv[j][d] = xb[d];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        double t = 0.0;
#pragma unroll
        for (int d = 0; d < BS; ++d) t += v[j][d] * xv[j][d];
        acc += k0 + j < len ? t : 0.0;
    }
}

// The same with the part's x in LDS (xs, rows row0 .. row0 + S - 1): a
// column inside the part reads LDS; every lane also issues the global load,
// at x_J for a column outside the part and at x_row0 (one line for the whole
// wavefront) inside it, so the chunk stays straight-line code.
template <int BS, int CH>
__device__ __forceinline__ void sell_chunk_lds(const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                               const double *__restrict__ x, const double *xs, int64_t row0, int S,
                                               int64_t base, int k0, int q, int len, int c, double &acc) {
    constexpr int RPW = 64 / BS, BB = BS * BS;
    int32_t J[CH];
    double v[CH][BS];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int64_t s = base + (int64_t)min(k0 + j, len - 1) * RPW + q;
        J[j] = ecol[s];
        const double *blk = eval + s * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) v[j][d] = blk[d];
    }
    __builtin_amdgcn_sched_barrier(0);
    double xl[CH][BS], xg[CH][BS];
    bool in[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int64_t jl = (int64_t)J[j] - row0;
        in[j] = jl >= 0 && jl < S;
        const double *xb = x + (in[j] ? row0 : (int64_t)J[j]) * BS;
        const double *lb = xs + (in[j] ? jl : 0) * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) {
            xg[j][d] = xb[d];
            xl[j][d] = lb[d];
        }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        double t = 0.0;
#pragma unroll
        for (int d = 0; d < BS; ++d) t += v[j][d] * (in[j] ? xl[j][d] : xg[j][d]);
        acc += k0 + j < len ? t : 0.0;
    }
}

// Chunks of four positions here: each holds both x candidates, and the
// part kernel's 1,024-lane workgroups leave 128 registers per lane.
constexpr int kSellChunkLds = 4;

template <int BS>
__device__ __forceinline__ double sell_row_lds(const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                               const double *__restrict__ x, const double *xs, int64_t row0, int S,
                                               int64_t base, int w, int q, int len, int c) {
    double acc = 0.0;
    int k0 = 0;
    for (; k0 + kSellChunkLds <= w; k0 += kSellChunkLds)
        sell_chunk_lds<BS, kSellChunkLds>(ecol, eval, x, xs, row0, S, base, k0, q, len, c, acc);
    switch (w - k0) {
        case 1: sell_chunk_lds<BS, 1>(ecol, eval, x, xs, row0, S, base, k0, q, len, c, acc); break;
        case 2: sell_chunk_lds<BS, 2>(ecol, eval, x, xs, row0, S, base, k0, q, len, c, acc); break;
        case 3: sell_chunk_lds<BS, 3>(ecol, eval, x, xs, row0, S, base, k0, q, len, c, acc); break;
        default: break;
    }
    return acc;
}

template <int BS>
__device__ __forceinline__ double sell_row(const int32_t *__restrict__ ecol, const double *__restrict__ eval,
                                           const double *__restrict__ x, int64_t base, int w, int q, int len,
                                           int c) {
    double acc = 0.0;
    int k0 = 0;
    for (; k0 + kSellChunk <= w; k0 += kSellChunk) sell_chunk<BS, kSellChunk>(ecol, eval, x, base, k0, q, len, c, acc);
    switch (w - k0) {
        case 1: sell_chunk<BS, 1>(ecol, eval, x, base, k0, q, len, c, acc); break;
        case 2: sell_chunk<BS, 2>(ecol, eval, x, base, k0, q, len, c, acc); break;
        case 3: sell_chunk<BS, 3>(ecol, eval, x, base, k0, q, len, c, acc); break;
        case 4: sell_chunk<BS, 4>(ecol, eval, x, base, k0, q, len, c, acc); break;
        case 5: sell_chunk<BS, 5>(ecol, eval, x, base, k0, q, len, c, acc); break;
        case 6: sell_chunk<BS, 6>(ecol, eval, x, base, k0, q, len, c, acc); break;
        case 7: sell_chunk<BS, 7>(ecol, eval, x, base, k0, q, len, c, acc); break;
        default: break;
    }
    return acc;
}

}  // namespace ddilu
