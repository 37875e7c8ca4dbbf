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

}  // namespace ddilu
