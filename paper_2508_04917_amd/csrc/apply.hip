// Fused domain-decomposed ILDU0 apply (Sections 4.2.2 and 4.4).
//
// One workgroup owns one subdomain.  The subdomain's vector lives in LDS for
// the whole apply: it is loaded once from r, transformed in place by the
// lower sweep (y = L^{-1} r), then by the upper sweep with the diagonal
// scaling folded in (z_I = inv_D_I y_I - sum_{K>I} Uhat_IK z_K), and
// stored once to z.  No workgroup waits on another.
//
// Each sweep walks the subdomain's levels; a barrier separates levels.  The
// factor blocks of a sweep are stored position by position in sweep order,
// so a workgroup reads its factor data as one forward stream.  Inside a
// level, BS consecutive lanes of one wavefront own one block row (lane c
// computes component c), so the BS lanes that read y_I and then overwrite it
// in the upper sweep belong to the same wavefront: all of its lanes issue
// their LDS reads before any lane issues the store.  64/BS rows per
// wavefront (21 for 3x3 blocks; the 64th lane idles).
//
// Types: TS is the storage type of the factor blocks (double or float), TC
// the type of the LDS vector and of the arithmetic (double for DD_FP64 and
// DD_MIXED, float for DD_FP32).  Input r and output z are always FP64.
#include <hip/hip_ext.h>

#include "internal.h"
#include "spmv.h"

// Prefetch depth (levels loaded ahead) of the slot-layout kernel, per factor
// storage type.  Once wavefronts without rows skip their loads, a level's
// time is mostly the latency of its own loads, which a deeper prefetch
// hides.  FP64 factors stop at 2: at 3 the four register sets of the upper
// sweep no longer fit the 128 registers a wavefront of a 1024-lane
// workgroup may hold.
#ifndef DDILU_PD64
#define DDILU_PD64 2
#endif
#ifndef DDILU_PD32
#define DDILU_PD32 3
#endif

namespace ddilu {

// Learned interface correction inside the apply: once the subdomain's r is
// in LDS, every row with cut faces adds sum_f C_f r_J (J in a neighbouring
// subdomain, read from r in global memory).  The work item is one
// (face, component) pair, and a subdomain's faces are stored rank-major: the
// first face of every row that has one (rank 0, rows ascending), then every
// row's second face (rank 1), and so on, each face as {local row, J} and its
// coefficient C_f, the copy of C in this order.  A lane takes up to
// kLicItems items; it fetches their records and coefficient rows before the
// subdomain's slice of r is loaded (lic_begin: nothing they read depends on
// the apply), their r_J once the records are in, and adds rank by rank with
// a barrier between ranks.  A row has at most one face of each rank, so no
// two items of a rank touch the same LDS entry, and every row adds its faces
// in CSR order (rank 0 first) whatever the number of passes: the item list
// is rank-major, so a pass holds the rest of one rank and a prefix of later
// ones.  One pass covers a subdomain of up to kLicItems * blockDim faces'
// components (at 16x20x20, 1,840 faces on 13 wavefronts).
struct LicArgs {
    const int32_t *fptr;    // [n+1] faces of each row (CSR order); fptr[s*S] = first face of subdomain s
    const int32_t *rb;      // [nsub*9] rank boundaries: faces of ranks < k of subdomain s at rb[9s + k]
    const int2 *lrec;       // [nf] rank-major faces {local row, J}
    const float *Cr;        // [nf*9] their coefficients C_f (row-major)
};

constexpr int kLicItems = 7;  // (face, component) items per lane and pass

template <int BS>
struct LicPass {
    int2 rec[kLicItems];
    float cf[kLicItems][BS];
    int item[kLicItems];
};

struct LicState {
    int32_t f0;   // first face of the subdomain
    int nitems;   // faces * BS
    int s;
};

// records and coefficient rows of items i0 + u*nt (positions past the end
// read item 0's, which exists when nitems > 0, and are not added)
template <int BS>
__device__ __forceinline__ void lic_fetch(LicPass<BS> &P, const LicArgs &la, const LicState &L, int i0, int nt) {
#pragma unroll
    for (int u = 0; u < kLicItems; ++u) {
        const int it = i0 + u * nt;
        P.item[u] = it;
        const int q = it < L.nitems ? it : 0;
        const int64_t f = L.f0 + q / BS;
        const int c = q % BS;
        P.rec[u] = la.lrec[f];
#pragma unroll
        for (int d = 0; d < BS; ++d) P.cf[u][d] = la.Cr[f * BS * BS + c * BS + d];
    }
}

template <int BS>
__device__ __forceinline__ void lic_begin(LicState &L, LicPass<BS> &P, int64_t base, int S, int s, const LicArgs &la,
                                          int tid, int nt) {
    L.s = s;
    L.f0 = la.fptr[base];
    L.nitems = (la.fptr[base + S] - L.f0) * BS;
    if (L.nitems > 0) lic_fetch<BS>(P, la, L, tid, nt);
}

// After the slice is in LDS and a barrier: r_J of the fetched items, the
// rank-ordered updates, further passes if the items did not fit one; then a
// barrier.
template <int BS, typename TC>
__device__ __forceinline__ void lic_finish(TC *__restrict__ y, const double *__restrict__ r, const LicState &L,
                                           LicPass<BS> &P, const LicArgs &la, int tid, int nt) {
    (void)tid;
    if (L.nitems == 0) return;  // uniform over the workgroup
    const int32_t *rb = la.rb + 9 * L.s;
    const int nf = L.nitems / BS;
    for (int p0 = 0;; p0 += kLicItems * nt) {  // passes: the same count for every lane
        double rv[kLicItems][BS];
#pragma unroll
        for (int u = 0; u < kLicItems; ++u)
#pragma unroll
            for (int d = 0; d < BS; ++d) rv[u][d] = r[(int64_t)P.rec[u].y * BS + d];
        // ranks present in this subdomain: k while rb[k] < nf (at most 8)
        for (int k = 0; k < 8 && rb[k] < nf; ++k) {
            const int lo = rb[k] * BS, hi = rb[k + 1] * BS;
#pragma unroll
            for (int u = 0; u < kLicItems; ++u) {
                const int it = P.item[u];
                if (it < L.nitems && it >= lo && it < hi) {
                    double t = 0.0;
#pragma unroll
                    for (int d = 0; d < BS; ++d) t += (double)P.cf[u][d] * rv[u][d];
                    const int c = it % BS;
                    y[P.rec[u].x * BS + c] += static_cast<TC>(t);
                }
            }
            __syncthreads();
        }
        if (p0 + kLicItems * nt >= L.nitems) break;
        lic_fetch<BS>(P, la, L, p0 + kLicItems * nt + tid, nt);
    }
}

// The subdomain's slice of r into LDS: each thread issues kLoadU loads
// before it waits for any (a plain strided loop would wait for every load
// in turn), positions past the end clamped to a valid one and not stored.
// With VEC, where the slice starts on a 16-byte boundary (an even number
// of values before it), pairs of values move as one 16-byte access: half as
// many load instructions for the same bytes in flight (an odd last value
// moves on its own).  The apply with the learned correction keeps the
// 8-byte accesses: with its face records in flight across the slice load,
// the paired form measured far slower there (368 against 284 us per apply).
constexpr int kLoadU = 8;
constexpr int kLoadU2 = kLoadU / 2;

template <typename TC>
struct Pair;
template <>
struct Pair<double> {
    using T = double2;
};
template <>
struct Pair<float> {
    using T = float2;
};

template <typename TC, bool VEC = false>
__device__ __forceinline__ void load_slice(TC *__restrict__ y, const double *__restrict__ rs, int m, int tid,
                                           int nt) {
    using P = typename Pair<TC>::T;
    if (VEC && (reinterpret_cast<uintptr_t>(rs) & 15) == 0) {  // uniform over the workgroup
        const int m2 = m >> 1;
        const double2 *__restrict__ r2 = reinterpret_cast<const double2 *>(rs);
        P *__restrict__ y2 = reinterpret_cast<P *>(y);
        for (int i0 = tid; i0 < m2; i0 += kLoadU2 * nt) {
            double2 v[kLoadU2];
#pragma unroll
            for (int u = 0; u < kLoadU2; ++u) v[u] = r2[min(i0 + u * nt, m2 - 1)];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < kLoadU2; ++u)
                if (i0 + u * nt < m2) {
                    P w;
                    w.x = static_cast<TC>(v[u].x);
                    w.y = static_cast<TC>(v[u].y);
                    y2[i0 + u * nt] = w;
                }
        }
        if ((m & 1) && tid == 0) y[m - 1] = static_cast<TC>(rs[m - 1]);
        return;
    }
    for (int i0 = tid; i0 < m; i0 += kLoadU * nt) {
        double v[kLoadU];
#pragma unroll
        for (int u = 0; u < kLoadU; ++u) v[u] = rs[min(i0 + u * nt, m - 1)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kLoadU; ++u)
            if (i0 + u * nt < m) y[i0 + u * nt] = static_cast<TC>(v[u]);
    }
}

// LDS back to the subdomain's slice of z, kLoadU values per thread at a
// time (with VEC in pairs where the slice starts on a 16-byte boundary).
template <typename TC, bool VEC = false>
__device__ __forceinline__ void store_slice(double *__restrict__ zs, const TC *__restrict__ y, int m, int tid,
                                            int nt) {
    using P = typename Pair<TC>::T;
    if (VEC && (reinterpret_cast<uintptr_t>(zs) & 15) == 0) {  // uniform over the workgroup
        const int m2 = m >> 1;
        double2 *__restrict__ z2 = reinterpret_cast<double2 *>(zs);
        const P *__restrict__ y2 = reinterpret_cast<const P *>(y);
        for (int i0 = tid; i0 < m2; i0 += kLoadU2 * nt) {
            P v[kLoadU2];
#pragma unroll
            for (int u = 0; u < kLoadU2; ++u) v[u] = y2[min(i0 + u * nt, m2 - 1)];
#pragma unroll
            for (int u = 0; u < kLoadU2; ++u)
                if (i0 + u * nt < m2) {
                    double2 w;
                    w.x = static_cast<double>(v[u].x);
                    w.y = static_cast<double>(v[u].y);
                    z2[i0 + u * nt] = w;
                }
        }
        if ((m & 1) && tid == 0) zs[m - 1] = static_cast<double>(y[m - 1]);
        return;
    }
    for (int i0 = tid; i0 < m; i0 += kLoadU * nt) {
        TC v[kLoadU];
#pragma unroll
        for (int u = 0; u < kLoadU; ++u) v[u] = y[min(i0 + u * nt, m - 1)];
#pragma unroll
        for (int u = 0; u < kLoadU; ++u)
            if (i0 + u * nt < m) zs[i0 + u * nt] = static_cast<double>(v[u]);
    }
}

// ------------------------------------------------------------------------
// Variant 1: plain level loop (levels of any width, rows of any length).
// The sweeps are shared with the ablation variants below.  VC selects the
// vertex-centric mapping (one thread per block row, all BS components)
// instead of BS lanes per row.
// acc[i] -= sum over the row's blocks b in [b0, b1) of block_b row (c0 + i)
// . y_{col b}, blocks in ascending order (the oracle's order).  The blocks
// come kRowChunk at a time with every load of a chunk issued before any is
// used: positions past the row's end re-read its last block and contribute a
// zero (a select, not a branch, so no load is sunk behind a condition), so a
// row costs one memory round trip per chunk instead of one per block.
constexpr int kRowChunk = 4;  // 8 measured slower (more re-read positions on short rows)

template <int BS, typename TS, typename TC, int NC>
__device__ __forceinline__ void row_blocks(TC (&acc)[NC], const TC *__restrict__ y, int32_t b0, int32_t b1,
                                           const uint16_t *__restrict__ col, const TS *__restrict__ val, int c0) {
    constexpr int BB = BS * BS;
    for (int32_t bb = b0; bb < b1; bb += kRowChunk) {
        int J[kRowChunk];
        TS v[kRowChunk][NC][BS];
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const int32_t b = min(bb + k, b1 - 1);
            J[k] = col[b];
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int d = 0; d < BS; ++d) v[k][i][d] = val[(int64_t)b * BB + (c0 + i) * BS + d];
        }
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) {
            const bool in = bb + k < b1;
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int d = 0; d < BS; ++d)
                    acc[i] -= (in ? static_cast<TC>(v[k][i][d]) : TC(0)) * y[J[k] * BS + d];
        }
    }
}

template <int NT, bool VC, int BS>
struct RowMap {
    static constexpr int RPW = kWave / BS;                     // block rows per wavefront (lane mapping)
    static constexpr int RPP = VC ? NT : RPW * (NT / kWave);  // block rows per pass of the workgroup
    int slot, c;
    bool ok;
    __device__ __forceinline__ RowMap() {
        const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
        slot = VC ? tid : wave * RPW + lane / BS;
        c = VC ? 0 : lane % BS;
        ok = VC || lane / BS < RPW;
    }
};

// y_I = y_I - sum_{J<I} L_IJ y_J, level by level.
template <int BS, typename TS, typename TC, int NT, bool VC>
__device__ __forceinline__ void plain_lower(TC *__restrict__ y, int64_t base, int s, const int32_t *__restrict__ Loff,
                                            const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow,
                                            const int32_t *__restrict__ Lbp, const uint16_t *__restrict__ Lcol,
                                            const TS *__restrict__ Lval) {
    const RowMap<NT, VC, BS> m;
    const int32_t o = Loff[s];
    const int nl = Loff[s + 1] - o - 1;
    for (int l = 0; l < nl; ++l) {
        const int32_t p0 = Llp[o + l], p1 = Llp[o + l + 1];
        for (int32_t pb = p0; pb < p1; pb += m.RPP) {
            const int32_t p = pb + m.slot;
            if (m.ok && p < p1) {
                const int64_t gp = base + p;
                const int I = Lrow[gp];
                const int32_t b1 = Lbp[gp + 1];
                if constexpr (VC) {
                    TC acc[BS];
#pragma unroll
                    for (int c = 0; c < BS; ++c) acc[c] = y[I * BS + c];
                    row_blocks<BS, TS, TC, BS>(acc, y, Lbp[gp], b1, Lcol, Lval, 0);
#pragma unroll
                    for (int c = 0; c < BS; ++c) y[I * BS + c] = acc[c];
                } else {
                    const int c = m.c;
                    TC acc[1] = {y[I * BS + c]};
                    row_blocks<BS, TS, TC, 1>(acc, y, Lbp[gp], b1, Lcol, Lval, c);
                    y[I * BS + c] = acc[0];
                }
            }
        }
        __syncthreads();
    }
}

// Upper sweep, level by level.  SCALE: z_I = inv_D_I y_I - sum_{K>I} Uhat_IK z_K
// (the diagonal scaling fused in); otherwise z_I = y_I - sum Uhat_IK z_K
// (unit diagonal, the scaling already applied).
template <int BS, typename TS, typename TC, int NT, bool VC, bool SCALE>
__device__ __forceinline__ void plain_upper(TC *__restrict__ y, int64_t base, int s, const int32_t *__restrict__ Uoff,
                                            const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow,
                                            const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol,
                                            const TS *__restrict__ Uval, const TS *__restrict__ Dval) {
    constexpr int BB = BS * BS;
    const RowMap<NT, VC, BS> m;
    const int32_t o = Uoff[s];
    const int nl = Uoff[s + 1] - o - 1;
    for (int l = 0; l < nl; ++l) {
        const int32_t p0 = Ulp[o + l], p1 = Ulp[o + l + 1];
        for (int32_t pb = p0; pb < p1; pb += m.RPP) {
            const int32_t p = pb + m.slot;
            if (m.ok && p < p1) {
                const int64_t gp = base + p;
                const int I = Urow[gp];
                const int32_t b1 = Ubp[gp + 1];
                if constexpr (VC) {
                    TC acc[BS];
#pragma unroll
                    for (int c = 0; c < BS; ++c) {
                        if constexpr (SCALE) {
                            acc[c] = 0;
#pragma unroll
                            for (int d = 0; d < BS; ++d)
                                acc[c] += static_cast<TC>(Dval[gp * BB + c * BS + d]) * y[I * BS + d];
                        } else {
                            acc[c] = y[I * BS + c];
                        }
                    }
                    row_blocks<BS, TS, TC, BS>(acc, y, Ubp[gp], b1, Ucol, Uval, 0);
#pragma unroll
                    for (int c = 0; c < BS; ++c) y[I * BS + c] = acc[c];
                } else {
                    const int c = m.c;
                    TC acc[1];
                    if constexpr (SCALE) {
                        const TS *dblk = Dval + gp * BB + c * BS;
                        acc[0] = 0;
#pragma unroll
                        for (int d = 0; d < BS; ++d) acc[0] += static_cast<TC>(dblk[d]) * y[I * BS + d];
                    } else {
                        acc[0] = y[I * BS + c];
                    }
                    row_blocks<BS, TS, TC, 1>(acc, y, Ubp[gp], b1, Ucol, Uval, c);
                    // every lane of this row has read y_I above (same wavefront)
                    __asm__ volatile("" ::: "memory");
                    y[I * BS + c] = acc[0];
                }
            }
        }
        __syncthreads();
    }
}

template <int BS, typename TS, typename TC, int NT, bool LIC>
__global__ __launch_bounds__(NT) void k_dd_apply(
    const double *__restrict__ r, double *__restrict__ z, int S,
    const int32_t *__restrict__ Loff, const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow,
    const int32_t *__restrict__ Lbp, const uint16_t *__restrict__ Lcol, const TS *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow,
    const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol, const TS *__restrict__ Uval,
    const TS *__restrict__ Dval, const int32_t *__restrict__ state, LicArgs la) {
    if (state != nullptr && *state != 0) return;  // enclosing solve already finished
    extern __shared__ unsigned char dd_smem[];
    TC *y = reinterpret_cast<TC *>(dd_smem);
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    LicState lst;
    LicPass<BS> lpass;
    if constexpr (LIC) lic_begin<BS>(lst, lpass, base, S, s, la, tid, NT);
    load_slice<TC>(y, r + base * BS, S * BS, tid, NT);
    __syncthreads();
    if constexpr (LIC) lic_finish<BS, TC>(y, r, lst, lpass, la, tid, NT);
    plain_lower<BS, TS, TC, NT, false>(y, base, s, Loff, Llp, Lrow, Lbp, Lcol, Lval);
    plain_upper<BS, TS, TC, NT, false, true>(y, base, s, Uoff, Ulp, Urow, Ubp, Ucol, Uval, Dval);
    store_slice<TC>(z + base * BS, y, S * BS, tid, NT);
}

// ------------------------------------------------------------------------
// Variant 2: rows in the CSR layout, levels of any width.  A sweep is a
// sequence of chunks — one workgroup pass of one level — with a barrier
// after the last chunk of each level only (the rows of a level are
// independent).  The factor data of a chunk does not depend on the solve,
// so it is fetched ahead: while chunk k computes from LDS, the blocks of
// chunk k+1 are in flight into registers and the row metadata of chunk k+2
// behind them.  The first MB blocks of a row are fetched without branches
// (positions past the row's end re-read its last block and contribute a
// zero through a select); rows with more blocks take the rest through a
// direct loop.
template <int BS, typename TS, int MB>
struct LevelRegs {
    bool ok;
    int I, b0, nb;
    int J[MB];
    TS v[MB][BS];
    TS d[BS];
};

struct LevelMeta {
    int64_t gp;
    bool ok;
    int I, b0, nb;
};

template <int BS, typename TS, int MB, bool UPPER>
__device__ __forceinline__ void csr_fetch(LevelRegs<BS, TS, MB> &R, const LevelMeta &m,
                                          const uint16_t *__restrict__ col, const TS *__restrict__ val,
                                          const TS *__restrict__ dval, int c) {
    constexpr int BB = BS * BS;
    R.ok = m.ok;
    R.I = m.I;
    R.b0 = m.b0;
    R.nb = m.nb;
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        const int64_t b = R.nb > 0 ? R.b0 + min(k, R.nb - 1) : 0;  // always a valid block
        R.J[k] = col[b];
        const TS *blk = val + b * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) R.v[k][d] = blk[d];
    }
    if constexpr (UPPER) {
        const TS *dblk = dval + (m.ok ? m.gp : 0) * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) R.d[d] = dblk[d];
    }
}

template <int BS, typename TS, typename TC, int MB, bool UPPER>
__device__ __forceinline__ void csr_compute(TC *__restrict__ y, const LevelRegs<BS, TS, MB> &R,
                                            const uint16_t *__restrict__ col, const TS *__restrict__ val, int c) {
    constexpr int BB = BS * BS;
    if (!R.ok) return;
    const int I = R.I;
    TC acc;
    if constexpr (UPPER) {
        acc = 0;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc += static_cast<TC>(R.d[d]) * y[I * BS + d];
    } else {
        acc = y[I * BS + c];
    }
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        const bool in = k < R.nb;
        const int J = R.J[k];
#pragma unroll
        for (int d = 0; d < BS; ++d) acc -= (in ? static_cast<TC>(R.v[k][d]) : TC(0)) * y[J * BS + d];
    }
    for (int k = MB; k < R.nb; ++k) {  // rows longer than the register window
        const int64_t b = R.b0 + k;
        const int J = col[b];
        const TS *blk = val + b * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc -= static_cast<TC>(blk[d]) * y[J * BS + d];
    }
    // all lanes of this row read y_I above (same wavefront)
    __asm__ volatile("" ::: "memory");
    y[I * BS + c] = acc;
}

// Position of a chunk: level l, first position pb of the pass, level end p1.
struct Chunk {
    int l;
    int32_t pb, p1;
};

template <int BS, typename TS, typename TC, int MB, bool UPPER>
__device__ __forceinline__ void sweep_csr(TC *__restrict__ y, int64_t base, int s, const int32_t *__restrict__ off,
                                          const int32_t *__restrict__ lp, const uint16_t *__restrict__ prow,
                                          const int32_t *__restrict__ bp, const uint16_t *__restrict__ col,
                                          const TS *__restrict__ val, const TS *__restrict__ dval, int slot,
                                          bool lane_ok, int c, int rpp) {
    const int32_t o = off[s];
    const int nl = off[s + 1] - o - 1;
    if (nl <= 0) return;
    auto next = [&](Chunk k) -> Chunk {
        k.pb += rpp;
        if (k.pb >= k.p1) {
            ++k.l;
            if (k.l < nl) {
                k.pb = lp[o + k.l];
                k.p1 = lp[o + k.l + 1];
            }
        }
        return k;
    };
    auto meta = [&](const Chunk &k) -> LevelMeta {
        LevelMeta m;
        const int32_t p = k.pb + slot;
        m.ok = lane_ok && k.l < nl && p < k.p1;
        m.gp = base + p;
        if (m.ok) {
            m.I = prow[m.gp];
            m.b0 = bp[m.gp];
            m.nb = bp[m.gp + 1] - m.b0;
        } else {
            m.I = 0;
            m.b0 = 0;
            m.nb = 0;
        }
        return m;
    };
    auto last_of_level = [&](const Chunk &k) { return k.pb + rpp >= k.p1; };
    // Two register sets alternate between "being computed" and "being
    // filled"; the loop is unrolled by two so that neither is copied (a copy
    // of a register with a load in flight would wait for the load).
    LevelRegs<BS, TS, MB> A, B;
    Chunk kA{0, lp[o], lp[o + 1]};
    LevelMeta mA = meta(kA);
    csr_fetch<BS, TS, MB, UPPER>(A, mA, col, val, dval, c);
    Chunk kB = next(kA);
    LevelMeta mB = meta(kB);
    while (kA.l < nl) {
        if (kB.l < nl) csr_fetch<BS, TS, MB, UPPER>(B, mB, col, val, dval, c);
        const Chunk kA2 = next(kB);
        if (kA2.l < nl) mA = meta(kA2);
        csr_compute<BS, TS, TC, MB, UPPER>(y, A, col, val, c);
        if (last_of_level(kA)) __syncthreads();
        if (kB.l >= nl) break;
        if (kA2.l < nl) csr_fetch<BS, TS, MB, UPPER>(A, mA, col, val, dval, c);
        const Chunk kB2 = next(kA2);
        if (kB2.l < nl) mB = meta(kB2);
        csr_compute<BS, TS, TC, MB, UPPER>(y, B, col, val, c);
        if (last_of_level(kB)) __syncthreads();
        kA = kA2;
        kB = kB2;
    }
}

template <int BS, typename TS, typename TC, int NT, int MB>
__global__ __launch_bounds__(NT) void k_dd_apply_pipe(
    const double *__restrict__ r, double *__restrict__ z, int S,
    const int32_t *__restrict__ Loff, const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow,
    const int32_t *__restrict__ Lbp, const uint16_t *__restrict__ Lcol, const TS *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow,
    const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol, const TS *__restrict__ Uval,
    const TS *__restrict__ Dval, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;
    constexpr int RPW = kWave / BS;
    extern __shared__ unsigned char dd_smem[];
    TC *y = reinterpret_cast<TC *>(dd_smem);
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int c = lane % BS, rl = lane / BS;
    const bool lane_ok = rl < RPW;
    const int slot = wave * RPW + rl;

    const double *rs = r + base * BS;
    load_slice<TC>(y, rs, S * BS, tid, NT);
    __syncthreads();
    constexpr int RPP = RPW * (NT / kWave);
    sweep_csr<BS, TS, TC, MB, false>(y, base, s, Loff, Llp, Lrow, Lbp, Lcol, Lval, nullptr, slot, lane_ok, c, RPP);
    sweep_csr<BS, TS, TC, MB, true>(y, base, s, Uoff, Ulp, Urow, Ubp, Ucol, Uval, Dval, slot, lane_ok, c, RPP);
    double *zs = z + base * BS;
    store_slice<TC>(zs, y, S * BS, tid, NT);
}

// ------------------------------------------------------------------------
// Variant 3: slot layout.  Position p's blocks sit in fixed slots
// p*MB..p*MB+MB-1 (zero blocks pad short rows), and its row and columns sit
// in one 64-bit descriptor.  No load depends on another load, so the loads of
// level l+PD are issued while level l computes: PD+1 register sets rotate,
// and the main loop is unrolled by PD+1 so that each set keeps its registers.
//
// A wavefront holding no row of a level skips that level's loads (about half
// of all wavefront-levels at 16x20x20 subdomains, whose levels run from 1 to
// 256 rows): the loads would only return zeros, and they cost issue slots of
// the vector memory pipeline the busy wavefronts need.  Because the number
// of loads a wavefront has in flight then depends on the level, the loads
// and their waits are written out here (the compiler's own waits, counted
// over both sides of the skip, would wait for the prefetched level too).
// The loads of one fetch are buffer loads behind one scalar branch on the
// wavefront's busy flag.  Before level l computes, the wavefront waits until
// only the loads of levels l+1..l+PD-1 it actually issued are outstanding,
// and then passes the registers of level l through an empty asm statement
// ("claim"), so that no read of them is scheduled before the wait.  The
// compiler does not know these registers are being loaded: the build checks
// the generated code, over its control-flow graph, for any instruction that
// touches a register between the load into it and its claim (a copy or a
// spill would read it before the data arrives).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Register image of the NB bytes one lane loads per position: 16-byte pieces,
// then an 8-byte and a 4-byte piece when NB is not a multiple of 16.
template <int NB>
struct RawRun {
    static constexpr int N16 = NB / 16;
    static constexpr bool T8 = (NB % 16) >= 8;
    static constexpr bool T4 = (NB % 8) >= 4;
    static constexpr int NLOAD = N16 + (T8 ? 1 : 0) + (T4 ? 1 : 0);
    u32x4 q[N16 > 0 ? N16 : 1];
    u32x2 h;
    uint32_t w;
};

template <int BS, typename TS, int MB, bool UPPER>
struct SlotRegs {
    static constexpr int NV = (MB + (UPPER ? 1 : 0)) * BS;  // values per lane and position
    static constexpr int NB = NV * (int)sizeof(TS);
    static constexpr int NLOAD = 1 + RawRun<NB>::NLOAD;    // descriptor + values
    bool ok;
    u32x2 desc;
    RawRun<NB> run;
};

// Buffer resource (base, byte size) in scalar registers.
__device__ __forceinline__ u32x4 slice_srd(const void *p, int64_t bytes) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    u32x4 r;
    r.x = (uint32_t)a;
    r.y = (uint32_t)(a >> 32) & 0xffffu;  // stride 0
    r.z = (uint32_t)bytes;
    r.w = 0x00020000u;                    // raw 32-bit data, as the buffer builtins use
    return r;
}

constexpr uint32_t kOobOffset = 0x80000000u;  // beyond every slice (slices < 2 GiB)

// One buffer load of a piece.  The destination is an in/out operand: on the
// path where the fetch is skipped it keeps its old (unused) value, so the
// compiler has no reason to copy it, and it cannot share a register with the
// offset, which is live across the loads of a fetch.
template <int OFF>
__device__ __forceinline__ void vm_load(u32x4 &d, uint32_t voff, const u32x4 &srd) {
    asm volatile("buffer_load_dwordx4 %[d], %[o], %[s], 0 offen offset:%[k]" : [d] "+v"(d) : [o] "v"(voff), [s] "s"(srd), [k] "n"(OFF));
}
template <int OFF>
__device__ __forceinline__ void vm_load(u32x2 &d, uint32_t voff, const u32x4 &srd) {
    asm volatile("buffer_load_dwordx2 %[d], %[o], %[s], 0 offen offset:%[k]" : [d] "+v"(d) : [o] "v"(voff), [s] "s"(srd), [k] "n"(OFF));
}
template <int OFF>
__device__ __forceinline__ void vm_load(uint32_t &d, uint32_t voff, const u32x4 &srd) {
    asm volatile("buffer_load_dword %[d], %[o], %[s], 0 offen offset:%[k]" : [d] "+v"(d) : [o] "v"(voff), [s] "s"(srd), [k] "n"(OFF));
}

// Wait until no vector memory operation is outstanding.
__device__ __forceinline__ void vm_wait_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wait until at most n*K vector memory operations are outstanding (n = 0, 1
// or 2, wavefront-uniform).
template <int K>
__device__ __forceinline__ void vm_wait_n(int n) {
    static_assert(K >= 0 && 2 * K < 64, "vmcnt has six bits");
    asm volatile(
        "s_cmp_eq_u32 %[n], 0\n\t"
        "s_cbranch_scc1 1f\n\t"
        "s_cmp_eq_u32 %[n], 1\n\t"
        "s_cbranch_scc1 2f\n\t"
        "s_waitcnt vmcnt(%[k2])\n\t"
        "s_branch 3f\n"
        "2:\n\t"
        "s_waitcnt vmcnt(%[k])\n\t"
        "s_branch 3f\n"
        "1:\n\t"
        "s_waitcnt vmcnt(0)\n"
        "3:"
        :
        : [n] "s"(__builtin_amdgcn_readfirstlane(n)), [k] "n"(K), [k2] "n"(2 * K)
        : "scc", "memory");
}

template <int I, int N>
struct LoadPieces {
    template <int NB>
    static __device__ __forceinline__ void run(RawRun<NB> &r, uint32_t off, const u32x4 &srd) {
        vm_load<16 * I>(r.q[I], off, srd);
        LoadPieces<I + 1, N>::run(r, off, srd);
    }
};
template <int N>
struct LoadPieces<N, N> {
    template <int NB>
    static __device__ __forceinline__ void run(RawRun<NB> &, uint32_t, const u32x4 &) {}
};

// Per position, the BS lanes of its row each read one contiguous run: lane c
// holds row c of every slot block (and, in the upper sweep, row c of inv_D).
// A lane without a row at the level passes an offset past the slice, for
// which the hardware returns zeros without a memory access (and no lane can
// address outside its subdomain's slice).
template <int BS, typename TS, int MB, bool UPPER>
__device__ __forceinline__ void slot_fetch(SlotRegs<BS, TS, MB, UPPER> &R, const u32x4 &srd_desc,
                                           const u32x4 &srd_val, int32_t p0, int32_t p1, int slot, bool lane_ok,
                                           int c, int busy) {
    using SR = SlotRegs<BS, TS, MB, UPPER>;
    using RR = RawRun<SR::NB>;
    const int32_t p = p0 + slot;
    R.ok = lane_ok && p < p1;
    const uint32_t pd = R.ok ? (uint32_t)p * 8u : kOobOffset;
    const uint32_t off = R.ok ? (uint32_t)((p * BS * SR::NV + c * SR::NV) * sizeof(TS)) : kOobOffset;
    if (busy) {
        vm_load<0>(R.desc, pd, srd_desc);
        LoadPieces<0, RR::N16>::run(R.run, off, srd_val);
        if constexpr (RR::T8) vm_load<16 * RR::N16>(R.run.h, off, srd_val);
        if constexpr (RR::T4) vm_load<16 * RR::N16 + (RR::T8 ? 8 : 0)>(R.run.w, off, srd_val);
    }
}

// Orders every later read of R's registers after the preceding wait.
template <int BS, typename TS, int MB, bool UPPER>
__device__ __forceinline__ void slot_claim(SlotRegs<BS, TS, MB, UPPER> &R) {
    using RR = RawRun<SlotRegs<BS, TS, MB, UPPER>::NB>;
    asm volatile("; claim %0" : "+v"(R.desc));
#pragma unroll
    for (int i = 0; i < RR::N16; ++i) asm volatile("; claim %0" : "+v"(R.run.q[i]));
    if constexpr (RR::T8) asm volatile("; claim %0" : "+v"(R.run.h));
    if constexpr (RR::T4) asm volatile("; claim %0" : "+v"(R.run.w));
}

// SEG: the segmented layout (15-bit descriptor fields, see Sweep).  A
// position computes the partial result of its segment: the owner (a row's
// first segment) starts from y_I (lower) or inv_D y_I (upper), a lower
// continuation from zero, an upper continuation from minus its extra block
// (in the inv_D slot) times z at the column its row field names; the owner
// then adds its continuations' partials, held by the next m - 1 positions
// of the same wavefront, in segment order through cross-lane reads, and
// alone writes the row.  All lanes take part in the reads (those without a
// position hold zero), so every value read is defined.
template <int BS, typename TS, typename TC, int MB, bool UPPER, bool SEG = false>
__device__ __forceinline__ void slot_compute(TC *__restrict__ y, const SlotRegs<BS, TS, MB, UPPER> &R, int c) {
    using SR = SlotRegs<BS, TS, MB, UPPER>;
    using RR = RawRun<SR::NB>;
    if constexpr (!SEG) {
        if (!R.ok) return;
    }
    uint32_t wd[SR::NB / 4];
#pragma unroll
    for (int i = 0; i < RR::N16; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) wd[4 * i + j] = R.run.q[i][j];
    if constexpr (RR::T8) {
        wd[4 * RR::N16] = R.run.h[0];
        wd[4 * RR::N16 + 1] = R.run.h[1];
    }
    if constexpr (RR::T4) wd[SR::NB / 4 - 1] = R.run.w;
    TS vals[SR::NV];
#pragma unroll
    for (int v = 0; v < SR::NV; ++v) {
        if constexpr (sizeof(TS) == 8)
            vals[v] = __builtin_bit_cast(TS, (uint64_t)wd[2 * v] | ((uint64_t)wd[2 * v + 1] << 32));
        else
            vals[v] = __builtin_bit_cast(TS, wd[v]);
    }
    const uint64_t desc = (uint64_t)R.desc[0] | ((uint64_t)R.desc[1] << 32);
    constexpr uint64_t FM = SEG ? 0x7fffu : 0xffffu;  // field mask; all ones = empty slot
    const int I = SEG && !R.ok ? 0 : (int)(desc & FM);
    // gather every LDS operand first (one round of LDS latency), then the
    // fixed-order arithmetic.  An empty slot holds a zero block: it is
    // applied to y_I (a valid LDS address) instead of being branched around.
    constexpr int NI = UPPER ? BS : 1;
    TC yi[NI], yj[MB][BS];
#pragma unroll
    for (int d = 0; d < NI; ++d) yi[d] = y[I * BS + (UPPER ? d : c)];
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        const int J = (int)((desc >> (16 * (k + 1))) & FM);
        const int Jc = (J != (int)FM && !(SEG && !R.ok)) ? J : I;
#pragma unroll
        for (int d = 0; d < BS; ++d) yj[k][d] = y[Jc * BS + d];
    }
    __builtin_amdgcn_sched_barrier(0);
    const bool cont = SEG && (((desc >> 15) & 1u) != 0 || !R.ok);
    TC acc;
    if constexpr (UPPER) {
        acc = 0;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc += static_cast<TC>(vals[MB * BS + d]) * yi[d];
        if constexpr (SEG)
            if (cont) acc = -acc;
    } else {
        acc = cont ? TC(0) : yi[0];
    }
#pragma unroll
    for (int k = 0; k < MB; ++k)
#pragma unroll
        for (int d = 0; d < BS; ++d) acc -= static_cast<TC>(vals[k * BS + d]) * yj[k][d];
    if constexpr (SEG) {
        if (!R.ok) acc = 0;
        const int m = cont ? 1
                           : 1 + (int)((desc >> 31) & 1u) + 2 * (int)((desc >> 47) & 1u) +
                                 4 * (int)((desc >> 63) & 1u);
        const int lane = threadIdx.x & (kWave - 1);
        for (int j = 1; j < kSegMax; ++j) {
            if (!__any(j < m)) break;  // wavefront-uniform
            const TC v = __shfl(acc, lane + BS * j);
            if (j < m) acc += v;
        }
        __asm__ volatile("" ::: "memory");
        if (!cont) y[I * BS + c] = acc;
    } else {
        // all lanes of this row read y_I above (same wavefront)
        __asm__ volatile("" ::: "memory");
        y[I * BS + c] = acc;
    }
}

// pbase, pcount: the subdomain's positions in the streams (s*S and S, or
// the segmented layout's offset and count).  SEG: the level table is the
// chunk table (starts in bits 0-29, bit 30 = barrier after the chunk).
template <int BS, typename TS, typename TC, int MB, int PD, bool UPPER, bool SEG = false>
__device__ __forceinline__ void sweep_slots(TC *__restrict__ y, int64_t pbase, int64_t pcount, int s,
                                            const int32_t *__restrict__ off, const int32_t *__restrict__ lp,
                                            const uint64_t *__restrict__ desc, const TS *__restrict__ sval,
                                            int slot, int wrow0, bool lane_ok, int c) {
    static_assert(PD >= 1 && PD <= 3, "prefetch depth 1 to 3");
    using SR = SlotRegs<BS, TS, MB, UPPER>;
    constexpr int PS = SR::NV * BS;  // values per position
    constexpr int32_t QM = SEG ? 0x3fffffff : 0x7fffffff;
    const u32x4 srd_desc = slice_srd(desc + pbase, pcount * 8);
    const u32x4 srd_val = slice_srd(sval + pbase * PS, pcount * PS * (int64_t)sizeof(TS));
    const int32_t o = off[s];
    const int nl = off[s + 1] - o - 1;
    SR R[PD + 1];
    int busy[PD + 1], bar[PD + 1];
    // level bounds are read one fetch ahead, so their scalar loads complete
    // during a level's update instead of after the barrier that follows it
    int32_t q0 = lp[o], q1 = lp[o + 1];
    auto fetch = [&](int k, int l) {
        const int32_t a0 = q0 & QM, a1 = q1 & QM;
        bar[k] = SEG ? (q0 >> 30) & 1 : 1;
        busy[k] = a0 + wrow0 < a1 ? 1 : 0;
        slot_fetch<BS, TS, MB, UPPER>(R[k], srd_desc, srd_val, a0, a1, slot, lane_ok, c, busy[k]);
        const int ln = l + 1 < nl ? l + 1 : nl - 1;
        q0 = lp[o + ln];
        q1 = lp[o + ln + 1];
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) fetch(u, u);
    const int nfull = nl - nl % (PD + 1);
    for (int l0 = 0; l0 < nfull; l0 += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) {
            // set u holds level l = l0+u; the loads issued after its own are
            // those of levels l+1..l+PD-1 (sets u+1..u+PD-1), by the
            // wavefronts that had rows there
            if constexpr (PD == 3)
                vm_wait_n<SR::NLOAD>(busy[(u + 1) % (PD + 1)] + busy[(u + 2) % (PD + 1)]);
            else if constexpr (PD == 2)
                vm_wait_n<SR::NLOAD>(busy[(u + 1) % (PD + 1)]);
            else
                vm_wait_all();
            slot_claim(R[u]);
            const int b = bar[u];
            fetch((u + PD) % (PD + 1), l0 + u + PD);
            slot_compute<BS, TS, TC, MB, UPPER, SEG>(y, R[u], c);
            if (b) __syncthreads();
        }
    }
    const int rem = nl - nfull;
#pragma unroll
    for (int u = 0; u < PD; ++u) {
        if (u < rem) {
            vm_wait_all();
            slot_claim(R[u]);
            slot_compute<BS, TS, TC, MB, UPPER, SEG>(y, R[u], c);
            if (bar[u]) __syncthreads();
        }
    }
    // nothing may still be loading into these registers once they are free
    vm_wait_all();
#pragma unroll
    for (int u = 0; u <= PD; ++u) slot_claim(R[u]);
}

// One subdomain's apply with the slot layout: r's slice into LDS (plus the
// learned correction), the lower sweep, the upper sweep with the diagonal
// scaling, and the slice back to z.
template <int BS, typename TS, typename TC, int MB, int PD, bool LIC, bool SEG = false>
__device__ __forceinline__ void apply_slots_sub(
    TC *__restrict__ y, int s, const double *__restrict__ r, double *__restrict__ z, int S,
    const int32_t *__restrict__ Loff, const int32_t *__restrict__ Llp, const uint64_t *__restrict__ Ldesc,
    const TS *__restrict__ Lval, const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp,
    const uint64_t *__restrict__ Udesc, const TS *__restrict__ Uval, const LicArgs &la,
    const int32_t *__restrict__ Lgpos = nullptr, const int32_t *__restrict__ Ugpos = nullptr) {
    constexpr int RPW = kWave / BS;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int c = lane % BS, rl = lane / BS;
    const bool lane_ok = rl < RPW;
    const int slot = wave * RPW + rl;

    // the launch may use fewer threads than the kernel's bound: just enough
    // wavefronts for the widest level, so no wavefront is idle at every level
    const int nt = blockDim.x;
    const double *rs = r + base * BS;
    LicState lst;
    LicPass<BS> lpass;
    if constexpr (LIC) lic_begin<BS>(lst, lpass, base, S, s, la, tid, nt);
    load_slice<TC, !LIC>(y, rs, S * BS, tid, nt);
    __syncthreads();
    if constexpr (LIC) lic_finish<BS, TC>(y, r, lst, lpass, la, tid, nt);
    const int wrow0 = __builtin_amdgcn_readfirstlane(wave) * RPW;  // first slot of this wavefront
    if constexpr (SEG) {
        const int64_t lb = Lgpos[s], ub = Ugpos[s];
        sweep_slots<BS, TS, TC, MB, PD, false, true>(y, lb, Lgpos[s + 1] - lb, s, Loff, Llp, Ldesc, Lval, slot,
                                                     wrow0, lane_ok, c);
        sweep_slots<BS, TS, TC, MB, PD, true, true>(y, ub, Ugpos[s + 1] - ub, s, Uoff, Ulp, Udesc, Uval, slot,
                                                    wrow0, lane_ok, c);
    } else {
        sweep_slots<BS, TS, TC, MB, PD, false>(y, base, S, s, Loff, Llp, Ldesc, Lval, slot, wrow0, lane_ok, c);
        sweep_slots<BS, TS, TC, MB, PD, true>(y, base, S, s, Uoff, Ulp, Udesc, Uval, slot, wrow0, lane_ok, c);
    }
    double *zs = z + base * BS;
    store_slice<TC, !LIC>(zs, y, S * BS, tid, nt);
}

template <int BS, typename TS, typename TC, int NT, int MB, int PD, bool LIC, bool SEG = false>
__global__ __launch_bounds__(NT) void k_dd_apply_slots(
    const double *__restrict__ r, double *__restrict__ z, int S, const int32_t *__restrict__ Loff,
    const int32_t *__restrict__ Llp, const uint64_t *__restrict__ Ldesc, const TS *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint64_t *__restrict__ Udesc,
    const TS *__restrict__ Uval, const int32_t *__restrict__ state, LicArgs la, int64_t vstride,
    const int32_t *__restrict__ Lgpos, const int32_t *__restrict__ Ugpos) {
    if (state != nullptr && *state != 0) return;
    extern __shared__ unsigned char dd_smem[];
    // right-hand side blockIdx.y of a batch stored one after another
    const int64_t off = (int64_t)blockIdx.y * vstride;
    apply_slots_sub<BS, TS, TC, MB, PD, LIC, SEG>(reinterpret_cast<TC *>(dd_smem), blockIdx.x, r + off, z + off, S,
                                                  Loff, Llp, Ldesc, Lval, Uoff, Ulp, Udesc, Uval, la, Lgpos, Ugpos);
}

// ------------------------------------------------------------------------
// The apply and the SpMV behind it (BiCGSTAB's y = A M^{-1} x) in one launch.
//
// Separate launches leave the chip half idle while the apply's last partial
// round of subdomains runs (640 subdomains on 256 CUs: the third round holds
// 128).  Here the launch has twice as many workgroups as subdomains; each
// takes a ticket from a device counter when it starts.  Tickets below nsub
// apply subdomain t; ticket nsub + k computes the product rows of subdomain
// k, after the subdomains its rows read (the range dep[2k]..dep[2k+1]) have
// finished.  All apply tickets are handed out before any product ticket, so
// a product workgroup only waits for workgroups that are already running
// and never wait themselves: every wait ends.  Each wait is still bounded;
// one that exhausts its bound sets the solve's state word to kWaitFailed
// (the solve returns an error) and releases the other waits.
//
// The price: every workgroup of the launch reserves the apply's LDS, so the
// product rows run at one workgroup per CU instead of the stand-alone SpMV's
// occupancy; at 160^3 (640 subdomains of 6400 rows) that loses more than the
// idle tail gives back (2.40 against 2.21 ms per BiCGSTAB iteration), which
// is why the solve uses it only on request.
//
// Visibility across the chip's L2 caches (one per XCD): an apply workgroup's
// wavefronts wait for their z stores to be acknowledged, meet at a barrier,
// and one lane publishes the subdomain's flag with a release store at agent
// scope (which writes the L2 back first).  A product workgroup's first
// wavefront polls the flags with relaxed agent-scope loads and then issues
// one agent-scope acquire fence (which invalidates the stale L1/L2 lines)
// before the barrier after which its rows read z.
struct FuseArgs {
    const int32_t *aptr, *acol;       // full reordered matrix
    const double *aval;
    double *y;                        // y = A z
    const double *w;                  // dot partner: r0 (mode 0) or s (mode 1)
    double *part;                     // partial sums [NV][part_stride], one per tile
    int32_t part_stride;
    int32_t nsub;
    const int32_t *dep;               // [2 nsub] lowest and highest subdomain a tile reads
    uint32_t *flag;                   // [nsub] epoch of the launch that last finished the subdomain
    unsigned long long *ticket;       // workgroup counter (zeroed at the start of each solve)
    unsigned long long ticket0;       // tickets handed out by the solve's earlier launches
    uint32_t epoch;                   // this launch's number within the solve (from 1)
    int32_t *state;                   // the solve's state word
};

constexpr int kWaitMax = 1 << 18;     // polls per flag (each at least 256 cycles apart)

template <int BS, typename TS, typename TC, int NT, int MB, int PD, bool LIC, int MODE>
__global__ __launch_bounds__(NT) void k_dd_apply_slots_spmv(
    const double *__restrict__ r, double *__restrict__ z, int S, const int32_t *__restrict__ Loff,
    const int32_t *__restrict__ Llp, const uint64_t *__restrict__ Ldesc, const TS *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint64_t *__restrict__ Udesc,
    const TS *__restrict__ Uval, LicArgs la, FuseArgs f) {
    constexpr int NV = MODE == 0 ? 1 : 2;
    __shared__ int ticket;
    __shared__ double red[NV][16];
    extern __shared__ unsigned char dd_smem[];
    if (threadIdx.x == 0) ticket = (int)(atomicAdd(f.ticket, 1ull) - f.ticket0);
    __syncthreads();
    const int t = ticket;
    const int nsub = f.nsub;
    // every workgroup has taken its ticket before this test, so the counter
    // advances by the grid size whether or not the solve is still running
    if (*f.state != 0) return;
    if ((unsigned)t >= 2u * (unsigned)nsub) {  // counter out of step with the host: fail the solve
        if (threadIdx.x == 0) __hip_atomic_store(f.state, kWaitFailed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (t < nsub) {
        apply_slots_sub<BS, TS, TC, MB, PD, LIC>(reinterpret_cast<TC *>(dd_smem), t, r, z, S, Loff, Llp, Ldesc,
                                                 Lval, Uoff, Ulp, Udesc, Uval, la);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) __hip_atomic_store(f.flag + t, f.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const int k = t - nsub;  // < nsub by the test above
    if (wave == 0) {
        const int lo = f.dep[2 * k], hi = f.dep[2 * k + 1];
        bool ok = true;
        for (int d = lo + lane; d <= hi && ok; d += kWave) {
            int polls = 0;
            while (__hip_atomic_load(f.flag + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != f.epoch) {
                if ((++polls & 63) == 0 &&
                    (polls > kWaitMax ||
                     __hip_atomic_load(f.state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
        }
        // the fence comes before the divergent store, so that the whole
        // wavefront executes it
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!ok) __hip_atomic_store(f.state, kWaitFailed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // rows of subdomain k, BS lanes per row as in the stand-alone SpMV
    constexpr int RPW = kWave / BS;
    const int c = lane % BS, rl = lane / BS;
    const int nw = blockDim.x / kWave;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    if (rl < RPW) {
        const int64_t row0 = (int64_t)k * S;
        for (int q = wave * RPW + rl; q < S; q += nw * RPW) {
            const int64_t row = row0 + q;
            const int64_t e = row * BS + c;
            const double tv = bsr_row<BS>(f.aptr, f.acol, f.aval, z, row, c);
            f.y[e] = tv;
            if constexpr (MODE == 0) {
                acc[0] += f.w[e] * tv;
            } else {
                acc[0] += tv * f.w[e];
                acc[1] += tv * tv;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double sum = wave_sum(acc[q]);
        if (lane == 0) red[q][wave] = sum;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double sum = 0.0;
            for (int i = 0; i < nw; ++i) sum += red[q][i];
            f.part[q * f.part_stride + k] = sum;
        }
    }
}

// ------------------------------------------------------------------------
// Ablation variants (FP64 factors and arithmetic, no learned correction).
// Each differs from the plain level loop (variant 1) in one respect, so that
// timing it against variant 1 isolates what that respect is worth on this
// GPU; together they recast the paper's kernel variants (Section 5.2 and
// Tables 3-4) for the lane-parallel mapping used here:
//   4  split: lower sweep + diagonal scaling, then the upper sweep with unit
//      diagonal, as two kernels with the intermediate vector in global memory
//      (the paper's ILD_U0 split against fused ILDU0);
//   5  no LDS: the subdomain's vector lives in z (global memory) throughout
//      (the paper's no_lds variant);
//   6  vertex-centric: one thread per block row computes all its components
//      (the paper's vertex-centric kernel) instead of BS lanes per row;
//   7  ILU0 form of the upper sweep: the U blocks as factored (same layout
//      and order as Uhat), and the row's sum is multiplied by inv(U_II) at
//      the end (the BS lanes of the row exchange their sums), instead of the
//      pre-scaled Uhat = inv(U_II) U of ILDU0 (the paper's ILU0 against
//      unit-diagonal ILDU0 comparison);
//   8  synchronisation-free sweeps (Algorithm 4): no level barriers, one
//      wavefront per row, each waiting on per-row completion flags in LDS.

// 4a: y = L^{-1} r, then w_I = inv_D_I y_I for every row, stored to z.
template <int BS, int NT>
__global__ __launch_bounds__(NT) void k_abl_lower_scale(
    const double *__restrict__ r, double *__restrict__ z, int S, const int32_t *__restrict__ Loff,
    const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow, const int32_t *__restrict__ Lbp,
    const uint16_t *__restrict__ Lcol, const double *__restrict__ Lval, const uint16_t *__restrict__ Urow,
    const double *__restrict__ Dval, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;
    constexpr int BB = BS * BS;
    extern __shared__ unsigned char dd_smem[];
    double *y = reinterpret_cast<double *>(dd_smem);
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    load_slice<double>(y, r + base * BS, S * BS, tid, NT);
    __syncthreads();
    plain_lower<BS, double, double, NT, false>(y, base, s, Loff, Llp, Lrow, Lbp, Lcol, Lval);
    const RowMap<NT, false, BS> m;
    for (int32_t pb = 0; pb < S; pb += m.RPP) {  // rows are independent here
        const int32_t p = pb + m.slot;
        if (m.ok && p < S) {
            const int64_t gp = base + p;
            const int I = Urow[gp];
            const double *dblk = Dval + gp * BB + m.c * BS;
            double acc = 0;
#pragma unroll
            for (int d = 0; d < BS; ++d) acc += dblk[d] * y[I * BS + d];
            __asm__ volatile("" ::: "memory");  // the row's lanes (one wavefront) read y_I first
            y[I * BS + m.c] = acc;
        }
    }
    __syncthreads();
    store_slice<double>(z + base * BS, y, S * BS, tid, NT);
}

// 4b: z_I = w_I - sum_{K>I} Uhat_IK z_K, in place on z.
template <int BS, int NT>
__global__ __launch_bounds__(NT) void k_abl_upper_unit(
    double *z, int S, const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp,
    const uint16_t *__restrict__ Urow, const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol,
    const double *__restrict__ Uval, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;
    extern __shared__ unsigned char dd_smem[];
    double *y = reinterpret_cast<double *>(dd_smem);
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    load_slice<double>(y, z + base * BS, S * BS, tid, NT);
    __syncthreads();
    plain_upper<BS, double, double, NT, false, false>(y, base, s, Uoff, Ulp, Urow, Ubp, Ucol, Uval, nullptr);
    store_slice<double>(z + base * BS, y, S * BS, tid, NT);
}

// 5 and 6: the plain level loop with the vector in global memory (z) or
// with one thread per row.
template <int BS, int NT, bool GLOBAL, bool VC>
__global__ __launch_bounds__(NT) void k_abl_plain(
    const double *__restrict__ r, double *__restrict__ z, int S, const int32_t *__restrict__ Loff,
    const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow, const int32_t *__restrict__ Lbp,
    const uint16_t *__restrict__ Lcol, const double *__restrict__ Lval, const int32_t *__restrict__ Uoff,
    const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow, const int32_t *__restrict__ Ubp,
    const uint16_t *__restrict__ Ucol, const double *__restrict__ Uval, const double *__restrict__ Dval,
    const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;
    extern __shared__ unsigned char dd_smem[];
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    double *y = GLOBAL ? z + base * BS : reinterpret_cast<double *>(dd_smem);
    if constexpr (GLOBAL) {
        for (int i = tid; i < S * BS; i += NT) y[i] = r[base * BS + i];
    } else {
        load_slice<double>(y, r + base * BS, S * BS, tid, NT);
    }
    __syncthreads();
    plain_lower<BS, double, double, NT, VC>(y, base, s, Loff, Llp, Lrow, Lbp, Lcol, Lval);
    plain_upper<BS, double, double, NT, VC, true>(y, base, s, Uoff, Ulp, Urow, Ubp, Ucol, Uval, Dval);
    if constexpr (!GLOBAL) store_slice<double>(z + base * BS, y, S * BS, tid, NT);
}

// 7: the upper sweep in ILU0 form, z_I = inv(U_II) (y_I - sum_{K>I} U_IK z_K):
// the U blocks as factored (packed in the same sweep order as Uhat), and the
// BS lanes of a row exchange their sums before the scaling.
template <int BS, int NT>
__global__ __launch_bounds__(NT) void k_abl_ilu0(
    const double *__restrict__ r, double *__restrict__ z, int S, const int32_t *__restrict__ Loff,
    const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow, const int32_t *__restrict__ Lbp,
    const uint16_t *__restrict__ Lcol, const double *__restrict__ Lval, const int32_t *__restrict__ Uoff,
    const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow, const int32_t *__restrict__ Ubp,
    const uint16_t *__restrict__ Ucol, const double *__restrict__ Uraw, const double *__restrict__ Dval,
    const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;
    constexpr int BB = BS * BS;
    extern __shared__ unsigned char dd_smem[];
    double *y = reinterpret_cast<double *>(dd_smem);
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    load_slice<double>(y, r + base * BS, S * BS, tid, NT);
    __syncthreads();
    plain_lower<BS, double, double, NT, false>(y, base, s, Loff, Llp, Lrow, Lbp, Lcol, Lval);
    const RowMap<NT, false, BS> m;
    const int32_t o = Uoff[s];
    const int nl = Uoff[s + 1] - o - 1;
    for (int l = 0; l < nl; ++l) {
        const int32_t p0 = Ulp[o + l], p1 = Ulp[o + l + 1];
        for (int32_t pb = p0; pb < p1; pb += m.RPP) {
            const int32_t p = pb + m.slot;
            const bool row = m.ok && p < p1;
            const int64_t gp = base + p;
            int I = 0;
            double acc[1] = {0.0};
            if (row) {
                I = Urow[gp];
                acc[0] = y[I * BS + m.c];
                row_blocks<BS, double, double, 1>(acc, y, Ubp[gp], Ubp[gp + 1], Ucol, Uraw, m.c);
            }
            // the row's BS sums, from its BS consecutive lanes (all lanes take part)
            double sum[BS];
#pragma unroll
            for (int d = 0; d < BS; ++d) sum[d] = __shfl(acc[0], lane - m.c + d);
            if (row) {
                const double *inv = Dval + gp * BB + m.c * BS;
                double zc = 0;
#pragma unroll
                for (int d = 0; d < BS; ++d) zc += inv[d] * sum[d];
                y[I * BS + m.c] = zc;
            }
        }
        __syncthreads();
    }
    store_slice<double>(z + base * BS, y, S * BS, tid, NT);
}

// 8: Algorithm 4 recast for the whole apply.  No barrier between levels:
// wavefront w takes the positions w, w + W, w + 2W, ... of a sweep (W
// wavefronts, positions in sweep order, so every dependency of a row sits at
// an earlier position).  The wavefront that holds the earliest unfinished
// row can therefore always proceed, and no wavefront waits on a row it holds
// itself.  Lane k of the row's wavefront owns its k-th off-diagonal block:
// it waits until the block's column row is complete (a byte flag per row in
// LDS), multiplies the block by that row's values, and lane 0 sums the
// products in block order, writes the row and then sets its flag.  Every
// wait is bounded: after kSpinMax polls the workgroup gives up (an abort
// flag in LDS ends every other wait too) and writes NaN over its slice of z,
// so a wait that could not end shows up as a wrong result, never as a hang.
constexpr int kSpinMax = 1 << 20;

struct SpinShared {
    uint8_t *done;
    int *abort;
};

template <int BS, int NT, bool UPPER>
__device__ __forceinline__ void spin_sweep(double *__restrict__ y, const SpinShared &sh, int64_t base, int S,
                                           const uint16_t *__restrict__ prow, const int32_t *__restrict__ bp,
                                           const uint16_t *__restrict__ col, const double *__restrict__ val,
                                           const double *__restrict__ dval) {
    constexpr int BB = BS * BS;
    constexpr uint8_t kWant = UPPER ? 2 : 1;
    constexpr int W = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    for (int32_t p = threadIdx.x / kWave; p < S; p += W) {
        if (__builtin_amdgcn_readfirstlane(*(volatile int *)sh.abort)) break;
        const int64_t gp = base + p;
        const int I = prow[gp];
        const int32_t b0 = bp[gp];
        const int nb = bp[gp + 1] - b0;  // at most 64 (kMaxRowBlocks)
        double prod[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) prod[c] = 0;
        if (lane < nb) {
            const int J = col[b0 + lane];
            for (int it = 0; *(volatile uint8_t *)(sh.done + J) < kWant; ++it) {
                if (it >= kSpinMax || *(volatile int *)sh.abort) {
                    *(volatile int *)sh.abort = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const double *blk = val + (int64_t)(b0 + lane) * BB;
#pragma unroll
            for (int c = 0; c < BS; ++c)
#pragma unroll
                for (int d = 0; d < BS; ++d) prod[c] += blk[c * BS + d] * y[J * BS + d];
        }
        double acc[BS];
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            if constexpr (UPPER) {
                acc[c] = 0;
#pragma unroll
                for (int d = 0; d < BS; ++d) acc[c] += dval[gp * BB + c * BS + d] * y[I * BS + d];
            } else {
                acc[c] = y[I * BS + c];
            }
        }
        for (int k = 0; k < nb; ++k)
#pragma unroll
            for (int c = 0; c < BS; ++c) acc[c] -= __shfl(prod[c], k);
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < BS; ++c) y[I * BS + c] = acc[c];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            *(volatile uint8_t *)(sh.done + I) = kWant;
        }
    }
}

template <int BS, int NT>
__global__ __launch_bounds__(NT) void k_abl_spin(
    const double *__restrict__ r, double *__restrict__ z, int S, const uint16_t *__restrict__ Lrow,
    const int32_t *__restrict__ Lbp, const uint16_t *__restrict__ Lcol, const double *__restrict__ Lval,
    const uint16_t *__restrict__ Urow, const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol,
    const double *__restrict__ Uval, const double *__restrict__ Dval, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;
    extern __shared__ unsigned char dd_smem[];
    double *y = reinterpret_cast<double *>(dd_smem);
    SpinShared sh;
    sh.done = dd_smem + (size_t)S * BS * sizeof(double);
    sh.abort = reinterpret_cast<int *>(dd_smem + (((size_t)S * BS * sizeof(double) + S + 3) & ~(size_t)3));
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    load_slice<double>(y, r + base * BS, S * BS, tid, NT);
    for (int i = tid; i < S; i += NT) sh.done[i] = 0;
    if (tid == 0) *sh.abort = 0;
    __syncthreads();
    spin_sweep<BS, NT, false>(y, sh, base, S, Lrow, Lbp, Lcol, Lval, nullptr);
    __syncthreads();  // the upper sweep reads y_I of rows other wavefronts finished
    spin_sweep<BS, NT, true>(y, sh, base, S, Urow, Ubp, Ucol, Uval, Dval);
    __syncthreads();
    if (*(volatile int *)sh.abort) {
        for (int i = tid; i < S * BS; i += NT) z[base * BS + i] = __builtin_nan("");
    } else {
        store_slice<double>(z + base * BS, y, S * BS, tid, NT);
    }
}

int spin_lds_bytes(const dd_ctx *h) {
    return (int)((((size_t)h->S * h->bs * sizeof(double) + h->S + 3) & ~(size_t)3) + sizeof(int));
}

// ------------------------------------------------------------------------
// Host side: variant choice and launch.
template <typename K>
static hipError_t allow_full_lds(K kern, bool &done) {
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
    if (e == hipSuccess) done = true;
    return e;
}

static bool compute_fp64(int precision) { return precision != DD_FP32; }

int apply_lds_bytes(const dd_ctx *h, int precision) {
    return h->S * h->bs * (compute_fp64(precision) ? 8 : 4);
}

const char *variant_unsupported(const dd_ctx *h, int v) {
    if (v < 4) return nullptr;
    if (h->precision != DD_FP64) return "apply variants 4-8 are FP64 ablations (set precision DD_FP64)";
    if (h->lic.active) return "apply variants 4-8 do not apply the learned correction (clear its parameters)";
    if (v == 8 && spin_lds_bytes(h) > 163840) return "apply variant 8: vector and row flags exceed the LDS";
    return nullptr;
}

template <typename TS>
static void factor_ptrs(const dd_ctx *h, bool slots, const TS **lv, const TS **uv, const TS **dv) {
    const Sweep &L = h->sw[0], &U = h->sw[1];
    if constexpr (sizeof(TS) == 8) {
        *lv = slots ? L.sval64 : L.val64;
        *uv = slots ? U.sval64 : U.val64;
        *dv = U.d64;
    } else {
        *lv = slots ? L.sval32 : L.val32;
        *uv = slots ? U.sval32 : U.val32;
        *dv = U.d32;
    }
}

static LicArgs lic_args(const dd_ctx *h) {
    return LicArgs{h->lic.fptr, h->lic.rb, h->lic.lrec, h->lic.Cr};
}

// Launch a slot kernel; with timing events pending on the handle, through
// hipExtLaunchKernel, which records them at the kernel's own start and end.
template <typename K, typename... A>
static void launch_timed(dd_ctx *h, K kern, dim3 grid, int nt, int lds, hipStream_t st, A... args) {
    if (h->tev[0]) {
        hipExtLaunchKernelGGL(kern, grid, dim3(nt), (uint32_t)lds, st, h->tev[0], h->tev[1], 0u, args...);
        h->tev_used = 1;
    } else {
        kern<<<grid, nt, lds, st>>>(args...);
    }
}

template <int BS, typename TS, typename TC, int NT, int MB, bool LIC>
static hipError_t launch_slots(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                               const TS *lv, const TS *uv, int nrhs) {
    constexpr int PD = sizeof(TS) == 8 ? DDILU_PD64 : DDILU_PD32;
    auto kern = k_dd_apply_slots<BS, TS, TC, NT, MB, PD, LIC>;
    static bool done = false;
    hipError_t e = allow_full_lds(kern, done);
    if (e != hipSuccess) return e;
    const int lds = h->S * BS * (int)sizeof(TC);
    // wavefronts for the widest level (at most NT / 64)
    constexpr int RPW = kWave / BS;
    const int nt = std::max(kWave, std::min(NT, (h->max_level_width + RPW - 1) / RPW * kWave));
    launch_timed(h, kern, dim3(h->nsub, nrhs), nt, lds, st, r, z, h->S, h->lev[0].off, h->lev[0].ptr,
                 h->sw[0].desc, lv, h->lev[1].off, h->lev[1].ptr, h->sw[1].desc, uv, state, lic_args(h),
                 (int64_t)h->n * BS, (const int32_t *)nullptr, (const int32_t *)nullptr);
    return hipGetLastError();
}

// The segmented slot layout (rows of more than three blocks): workgroups of
// 1,024 lanes (the layout's chunks are cut for that width), chunk tables as
// level tables, MB = the layout's blocks per segment (2 or 3).
template <int BS, typename TS, typename TC>
static hipError_t launch_seg(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                             const TS *lv, const TS *uv, int nrhs) {
    constexpr int PD = sizeof(TS) == 8 ? DDILU_PD64 : DDILU_PD32;
    auto go = [&](auto kern, bool &done) -> hipError_t {
        hipError_t e = allow_full_lds(kern, done);
        if (e != hipSuccess) return e;
        const int lds = h->S * BS * (int)sizeof(TC);
        const Sweep &L = h->sw[0], &U = h->sw[1];
        launch_timed(h, kern, dim3(h->nsub, nrhs), 1024, lds, st, r, z, h->S, (const int32_t *)L.gchk,
                     (const int32_t *)L.chk, (const uint64_t *)L.desc, lv, (const int32_t *)U.gchk,
                     (const int32_t *)U.chk, (const uint64_t *)U.desc, uv, state, lic_args(h), (int64_t)h->n * BS,
                     (const int32_t *)L.gpos, (const int32_t *)U.gpos);
        return hipGetLastError();
    };
    static bool done2 = false, done3 = false;
    if (h->seg == 2) return go(k_dd_apply_slots<BS, TS, TC, 1024, 2, PD, false, true>, done2);
    return go(k_dd_apply_slots<BS, TS, TC, 1024, 3, PD, false, true>, done3);
}

template <int BS, typename TS, typename TC, int NT, bool LIC>
static hipError_t launch_slots_mb(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                                  const TS *lv, const TS *uv, int nrhs = 1) {
    switch (h->slots) {
        case 1: return launch_slots<BS, TS, TC, NT, 1, LIC>(h, r, z, state, st, lv, uv, nrhs);
        case 2: return launch_slots<BS, TS, TC, NT, 2, LIC>(h, r, z, state, st, lv, uv, nrhs);
        default: return launch_slots<BS, TS, TC, NT, 3, LIC>(h, r, z, state, st, lv, uv, nrhs);
    }
}

// ------------------------------------------------------- apply + SpMV launch
constexpr int kFusedStaticLds = 512;  // the kernel's ticket and partial sums (bound)

int fused_unsupported(const dd_ctx *h) {
    constexpr int kMaxNT = 1024;
    const int rpp = (kWave / h->bs) * (kMaxNT / kWave);
    if (h->pc_kind != 0 || h->profile) return 1;
    if (!(h->variant == 0 || h->variant == 3) || !h->slots || h->max_level_width > rpp) return 2;
    if (h->nsub > h->spmv_part_stride) return 3;
    if (apply_lds_bytes(h, h->precision) > 163840 - kFusedStaticLds) return 4;
    return 0;
}

template <int BS, typename TS, typename TC, int MB, bool LIC, int MODE>
static hipError_t launch_fused_k(dd_ctx *h, const double *r, double *z, const FuseArgs &f, hipStream_t st) {
    constexpr int PD = sizeof(TS) == 8 ? DDILU_PD64 : DDILU_PD32;
    auto kern = k_dd_apply_slots_spmv<BS, TS, TC, 1024, MB, PD, LIC, MODE>;
    static bool done = false;
    if (!done) {
        hipFuncAttributes a{};
        hipError_t e = hipFuncGetAttributes(&a, reinterpret_cast<const void *>(kern));
        if (e != hipSuccess) return e;
        if (a.sharedSizeBytes > (size_t)kFusedStaticLds) return hipErrorInvalidValue;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                163840 - kFusedStaticLds);
        if (e != hipSuccess) return e;
        done = true;
    }
    const TS *lv, *uv, *dv;
    factor_ptrs<TS>(h, true, &lv, &uv, &dv);
    const int lds = h->S * BS * (int)sizeof(TC);
    constexpr int RPW = kWave / BS;
    const int nt = std::max(kWave, std::min(1024, (h->max_level_width + RPW - 1) / RPW * kWave));
    kern<<<2 * h->nsub, nt, lds, st>>>(r, z, h->S, h->lev[0].off, h->lev[0].ptr, h->sw[0].desc, lv, h->lev[1].off,
                                       h->lev[1].ptr, h->sw[1].desc, uv, lic_args(h), f);
    return hipGetLastError();
}

template <int BS, typename TS, typename TC, bool LIC>
static hipError_t fused_mb(dd_ctx *h, int mode, const double *r, double *z, const FuseArgs &f, hipStream_t st) {
    switch (h->slots * 2 + (mode != 0)) {
        case 2: return launch_fused_k<BS, TS, TC, 1, LIC, 0>(h, r, z, f, st);
        case 3: return launch_fused_k<BS, TS, TC, 1, LIC, 1>(h, r, z, f, st);
        case 4: return launch_fused_k<BS, TS, TC, 2, LIC, 0>(h, r, z, f, st);
        case 5: return launch_fused_k<BS, TS, TC, 2, LIC, 1>(h, r, z, f, st);
        case 6: return launch_fused_k<BS, TS, TC, 3, LIC, 0>(h, r, z, f, st);
        default: return launch_fused_k<BS, TS, TC, 3, LIC, 1>(h, r, z, f, st);
    }
}

template <int BS, typename TS, typename TC>
static hipError_t fused_lic(dd_ctx *h, int mode, const double *r, double *z, const FuseArgs &f, hipStream_t st) {
    if constexpr (BS == 3)
        if (h->lic.active) return fused_mb<BS, TS, TC, true>(h, mode, r, z, f, st);
    return fused_mb<BS, TS, TC, false>(h, mode, r, z, f, st);
}

template <int BS>
static hipError_t fused_bs(dd_ctx *h, int mode, const double *r, double *z, const FuseArgs &f, hipStream_t st) {
    switch (h->precision) {
        case DD_FP32: return fused_lic<BS, float, float>(h, mode, r, z, f, st);
        case DD_MIXED: return fused_lic<BS, float, double>(h, mode, r, z, f, st);
        default: return fused_lic<BS, double, double>(h, mode, r, z, f, st);
    }
}

hipError_t launch_apply_spmv(dd_ctx *h, int mode, const double *r, double *z, double *y, const double *w,
                             double *part, int part_stride, uint32_t epoch, unsigned long long ticket0,
                             int32_t *state, hipStream_t st) {
    if (fused_unsupported(h) || !h->fdep) return hipErrorInvalidValue;
    const FuseArgs f{h->aptr, h->acol,  h->aval,   y,     w,       part,   part_stride,
                     h->nsub, h->fdep,  h->fflag,  h->fticket,     ticket0, epoch, state};
    return h->bs == 3 ? fused_bs<3>(h, mode, r, z, f, st) : fused_bs<1>(h, mode, r, z, f, st);
}

__global__ __launch_bounds__(256) void k_dep_range(int S, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, int32_t *__restrict__ dep) {
    __shared__ int lo, hi;
    const int k = blockIdx.x;
    if (threadIdx.x == 0) {
        lo = INT32_MAX;
        hi = -1;
    }
    __syncthreads();
    int l = INT32_MAX, u = -1;
    for (int q = threadIdx.x; q < S; q += blockDim.x) {
        const int64_t row = (int64_t)k * S + q;
        for (int32_t b = ptr[row]; b < ptr[row + 1]; ++b) {
            const int d = col[b] / S;
            l = min(l, d);
            u = max(u, d);
        }
    }
    atomicMin(&lo, l);
    atomicMax(&hi, u);
    __syncthreads();
    if (threadIdx.x == 0) {
        dep[2 * k] = lo <= hi ? lo : k;
        dep[2 * k + 1] = lo <= hi ? hi : k;
    }
}

hipError_t launch_dep_range(dd_ctx *h, hipStream_t st) {
    k_dep_range<<<h->nsub, 256, 0, st>>>(h->S, h->aptr, h->acol, h->fdep);
    return hipGetLastError();
}

// Ablation variants 4-8 (FP64; the API rejects other precisions and the
// learned correction for them).
template <int BS, int NT>
static hipError_t launch_ablation(dd_ctx *h, int variant, const double *r, double *z, const int32_t *state,
                                  hipStream_t st) {
    const Sweep &L = h->sw[0], &U = h->sw[1];
    const Levels &LL = h->lev[0], &UL = h->lev[1];
    const int lds = h->S * BS * (int)sizeof(double);
    const unsigned g = (unsigned)h->nsub;
    hipError_t e = hipSuccess;
    switch (variant) {
        case 4: {
            auto k1 = k_abl_lower_scale<BS, NT>;
            auto k2 = k_abl_upper_unit<BS, NT>;
            static bool d1 = false, d2 = false;
            if ((e = allow_full_lds(k1, d1)) != hipSuccess || (e = allow_full_lds(k2, d2)) != hipSuccess) return e;
            k1<<<g, NT, lds, st>>>(r, z, h->S, LL.off, LL.ptr, L.prow, L.bptr, L.bcol, L.val64, U.prow, U.d64, state);
            k2<<<g, NT, lds, st>>>(z, h->S, UL.off, UL.ptr, U.prow, U.bptr, U.bcol, U.val64, state);
            break;
        }
        case 5:
            k_abl_plain<BS, NT, true, false><<<g, NT, 0, st>>>(r, z, h->S, LL.off, LL.ptr, L.prow, L.bptr, L.bcol,
                                                               L.val64, UL.off, UL.ptr, U.prow, U.bptr, U.bcol,
                                                               U.val64, U.d64, state);
            break;
        case 6: {
            auto k = k_abl_plain<BS, NT, false, true>;
            static bool d = false;
            if ((e = allow_full_lds(k, d)) != hipSuccess) return e;
            k<<<g, NT, lds, st>>>(r, z, h->S, LL.off, LL.ptr, L.prow, L.bptr, L.bcol, L.val64, UL.off, UL.ptr,
                                  U.prow, U.bptr, U.bcol, U.val64, U.d64, state);
            break;
        }
        case 7: {
            auto k = k_abl_ilu0<BS, NT>;
            static bool d = false;
            if ((e = allow_full_lds(k, d)) != hipSuccess) return e;
            if (!U.uraw) return hipErrorInvalidValue;  // built by the API before the first launch
            k<<<g, NT, lds, st>>>(r, z, h->S, LL.off, LL.ptr, L.prow, L.bptr, L.bcol, L.val64, UL.off, UL.ptr,
                                  U.prow, U.bptr, U.bcol, U.uraw, U.d64, state);
            break;
        }
        case 8: {
            auto k = k_abl_spin<BS, NT>;
            static bool d = false;
            const int sl = spin_lds_bytes(h);
            if (sl > 163840) return hipErrorInvalidValue;  // vector + flags must fit the LDS
            if ((e = allow_full_lds(k, d)) != hipSuccess) return e;
            k<<<g, NT, sl, st>>>(r, z, h->S, L.prow, L.bptr, L.bcol, L.val64, U.prow, U.bptr, U.bcol, U.val64,
                                 U.d64, state);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int BS, typename TS, typename TC, int NT>
static hipError_t launch_typed(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                               int nrhs) {
    const Sweep &L = h->sw[0], &U = h->sw[1];
    const int lds = h->S * BS * (int)sizeof(TC);
    constexpr int RPP = (kWave / BS) * (NT / kWave);
    const bool one_pass = h->max_level_width <= RPP;
    const bool lic = BS == 3 && h->lic.active;
    int variant = h->variant;
    if (variant >= 4) {
        if constexpr (sizeof(TS) == 8 && sizeof(TC) == 8)
            return launch_ablation<BS, NT>(h, variant, r, z, state, st);
        return hipErrorInvalidValue;  // rejected by the API before launch
    }
    // automatic: the slot kernel where the shape allows it, else the plain
    // loop (measured faster than the pipelined one on rows of up to 17
    // blocks: 438 against 730 us at 2M unstructured rows)
    if (variant == 0) variant = 3;
    // rows of more than three blocks: the segmented slot layout
    if (variant == 3 && h->seg && !lic) {
        const TS *lv, *uv, *dv;
        factor_ptrs<TS>(h, true, &lv, &uv, &dv);
        return launch_seg<BS, TS, TC>(h, r, z, state, st, lv, uv, nrhs);
    }
    if (variant == 3 && (!one_pass || !h->slots)) variant = 1;
    if (variant == 2 && lic) variant = 1;  // the correction runs in 1 and 3
    if (variant == 3) {
        const TS *lv, *uv, *dv;
        factor_ptrs<TS>(h, true, &lv, &uv, &dv);
        if constexpr (BS == 3)
            if (lic) return launch_slots_mb<BS, TS, TC, NT, true>(h, r, z, state, st, lv, uv, nrhs);
        return launch_slots_mb<BS, TS, TC, NT, false>(h, r, z, state, st, lv, uv, nrhs);
    }
    if (nrhs > 1) {  // the other kernels take one right-hand side per launch
        const int64_t m = h->n * BS;
        for (int q = 0; q < nrhs; ++q) {
            hipError_t e = launch_typed<BS, TS, TC, NT>(h, r + q * m, z + q * m, state, st, 1);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const TS *lv, *uv, *dv;
    factor_ptrs<TS>(h, false, &lv, &uv, &dv);
    if (variant == 2) {
        auto kern = k_dd_apply_pipe<BS, TS, TC, NT, 3>;
        static bool done = false;
        hipError_t e = allow_full_lds(kern, done);
        if (e != hipSuccess) return e;
        kern<<<h->nsub, NT, lds, st>>>(r, z, h->S, h->lev[0].off, h->lev[0].ptr, L.prow, L.bptr, L.bcol, lv,
                                       h->lev[1].off, h->lev[1].ptr, U.prow, U.bptr, U.bcol, uv, dv, state);
        return hipGetLastError();
    }
    auto launch_simple = [&](auto kern, bool &done) -> hipError_t {
        hipError_t e = allow_full_lds(kern, done);
        if (e != hipSuccess) return e;
        kern<<<h->nsub, NT, lds, st>>>(r, z, h->S, h->lev[0].off, h->lev[0].ptr, L.prow, L.bptr, L.bcol, lv,
                                       h->lev[1].off, h->lev[1].ptr, U.prow, U.bptr, U.bcol, uv, dv, state,
                                       lic_args(h));
        return hipGetLastError();
    };
    if constexpr (BS == 3) {
        if (lic) {
            static bool done_l = false;
            return launch_simple(k_dd_apply<BS, TS, TC, NT, true>, done_l);
        }
    }
    static bool done = false;
    return launch_simple(k_dd_apply<BS, TS, TC, NT, false>, done);
}

// Workgroup size: enough wavefronts to cover the widest level in one pass,
// rounded up to a power of two between 64 and 1024 lanes.
static int pick_threads(const dd_ctx *h) {
    const int width = h->lev[0].max_levels > 0 ? h->max_level_width : h->S;
    const int rpw = kWave / h->bs;
    const int waves = (width + rpw - 1) / rpw;
    int nt = 64;
    while (nt < waves * kWave && nt < 1024) nt *= 2;
    return nt;
}

template <int BS, typename TS, typename TC>
static hipError_t launch_nt(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st, int nrhs) {
    switch (pick_threads(h)) {
        case 64: return launch_typed<BS, TS, TC, 64>(h, r, z, state, st, nrhs);
        case 128: return launch_typed<BS, TS, TC, 128>(h, r, z, state, st, nrhs);
        case 256: return launch_typed<BS, TS, TC, 256>(h, r, z, state, st, nrhs);
        case 512: return launch_typed<BS, TS, TC, 512>(h, r, z, state, st, nrhs);
        default: return launch_typed<BS, TS, TC, 1024>(h, r, z, state, st, nrhs);
    }
}

template <int BS>
static hipError_t launch_bs(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st, int nrhs) {
    switch (h->precision) {
        case DD_FP32: return launch_nt<BS, float, float>(h, r, z, state, st, nrhs);
        case DD_MIXED: return launch_nt<BS, float, double>(h, r, z, state, st, nrhs);
        default: return launch_nt<BS, double, double>(h, r, z, state, st, nrhs);
    }
}

hipError_t launch_apply(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    return launch_apply_batch(h, r, z, 1, st, state);
}

hipError_t launch_apply_batch(dd_ctx *h, const double *r, double *z, int nrhs, hipStream_t st,
                              const int32_t *state) {
    return h->bs == 3 ? launch_bs<3>(h, r, z, state, st, nrhs) : launch_bs<1>(h, r, z, state, st, nrhs);
}

// a = M_DD^{-T} g: the slot kernel run on the transposed factor streams (FP64,
// no correction); needs 3x3 blocks, the slot layout and one-pass levels.
template <int NT>
static hipError_t launch_adjoint_nt(dd_ctx *h, const double *g, double *a, int nrhs, hipStream_t st) {
    constexpr int RPP = (kWave / 3) * (NT / kWave);
    if (h->max_level_width > RPP) return hipErrorInvalidValue;
    const double *lv = h->lic.adj_val[0], *uv = h->lic.adj_val[1];
    return launch_slots_mb<3, double, double, NT, false>(h, g, a, nullptr, st, lv, uv, nrhs);
}

hipError_t launch_apply_adjoint(dd_ctx *h, const double *g, double *a, int nrhs, hipStream_t st) {
    if (h->bs != 3 || !h->slots || !h->lic.ready || !h->lic.adj_val[1]) return hipErrorInvalidValue;
    switch (pick_threads(h)) {
        case 64: return launch_adjoint_nt<64>(h, g, a, nrhs, st);
        case 128: return launch_adjoint_nt<128>(h, g, a, nrhs, st);
        case 256: return launch_adjoint_nt<256>(h, g, a, nrhs, st);
        case 512: return launch_adjoint_nt<512>(h, g, a, nrhs, st);
        default: return launch_adjoint_nt<1024>(h, g, a, nrhs, st);
    }
}

hipError_t launch_precond(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                          hipEvent_t ev0, hipEvent_t ev1) {
    if (!ev0) {
        if (h->pc_kind == 1) return launch_global_apply(h, r, z, 1, st);
        return launch_apply(h, r, z, state, st);
    }
    // the stream-ordered record stands for paths of several launches; a slot
    // kernel records both events again at its own start and end
    hipError_t e = hipEventRecord(ev0, st);
    if (e != hipSuccess) return e;
    h->tev[0] = ev0;
    h->tev[1] = ev1;
    h->tev_used = 0;
    e = h->pc_kind == 1 ? launch_global_apply(h, r, z, 1, st) : launch_apply(h, r, z, state, st);
    h->tev[0] = h->tev[1] = nullptr;
    if (e == hipSuccess && !h->tev_used) e = hipEventRecord(ev1, st);
    return e;
}

}  // namespace ddilu
