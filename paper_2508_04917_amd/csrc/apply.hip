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
#include "internal.h"

// Prefetch depth (levels loaded ahead) of the slot-layout kernel, per factor
// storage type.  Depths 1 to 3 measure the same at 160^3 (the per-level time
// is not set by load latency), so the default takes the fewest registers.
#ifndef DDILU_PD64
#define DDILU_PD64 1
#endif
#ifndef DDILU_PD32
#define DDILU_PD32 1
#endif

namespace ddilu {

// Learned interface correction inside the apply: once the subdomain's r is
// in LDS, every row with cut faces adds sum_f C_f r_J (J in a neighbouring
// subdomain, read from r in global memory; faces in CSR order).  One lane per
// (row, component), so the update order is fixed.  Each lane handles two
// rows per pass and fetches in three dependent steps (row record; column
// and coefficients of up to kLicFaces faces; r_J), with positions past the
// end clamped to valid ones and discarded by selects, so the loads of a step
// are all in flight together.  Rows with more faces finish in a loop.
struct LicArgs {
    const int32_t *bsub;
    const int4 *brow;  // {row, first face, face count, 0}
    const int32_t *fJ;
    const float *C;
};

constexpr int kLicFaces = 3;  // a 7-point row has at most 3 cut faces unless a subdomain is one cell thin

template <int BS, typename TC>
__device__ __forceinline__ void lic_correct_lds(TC *__restrict__ y, const double *__restrict__ r, int64_t base, int s,
                                                const LicArgs &la, int tid, int nt) {
    const int32_t b0 = la.bsub[s], b1 = la.bsub[s + 1];
    const int nitems = (b1 - b0) * BS;
    for (int i0 = tid; i0 < nitems; i0 += 2 * nt) {
        int item[2];
        bool ok[2];
        int4 ri[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            ok[u] = i0 + u * nt < nitems;
            item[u] = ok[u] ? i0 + u * nt : i0;
            ri[u] = la.brow[b0 + item[u] / BS];
        }
        __builtin_amdgcn_sched_barrier(0);
        int64_t J[2][kLicFaces];
        float cf[2][kLicFaces][BS];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = item[u] % BS;
#pragma unroll
            for (int k = 0; k < kLicFaces; ++k) {
                const int32_t f = ri[u].y + min(k, ri[u].z - 1);
                J[u][k] = la.fJ[f];
                const float *Cf = la.C + (int64_t)f * BS * BS + c * BS;
#pragma unroll
                for (int d = 0; d < BS; ++d) cf[u][k][d] = Cf[d];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        double rv[2][kLicFaces][BS];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int k = 0; k < kLicFaces; ++k)
#pragma unroll
                for (int d = 0; d < BS; ++d) rv[u][k][d] = r[J[u][k] * BS + d];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!ok[u]) continue;
            const int c = item[u] % BS;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < kLicFaces; ++k) {
                double t = acc;
#pragma unroll
                for (int d = 0; d < BS; ++d) t += (double)cf[u][k][d] * rv[u][k][d];
                acc = k < ri[u].z ? t : acc;
            }
            for (int32_t f = ri[u].y + kLicFaces; f < ri[u].y + ri[u].z; ++f) {
                const int64_t Jf = la.fJ[f];
                const float *Cf = la.C + (int64_t)f * BS * BS + c * BS;
#pragma unroll
                for (int d = 0; d < BS; ++d) acc += (double)Cf[d] * r[Jf * BS + d];
            }
            y[(ri[u].x - base) * BS + c] += static_cast<TC>(acc);
        }
    }
    __syncthreads();
}

// The subdomain's slice of r into LDS: each thread issues kLoadU loads
// before it waits for any (a plain strided loop would wait for every load
// in turn), positions past the end clamped to a valid one and not stored.
constexpr int kLoadU = 8;

template <typename TC>
__device__ __forceinline__ void load_slice(TC *__restrict__ y, const double *__restrict__ rs, int m, int tid,
                                           int nt) {
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

// LDS back to the subdomain's slice of z, kLoadU values per thread at a time.
template <typename TC>
__device__ __forceinline__ void store_slice(double *__restrict__ zs, const TC *__restrict__ y, int m, int tid,
                                            int nt) {
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
template <int BS, typename TS, typename TC, int NT, bool LIC>
__global__ __launch_bounds__(NT) void k_dd_apply(
    const double *__restrict__ r, double *__restrict__ z, int S,
    const int32_t *__restrict__ Loff, const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow,
    const int32_t *__restrict__ Lbp, const uint16_t *__restrict__ Lcol, const TS *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow,
    const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol, const TS *__restrict__ Uval,
    const TS *__restrict__ Dval, const int32_t *__restrict__ state, LicArgs la) {
    if (state != nullptr && *state != 0) return;  // enclosing solve already finished
    constexpr int BB = BS * BS;
    constexpr int RPW = kWave / BS;          // block rows per wavefront
    constexpr int RPP = RPW * (NT / kWave);  // block rows per pass of the workgroup
    extern __shared__ unsigned char dd_smem[];
    TC *y = reinterpret_cast<TC *>(dd_smem);

    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int c = lane % BS, rl = lane / BS;
    const bool lane_ok = rl < RPW;

    const double *rs = r + base * BS;
    load_slice<TC>(y, rs, S * BS, tid, NT);
    __syncthreads();
    if constexpr (LIC) lic_correct_lds<BS, TC>(y, r, base, s, la, tid, NT);

    // lower sweep: y_I = r_I - sum_{J<I} L_IJ y_J
    {
        const int32_t o = Loff[s];
        const int nl = Loff[s + 1] - o - 1;
        for (int l = 0; l < nl; ++l) {
            const int32_t p0 = Llp[o + l], p1 = Llp[o + l + 1];
            for (int32_t pb = p0; pb < p1; pb += RPP) {
                const int32_t p = pb + wave * RPW + rl;
                if (lane_ok && p < p1) {
                    const int64_t gp = base + p;
                    const int I = Lrow[gp];
                    TC acc = y[I * BS + c];
                    const int32_t b1 = Lbp[gp + 1];
                    for (int32_t b = Lbp[gp]; b < b1; ++b) {
                        const int J = Lcol[b];
                        const TS *blk = Lval + (int64_t)b * BB + c * BS;
#pragma unroll
                        for (int d = 0; d < BS; ++d) acc -= static_cast<TC>(blk[d]) * y[J * BS + d];
                    }
                    y[I * BS + c] = acc;
                }
            }
            __syncthreads();
        }
    }

    // upper sweep with the scaling fused: z_I = inv_D_I y_I - sum_{K>I} Uhat_IK z_K
    {
        const int32_t o = Uoff[s];
        const int nl = Uoff[s + 1] - o - 1;
        for (int l = 0; l < nl; ++l) {
            const int32_t p0 = Ulp[o + l], p1 = Ulp[o + l + 1];
            for (int32_t pb = p0; pb < p1; pb += RPP) {
                const int32_t p = pb + wave * RPW + rl;
                if (lane_ok && p < p1) {
                    const int64_t gp = base + p;
                    const int I = Urow[gp];
                    const TS *dblk = Dval + gp * BB + c * BS;
                    TC acc = 0;
#pragma unroll
                    for (int d = 0; d < BS; ++d) acc += static_cast<TC>(dblk[d]) * y[I * BS + d];
                    const int32_t b1 = Ubp[gp + 1];
                    for (int32_t b = Ubp[gp]; b < b1; ++b) {
                        const int K = Ucol[b];
                        const TS *blk = Uval + (int64_t)b * BB + c * BS;
#pragma unroll
                        for (int d = 0; d < BS; ++d) acc -= static_cast<TC>(blk[d]) * y[K * BS + d];
                    }
                    // every lane of this row has read y_I above (same wavefront)
                    __asm__ volatile("" ::: "memory");
                    y[I * BS + c] = acc;
                }
            }
            __syncthreads();
        }
    }

    double *zs = z + base * BS;
    store_slice<TC>(zs, y, S * BS, tid, NT);
}

// ------------------------------------------------------------------------
// Variant 2: levels no wider than one workgroup pass, rows in the CSR
// layout.  The factor data of a level does not depend on the solve, so it is
// fetched ahead: while level l computes from LDS, the blocks of level l+1 are
// in flight into registers and the row metadata of level l+2 behind them.
// The level barrier only orders LDS traffic, so HBM latency overlaps the
// level chain.  Rows with more than MB blocks take the extra blocks through a
// direct (unpipelined) loop.
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
        if (k < R.nb) {
            const int64_t b = R.b0 + k;
            R.J[k] = col[b];
            const TS *blk = val + b * BB + c * BS;
#pragma unroll
            for (int d = 0; d < BS; ++d) R.v[k][d] = blk[d];
        }
    }
    if constexpr (UPPER) {
        if (m.ok) {
            const TS *dblk = dval + m.gp * BB + c * BS;
#pragma unroll
            for (int d = 0; d < BS; ++d) R.d[d] = dblk[d];
        }
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
        if (k < R.nb) {
            const int J = R.J[k];
#pragma unroll
            for (int d = 0; d < BS; ++d) acc -= static_cast<TC>(R.v[k][d]) * y[J * BS + d];
        }
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

template <int BS, typename TS, typename TC, int MB, bool UPPER>
__device__ __forceinline__ void sweep_csr(TC *__restrict__ y, int64_t base, int s, const int32_t *__restrict__ off,
                                          const int32_t *__restrict__ lp, const uint16_t *__restrict__ prow,
                                          const int32_t *__restrict__ bp, const uint16_t *__restrict__ col,
                                          const TS *__restrict__ val, const TS *__restrict__ dval, int slot,
                                          bool lane_ok, int c) {
    const int32_t o = off[s];
    const int nl = off[s + 1] - o - 1;
    if (nl <= 0) return;
    auto meta = [&](int l) -> LevelMeta {
        LevelMeta m;
        const int32_t p0 = lp[o + l], p1 = lp[o + l + 1];
        const int32_t p = p0 + slot;
        m.ok = lane_ok && p < p1;
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
    // Two register sets alternate between "being computed" and "being
    // filled"; the loop is unrolled by two so that neither is copied (a copy
    // of a register with a load in flight would wait for the load).
    LevelRegs<BS, TS, MB> A, B;
    LevelMeta mA = meta(0);
    csr_fetch<BS, TS, MB, UPPER>(A, mA, col, val, dval, c);
    LevelMeta mB;
    mB.ok = false;
    if (nl > 1) mB = meta(1);
    for (int l = 0; l < nl; l += 2) {
        if (l + 1 < nl) csr_fetch<BS, TS, MB, UPPER>(B, mB, col, val, dval, c);
        if (l + 2 < nl) mA = meta(l + 2);
        csr_compute<BS, TS, TC, MB, UPPER>(y, A, col, val, c);
        __syncthreads();
        if (l + 1 >= nl) break;
        if (l + 2 < nl) csr_fetch<BS, TS, MB, UPPER>(A, mA, col, val, dval, c);
        if (l + 3 < nl) mB = meta(l + 3);
        csr_compute<BS, TS, TC, MB, UPPER>(y, B, col, val, c);
        __syncthreads();
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
    sweep_csr<BS, TS, TC, MB, false>(y, base, s, Loff, Llp, Lrow, Lbp, Lcol, Lval, nullptr, slot, lane_ok, c);
    sweep_csr<BS, TS, TC, MB, true>(y, base, s, Uoff, Ulp, Urow, Ubp, Ucol, Uval, Dval, slot, lane_ok, c);
    double *zs = z + base * BS;
    store_slice<TC>(zs, y, S * BS, tid, NT);
}

// ------------------------------------------------------------------------
// Variant 3: slot layout.  Position p's blocks sit in fixed slots
// p*MB..p*MB+MB-1 (zero blocks pad short rows), and its row and columns sit
// in one 64-bit descriptor.  No load depends on another load, so the loads of
// level l+PD are issued while level l computes: PD+1 register sets rotate.
// The main loop is unrolled by PD+1 (each set keeps its registers) and has no
// early exit, and every lane issues the same loads in the same order (fetches
// past the last level re-read the last level), so the compiler can count
// outstanding loads exactly and each level waits only for its own set, not
// for the whole queue.
template <int BS, typename TS, int MB>
struct SlotRegs {
    bool ok;
    uint64_t desc;
    TS v[MB][BS];
    TS d[BS];
};

template <int BS, typename TS, typename TC, int MB, bool UPPER>
__device__ __forceinline__ void slot_compute(TC *__restrict__ y, const SlotRegs<BS, TS, MB> &R, int c) {
    if (!R.ok) return;
    const int I = (int)(R.desc & 0xffffu);
    // gather every LDS operand first (one round of LDS latency), then the
    // fixed-order arithmetic.  An empty slot holds a zero block: it is
    // applied to y_I (a valid LDS address) instead of being branched around,
    // so every loaded value has an unconditional use and the factor loads
    // stay where they were issued.
    constexpr int NI = UPPER ? BS : 1;
    TC yi[NI], yj[MB][BS];
#pragma unroll
    for (int d = 0; d < NI; ++d) yi[d] = y[I * BS + (UPPER ? d : c)];
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        const int J = (int)((R.desc >> (16 * (k + 1))) & 0xffffu);
        const int Jc = J != 0xffff ? J : I;
#pragma unroll
        for (int d = 0; d < BS; ++d) yj[k][d] = y[Jc * BS + d];
    }
    __builtin_amdgcn_sched_barrier(0);
    TC acc;
    if constexpr (UPPER) {
        acc = 0;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc += static_cast<TC>(R.d[d]) * yi[d];
    } else {
        acc = yi[0];
    }
#pragma unroll
    for (int k = 0; k < MB; ++k)
#pragma unroll
        for (int d = 0; d < BS; ++d) acc -= static_cast<TC>(R.v[k][d]) * yj[k][d];
    // all lanes of this row read y_I above (same wavefront)
    __asm__ volatile("" ::: "memory");
    y[I * BS + c] = acc;
}

// Loads go through buffer resources over the workgroup's slice of the
// descriptor, block and inv_D streams: a lane without a row at a level passes
// an offset past the slice, for which the hardware returns zeros without a
// memory access (and no lane can address outside its subdomain's slice).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice_rsrc(const void *p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

constexpr uint32_t kOobOffset = 0x80000000u;  // beyond every slice (slices < 2 GiB)

// N consecutive values starting at byte offset off, in the widest loads
// that fit (16, then 8, then 4 bytes).
template <typename TS, int N>
__device__ __forceinline__ void buf_load_run(__amdgpu_buffer_rsrc_t rs, uint32_t off, TS (&v)[N]) {
    constexpr int PER16 = 16 / (int)sizeof(TS);
    int i = 0;
#pragma unroll
    for (; i + PER16 <= N; i += PER16) {
        struct Q { TS x[PER16]; };
        const Q q = __builtin_bit_cast(Q, __builtin_amdgcn_raw_buffer_load_b128(rs, off + i * (uint32_t)sizeof(TS), 0, 0));
#pragma unroll
        for (int j = 0; j < PER16; ++j) v[i + j] = q.x[j];
    }
    if constexpr (sizeof(TS) == 4) {
        if (i + 2 <= N) {
            struct F2 { float x, y; };
            const F2 q = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(rs, off + i * 4u, 0, 0));
            v[i] = q.x;
            v[i + 1] = q.y;
            i += 2;
        }
        if (i < N) v[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off + i * 4u, 0, 0));
    } else {
        if (i < N) v[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off + i * 8u, 0, 0));
    }
}

struct SlotRsrc {
    __amdgpu_buffer_rsrc_t desc, val;
};

// Per position, the BS lanes of its row each read one contiguous run: lane c
// holds row c of every slot block (and, in the upper sweep, row c of inv_D),
// NV = (MB [+1]) * BS values, so a lane issues ceil(NV * sizeof(TS) / 16)
// loads rather than two per block.
template <int BS, typename TS, int MB, bool UPPER>
__device__ __forceinline__ void slot_fetch(SlotRegs<BS, TS, MB> &R, const SlotRsrc &rs, int32_t p0, int32_t p1,
                                           int slot, bool lane_ok, int c) {
    constexpr int NV = (MB + (UPPER ? 1 : 0)) * BS;
    const int32_t p = p0 + slot;
    R.ok = lane_ok && p < p1;
    const uint32_t pd = R.ok ? (uint32_t)p * 8u : kOobOffset;
    R.desc = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(rs.desc, pd, 0, 0));
    TS vals[NV];
    const uint32_t off = R.ok ? (uint32_t)((p * BS * NV + c * NV) * sizeof(TS)) : kOobOffset;
    buf_load_run<TS, NV>(rs.val, off, vals);
#pragma unroll
    for (int k = 0; k < MB; ++k)
#pragma unroll
        for (int d = 0; d < BS; ++d) R.v[k][d] = vals[k * BS + d];
    if constexpr (UPPER)
#pragma unroll
        for (int d = 0; d < BS; ++d) R.d[d] = vals[MB * BS + d];
}

template <int BS, typename TS, typename TC, int MB, int PD, bool UPPER>
__device__ __forceinline__ void sweep_slots(TC *__restrict__ y, int64_t base, int S, int s,
                                            const int32_t *__restrict__ off, const int32_t *__restrict__ lp,
                                            const uint64_t *__restrict__ desc, const TS *__restrict__ sval,
                                            int slot, bool lane_ok, int c) {
    constexpr int PS = (MB + (UPPER ? 1 : 0)) * BS * BS;  // values per position
    SlotRsrc rs;
    rs.desc = slice_rsrc(desc + base, (int64_t)S * 8);
    rs.val = slice_rsrc(sval + base * PS, (int64_t)S * PS * sizeof(TS));
    const int32_t o = off[s];
    const int nl = off[s + 1] - o - 1;
    SlotRegs<BS, TS, MB> R[PD + 1];
    // level bounds are read one fetch ahead, so their scalar loads complete
    // during a level's update instead of after the barrier that follows it
    int32_t q0 = lp[o], q1 = lp[o + 1];
    auto fetch = [&](SlotRegs<BS, TS, MB> &Rk, int l) {
        slot_fetch<BS, TS, MB, UPPER>(Rk, rs, q0, q1, slot, lane_ok, c);
        const int ln = l + 1 < nl ? l + 1 : nl - 1;
        q0 = lp[o + ln];
        q1 = lp[o + ln + 1];
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) fetch(R[u], u);
    const int nfull = nl - nl % (PD + 1);
    for (int l0 = 0; l0 < nfull; l0 += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) {
            fetch(R[(u + PD) % (PD + 1)], l0 + u + PD);
            slot_compute<BS, TS, TC, MB, UPPER>(y, R[u], c);
            __syncthreads();
        }
    }
    const int rem = nl - nfull;
#pragma unroll
    for (int u = 0; u < PD; ++u) {
        if (u < rem) {
            slot_compute<BS, TS, TC, MB, UPPER>(y, R[u], c);
            __syncthreads();
        }
    }
}

template <int BS, typename TS, typename TC, int NT, int MB, int PD, bool LIC>
__global__ __launch_bounds__(NT) void k_dd_apply_slots(
    const double *__restrict__ r, double *__restrict__ z, int S, const int32_t *__restrict__ Loff,
    const int32_t *__restrict__ Llp, const uint64_t *__restrict__ Ldesc, const TS *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint64_t *__restrict__ Udesc,
    const TS *__restrict__ Uval, const int32_t *__restrict__ state, LicArgs la) {
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

    // the launch may use fewer threads than NT: just enough wavefronts for
    // the widest level, so no wavefront is idle at every level
    const int nt = blockDim.x;
    const double *rs = r + base * BS;
    load_slice<TC>(y, rs, S * BS, tid, nt);
    __syncthreads();
    if constexpr (LIC) lic_correct_lds<BS, TC>(y, r, base, s, la, tid, nt);
    sweep_slots<BS, TS, TC, MB, PD, false>(y, base, S, s, Loff, Llp, Ldesc, Lval, slot, lane_ok, c);
    sweep_slots<BS, TS, TC, MB, PD, true>(y, base, S, s, Uoff, Ulp, Udesc, Uval, slot, lane_ok, c);
    double *zs = z + base * BS;
    store_slice<TC>(zs, y, S * BS, tid, nt);
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
    return LicArgs{h->lic.bsub, h->lic.brow, h->lic.fJ, h->lic.C};
}

template <int BS, typename TS, typename TC, int NT, int MB, bool LIC>
static hipError_t launch_slots(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                               const TS *lv, const TS *uv) {
    constexpr int PD = sizeof(TS) == 8 ? DDILU_PD64 : DDILU_PD32;
    auto kern = k_dd_apply_slots<BS, TS, TC, NT, MB, PD, LIC>;
    static bool done = false;
    hipError_t e = allow_full_lds(kern, done);
    if (e != hipSuccess) return e;
    const int lds = h->S * BS * (int)sizeof(TC);
    // wavefronts for the widest level (at most NT / 64)
    constexpr int RPW = kWave / BS;
    const int nt = std::max(kWave, std::min(NT, (h->max_level_width + RPW - 1) / RPW * kWave));
    kern<<<h->nsub, nt, lds, st>>>(r, z, h->S, h->lev[0].off, h->lev[0].ptr, h->sw[0].desc, lv, h->lev[1].off,
                                   h->lev[1].ptr, h->sw[1].desc, uv, state, lic_args(h));
    return hipGetLastError();
}

template <int BS, typename TS, typename TC, int NT, bool LIC>
static hipError_t launch_slots_mb(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st,
                                  const TS *lv, const TS *uv) {
    switch (h->slots) {
        case 1: return launch_slots<BS, TS, TC, NT, 1, LIC>(h, r, z, state, st, lv, uv);
        case 2: return launch_slots<BS, TS, TC, NT, 2, LIC>(h, r, z, state, st, lv, uv);
        default: return launch_slots<BS, TS, TC, NT, 3, LIC>(h, r, z, state, st, lv, uv);
    }
}

template <int BS, typename TS, typename TC, int NT>
static hipError_t launch_typed(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    const Sweep &L = h->sw[0], &U = h->sw[1];
    const int lds = h->S * BS * (int)sizeof(TC);
    constexpr int RPP = (kWave / BS) * (NT / kWave);
    const bool one_pass = h->max_level_width <= RPP;
    const bool lic = BS == 3 && h->lic.active;
    int variant = h->variant;
    if (variant == 0) variant = h->slots ? 3 : 2;
    if (variant == 3 && (!one_pass || !h->slots)) variant = 1;
    if (variant == 2 && (!one_pass || lic)) variant = 1;
    if (variant == 3) {
        const TS *lv, *uv, *dv;
        factor_ptrs<TS>(h, true, &lv, &uv, &dv);
        if constexpr (BS == 3)
            if (lic) return launch_slots_mb<BS, TS, TC, NT, true>(h, r, z, state, st, lv, uv);
        return launch_slots_mb<BS, TS, TC, NT, false>(h, r, z, state, st, lv, uv);
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
static hipError_t launch_nt(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    switch (pick_threads(h)) {
        case 64: return launch_typed<BS, TS, TC, 64>(h, r, z, state, st);
        case 128: return launch_typed<BS, TS, TC, 128>(h, r, z, state, st);
        case 256: return launch_typed<BS, TS, TC, 256>(h, r, z, state, st);
        case 512: return launch_typed<BS, TS, TC, 512>(h, r, z, state, st);
        default: return launch_typed<BS, TS, TC, 1024>(h, r, z, state, st);
    }
}

template <int BS>
static hipError_t launch_bs(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    switch (h->precision) {
        case DD_FP32: return launch_nt<BS, float, float>(h, r, z, state, st);
        case DD_MIXED: return launch_nt<BS, float, double>(h, r, z, state, st);
        default: return launch_nt<BS, double, double>(h, r, z, state, st);
    }
}

hipError_t launch_apply(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    return h->bs == 3 ? launch_bs<3>(h, r, z, state, st) : launch_bs<1>(h, r, z, state, st);
}

// a = M_DD^{-T} g: the slot kernel run on the transposed factor streams (FP64,
// no correction); needs 3x3 blocks, the slot layout and one-pass levels.
template <int NT>
static hipError_t launch_adjoint_nt(dd_ctx *h, const double *g, double *a, hipStream_t st) {
    constexpr int RPP = (kWave / 3) * (NT / kWave);
    if (h->max_level_width > RPP) return hipErrorInvalidValue;
    const double *lv = h->lic.adj_val[0], *uv = h->lic.adj_val[1];
    return launch_slots_mb<3, double, double, NT, false>(h, g, a, nullptr, st, lv, uv);
}

hipError_t launch_apply_adjoint(dd_ctx *h, const double *g, double *a, hipStream_t st) {
    if (h->bs != 3 || !h->slots || !h->lic.ready) return hipErrorInvalidValue;
    switch (pick_threads(h)) {
        case 64: return launch_adjoint_nt<64>(h, g, a, st);
        case 128: return launch_adjoint_nt<128>(h, g, a, st);
        case 256: return launch_adjoint_nt<256>(h, g, a, st);
        case 512: return launch_adjoint_nt<512>(h, g, a, st);
        default: return launch_adjoint_nt<1024>(h, g, a, st);
    }
}

hipError_t launch_precond(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    if (h->pc_kind == 1) return launch_global_apply(h, r, z, 1, st);
    return launch_apply(h, r, z, state, st);
}

}  // namespace ddilu
