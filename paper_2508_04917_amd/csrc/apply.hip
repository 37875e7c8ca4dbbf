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
#include "internal.h"

namespace ddilu {

template <int BS, typename T, int NT>
__global__ __launch_bounds__(NT) void k_dd_apply(
    const double *__restrict__ r, double *__restrict__ z, int S,
    const int32_t *__restrict__ Loff, const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow,
    const int32_t *__restrict__ Lbp, const uint16_t *__restrict__ Lcol, const T *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow,
    const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol, const T *__restrict__ Uval,
    const T *__restrict__ Dval, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;  // enclosing solve already finished
    constexpr int BB = BS * BS;
    constexpr int RPW = kWave / BS;         // block rows per wavefront
    constexpr int RPP = RPW * (NT / kWave); // block rows per pass of the workgroup
    extern __shared__ unsigned char dd_smem[];
    T *y = reinterpret_cast<T *>(dd_smem);

    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int c = lane % BS, rl = lane / BS;
    const bool lane_ok = rl < RPW;

    const double *rs = r + base * BS;
    for (int i = tid; i < S * BS; i += NT) y[i] = static_cast<T>(rs[i]);
    __syncthreads();

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
                    T acc = y[I * BS + c];
                    const int32_t b1 = Lbp[gp + 1];
                    for (int32_t b = Lbp[gp]; b < b1; ++b) {
                        const int J = Lcol[b];
                        const T *blk = Lval + (int64_t)b * BB + c * BS;
#pragma unroll
                        for (int d = 0; d < BS; ++d) acc -= blk[d] * y[J * BS + d];
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
                    const T *dblk = Dval + gp * BB + c * BS;
                    T acc = 0;
#pragma unroll
                    for (int d = 0; d < BS; ++d) acc += dblk[d] * y[I * BS + d];
                    const int32_t b1 = Ubp[gp + 1];
                    for (int32_t b = Ubp[gp]; b < b1; ++b) {
                        const int K = Ucol[b];
                        const T *blk = Uval + (int64_t)b * BB + c * BS;
#pragma unroll
                        for (int d = 0; d < BS; ++d) acc -= blk[d] * y[K * BS + d];
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
    for (int i = tid; i < S * BS; i += NT) zs[i] = static_cast<double>(y[i]);
}

// Software-pipelined variant for subdomains whose widest level fits one pass
// of the workgroup (every level is handled by one lane group per row).
// The factor data of a level does not depend on the solve, so it is fetched
// ahead: while level l computes from LDS, the blocks of level l+1 are already
// in flight into registers and the row metadata of level l+2 behind them.
// The level barrier only orders LDS traffic; it does not wait for these
// global loads, so HBM latency overlaps the level chain.  Rows with more
// than MB blocks take the extra blocks through a direct (unpipelined) loop.
template <int BS, typename T, int MB>
struct LevelRegs {
    bool ok;
    int I, b0, nb;
    int J[MB];
    T v[MB][BS];
    T d[BS];
};

template <int BS, typename T, int MB, bool UPPER>
__device__ __forceinline__ void load_meta(const uint16_t *__restrict__ prow, const int32_t *__restrict__ bp,
                                          int64_t gp, bool ok, int &I, int &b0, int &nb) {
    if (ok) {
        I = prow[gp];
        b0 = bp[gp];
        nb = bp[gp + 1] - b0;
    } else {
        I = 0;
        b0 = 0;
        nb = 0;
    }
}

template <int BS, typename T, int MB, bool UPPER>
__device__ __forceinline__ void load_vals(LevelRegs<BS, T, MB> &R, const uint16_t *__restrict__ col,
                                          const T *__restrict__ val, const T *__restrict__ dval, int64_t gp,
                                          bool ok, int c) {
    constexpr int BB = BS * BS;
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        if (k < R.nb) {
            const int64_t b = R.b0 + k;
            R.J[k] = col[b];
            const T *blk = val + b * BB + c * BS;
#pragma unroll
            for (int d = 0; d < BS; ++d) R.v[k][d] = blk[d];
        }
    }
    if constexpr (UPPER) {
        if (ok) {
            const T *dblk = dval + gp * BB + c * BS;
#pragma unroll
            for (int d = 0; d < BS; ++d) R.d[d] = dblk[d];
        }
    }
}

// Row metadata of one lane at one level.
struct LevelMeta {
    int64_t gp;
    bool ok;
    int I, b0, nb;
};

// Compute one level from the registers R and the LDS vector y.
template <int BS, typename T, int MB, bool UPPER>
__device__ __forceinline__ void level_compute(T *__restrict__ y, const LevelRegs<BS, T, MB> &R,
                                              const uint16_t *__restrict__ col, const T *__restrict__ val, int c) {
    constexpr int BB = BS * BS;
    if (!R.ok) return;
    const int I = R.I;
    T acc;
    if constexpr (UPPER) {
        acc = 0;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc += R.d[d] * y[I * BS + d];
    } else {
        acc = y[I * BS + c];
    }
#pragma unroll
    for (int k = 0; k < MB; ++k) {
        if (k < R.nb) {
            const int J = R.J[k];
#pragma unroll
            for (int d = 0; d < BS; ++d) acc -= R.v[k][d] * y[J * BS + d];
        }
    }
    for (int k = MB; k < R.nb; ++k) {  // rows longer than the register window
        const int64_t b = R.b0 + k;
        const int J = col[b];
        const T *blk = val + b * BB + c * BS;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc -= blk[d] * y[J * BS + d];
    }
    // all lanes of this row read y_I above (same wavefront)
    __asm__ volatile("" ::: "memory");
    y[I * BS + c] = acc;
}

template <int BS, typename T, int NT, int MB, bool UPPER>
__device__ __forceinline__ void sweep_pipelined(T *__restrict__ y, int64_t base, int s,
                                                const int32_t *__restrict__ off, const int32_t *__restrict__ lp,
                                                const uint16_t *__restrict__ prow, const int32_t *__restrict__ bp,
                                                const uint16_t *__restrict__ col, const T *__restrict__ val,
                                                const T *__restrict__ dval, int slot, bool lane_ok, int c) {
    const int32_t o = off[s];
    const int nl = off[s + 1] - o - 1;
    if (nl <= 0) return;
    auto meta = [&](int l) -> LevelMeta {
        LevelMeta m;
        const int32_t p0 = lp[o + l], p1 = lp[o + l + 1];
        const int32_t p = p0 + slot;
        m.ok = lane_ok && p < p1;
        m.gp = base + p;
        load_meta<BS, T, MB, UPPER>(prow, bp, m.gp, m.ok, m.I, m.b0, m.nb);
        return m;
    };
    auto fetch = [&](LevelRegs<BS, T, MB> &R, const LevelMeta &m) {
        R.ok = m.ok;
        R.I = m.I;
        R.b0 = m.b0;
        R.nb = m.nb;
        load_vals<BS, T, MB, UPPER>(R, col, val, dval, m.gp, m.ok, c);
    };
    // Two register sets, A and B, alternate between "being computed" and
    // "being filled"; the loop is unrolled by two so that neither is copied
    // (a copy of a register with a load in flight would wait for the load).
    LevelRegs<BS, T, MB> A, B;
    LevelMeta mA = meta(0);
    fetch(A, mA);
    LevelMeta mB;
    mB.ok = false;
    if (nl > 1) mB = meta(1);
    for (int l = 0; l < nl; l += 2) {
        // level l from A; fill B with level l+1; metadata of level l+2
        if (l + 1 < nl) fetch(B, mB);
        if (l + 2 < nl) mA = meta(l + 2);
        level_compute<BS, T, MB, UPPER>(y, A, col, val, c);
        __syncthreads();
        if (l + 1 >= nl) break;
        // level l+1 from B; fill A with level l+2; metadata of level l+3
        if (l + 2 < nl) fetch(A, mA);
        if (l + 3 < nl) mB = meta(l + 3);
        level_compute<BS, T, MB, UPPER>(y, B, col, val, c);
        __syncthreads();
    }
}

template <int BS, typename T, int NT, int MB>
__global__ __launch_bounds__(NT) void k_dd_apply_pipe(
    const double *__restrict__ r, double *__restrict__ z, int S,
    const int32_t *__restrict__ Loff, const int32_t *__restrict__ Llp, const uint16_t *__restrict__ Lrow,
    const int32_t *__restrict__ Lbp, const uint16_t *__restrict__ Lcol, const T *__restrict__ Lval,
    const int32_t *__restrict__ Uoff, const int32_t *__restrict__ Ulp, const uint16_t *__restrict__ Urow,
    const int32_t *__restrict__ Ubp, const uint16_t *__restrict__ Ucol, const T *__restrict__ Uval,
    const T *__restrict__ Dval, const int32_t *__restrict__ state) {
    if (state != nullptr && *state != 0) return;
    constexpr int RPW = kWave / BS;
    extern __shared__ unsigned char dd_smem[];
    T *y = reinterpret_cast<T *>(dd_smem);
    const int s = blockIdx.x;
    const int64_t base = (int64_t)s * S;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int c = lane % BS, rl = lane / BS;
    const bool lane_ok = rl < RPW;
    const int slot = wave * RPW + rl;

    const double *rs = r + base * BS;
    for (int i = tid; i < S * BS; i += NT) y[i] = static_cast<T>(rs[i]);
    __syncthreads();
    sweep_pipelined<BS, T, NT, MB, false>(y, base, s, Loff, Llp, Lrow, Lbp, Lcol, Lval, nullptr, slot, lane_ok, c);
    sweep_pipelined<BS, T, NT, MB, true>(y, base, s, Uoff, Ulp, Urow, Ubp, Ucol, Uval, Dval, slot, lane_ok, c);
    double *zs = z + base * BS;
    for (int i = tid; i < S * BS; i += NT) zs[i] = static_cast<double>(y[i]);
}

int apply_lds_bytes(const dd_ctx *h, int precision) {
    return h->S * h->bs * (precision == DD_FP32 ? 4 : 8);
}

template <typename K>
static hipError_t allow_full_lds(K kern) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               163840);
}

template <int BS, typename T, int NT>
static hipError_t launch_typed(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    const Sweep &L = h->sw[0], &U = h->sw[1];
    const T *lv, *uv, *dv;
    if constexpr (sizeof(T) == 8) {
        lv = L.val64; uv = U.val64; dv = U.d64;
    } else {
        lv = L.val32; uv = U.val32; dv = U.d32;
    }
    const int lds = h->S * BS * (int)sizeof(T);
    constexpr int RPP = (kWave / BS) * (NT / kWave);
    if (h->max_level_width <= RPP && h->use_pipeline) {
        constexpr int MB = BS == 3 ? 3 : 3;
        auto kern = k_dd_apply_pipe<BS, T, NT, MB>;
        static bool attr_done = false;
        if (!attr_done) {
            hipError_t e = allow_full_lds(kern);
            if (e != hipSuccess) return e;
            attr_done = true;
        }
        kern<<<h->nsub, NT, lds, st>>>(r, z, h->S, h->lev[0].off, h->lev[0].ptr, L.prow, L.bptr, L.bcol, lv,
                                       h->lev[1].off, h->lev[1].ptr, U.prow, U.bptr, U.bcol, uv, dv, state);
        return hipGetLastError();
    }
    auto kern = k_dd_apply<BS, T, NT>;
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = allow_full_lds(kern);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    kern<<<h->nsub, NT, lds, st>>>(r, z, h->S, h->lev[0].off, h->lev[0].ptr, L.prow, L.bptr, L.bcol, lv,
                                   h->lev[1].off, h->lev[1].ptr, U.prow, U.bptr, U.bcol, uv, dv, state);
    return hipGetLastError();
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

template <int BS, typename T>
static hipError_t launch_nt(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    switch (pick_threads(h)) {
        case 64: return launch_typed<BS, T, 64>(h, r, z, state, st);
        case 128: return launch_typed<BS, T, 128>(h, r, z, state, st);
        case 256: return launch_typed<BS, T, 256>(h, r, z, state, st);
        case 512: return launch_typed<BS, T, 512>(h, r, z, state, st);
        default: return launch_typed<BS, T, 1024>(h, r, z, state, st);
    }
}

hipError_t launch_apply(dd_ctx *h, const double *r, double *z, const int32_t *state, hipStream_t st) {
    if (h->bs == 3)
        return h->precision == DD_FP32 ? launch_nt<3, float>(h, r, z, state, st)
                                       : launch_nt<3, double>(h, r, z, state, st);
    return h->precision == DD_FP32 ? launch_nt<1, float>(h, r, z, state, st)
                                   : launch_nt<1, double>(h, r, z, state, st);
}

}  // namespace ddilu
