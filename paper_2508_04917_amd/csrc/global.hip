// Global (undecomposed) ILU0 of the full reordered matrix: the preconditioner
// the decomposition approximates.  It serves as the regression target of the
// learned interface correction and as the reference for the iterations the
// decomposition costs.
//
// Everything runs level by level over the whole matrix, one kernel launch per
// level, with the vector in global memory: rows whose level equals the
// launch's level are processed ("if hmap[i] == level", Section 4.2.2); the
// level of a row is its longest dependency path (Section 4.2.1), computed by
// repeated relaxation lev_I = max over dependencies J of lev_J + 1.
#include "internal.h"

namespace ddilu {

// One relaxation step of the longest-path levels (which = 0: J < I, 1: J > I).
__global__ void k_glev_relax(int64_t n, int which, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             const int32_t *__restrict__ lev_in, int32_t *__restrict__ lev_out, int32_t *changed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t l = 0;
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int32_t c = col[q];
        if (which == 0 ? (c < i) : (c > i)) l = max(l, lev_in[c] + 1);
    }
    lev_out[i] = l;
    if (l != lev_in[i]) atomicOr(changed, 1);
}

__global__ void k_gdiag(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col, int32_t *diag,
                        int32_t *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t d = -1;
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q)
        if (col[q] == i) d = q;
    diag[i] = d;
    if (d < 0) atomicMin(&status[1], (int32_t)i);
}

template <int BS>
__device__ __forceinline__ void gblk_mul(const double *A, const double *B, double *C) {
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
__device__ bool gblk_inverse(const double *a, double *inv) {
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
        double n1 = 0.0, n2 = 0.0;
        for (int j = 0; j < 3; ++j) {
            n1 = fmax(n1, fabs(a[j]) + fabs(a[3 + j]) + fabs(a[6 + j]));
            n2 = fmax(n2, fabs(inv[j]) + fabs(inv[3 + j]) + fabs(inv[6 + j]));
        }
        return n1 * n2 <= 1e14;
    }
}

// Block ILU0 (Algorithm 5, IKJ order) for the rows of one level.
template <int BS>
__global__ void k_gbilu0_level(int64_t n, int level, const int32_t *__restrict__ lev, const int32_t *__restrict__ ptr,
                               const int32_t *__restrict__ col, const int32_t *__restrict__ diag, double *lu,
                               double *invd, int32_t *status) {
    constexpr int BB = BS * BS;
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n || lev[gi] != level) return;
    const int32_t tb = ptr[gi], te = ptr[gi + 1];
    for (int32_t pj = tb; pj < te; ++pj) {
        const int32_t J = col[pj];
        if (J >= gi) break;
        double Lij[BB];
        gblk_mul<BS>(lu + (int64_t)pj * BB, invd + (int64_t)J * BB, Lij);
#pragma unroll
        for (int e = 0; e < BB; ++e) lu[(int64_t)pj * BB + e] = Lij[e];
        const int32_t je = ptr[J + 1];
        int32_t q = ptr[J];
        for (int32_t pk = pj + 1; pk < te; ++pk) {
            const int32_t K = col[pk];
            while (q < je && col[q] < K) ++q;
            if (q < je && col[q] == K) {
                double t[BB];
                gblk_mul<BS>(Lij, lu + (int64_t)q * BB, t);
#pragma unroll
                for (int e = 0; e < BB; ++e) lu[(int64_t)pk * BB + e] -= t[e];
            }
        }
    }
    double inv[BB];
    if (!gblk_inverse<BS>(lu + (int64_t)diag[gi] * BB, inv)) {
        atomicMin(&status[2], (int32_t)gi);
#pragma unroll
        for (int e = 0; e < BB; ++e) inv[e] = (e % (BS + 1) == 0) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < BB; ++e) invd[gi * BB + e] = inv[e];
}

// ILDU0 form in the full pattern: L (lower), inv_D (diagonal), Uhat = inv_D U.
template <int BS>
__global__ void k_gildu0(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                         const double *__restrict__ lu, const double *__restrict__ invd, double *f) {
    constexpr int BB = BS * BS;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *inv = invd + i * BB;
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int32_t c = col[q];
        double t[BB];
        if (c < i) {
#pragma unroll
            for (int e = 0; e < BB; ++e) t[e] = lu[(int64_t)q * BB + e];
        } else if (c == i) {
#pragma unroll
            for (int e = 0; e < BB; ++e) t[e] = inv[e];
        } else {
            gblk_mul<BS>(inv, lu + (int64_t)q * BB, t);
        }
#pragma unroll
        for (int e = 0; e < BB; ++e) f[(int64_t)q * BB + e] = t[e];
    }
}

// One level of the global forward (UPPER = false: y_I = r_I - sum_{J<I} L_IJ y_J,
// y kept in z) or backward sweep (z_I = inv_D_I y_I - sum_{K>I} Uhat_IK z_K).
// BS lanes of one wavefront per row; nrhs right-hand sides along grid y.
template <int BS, bool UPPER>
__global__ void k_gsweep_level(int64_t n, int level, const int32_t *__restrict__ lev,
                               const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                               const int32_t *__restrict__ diag, const double *__restrict__ f,
                               const double *__restrict__ r, double *z) {
    constexpr int BB = BS * BS, RPW = kWave / BS;
    const int lane = threadIdx.x & 63;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t i = gw * RPW + lane / BS;
    const int c = lane % BS;
    const int64_t off = (int64_t)blockIdx.y * n * BS;
    if (lane / BS >= RPW || i >= n || lev[i] != level) return;
    const double *rr = r + off;
    double *zz = z + off;
    double acc;
    if constexpr (UPPER) {
        const double *dblk = f + (int64_t)diag[i] * BB + c * BS;
        acc = 0.0;
#pragma unroll
        for (int d = 0; d < BS; ++d) acc += dblk[d] * zz[i * BS + d];
    } else {
        acc = rr[i * BS + c];
    }
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int64_t J = col[q];
        if (UPPER ? (J > i) : (J < i)) {
            const double *blk = f + (int64_t)q * BB + c * BS;
#pragma unroll
            for (int d = 0; d < BS; ++d) acc -= blk[d] * zz[J * BS + d];
        }
    }
    // the BS lanes of row i (one wavefront) have read z_i above
    __asm__ volatile("" ::: "memory");
    zz[i * BS + c] = acc;
}

static int glevels(dd_ctx *h, int which, int32_t *lev, int32_t *tmp, int32_t *flag, hipStream_t st, int *nlev) {
    const int T = 256;
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    (void)hipMemsetAsync(lev, 0, h->n * sizeof(int32_t), st);
    int32_t *a = lev, *b = tmp;
    for (int it = 0;; ++it) {
        int32_t changed = 0;
        hipError_t e = hipMemsetAsync(flag, 0, sizeof(int32_t), st);
        if (e != hipSuccess) return h->fail(DD_EHIP, "memset: %s", hipGetErrorString(e));
        k_glev_relax<<<g, T, 0, st>>>(h->n, which, h->aptr, h->acol, a, b, flag);
        e = hipMemcpyAsync(&changed, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return h->fail(DD_EHIP, "global levels: %s", hipGetErrorString(e));
        std::swap(a, b);
        if (!changed) break;
        if (it > h->n) return h->fail(DD_EINVAL, "global levels did not converge");
    }
    if (a != lev) {
        hipError_t e = hipMemcpyAsync(lev, a, h->n * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return h->fail(DD_EHIP, "copy: %s", hipGetErrorString(e));
    }
    // number of levels = 1 + max level
    std::vector<int32_t> host(h->n);
    hipError_t e = hipMemcpyAsync(host.data(), lev, h->n * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "level readback: %s", hipGetErrorString(e));
    int m = 0;
    for (int32_t v : host) m = std::max(m, v);
    *nlev = m + 1;
    return DD_OK;
}

hipError_t launch_diag_positions(dd_ctx *h, int32_t *diag, hipStream_t st) {
    const int T = 256;
    k_gdiag<<<(unsigned)((h->n + T - 1) / T), T, 0, st>>>(h->n, h->aptr, h->acol, diag, h->status);
    return hipGetLastError();
}

int global_factor(dd_ctx *h, hipStream_t st) {
    const int bb = h->bs * h->bs;
    if (!h->glev[0]) {
        for (int w = 0; w < 2; ++w) {
            int rc = h->alloc(&h->glev[w], h->n);
            if (rc) return rc;
        }
        int rc = h->alloc(&h->gdiag, h->n);
        if (!rc) rc = h->alloc(&h->glu, h->nnzb * bb);
        if (!rc) rc = h->alloc(&h->ginvd, h->n * bb);
        if (!rc) rc = h->alloc(&h->gf, h->nnzb * bb);
        if (rc) return rc;
    }
    int32_t *tmp = nullptr;
    int rc = h->alloc(&tmp, h->n);
    if (rc) return rc;
    int32_t init_status[8] = {0, 0x7fffffff, 0x7fffffff, 0, 0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(h->status, init_status, sizeof(init_status), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "memcpy: %s", hipGetErrorString(e));
    for (int w = 0; w < 2; ++w) {
        rc = glevels(h, w, h->glev[w], tmp, h->status + 5, st, &h->gnlev[w]);
        if (rc) return rc;
    }
    const int T = 256;
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    k_gdiag<<<g, T, 0, st>>>(h->n, h->aptr, h->acol, h->gdiag, h->status);
    e = hipMemcpyAsync(h->glu, h->aval, h->nnzb * bb * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "memcpy: %s", hipGetErrorString(e));
    for (int l = 0; l < h->gnlev[0]; ++l) {
        if (h->bs == 3)
            k_gbilu0_level<3><<<g, T, 0, st>>>(h->n, l, h->glev[0], h->aptr, h->acol, h->gdiag, h->glu, h->ginvd,
                                               h->status);
        else
            k_gbilu0_level<1><<<g, T, 0, st>>>(h->n, l, h->glev[0], h->aptr, h->acol, h->gdiag, h->glu, h->ginvd,
                                               h->status);
    }
    if (h->bs == 3)
        k_gildu0<3><<<g, T, 0, st>>>(h->n, h->aptr, h->acol, h->glu, h->ginvd, h->gf);
    else
        k_gildu0<1><<<g, T, 0, st>>>(h->n, h->aptr, h->acol, h->glu, h->ginvd, h->gf);
    int32_t status[8];
    e = hipMemcpyAsync(status, h->status, sizeof(status), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void *)tmp));
    (void)hipFree(tmp);
    if (e != hipSuccess) return h->fail(DD_EHIP, "global factor: %s", hipGetErrorString(e));
    if (status[1] != 0x7fffffff) return h->fail(DD_EZEROPIVOT, "block row %d has no diagonal block", status[1]);
    if (status[2] != 0x7fffffff)
        return h->fail(DD_EZEROPIVOT, "global ILU0: singular pivot at reordered block row %d", status[2]);
    h->gfactored = 1;
    return DD_OK;
}

hipError_t launch_global_apply(dd_ctx *h, const double *r, double *z, int nrhs, hipStream_t st) {
    const int T = 256;
    const int rpb = (kWave / h->bs) * (T / kWave);
    const dim3 grid((unsigned)((h->n + rpb - 1) / rpb), (unsigned)nrhs);
    for (int l = 0; l < h->gnlev[0]; ++l) {
        if (h->bs == 3)
            k_gsweep_level<3, false><<<grid, T, 0, st>>>(h->n, l, h->glev[0], h->aptr, h->acol, h->gdiag, h->gf, r, z);
        else
            k_gsweep_level<1, false><<<grid, T, 0, st>>>(h->n, l, h->glev[0], h->aptr, h->acol, h->gdiag, h->gf, r, z);
    }
    for (int l = 0; l < h->gnlev[1]; ++l) {
        if (h->bs == 3)
            k_gsweep_level<3, true><<<grid, T, 0, st>>>(h->n, l, h->glev[1], h->aptr, h->acol, h->gdiag, h->gf, r, z);
        else
            k_gsweep_level<1, true><<<grid, T, 0, st>>>(h->n, l, h->glev[1], h->aptr, h->acol, h->gdiag, h->gf, r, z);
    }
    return hipGetLastError();
}

}  // namespace ddilu
