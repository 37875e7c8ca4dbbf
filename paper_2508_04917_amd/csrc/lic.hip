// Learned interface correction (an addition to the paper's method; the paper
// has no learned component).
//
// Faces are the directed cut pairs (I, J): the blocks A_IJ of the full
// reordered matrix whose row and column lie in different subdomains (the
// blocks the drop removes), in CSR order.  A per-face MLP 27 -> 64 -> 64 -> 9
// (FP32) maps x_f = [A_II, A_IJ, A_JJ] / sigma_f, sigma_f =
// sqrt(|tr A_II| |tr A_JJ|) / 3, to a 3x3 coefficient C_f, and the
// preconditioner becomes z = M_DD^{-1} (r + C r), (C r)_I = sum_f C_f r_J:
// a fixed linear operator once C is set, so BiCGSTAB stays valid.  The
// correction is applied inside the apply kernel right after the subdomain's
// r is staged in LDS (it reads only r).
//
// Training regresses the corrected apply onto the global ILU0 apply on probe
// vectors: loss = mean_q ||z_q - z*_q||^2 / ||z_DD,q - z*_q||^2; its
// gradient is dL/dC_f = sum_q a_q[I] r_q[J]^T with a_q = M_DD^{-T} g_q,
// g_q = 2 (z_q - z*_q) / (Q den_q), computed with the same apply kernel run
// on the transposed factors, then backpropagated through the MLP.
#include "internal.h"

namespace ddilu {

constexpr int kIn = 27, kHid = 64, kOut = 9;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid, kNParam = oB3 + kOut;
static_assert(kNParam == 6537, "parameter count");

// ------------------------------------------------------------------ faces
__global__ void k_face_count(int64_t n, int S, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                             int32_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = i / S;
    int c = 0;
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) c += (col[q] / S != s);
    cnt[i] = c;
}

__global__ void k_face_fill(int64_t n, int S, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ fptr, int32_t *fI, int32_t *fJ, int32_t *fq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = i / S;
    int32_t f = fptr[i];
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q)
        if (col[q] / S != s) {
            fI[f] = (int32_t)i;
            fJ[f] = col[q];
            fq[f] = q;
            ++f;
        }
}

// rows with at least one face: flag for the boundary-row compaction
__global__ void k_bflag(int64_t n, const int32_t *__restrict__ fptr, int32_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = fptr[i + 1] > fptr[i];
}

__global__ void k_bfill(int64_t n, int S, const int32_t *__restrict__ fptr, const int32_t *__restrict__ bpos,
                        int4 *brow, int32_t *bsub) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (fptr[i + 1] > fptr[i]) brow[bpos[i]] = make_int4((int32_t)i, fptr[i], fptr[i + 1] - fptr[i], 0);
    if (i % S == 0) bsub[i / S] = bpos[i];  // first boundary row of the subdomain
}

__global__ void k_sym_check(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            int32_t *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t q = ptr[i]; q < ptr[i + 1]; ++q) {
        const int32_t j = col[q];
        bool found = false;
        for (int32_t r = ptr[j]; r < ptr[j + 1]; ++r) found |= (col[r] == i);
        if (!found) atomicMax(&status[6], 1);
    }
}

__global__ void k_features(int64_t nf, const int32_t *__restrict__ fI, const int32_t *__restrict__ fJ,
                           const int32_t *__restrict__ fq, const int32_t *__restrict__ diag,
                           const double *__restrict__ val, float *X) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const double *Aii = val + (int64_t)diag[fI[f]] * 9, *Aij = val + (int64_t)fq[f] * 9;
    const double *Ajj = val + (int64_t)diag[fJ[f]] * 9;
    const double ti = Aii[0] + Aii[4] + Aii[8], tj = Ajj[0] + Ajj[4] + Ajj[8];
    const double sigma = sqrt(fabs(ti) * fabs(tj)) / 3.0;
    float *x = X + f * kIn;
    for (int e = 0; e < 9; ++e) {
        x[e] = (float)(Aii[e] / sigma);
        x[9 + e] = (float)(Aij[e] / sigma);
        x[18 + e] = (float)(Ajj[e] / sigma);
    }
}

// ---------------------------------------------------------------- MLP (FP32)
// One thread per face; the 6,537 parameters are staged in LDS.  When H1/H2
// are given the hidden activations are kept for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_forward(int64_t nf, const float *__restrict__ P,
                                                     const float *__restrict__ X, float *__restrict__ C,
                                                     float *__restrict__ H1, float *__restrict__ H2) {
    __shared__ float w[kNParam];
    for (int i = threadIdx.x; i < kNParam; i += blockDim.x) w[i] = P[i];
    __syncthreads();
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    float x[kIn], h1[kHid], h2[kHid];
#pragma unroll
    for (int k = 0; k < kIn; ++k) x[k] = X[f * kIn + k];
#pragma unroll
    for (int i = 0; i < kHid; ++i) {
        float s = w[oB1 + i];
#pragma unroll
        for (int k = 0; k < kIn; ++k) s += w[oW1 + i * kIn + k] * x[k];
        h1[i] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kHid; ++i) {
        float s = w[oB2 + i];
#pragma unroll
        for (int k = 0; k < kHid; ++k) s += w[oW2 + i * kHid + k] * h1[k];
        h2[i] = s > 0.f ? s : 0.f;
    }
    for (int i = 0; i < kOut; ++i) {
        float s = w[oB3 + i];
#pragma unroll
        for (int k = 0; k < kHid; ++k) s += w[oW3 + i * kHid + k] * h2[k];
        C[f * kOut + i] = s;
    }
    if (H1) {
#pragma unroll
        for (int k = 0; k < kHid; ++k) {
            H1[f * kHid + k] = h1[k];
            H2[f * kHid + k] = h2[k];
        }
    }
}

// Backward through the two hidden layers, per face: G2 = W3^T dOUT (masked by
// h2 > 0), G1 = W2^T G2 (masked by h1 > 0).
__global__ __launch_bounds__(256) void k_mlp_backprop(int64_t nf, const float *__restrict__ P,
                                                      const float *__restrict__ dOUT, const float *__restrict__ H1,
                                                      const float *__restrict__ H2, float *__restrict__ G1,
                                                      float *__restrict__ G2) {
    __shared__ float w[kNParam];
    for (int i = threadIdx.x; i < kNParam; i += blockDim.x) w[i] = P[i];
    __syncthreads();
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    float d[kOut], g2[kHid];
#pragma unroll
    for (int i = 0; i < kOut; ++i) d[i] = dOUT[f * kOut + i];
#pragma unroll
    for (int k = 0; k < kHid; ++k) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < kOut; ++i) s += w[oW3 + i * kHid + k] * d[i];
        g2[k] = H2[f * kHid + k] > 0.f ? s : 0.f;
        G2[f * kHid + k] = g2[k];
    }
#pragma unroll
    for (int k = 0; k < kHid; ++k) {
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < kHid; ++i) s += w[oW2 + i * kHid + k] * g2[i];
        G1[f * kHid + k] = H1[f * kHid + k] > 0.f ? s : 0.f;
    }
}

// Weight gradients as sums over faces, deterministic: workgroup (chunk, layer)
// sums its chunk of faces for every output entry in a fixed order into a FP64
// partial; k_wgrad_sum adds the chunk partials in order.
// Layer l: out[i][k] = sum_f A[f][i] B[f][k] (A = dOUT/G2/G1, B = H2/H1/X),
// bias[i] = sum_f A[f][i].
constexpr int kFaceChunk = 1024;

__global__ __launch_bounds__(256) void k_wgrad_partial(int64_t nf, const float *__restrict__ dOUT,
                                                       const float *__restrict__ G2, const float *__restrict__ G1,
                                                       const float *__restrict__ H2, const float *__restrict__ H1,
                                                       const float *__restrict__ X, double *__restrict__ part) {
    const int chunk = blockIdx.x, layer = blockIdx.y;
    const float *A, *B;
    int na, nb, ow, ob;
    if (layer == 0) { A = dOUT; na = kOut; B = H2; nb = kHid; ow = oW3; ob = oB3; }
    else if (layer == 1) { A = G2; na = kHid; B = H1; nb = kHid; ow = oW2; ob = oB2; }
    else { A = G1; na = kHid; B = X; nb = kIn; ow = oW1; ob = oB1; }
    const int64_t f0 = (int64_t)chunk * kFaceChunk;
    const int64_t f1 = f0 + kFaceChunk < nf ? f0 + kFaceChunk : nf;
    double *out = part + (int64_t)chunk * kNParam;
    for (int e = threadIdx.x; e < na * (nb + 1); e += blockDim.x) {
        const int i = e / (nb + 1), k = e % (nb + 1);
        double s = 0.0;
        if (k < nb) {
            for (int64_t f = f0; f < f1; ++f) s += (double)A[f * na + i] * (double)B[f * nb + k];
            out[ow + i * nb + k] = s;
        } else {
            for (int64_t f = f0; f < f1; ++f) s += (double)A[f * na + i];
            out[ob + i] = s;
        }
    }
}

__global__ void k_wgrad_sum(int nchunk, const double *__restrict__ part, float *grad, int accumulate) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNParam) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * kNParam + e];
    grad[e] = accumulate ? grad[e] + (float)s : (float)s;
}

// ----------------------------------------------------------- training steps
// g = 2 (z - z*) / (Q den_q) for probe q (grid.y), and per-workgroup partial
// sums of ||z - z*||^2.
__global__ __launch_bounds__(256) void k_lic_residual(int64_t m, const double *__restrict__ z,
                                                      const double *__restrict__ zs, const double *__restrict__ den,
                                                      int Q, double *__restrict__ g, double *__restrict__ part,
                                                      int part_stride) {
    const int q = blockIdx.y;
    const double sc = 2.0 / (Q * den[q]);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const double e = z[q * m + i] - zs[q * m + i];
        g[q * m + i] = sc * e;
        acc += e * e;
    }
    __shared__ double sh[4];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
        part[q * part_stride + blockIdx.x] = t;
    }
}

// loss += sum_q (sum of partials of probe q) / (Q den_q); one thread.
__global__ void k_lic_loss(int Q, int nblk, int part_stride, const double *__restrict__ part,
                           const double *__restrict__ den, double *loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double L = 0.0;
    for (int q = 0; q < Q; ++q) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[q * part_stride + b];
        L += s / (Q * den[q]);
    }
    *loss += L;
}

// den_q = ||z_DD,q - z*_q||^2 (one workgroup per probe, fixed order).
__global__ __launch_bounds__(256) void k_lic_den(int64_t m, const double *__restrict__ zdd,
                                                 const double *__restrict__ zs, double *den) {
    const int q = blockIdx.x;
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
        const double e = zdd[q * m + i] - zs[q * m + i];
        acc += e * e;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) den[q] = sh[0];
}

// dC_f[a][b] = sum_q a_q[I][a] r_q[J][b] (FP32 result, FP64 sum).
__global__ void k_lic_dC(int64_t nf, int64_t m, int Q, const int32_t *__restrict__ fI, const int32_t *__restrict__ fJ,
                         const double *__restrict__ A, const double *__restrict__ R, float *dC) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nf * 9) return;
    const int64_t f = t / 9;
    const int a = (int)(t % 9) / 3, b = (int)(t % 3);
    const int64_t I = fI[f], J = fJ[f];
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += A[q * m + I * 3 + a] * R[q * m + J * 3 + b];
    dC[t] = (float)s;
}

// Adam (Kingma & Ba) on FP32 parameters.
__global__ void k_adam(int np, float *P, const float *__restrict__ G, float *M, float *V, float c1, float c2, float lr,
                       float b1, float b2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float g = G[i];
    const float m = b1 * M[i] + (1.f - b1) * g;
    const float v = b2 * V[i] + (1.f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ------------------------------------------------------------ adjoint streams
// Values of the transposed sweeps in the slot layout (same positions and
// columns as the forward sweeps, which requires a structurally symmetric
// pattern; lane-contiguous runs as in the forward streams): lower sweep of
// U^T: slot k of row I holds (Uhat_{J_k I})^T; upper sweep of L^T: slot k
// holds (L_{K_k I})^T, followed by inv_D_I^T.
__global__ void k_pack_adjoint(int64_t n, int S, int which, int MB, const int32_t *__restrict__ tptr,
                               const int32_t *__restrict__ tcol, const double *__restrict__ lu,
                               const double *__restrict__ invd, const int32_t *__restrict__ rows, double *sval) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t base = (p / S) * (int64_t)S;
    const int64_t gi = base + rows[p];
    const int NV = (MB + which) * 3;
    double *o = sval + p * 3 * NV;
    int k = 0;
    for (int32_t q = tptr[gi]; q < tptr[gi + 1] && k < MB; ++q) {
        const int32_t c = tcol[q];
        if (which == 0 ? (c < gi) : (c > gi)) {
            int32_t qt = -1;  // position of (c, gi) in row c (exists: symmetric pattern)
            for (int32_t r = tptr[c]; r < tptr[c + 1]; ++r)
                if (tcol[r] == gi) qt = r;
            double blk[9];
            if (qt < 0) {
                for (int e = 0; e < 9; ++e) blk[e] = 0.0;
            } else if (which == 0) {  // Uhat_{c,gi} = inv_D_c U_{c,gi}
                const double *a = invd + (int64_t)c * 9, *b = lu + (int64_t)qt * 9;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double s = 0.0;
                        for (int l = 0; l < 3; ++l) s += a[i * 3 + l] * b[l * 3 + j];
                        blk[i * 3 + j] = s;
                    }
            } else {  // L_{c,gi}
                for (int e = 0; e < 9; ++e) blk[e] = lu[(int64_t)qt * 9 + e];
            }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) o[i * NV + k * 3 + j] = blk[j * 3 + i];
            ++k;
        }
    }
    for (; k < MB; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) o[i * NV + k * 3 + j] = 0.0;
    if (which == 1) {
        const double *a = invd + gi * 9;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) o[i * NV + MB * 3 + j] = a[j * 3 + i];
    }
}

// ------------------------------------------------------------------ setup
int lic_setup(dd_ctx *h, hipStream_t st) {
    if (h->bs != 3) return h->fail(DD_EINVAL, "the learned correction needs 3x3 blocks");
    if (!h->factored) return h->fail(DD_ESTATE, "lic_setup before ilu0_factor");
    if (h->slots == 0) return h->fail(DD_EINVAL, "the learned correction needs the slot layout (rows of <= 3 blocks)");
    const int T = 256;
    const unsigned g = (unsigned)((h->n + T - 1) / T);
    Lic &L = h->lic;
    hipError_t e;
    int32_t st6 = 0;
    e = hipMemcpyAsync(h->status + 6, &st6, sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "memcpy: %s", hipGetErrorString(e));
    k_sym_check<<<g, T, 0, st>>>(h->n, h->aptr, h->acol, h->status);
    int32_t *cnt = nullptr, *flag = nullptr, *bpos = nullptr;
    int rc = h->alloc(&cnt, h->n);
    if (!rc) rc = h->alloc(&flag, h->n);
    if (!rc) rc = h->alloc(&bpos, h->n + 1);
    if (!rc && !L.fptr) rc = h->alloc(&L.fptr, h->n + 1);
    if (!rc && !L.diag) rc = h->alloc(&L.diag, h->n);
    if (!rc && !L.bsub) rc = h->alloc(&L.bsub, h->nsub + 1);
    if (rc) return rc;
    k_face_count<<<g, T, 0, st>>>(h->n, h->S, h->aptr, h->acol, cnt);
    e = exclusive_scan(cnt, L.fptr, h->n, h->scan_tmp, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "scan: %s", hipGetErrorString(e));
    int32_t nf = 0, sym = 0;
    e = hipMemcpyAsync(&nf, L.fptr + h->n, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&sym, h->status + 6, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic setup: %s", hipGetErrorString(e));
    if (sym) return h->fail(DD_EINVAL, "the learned correction needs a structurally symmetric pattern");
    L.nf = nf;
    for (void *q : {(void *)L.fI, (void *)L.fJ, (void *)L.fq, (void *)L.X, (void *)L.C, (void *)L.brow})
        if (q) {
            h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), q));
            (void)hipFree(q);
        }
    rc = h->alloc(&L.fI, nf);
    if (!rc) rc = h->alloc(&L.fJ, nf);
    if (!rc) rc = h->alloc(&L.fq, nf);
    if (!rc) rc = h->alloc(&L.X, (int64_t)nf * kIn);
    if (!rc) rc = h->alloc(&L.C, (int64_t)nf * kOut);
    if (rc) return rc;
    k_face_fill<<<g, T, 0, st>>>(h->n, h->S, h->aptr, h->acol, L.fptr, L.fI, L.fJ, L.fq);
    // diagonal position of every row of the full matrix
    k_bflag<<<g, T, 0, st>>>(h->n, L.fptr, flag);
    e = exclusive_scan(flag, bpos, h->n, h->scan_tmp, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "scan: %s", hipGetErrorString(e));
    int32_t nb = 0;
    e = hipMemcpyAsync(&nb, bpos + h->n, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic setup: %s", hipGetErrorString(e));
    L.nb = nb;
    rc = h->alloc(&L.brow, nb);
    if (rc) return rc;
    k_bfill<<<g, T, 0, st>>>(h->n, h->S, L.fptr, bpos, L.brow, L.bsub);
    e = hipMemcpyAsync(L.bsub + h->nsub, &nb, sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return h->fail(DD_EHIP, "memcpy: %s", hipGetErrorString(e));
    hipError_t ed = launch_diag_positions(h, L.diag, st);
    if (ed != hipSuccess) return h->fail(DD_EHIP, "diag: %s", hipGetErrorString(ed));
    if (nf) k_features<<<(unsigned)((nf + T - 1) / T), T, 0, st>>>(nf, L.fI, L.fJ, L.fq, L.diag, h->aval, L.X);
    // adjoint slot streams
    const int bb = 9;
    for (int w = 0; w < 2; ++w) {
        if (!L.adj_val[w]) {
            rc = h->alloc(&L.adj_val[w], h->n * (h->slots + w) * bb);
            if (rc) return rc;
        }
    }
    for (int w = 0; w < 2; ++w)
        k_pack_adjoint<<<g, T, 0, st>>>(h->n, h->S, w, h->slots, h->tptr, h->tcol, h->lu, h->invd,
                                        h->lev[w].rows, L.adj_val[w]);
    e = hipStreamSynchronize(st);
    for (void *q : {(void *)cnt, (void *)flag, (void *)bpos}) {
        h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), q));
        (void)hipFree(q);
    }
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic setup: %s", hipGetErrorString(e));
    L.ready = 1;
    L.active = 0;
    return DD_OK;
}

int lic_coeffs_from_params(dd_ctx *h, const float *params, bool keep_hidden, hipStream_t st) {
    Lic &L = h->lic;
    if (keep_hidden && !L.H1) {
        int rc = h->alloc(&L.H1, (int64_t)std::max(L.nf, 1) * kHid);
        if (!rc) rc = h->alloc(&L.H2, (int64_t)std::max(L.nf, 1) * kHid);
        if (rc) return rc;
    }
    if (L.nf)
        k_mlp_forward<<<(unsigned)((L.nf + 255) / 256), 256, 0, st>>>(L.nf, params, L.X, L.C, keep_hidden ? L.H1 : nullptr,
                                                                     keep_hidden ? L.H2 : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return h->fail(DD_EHIP, "mlp forward: %s", hipGetErrorString(e));
    return DD_OK;
}

// Loss and gradient of one problem (see the file comment); adds to *loss and
// (accumulate != 0) to grad.
int lic_loss_grad_run(dd_ctx *h, const float *params, int Q, const double *R, const double *Zs, const double *den,
                      double *loss, float *grad, int accumulate, hipStream_t st) {
    Lic &L = h->lic;
    const int64_t m = h->n * 3;
    int rc = lic_coeffs_from_params(h, params, true, st);
    if (rc) return rc;
    if (L.work_q < Q) {
        for (void *q : {(void *)L.Z, (void *)L.G, (void *)L.A, (void *)L.rpart})
            if (q) {
                h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), q));
                (void)hipFree(q);
            }
        rc = h->alloc(&L.Z, Q * m);
        if (!rc) rc = h->alloc(&L.G, Q * m);
        if (!rc) rc = h->alloc(&L.A, Q * m);
        if (!rc) rc = h->alloc(&L.rpart, (int64_t)Q * 2048);
        if (rc) return rc;
        L.work_q = Q;
    }
    if (!L.dC) {
        rc = h->alloc(&L.dC, (int64_t)std::max(L.nf, 1) * 9);
        if (!rc) rc = h->alloc(&L.G1, (int64_t)std::max(L.nf, 1) * kHid);
        if (!rc) rc = h->alloc(&L.G2, (int64_t)std::max(L.nf, 1) * kHid);
        const int nchunk = (int)((std::max(L.nf, 1) + kFaceChunk - 1) / kFaceChunk);
        if (!rc) rc = h->alloc(&L.wpart, (int64_t)nchunk * kNParam);
        if (rc) return rc;
    }
    const int32_t saved_prec = h->precision, saved_active = L.active;
    h->precision = DD_FP64;
    L.active = 1;
    hipError_t e = hipSuccess;
    for (int q = 0; q < Q && e == hipSuccess; ++q) e = launch_apply(h, R + q * m, L.Z + q * m, nullptr, st);
    L.active = saved_active;
    const int gres = (int)std::min<int64_t>((m + 255) / 256, 2048);
    if (e == hipSuccess) {
        k_lic_residual<<<dim3(gres, Q), 256, 0, st>>>(m, L.Z, Zs, den, Q, L.G, L.rpart, 2048);
        k_lic_loss<<<1, 1, 0, st>>>(Q, gres, 2048, L.rpart, den, loss);
        e = hipGetLastError();
    }
    for (int q = 0; q < Q && e == hipSuccess; ++q) e = launch_apply_adjoint(h, L.G + q * m, L.A + q * m, st);
    h->precision = saved_prec;
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic applies: %s", hipGetErrorString(e));
    if (L.nf) {
        k_lic_dC<<<(unsigned)((L.nf * 9 + 255) / 256), 256, 0, st>>>(L.nf, m, Q, L.fI, L.fJ, L.A, R, L.dC);
        const unsigned gf = (unsigned)((L.nf + 255) / 256);
        k_mlp_backprop<<<gf, 256, 0, st>>>(L.nf, params, L.dC, L.H1, L.H2, L.G1, L.G2);
        const int nchunk = (int)((L.nf + kFaceChunk - 1) / kFaceChunk);
        k_wgrad_partial<<<dim3(nchunk, 3), 256, 0, st>>>(L.nf, L.dC, L.G2, L.G1, L.H2, L.H1, L.X, L.wpart);
        k_wgrad_sum<<<(kNParam + 255) / 256, 256, 0, st>>>(nchunk, L.wpart, grad, accumulate);
    } else if (!accumulate) {
        e = hipMemsetAsync(grad, 0, kNParam * sizeof(float), st);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic gradient: %s", hipGetErrorString(e));
    return DD_OK;
}

int lic_targets_run(dd_ctx *h, int Q, const double *R, double *Zs, double *den, hipStream_t st) {
    const int64_t m = h->n * 3;
    double *zdd = nullptr;
    int rc = h->alloc(&zdd, Q * m);
    if (rc) return rc;
    const int32_t saved_prec = h->precision;
    const int32_t saved_active = h->lic.active;
    h->precision = DD_FP64;
    h->lic.active = 0;
    hipError_t e = launch_global_apply(h, R, Zs, Q, st);
    for (int q = 0; q < Q && e == hipSuccess; ++q) e = launch_apply(h, R + q * m, zdd + q * m, nullptr, st);
    h->precision = saved_prec;
    h->lic.active = saved_active;
    if (e == hipSuccess) {
        k_lic_den<<<Q, 256, 0, st>>>(m, zdd, Zs, den);
        e = hipStreamSynchronize(st);
    }
    h->allocs.erase(std::find(h->allocs.begin(), h->allocs.end(), (void *)zdd));
    (void)hipFree(zdd);
    if (e != hipSuccess) return h->fail(DD_EHIP, "lic targets: %s", hipGetErrorString(e));
    return DD_OK;
}

hipError_t launch_adam(int np, float *P, const float *G, float *M, float *V, int t, float lr, float b1, float b2,
                       float eps, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    k_adam<<<(np + 255) / 256, 256, 0, st>>>(np, P, G, M, V, c1, c2, lr, b1, b2, eps);
    return hipGetLastError();
}

}  // namespace ddilu
